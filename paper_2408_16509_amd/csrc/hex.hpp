// Hexahedral FR kernels (order P, Gauss--Legendre points), FP64.
//
// Native layout: state u[(pt*5 + v)*E + e] (element fastest, E = padded count),
// traces uf[(fp*5 + v)*E + e], gradients grad[(pt*15 + v*3 + j)*E + e] and
// gradf[(fp*15 + v*3 + j)*E + e].  Solution point pt = i + N1*(j + N1*k); flux point
// fp = face*N1^2 + q, face = 2*d + (xi_d > 0), q = t0 + N1*t1 over the two tangential
// axes of the face in increasing order.
//
// The element kernels work line by line: a line in direction d through the
// solution points (t0, t1) holds the N1 points that the 1-D operators act on, and
// both of its ends are flux points.  Along such a line the corrected divergence
// of eq:FRfinal with the DG correction reduces to
//     div_d = Dh f~_d + cp F^C(+) + cm F^C(-)
// (Dh = D - gR' l(+1)^T - gL' l(-1)^T, cp = gR', cm = -gL'), so the discontinuous
// normal flux at the ends never needs forming.  Each thread owns one line of one
// element per direction pass; the three directions' contributions meet in LDS.
// The geometric map is trilinear and evaluated on the fly from its 24 monomial
// coefficients (metric terms of linear elements computed from the corners).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "physics.hpp"

namespace frmi {

struct HexK {
  double x[5], lm[5], lp[5], Dh[5][5], cp[5], cm[5];
};

struct Conn {
  const int32_t* nbr_elem;   // [6][E]
  const int32_t* nbr_info;   // [6][E] nbr_face | orient << 3 | is_left << 12
  const int32_t* perm;       // [n_orient][stride]
  int32_t perm_stride;
};

// Columns of G = dx/dxi at reference point (a, b, d) of a trilinear map with
// monomial coefficients c[comp*8 + S], S in {1, a, b, d, ab, ad, bd, abd}.
__device__ __forceinline__ void hex_cols(const double* c, double a, double b, double d, double g[3][3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double* q = c + k * 8;
    g[0][k] = q[1] + q[4] * b + q[5] * d + q[7] * b * d;
    g[1][k] = q[2] + q[4] * a + q[6] * d + q[7] * a * d;
    g[2][k] = q[3] + q[5] * a + q[6] * b + q[7] * a * b;
  }
}

__device__ __forceinline__ void cross3(const double* u, const double* v, double* w) {
  w[0] = u[1] * v[2] - u[2] * v[1];
  w[1] = u[2] * v[0] - u[0] * v[2];
  w[2] = u[0] * v[1] - u[1] * v[0];
}

template <int N1>
__device__ __forceinline__ int line_pt(int d, int a, int t0, int t1) {
  return d == 0 ? a + N1 * (t0 + N1 * t1) : (d == 1 ? t0 + N1 * (a + N1 * t1) : t0 + N1 * (t1 + N1 * a));
}

template <int N1>
__device__ __forceinline__ void line_xi(const HexK& K, int d, int a, int t0, int t1, double xi[3]) {
  const double ta = K.x[t0], tb = K.x[t1], xa = K.x[a];
  xi[0] = d == 0 ? xa : ta;
  xi[1] = d == 0 ? ta : (d == 1 ? xa : tb);
  xi[2] = d == 2 ? xa : tb;
}

template <int N1>
__device__ __forceinline__ void end_xi(const HexK& K, int d, int s, int t0, int t1, double xi[3]) {
  const double ta = K.x[t0], tb = K.x[t1], xe = s ? 1.0 : -1.0;
  xi[0] = d == 0 ? xe : ta;
  xi[1] = d == 0 ? ta : (d == 1 ? xe : tb);
  xi[2] = d == 2 ? xe : tb;
}

// S row d = g_{d+1} x g_{d+2}: row d of J G^{-1}.
__device__ __forceinline__ void srow(const double g[3][3], int d, double s[3]) {
  if (d == 0) cross3(g[1], g[2], s);
  else if (d == 1) cross3(g[2], g[0], s);
  else cross3(g[0], g[1], s);
}

// Neighbour flux-point slot of end s of line (d, q) of element e.
struct NbrSlot {
  int64_t elem;
  int fp;
  bool left;
};

template <int N1>
__device__ __forceinline__ NbrSlot nbr_slot(const Conn& C, int64_t E, int64_t e, int face, int q) {
  const int info = C.nbr_info[(int64_t)face * E + e];
  NbrSlot s;
  s.elem = C.nbr_elem[(int64_t)face * E + e];
  const int nf = info & 7, orient = (info >> 3) & 511;
  s.left = (info >> 12) & 1;
  s.fp = nf * N1 * N1 + C.perm[orient * C.perm_stride + q];
  return s;
}

// ---------------------------------------------------------------------------
// Step 1 (eq:disu) at the flux points: traces of u at both ends of every line.
template <int P>
__global__ void __launch_bounds__(256) hex_trace(const double* __restrict__ u, double* __restrict__ uf,
                                                 int64_t E, HexK K) {
  constexpr int N1 = P + 1, NL = 3 * N1 * N1;
  const int64_t gtid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t wave = gtid >> 6;
  const int lane = (int)(gtid & 63);
  const int64_t tile = wave / NL;
  const int l = (int)(wave % NL);
  const int64_t e = tile * 64 + lane;
  if (e >= E) return;
  const int d = l / (N1 * N1), q = l % (N1 * N1), t0 = q % N1, t1 = q / N1;
  double m[5] = {0, 0, 0, 0, 0}, p[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int a = 0; a < N1; ++a) {
    const int pt = line_pt<N1>(d, a, t0, t1);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double val = u[((int64_t)pt * 5 + v) * E + e];
      m[v] += K.lm[a] * val;
      p[v] += K.lp[a] * val;
    }
  }
  const int fm = (2 * d) * N1 * N1 + q, fp = (2 * d + 1) * N1 * N1 + q;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    uf[((int64_t)fm * 5 + v) * E + e] = m[v];
    uf[((int64_t)fp * 5 + v) * E + e] = p[v];
  }
}

// ---------------------------------------------------------------------------
// Steps 2-4 for Euler, fused: per line, own traces, neighbour traces, common flux
// (eq:comm_flux) at both ends, transformed flux at the line points and the
// corrected divergence (eq:FRfinal); R = -div / J.
template <int P, int NE>
__global__ void __launch_bounds__(NE*(P + 1)*(P + 1)) hex_div_euler(
    const double* __restrict__ u, const double* __restrict__ uf, const double* __restrict__ geo,
    Conn C, double* __restrict__ r, int64_t E, int64_t n, HexK K, Phys ph) {
  constexpr int N1 = P + 1, NSP = N1 * N1 * N1;
  __shared__ double DIV[5 * NSP * NE];
  const int el = threadIdx.x % NE, l = threadIdx.x / NE;
  const int64_t e = (int64_t)blockIdx.x * NE + el;
  const int t0 = l % N1, t1 = l / N1;
  double c[24];
#pragma unroll
  for (int g = 0; g < 24; ++g) c[g] = geo[(int64_t)g * E + e];
  const double gam = ph.gamma, gm1 = ph.gamma - 1.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double ft[5][N1], tm[5] = {0, 0, 0, 0, 0}, tp[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < N1; ++a) {
      const int pt = line_pt<N1>(d, a, t0, t1);
      double uu[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        uu[v] = u[((int64_t)pt * 5 + v) * E + e];
        tm[v] += K.lm[a] * uu[v];
        tp[v] += K.lp[a] * uu[v];
      }
      double xi[3], g[3][3], s[3], f[5], vs, pr;
      line_xi<N1>(K, d, a, t0, t1, xi);
      hex_cols(c, xi[0], xi[1], xi[2], g);
      srow(g, d, s);
      flux_dir(uu, s[0], s[1], s[2], gm1, f, vs, pr);
#pragma unroll
      for (int v = 0; v < 5; ++v) ft[v][a] = f[v];
    }
    double Fc[2][5];
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      double xi[3], g[3][3], nv[3];
      end_xi<N1>(K, d, sd, t0, t1, xi);
      hex_cols(c, xi[0], xi[1], xi[2], g);
      srow(g, d, nv);
      const double sg = sd ? 1.0 : -1.0;
      const double mag = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
      const int face = 2 * d + sd;
      const NbrSlot ns = nbr_slot<N1>(C, E, e, face, l);
      double un[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) un[v] = uf[((int64_t)ns.fp * 5 + v) * E + ns.elem];
      const double* own = sd ? tp : tm;
      double uL[5], uR[5], nL[3], F[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) { uL[v] = ns.left ? own[v] : un[v]; uR[v] = ns.left ? un[v] : own[v]; }
      const double sl = (ns.left ? sg : -sg) / mag;
#pragma unroll
      for (int k = 0; k < 3; ++k) nL[k] = nv[k] * sl;
      riemann(ph.riemann, uL, uR, nL, gam, F);
      const double fs = ns.left ? mag : -mag;
#pragma unroll
      for (int v = 0; v < 5; ++v) Fc[sd][v] = fs * F[v];
    }
#pragma unroll
    for (int a = 0; a < N1; ++a) {
      const int pt = line_pt<N1>(d, a, t0, t1);
      double div[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        double acc = K.cp[a] * Fc[1][v] + K.cm[a] * Fc[0][v];
#pragma unroll
        for (int b = 0; b < N1; ++b) acc += K.Dh[a][b] * ft[v][b];
        div[v] = acc;
      }
      double* D = DIV + (pt * NE + el);
      if (d == 0) {
#pragma unroll
        for (int v = 0; v < 5; ++v) D[v * NSP * NE] = div[v];
      } else if (d == 1) {
#pragma unroll
        for (int v = 0; v < 5; ++v) D[v * NSP * NE] += div[v];
      } else {
        double xi[3], g[3][3], s[3];
        line_xi<N1>(K, d, a, t0, t1, xi);
        hex_cols(c, xi[0], xi[1], xi[2], g);
        cross3(g[1], g[2], s);
        const double iJ = -1.0 / (g[0][0] * s[0] + g[0][1] * s[1] + g[0][2] * s[2]);
        if (e < n) {
#pragma unroll
          for (int v = 0; v < 5; ++v) r[((int64_t)pt * 5 + v) * E + e] = (D[v * NSP * NE] + div[v]) * iJ;
        }
      }
    }
    if (d < 2) __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Navier--Stokes phase 1: corrected gradient (LDG common solution u^ at the
// flux points), physical gradient at the solution points, and its traces.
template <int P, int NE>
__global__ void __launch_bounds__(NE*(P + 1)*(P + 1)) hex_grad(
    const double* __restrict__ u, const double* __restrict__ uf, const double* __restrict__ geo,
    Conn C, double* __restrict__ grad, double* __restrict__ gradf, int64_t E, HexK K, Phys ph) {
  constexpr int N1 = P + 1, NSP = N1 * N1 * N1, NF = N1 * N1;
  __shared__ double GR[3 * NSP * NE];
  const int el = threadIdx.x % NE, l = threadIdx.x / NE;
  const int64_t e = (int64_t)blockIdx.x * NE + el;
  const int t0 = l % N1, t1 = l / N1;
  double c[24];
#pragma unroll
  for (int g = 0; g < 24; ++g) c[g] = geo[(int64_t)g * E + e];
  const double beta = ph.beta;
  for (int v = 0; v < 5; ++v) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double uv[N1], tm = 0, tp = 0;
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        uv[a] = u[((int64_t)line_pt<N1>(d, a, t0, t1) * 5 + v) * E + e];
        tm += K.lm[a] * uv[a];
        tp += K.lp[a] * uv[a];
      }
      double uh[2];
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        const NbrSlot ns = nbr_slot<N1>(C, E, e, 2 * d + sd, l);
        const double un = uf[((int64_t)ns.fp * 5 + v) * E + ns.elem];
        const double own = sd ? tp : tm;
        const double uL = ns.left ? own : un, uR = ns.left ? un : own;
        uh[sd] = 0.5 * (uL + uR) + beta * (uL - uR);
      }
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        double gt = K.cp[a] * uh[1] - K.cm[a] * uh[0];
#pragma unroll
        for (int b = 0; b < N1; ++b) gt += K.Dh[a][b] * uv[b];
        double xi[3], g[3][3], s[3], cr[3];
        line_xi<N1>(K, d, a, t0, t1, xi);
        hex_cols(c, xi[0], xi[1], xi[2], g);
        srow(g, d, s);
        cross3(g[1], g[2], cr);
        const double sc = gt / (g[0][0] * cr[0] + g[0][1] * cr[1] + g[0][2] * cr[2]);
        const int pt = line_pt<N1>(d, a, t0, t1);
        double* G = GR + (pt * NE + el);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          if (d == 0) G[j * NSP * NE] = s[j] * sc;
          else G[j * NSP * NE] += s[j] * sc;
        }
      }
      __syncthreads();
    }
    // gradient at the solution points of this thread's column, then traces
#pragma unroll
    for (int a = 0; a < N1; ++a) {
      const int pt = line_pt<N1>(2, a, t0, t1);
#pragma unroll
      for (int j = 0; j < 3; ++j) grad[((int64_t)pt * 15 + v * 3 + j) * E + e] = GR[(j * NSP + pt) * NE + el];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double gm[3] = {0, 0, 0}, gp[3] = {0, 0, 0};
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        const int pt = line_pt<N1>(d, a, t0, t1);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const double val = GR[(j * NSP + pt) * NE + el];
          gm[j] += K.lm[a] * val;
          gp[j] += K.lp[a] * val;
        }
      }
      const int fm = 2 * d * NF + l, fp = (2 * d + 1) * NF + l;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        gradf[((int64_t)fm * 15 + v * 3 + j) * E + e] = gm[j];
        gradf[((int64_t)fp * 15 + v * 3 + j) * E + e] = gp[j];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Navier--Stokes phase 2: f = f_inv - f_v at the solution points, LDG common
// flux (inviscid Riemann flux minus the switched viscous flux plus the penalty)
// at the line ends, corrected divergence.
template <int P, int NE>
__global__ void __launch_bounds__(NE*(P + 1)*(P + 1)) hex_div_ns(
    const double* __restrict__ u, const double* __restrict__ uf, const double* __restrict__ grad,
    const double* __restrict__ gradf, const double* __restrict__ geo, Conn C, double* __restrict__ r,
    int64_t E, int64_t n, HexK K, Phys ph) {
  constexpr int N1 = P + 1, NSP = N1 * N1 * N1;
  __shared__ double DIV[5 * NSP * NE];
  const int el = threadIdx.x % NE, l = threadIdx.x / NE;
  const int64_t e = (int64_t)blockIdx.x * NE + el;
  const int t0 = l % N1, t1 = l / N1;
  double c[24];
#pragma unroll
  for (int g = 0; g < 24; ++g) c[g] = geo[(int64_t)g * E + e];
  const double gam = ph.gamma, gm1 = ph.gamma - 1.0, mu = ph.mu, pr = ph.prandtl;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double ft[5][N1], tm[5] = {0, 0, 0, 0, 0}, tp[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < N1; ++a) {
      const int pt = line_pt<N1>(d, a, t0, t1);
      double uu[5], gg[15];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        uu[v] = u[((int64_t)pt * 5 + v) * E + e];
        tm[v] += K.lm[a] * uu[v];
        tp[v] += K.lp[a] * uu[v];
      }
#pragma unroll
      for (int k = 0; k < 15; ++k) gg[k] = grad[((int64_t)pt * 15 + k) * E + e];
      double xi[3], g[3][3], s[3], f[5], fv[5], vs, prs;
      line_xi<N1>(K, d, a, t0, t1, xi);
      hex_cols(c, xi[0], xi[1], xi[2], g);
      srow(g, d, s);
      flux_dir(uu, s[0], s[1], s[2], gm1, f, vs, prs);
      viscous_dir(uu, gg, s[0], s[1], s[2], gam, mu, pr, fv);
#pragma unroll
      for (int v = 0; v < 5; ++v) ft[v][a] = f[v] - fv[v];
    }
    double Fc[2][5];
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      double xi[3], g[3][3], nv[3];
      end_xi<N1>(K, d, sd, t0, t1, xi);
      hex_cols(c, xi[0], xi[1], xi[2], g);
      srow(g, d, nv);
      const double sg = sd ? 1.0 : -1.0;
      const double mag = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
      const int face = 2 * d + sd;
      const int fown = face * N1 * N1 + l;
      const NbrSlot ns = nbr_slot<N1>(C, E, e, face, l);
      double un[5], gn[15], go[15];
#pragma unroll
      for (int v = 0; v < 5; ++v) un[v] = uf[((int64_t)ns.fp * 5 + v) * E + ns.elem];
#pragma unroll
      for (int k = 0; k < 15; ++k) {
        gn[k] = gradf[((int64_t)ns.fp * 15 + k) * E + ns.elem];
        go[k] = gradf[((int64_t)fown * 15 + k) * E + e];
      }
      const double* own = sd ? tp : tm;
      double uL[5], uR[5], gL[15], gR[15], nL[3], F[5], fvL[5], fvR[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) { uL[v] = ns.left ? own[v] : un[v]; uR[v] = ns.left ? un[v] : own[v]; }
#pragma unroll
      for (int k = 0; k < 15; ++k) { gL[k] = ns.left ? go[k] : gn[k]; gR[k] = ns.left ? gn[k] : go[k]; }
      const double sl = (ns.left ? sg : -sg) / mag;
#pragma unroll
      for (int k = 0; k < 3; ++k) nL[k] = nv[k] * sl;
      riemann(ph.riemann, uL, uR, nL, gam, F);
      viscous_dir(uL, gL, nL[0], nL[1], nL[2], gam, mu, pr, fvL);
      viscous_dir(uR, gR, nL[0], nL[1], nL[2], gam, mu, pr, fvR);
      const double fs = ns.left ? mag : -mag;
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const double fvc = 0.5 * (fvL[v] + fvR[v]) - ph.beta * (fvL[v] - fvR[v]);
        Fc[sd][v] = fs * (F[v] - fvc + ph.tau * (uL[v] - uR[v]));
      }
    }
#pragma unroll
    for (int a = 0; a < N1; ++a) {
      const int pt = line_pt<N1>(d, a, t0, t1);
      double div[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        double acc = K.cp[a] * Fc[1][v] + K.cm[a] * Fc[0][v];
#pragma unroll
        for (int b = 0; b < N1; ++b) acc += K.Dh[a][b] * ft[v][b];
        div[v] = acc;
      }
      double* D = DIV + (pt * NE + el);
      if (d == 0) {
#pragma unroll
        for (int v = 0; v < 5; ++v) D[v * NSP * NE] = div[v];
      } else if (d == 1) {
#pragma unroll
        for (int v = 0; v < 5; ++v) D[v * NSP * NE] += div[v];
      } else {
        double xi[3], g[3][3], s[3];
        line_xi<N1>(K, d, a, t0, t1, xi);
        hex_cols(c, xi[0], xi[1], xi[2], g);
        cross3(g[1], g[2], s);
        const double iJ = -1.0 / (g[0][0] * s[0] + g[0][1] * s[1] + g[0][2] * s[2]);
        if (e < n) {
#pragma unroll
          for (int v = 0; v < 5; ++v) r[((int64_t)pt * 5 + v) * E + e] = (D[v * NSP * NE] + div[v]) * iJ;
        }
      }
    }
    if (d < 2) __syncthreads();
  }
}

}  // namespace frmi
