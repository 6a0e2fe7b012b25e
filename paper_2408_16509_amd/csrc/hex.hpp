// Hexahedral FR kernels (order P, Gauss--Legendre points).
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
// normal flux at the ends never needs forming.  In the trace, Euler and gradient
// kernels each thread owns one line of one element per direction pass and the three
// directions' contributions meet in LDS; the NS divergence gives each thread one
// column of points and pulls the three line contractions through its points from LDS.
// The geometric map is trilinear and evaluated on the fly from its 24 monomial
// coefficients (metric terms of linear elements computed from the corners),
// staged per block in LDS.  Curved elements (CUR = true) instead read metric terms
// stored per point (Sec. "Curved elements"), layout cm (element fastest):
//   cm[(pt*9 + d*3 + j)*E + e]      row d of S = J G^{-1} at solution point pt
//   cm[(9*NSP + pt)*E + e]          1/J at solution point pt
//   cm[(10*NSP + fp*3 + j)*E + e]   row d of S at flux point fp of face 2d+s
//
// Arithmetic type T: double (the plain form) or float.  In the float form the
// state is the deviation du = u - u_ref from a constant state at rest and every
// flux is evaluated as f(u) - f(u_ref) in cancellation-free form (Flux<T, DEV>);
// this changes nothing in exact arithmetic because the transformed flux of a
// constant state has zero discrete divergence and zero interface jump.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "physics.hpp"

namespace frmi {

// Workgroups of a launch are dispatched round-robin over the 8 XCDs, each with its
// own L2.  Renumber them so that every XCD works through one contiguous range of
// logical blocks: blocks that read the same cache lines (neighbouring element tiles,
// the lines of one tile) then meet in the same L2 instead of fetching from HBM once
// per XCD.  A bijection on [0, gridDim.x).
__device__ __forceinline__ int64_t xcd_block() {
  const uint32_t b = blockIdx.x, nb = gridDim.x;
  const uint32_t x = b & 7u, i = b >> 3, q = nb >> 3, r = nb & 7u;
  return (int64_t)x * q + (x < r ? x : r) + i;
}

template <typename T>
struct HexK {
  T x[5], lm[5], lp[5], Dh[5][5], cp[5], cm[5];
};

// Reference state of the deviation form (at rest): rho0, E0, p0 = (gamma-1)E0, H0 = E0 + p0.
template <typename T>
struct RefState {
  T rho0, E0, p0, H0;
};

struct Conn {
  const int32_t* nbr_elem;   // [nfaces][E]
  const int32_t* nbr_info;   // [nfaces][E] nbr_face | orient << 3 | is_left << 12
  const int32_t* perm;       // [n_orient][stride]
  int32_t perm_stride;
};

// Inviscid flux along s and the quantities the Riemann solvers need.  DEV: the
// state holds du and the flux returned is f(u).s - f(u_ref).s.
template <typename T, bool DEV>
struct Flux {
  __device__ __forceinline__ static void eval(const T w[5], T sx, T sy, T sz, T gm1, const RefState<T>& R,
                                              T f[5], T& vs, T& p_full) {
    if constexpr (!DEV) {
      flux_dir(w, sx, sy, sz, gm1, f, vs, p_full);
    } else {
      const T rho = R.rho0 + w[0];
      const T ir = rcp(rho);
      const T vx = w[1] * ir, vy = w[2] * ir, vz = w[3] * ir;
      const T dp = gm1 * (w[4] - T(0.5) * (w[1] * vx + w[2] * vy + w[3] * vz));
      vs = vx * sx + vy * sy + vz * sz;
      f[0] = w[1] * sx + w[2] * sy + w[3] * sz;
      f[1] = w[1] * vs + dp * sx;
      f[2] = w[2] * vs + dp * sy;
      f[3] = w[3] * vs + dp * sz;
      f[4] = (R.H0 + w[4] + dp) * vs;
      p_full = R.p0 + dp;
    }
  }
  __device__ __forceinline__ static T rho(const T w[5], const RefState<T>& R) {
    if constexpr (DEV) return R.rho0 + w[0];
    else return w[0];
  }
};

// Rusanov / HLLC on (possibly deviation) states.  In the deviation form the
// constant f(u_ref).n is subtracted, which leaves every solver's formula intact
// because solvers are consistent (𝔉(u, u, n) = f(u).n).
template <typename T, bool DEV>
__device__ __forceinline__ void common_inviscid(int kind, const T uL[5], const T uR[5], const T n[3], T gamma,
                                                const RefState<T>& R, T F[5]) {
  const T gm1 = gamma - T(1);
  T fL[5], fR[5], vnL, vnR, pL, pR;
  Flux<T, DEV>::eval(uL, n[0], n[1], n[2], gm1, R, fL, vnL, pL);
  Flux<T, DEV>::eval(uR, n[0], n[1], n[2], gm1, R, fR, vnR, pR);
  const T rL = Flux<T, DEV>::rho(uL, R), rR = Flux<T, DEV>::rho(uR, R);
  const T cL = fsqrt(fdiv(gamma * pL, rL)), cR = fsqrt(fdiv(gamma * pR, rR));
  if (kind != 1) {
    const T lam = fmax(fabs(vnL) + cL, fabs(vnR) + cR);
#pragma unroll
    for (int v = 0; v < 5; ++v) F[v] = T(0.5) * (fL[v] + fR[v]) - T(0.5) * lam * (uR[v] - uL[v]);
    return;
  }
  const T SL = fmin(vnL - cL, vnR - cR);
  const T SR = fmax(vnL + cL, vnR + cR);
  // pR - pL from the deviation pressures in the float form (same value in exact arithmetic)
  const T dpLR = pR - pL;
  const T Ss = fdiv(dpLR + rL * vnL * (SL - vnL) - rR * vnR * (SR - vnR), rL * (SL - vnL) - rR * (SR - vnR));
  if (T(0) <= SL) {
#pragma unroll
    for (int v = 0; v < 5; ++v) F[v] = fL[v];
    return;
  }
  const bool left = T(0) <= Ss;
  if (!left && !(T(0) < SR)) {
#pragma unroll
    for (int v = 0; v < 5; ++v) F[v] = fR[v];
    return;
  }
  const T* wK = left ? uL : uR;
  const T* fK = left ? fL : fR;
  const T S = left ? SL : SR, vn = left ? vnL : vnR, p = left ? pL : pR, r = left ? rL : rR;
  // U*_K - U_K written without forming U*_K (no cancellation of the total energy):
  //   mass: r (Ss - vn)/(S - Ss); momentum: that times v + fac (Ss - vn) n;
  //   energy: (Ss - vn)/(S - Ss) [r (S - vn) Ss + p + E]
  const T fac = fdiv(r * (S - vn), S - Ss);
  const T q = fdiv(Ss - vn, S - Ss);
  const T E = DEV ? R.E0 + wK[4] : wK[4];
  T dU[5];
  dU[0] = r * q;
  dU[1] = wK[1] * q + fac * (Ss - vn) * n[0];
  dU[2] = wK[2] * q + fac * (Ss - vn) * n[1];
  dU[3] = wK[3] * q + fac * (Ss - vn) * n[2];
  dU[4] = q * (r * (S - vn) * Ss + p + E);
#pragma unroll
  for (int v = 0; v < 5; ++v) F[v] = fK[v] + S * dU[v];
}

// Viscous flux along s from (possibly deviation) state and its gradient.
template <typename T, bool DEV>
__device__ __forceinline__ void viscous(const T w[5], const T g[15], T sx, T sy, T sz, T gamma, T mu, T pr,
                                        const RefState<T>& R, T fv[5]) {
  T u[5] = {w[0], w[1], w[2], w[3], w[4]};
  if constexpr (DEV) { u[0] += R.rho0; u[4] += R.E0; }
  viscous_dir(u, g, sx, sy, sz, gamma, mu, pr, fv);
}

// Navier--Stokes flux of one solution point along several directions s:
// (f_inv - f_v).s.  The velocity, (deviation) pressure and enthalpy, the viscous stress
// tau and the energy flux vector tau v + kappa grad e are formed once per point (the same
// formulas as Flux::eval and viscous_dir); each direction then costs a few products.
template <typename T, bool DEV>
struct PointFluxNS {
  T m[3], vx, vy, vz, dp, h;       // momentum, velocity, (deviation) pressure, (deviation) H v factor
  T tau[6], qe[3];                 // tau_xx, tau_yy, tau_zz, tau_xy, tau_xz, tau_yz; energy flux vector
  __device__ __forceinline__ PointFluxNS(const T w[5], const T g[15], T gamma, T mu, T pr, const RefState<T>& R) {
    const T gm1 = gamma - T(1);
    const T rho = DEV ? R.rho0 + w[0] : w[0];
    const T Et = DEV ? R.E0 + w[4] : w[4];
    const T ir = rcp(rho);
    m[0] = w[1]; m[1] = w[2]; m[2] = w[3];
    vx = w[1] * ir; vy = w[2] * ir; vz = w[3] * ir;
    dp = gm1 * (w[4] - T(0.5) * (w[1] * vx + w[2] * vy + w[3] * vz));
    // DEV: (H0 + dE + dp) multiplies v.s (f(u).s - f(u_ref).s); else (E + p)
    h = DEV ? R.H0 + w[4] + dp : w[4] + dp;
    const T v[3] = {vx, vy, vz};
    T gv[3][3];                                   // gv[i][j] = d v_i / d x_j
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) gv[i][j] = (g[(1 + i) * 3 + j] - v[i] * g[j]) * ir;
    const T Er = Et * ir;
    T ge[3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
      ge[j] = (g[12 + j] - Er * g[j] - (w[1] * gv[0][j] + w[2] * gv[1][j] + w[3] * gv[2][j])) * ir;
    const T div = gv[0][0] + gv[1][1] + gv[2][2];
    const T d23 = T(2.0 / 3.0) * div;
    tau[0] = mu * (T(2) * gv[0][0] - d23);
    tau[1] = mu * (T(2) * gv[1][1] - d23);
    tau[2] = mu * (T(2) * gv[2][2] - d23);
    tau[3] = mu * (gv[0][1] + gv[1][0]);
    tau[4] = mu * (gv[0][2] + gv[2][0]);
    tau[5] = mu * (gv[1][2] + gv[2][1]);
    const T kappa = fdiv(mu * gamma, pr);
    qe[0] = tau[0] * vx + tau[3] * vy + tau[4] * vz + kappa * ge[0];
    qe[1] = tau[3] * vx + tau[1] * vy + tau[5] * vz + kappa * ge[1];
    qe[2] = tau[4] * vx + tau[5] * vy + tau[2] * vz + kappa * ge[2];
  }
  __device__ __forceinline__ void dir(T sx, T sy, T sz, T f[5]) const {
    const T vs = vx * sx + vy * sy + vz * sz;
    f[0] = DEV ? m[0] * sx + m[1] * sy + m[2] * sz : (m[0] * sx + m[1] * sy + m[2] * sz);
    f[1] = m[0] * vs + dp * sx - (tau[0] * sx + tau[3] * sy + tau[4] * sz);
    f[2] = m[1] * vs + dp * sy - (tau[3] * sx + tau[1] * sy + tau[5] * sz);
    f[3] = m[2] * vs + dp * sz - (tau[4] * sx + tau[5] * sy + tau[2] * sz);
    f[4] = h * vs - (qe[0] * sx + qe[1] * sy + qe[2] * sz);
  }
  // the viscous part alone, f_v.s, without its zero mass component (4 values)
  __device__ __forceinline__ void visc(T sx, T sy, T sz, T fv[4]) const {
    fv[0] = tau[0] * sx + tau[3] * sy + tau[4] * sz;
    fv[1] = tau[3] * sx + tau[1] * sy + tau[5] * sz;
    fv[2] = tau[4] * sx + tau[5] * sy + tau[2] * sz;
    fv[3] = qe[0] * sx + qe[1] * sy + qe[2] * sz;
  }
};

// The inviscid part of PointFluxNS: f_inv.s along several directions of one point.
template <typename T, bool DEV>
struct PointInv {
  T m[3], vx, vy, vz, dp, h;
  __device__ __forceinline__ PointInv(const T w[5], T gamma, const RefState<T>& R) {
    const T gm1 = gamma - T(1);
    const T rho = DEV ? R.rho0 + w[0] : w[0];
    const T ir = rcp(rho);
    m[0] = w[1]; m[1] = w[2]; m[2] = w[3];
    vx = w[1] * ir; vy = w[2] * ir; vz = w[3] * ir;
    dp = gm1 * (w[4] - T(0.5) * (w[1] * vx + w[2] * vy + w[3] * vz));
    h = DEV ? R.H0 + w[4] + dp : w[4] + dp;
  }
  __device__ __forceinline__ void dir(T sx, T sy, T sz, T f[5]) const {
    const T vs = vx * sx + vy * sy + vz * sz;
    f[0] = m[0] * sx + m[1] * sy + m[2] * sz;
    f[1] = m[0] * vs + dp * sx;
    f[2] = m[1] * vs + dp * sy;
    f[3] = m[2] * vs + dp * sz;
    f[4] = h * vs;
  }
};

// Columns of G = dx/dxi at reference point (a, b, d) of a trilinear map with
// monomial coefficients c[comp*8 + S], S in {1, a, b, d, ab, ad, bd, abd}; c is
// read through the stride `cs` (LDS staging).
template <typename T>
__device__ __forceinline__ void hex_cols(const T* c, int cs, T a, T b, T d, T g[3][3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T* q = c + k * 8 * cs;
    const T q1 = q[1 * cs], q2 = q[2 * cs], q3 = q[3 * cs], q4 = q[4 * cs];
    const T q5 = q[5 * cs], q6 = q[6 * cs], q7 = q[7 * cs];
    g[0][k] = q1 + q4 * b + q5 * d + q7 * b * d;
    g[1][k] = q2 + q4 * a + q6 * d + q7 * a * d;
    g[2][k] = q3 + q5 * a + q6 * b + q7 * a * b;
  }
}

template <typename T>
__device__ __forceinline__ void cross3(const T* u, const T* v, T* w) {
  w[0] = u[1] * v[2] - u[2] * v[1];
  w[1] = u[2] * v[0] - u[0] * v[2];
  w[2] = u[0] * v[1] - u[1] * v[0];
}

template <int N1>
__device__ __forceinline__ int line_pt(int d, int a, int t0, int t1) {
  return d == 0 ? a + N1 * (t0 + N1 * t1) : (d == 1 ? t0 + N1 * (a + N1 * t1) : t0 + N1 * (t1 + N1 * a));
}

template <typename T>
__device__ __forceinline__ void line_xi(const HexK<T>& K, int d, int a, int t0, int t1, T xi[3]) {
  const T ta = K.x[t0], tb = K.x[t1], xa = K.x[a];
  xi[0] = d == 0 ? xa : ta;
  xi[1] = d == 0 ? ta : (d == 1 ? xa : tb);
  xi[2] = d == 2 ? xa : tb;
}

template <typename T>
__device__ __forceinline__ void end_xi(const HexK<T>& K, int d, int s, int t0, int t1, T xi[3]) {
  const T ta = K.x[t0], tb = K.x[t1], xe = s ? T(1) : T(-1);
  xi[0] = d == 0 ? xe : ta;
  xi[1] = d == 0 ? ta : (d == 1 ? xe : tb);
  xi[2] = d == 2 ? xe : tb;
}

// S row d = g_{d+1} x g_{d+2}: row d of J G^{-1}.
template <typename T>
__device__ __forceinline__ void srow(const T g[3][3], int d, T s[3]) {
  if (d == 0) cross3(g[1], g[2], s);
  else if (d == 1) cross3(g[2], g[0], s);
  else cross3(g[0], g[1], s);
}

template <typename T>
__device__ __forceinline__ T det_cols(const T g[3][3]) {
  T cr[3];
  cross3(g[1], g[2], cr);
  return g[0][0] * cr[0] + g[0][1] * cr[1] + g[0][2] * cr[2];
}

// Neighbour flux-point slot of end `face` / face-local point q of element e.
struct NbrSlot {
  int64_t elem;
  int fp;
  bool left;
};

template <int NFPF>
__device__ __forceinline__ NbrSlot nbr_slot(const Conn& C, int64_t E, int64_t e, int face, int q) {
  const int info = C.nbr_info[(int64_t)face * E + e];
  NbrSlot s;
  s.elem = C.nbr_elem[(int64_t)face * E + e];
  const int nf = info & 7, orient = (info >> 3) & 511;
  s.left = (info >> 12) & 1;
  s.fp = nf * NFPF + C.perm[orient * C.perm_stride + q];
  return s;
}

template <typename T, int NSP>
__device__ __forceinline__ void cm_srow(const T* __restrict__ cm, int64_t E, int64_t e, int pt, int d, T s[3]) {
#pragma unroll
  for (int j = 0; j < 3; ++j) s[j] = cm[((int64_t)pt * 9 + d * 3 + j) * E + e];
}

template <typename T, int NSP>
__device__ __forceinline__ T cm_rjac(const T* __restrict__ cm, int64_t E, int64_t e, int pt) {
  return cm[((int64_t)9 * NSP + pt) * E + e];
}

template <typename T, int NSP>
__device__ __forceinline__ void cm_fnrm(const T* __restrict__ cm, int64_t E, int64_t e, int fp, T s[3]) {
#pragma unroll
  for (int j = 0; j < 3; ++j) s[j] = cm[((int64_t)10 * NSP + fp * 3 + j) * E + e];
}

// Stage the block's geometry coefficients into LDS: G[g*NE + el].
template <typename T, int NE, int NT>
__device__ __forceinline__ void stage_geo(const T* __restrict__ geo, int64_t E, int64_t e0, T* G) {
  for (int i = threadIdx.x; i < 24 * NE; i += NT) {
    const int g = i / NE, el = i % NE;
    G[i] = geo[(int64_t)g * E + e0 + el];
  }
}

// ---------------------------------------------------------------------------
// Step 1 (eq:disu) at the flux points: traces of u at both ends of every line.
template <typename T, int P>
__global__ void __launch_bounds__(256) hex_trace(const T* __restrict__ u, T* __restrict__ uf, int64_t E, HexK<T> K) {
  constexpr int N1 = P + 1, NL = 3 * N1 * N1;
  const int64_t gtid = xcd_block() * 256 + threadIdx.x;
  const int64_t wave = gtid >> 6;
  const int lane = (int)(gtid & 63);
  const int64_t tile = wave / NL;
  const int l = (int)(wave % NL);
  const int64_t e = tile * 64 + lane;
  if (e >= E) return;
  const int d = l / (N1 * N1), q = l % (N1 * N1), t0 = q % N1, t1 = q / N1;
  T m[5] = {0, 0, 0, 0, 0}, p[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int a = 0; a < N1; ++a) {
    const int pt = line_pt<N1>(d, a, t0, t1);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const T val = u[((int64_t)pt * 5 + v) * E + e];
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

// Accumulate one direction's divergence contribution into LDS and, in the last
// pass, write R = -div / J.
template <typename T, int N1, int NE, bool CUR>
__device__ __forceinline__ void accumulate_div(int d, const T (&ft)[5][N1], const T (&Fc)[2][5], const HexK<T>& K,
                                               T* DIV, const T* G, const T* __restrict__ cm, int el, int t0, int t1,
                                               int64_t e, int64_t n, int64_t E, T* __restrict__ r) {
  constexpr int NSP = N1 * N1 * N1;
#pragma unroll
  for (int a = 0; a < N1; ++a) {
    const int pt = line_pt<N1>(d, a, t0, t1);
    T div[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      T acc = K.cp[a] * Fc[1][v] + K.cm[a] * Fc[0][v];
#pragma unroll
      for (int b = 0; b < N1; ++b) acc += K.Dh[a][b] * ft[v][b];
      div[v] = acc;
    }
    T* D = DIV + (pt * NE + el);
    if (d == 0) {
#pragma unroll
      for (int v = 0; v < 5; ++v) D[v * NSP * NE] = div[v];
    } else if (d == 1) {
#pragma unroll
      for (int v = 0; v < 5; ++v) D[v * NSP * NE] += div[v];
    } else {
      T iJ;
      if constexpr (CUR) {
        iJ = -cm_rjac<T, NSP>(cm, E, e, pt);
      } else {
        T xi[3], g[3][3];
        line_xi(K, d, a, t0, t1, xi);
        hex_cols(G + el, NE, xi[0], xi[1], xi[2], g);
        iJ = -rcp(det_cols(g));
      }
      if (e < n) {
#pragma unroll
        for (int v = 0; v < 5; ++v) r[((int64_t)pt * 5 + v) * E + e] = (D[v * NSP * NE] + div[v]) * iJ;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Steps 2-4 for Euler, fused: per line, own traces, neighbour traces, common flux
// (eq:comm_flux) at both ends, transformed flux at the line points and the
// corrected divergence (eq:FRfinal); R = -div / J.
template <typename T, bool DEV, int P, int NE, bool CUR = false>
__global__ void __launch_bounds__(NE*(P + 1)*(P + 1)) hex_div_euler(
    const T* __restrict__ u, const T* __restrict__ uf, const T* __restrict__ geo, const T* __restrict__ cm,
    Conn C, T* __restrict__ r, int64_t E, int64_t n, HexK<T> K, T gamma, int riemann, RefState<T> R) {
  constexpr int N1 = P + 1, NSP = N1 * N1 * N1, NF = N1 * N1, NT = NE * N1 * N1;
  __shared__ T DIV[5 * NSP * NE];
  __shared__ T G[CUR ? 1 : 24 * NE];
  const int el = threadIdx.x % NE, l = threadIdx.x / NE;
  const int64_t e0 = xcd_block() * NE, e = e0 + el;
  const int t0 = l % N1, t1 = l / N1;
  if constexpr (!CUR) stage_geo<T, NE, NT>(geo, E, e0, G);
  __syncthreads();
  const T gm1 = gamma - T(1);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    T ft[5][N1], tm[5] = {0, 0, 0, 0, 0}, tp[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < N1; ++a) {
      const int pt = line_pt<N1>(d, a, t0, t1);
      T uu[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        uu[v] = u[((int64_t)pt * 5 + v) * E + e];
        tm[v] += K.lm[a] * uu[v];
        tp[v] += K.lp[a] * uu[v];
      }
      T s[3], f[5], vs, pr;
      if constexpr (CUR) {
        cm_srow<T, NSP>(cm, E, e, pt, d, s);
      } else {
        T xi[3], g[3][3];
        line_xi(K, d, a, t0, t1, xi);
        hex_cols(G + el, NE, xi[0], xi[1], xi[2], g);
        srow(g, d, s);
      }
      Flux<T, DEV>::eval(uu, s[0], s[1], s[2], gm1, R, f, vs, pr);
#pragma unroll
      for (int v = 0; v < 5; ++v) ft[v][a] = f[v];
    }
    T Fc[2][5];
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      T nv[3];
      if constexpr (CUR) {
        cm_fnrm<T, NSP>(cm, E, e, (2 * d + sd) * NF + l, nv);
      } else {
        T xi[3], g[3][3];
        end_xi(K, d, sd, t0, t1, xi);
        hex_cols(G + el, NE, xi[0], xi[1], xi[2], g);
        srow(g, d, nv);
      }
      const T sg = sd ? T(1) : T(-1);
      const T mag = fsqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
      const NbrSlot ns = nbr_slot<NF>(C, E, e, 2 * d + sd, l);
      T un[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) un[v] = uf[((int64_t)ns.fp * 5 + v) * E + ns.elem];
      const T* own = sd ? tp : tm;
      T uL[5], uR[5], nL[3], F[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) { uL[v] = ns.left ? own[v] : un[v]; uR[v] = ns.left ? un[v] : own[v]; }
      const T sl = fdiv(ns.left ? sg : -sg, mag);
#pragma unroll
      for (int k = 0; k < 3; ++k) nL[k] = nv[k] * sl;
      common_inviscid<T, DEV>(riemann, uL, uR, nL, gamma, R, F);
      const T fs = ns.left ? mag : -mag;
#pragma unroll
      for (int v = 0; v < 5; ++v) Fc[sd][v] = fs * F[v];
    }
    accumulate_div<T, N1, NE, CUR>(d, ft, Fc, K, DIV, G, cm, el, t0, t1, e, n, E, r);
    if (d < 2) __syncthreads();
  }
}

// LDS slot of point pt in the gradient kernel's [component][point][element] buffer.
// With 4 points per line and 16 FP32 elements a point row is 16 banks, and the rows
// a wave touches on a line along xi_1 are 4 apart (same 16 banks of 64): the XOR of
// the point's low two bits with the next two spreads the four rows of every line
// direction over different bank groups.  A bijection on [0, 64).
template <typename T, int N1, int NE>
__device__ __forceinline__ int gr_slot(int pt) {
  if constexpr (N1 == 4 && NE * sizeof(T) == 64) return pt ^ ((pt >> 2) & 3);
  else return pt;
}

// ---------------------------------------------------------------------------
// Navier--Stokes phase 1: corrected gradient (LDG common solution u^ at the flux
// points), physical gradient at the solution points, and its traces at the flux
// points that the viscous common flux will read.  side_mode: +1 when beta = +1/2
// (u^ = u_L, the viscous common flux takes the right side only: the left side's
// jump vanishes and only right-side traces are stored), -1 for beta = -1/2 (the
// mirror case), 0 in general.
template <typename T, int P, int NE, bool CUR = false>
__global__ void __launch_bounds__(NE*(P + 1)*(P + 1)) hex_grad(
    const T* __restrict__ u, const T* __restrict__ uf, const T* __restrict__ geo, const T* __restrict__ cm,
    Conn C, T* __restrict__ grad, T* __restrict__ gradf, int64_t E, HexK<T> K, T beta, int side_mode) {
  constexpr int N1 = P + 1, NSP = N1 * N1 * N1, NF = N1 * N1, NT = NE * N1 * N1;
  __shared__ T GR[3 * NSP * NE];
  __shared__ T U[5 * NSP * NE];       // the block's state, [pt*5 + v][el]
  __shared__ T G[CUR ? 1 : 24 * NE];
  const int el = threadIdx.x % NE, l = threadIdx.x / NE;
  const int64_t e0 = xcd_block() * NE, e = e0 + el;
  const int t0 = l % N1, t1 = l / N1;
  // the global reads up front: geometry, the block's state and the neighbour traces at
  // this thread's 6 line ends (only where the common value is not the own trace)
  if constexpr (!CUR) stage_geo<T, NE, NT>(geo, E, e0, G);
  for (int i = threadIdx.x; i < 5 * NSP * NE; i += NT) U[i] = u[(int64_t)(i / NE) * E + e0 + i % NE];
  auto uval = [&](int pt, int v) -> T { return U[(pt * 5 + v) * NE + el]; };
  T uh[3][2][5];
  bool need[3][2], left[3][2];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      const NbrSlot s = nbr_slot<NF>(C, E, e, 2 * d + sd, l);
      left[d][sd] = s.left;
      need[d][sd] = side_mode == 0 || (side_mode > 0 ? !s.left : s.left);
#pragma unroll
      for (int v = 0; v < 5; ++v) uh[d][sd][v] = need[d][sd] ? uf[((int64_t)s.fp * 5 + v) * E + s.elem] : T(0);
    }
  __syncthreads();
  // metric of this thread's line points, once for all five variables: row d of S over J
  T sJ[3][N1][3];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int a = 0; a < N1; ++a) {
      T s[3], iJ;
      if constexpr (CUR) {
        const int pt = line_pt<N1>(d, a, t0, t1);
        cm_srow<T, NSP>(cm, E, e, pt, d, s);
        iJ = cm_rjac<T, NSP>(cm, E, e, pt);
      } else {
        T xi[3], g[3][3];
        line_xi(K, d, a, t0, t1, xi);
        hex_cols(G + el, NE, xi[0], xi[1], xi[2], g);
        srow(g, d, s);
        iJ = rcp(det_cols(g));
      }
#pragma unroll
      for (int j = 0; j < 3; ++j) sJ[d][a][j] = s[j] * iJ;
    }
  // common solution values u^ (LDG) at the 6 line ends
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      T tm = 0, tp = 0;
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        const T x = uval(line_pt<N1>(d, a, t0, t1), v);
        tm += K.lm[a] * x;
        tp += K.lp[a] * x;
      }
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        const T own = sd ? tp : tm, un = uh[d][sd][v];
        const T uL = left[d][sd] ? own : un, uR = left[d][sd] ? un : own;
        uh[d][sd][v] = need[d][sd] ? T(0.5) * (uL + uR) + beta * (uL - uR) : own;
      }
    }
#pragma unroll
  for (int v = 0; v < 5; ++v) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T uv[N1];
#pragma unroll
      for (int a = 0; a < N1; ++a) uv[a] = uval(line_pt<N1>(d, a, t0, t1), v);
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        T gt = K.cp[a] * uh[d][1][v] - K.cm[a] * uh[d][0][v];
#pragma unroll
        for (int b = 0; b < N1; ++b) gt += K.Dh[a][b] * uv[b];
        const int pt = line_pt<N1>(d, a, t0, t1);
        T* Gp = GR + (gr_slot<T, N1, NE>(pt) * NE + el);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          if (d == 0) Gp[j * NSP * NE] = sJ[d][a][j] * gt;
          else Gp[j * NSP * NE] += sJ[d][a][j] * gt;
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < N1; ++a) {
      const int pt = line_pt<N1>(2, a, t0, t1);
#pragma unroll
      for (int j = 0; j < 3; ++j)
        grad[((int64_t)pt * 15 + v * 3 + j) * E + e] = GR[(j * NSP + gr_slot<T, N1, NE>(pt)) * NE + el];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T gm[3] = {0, 0, 0}, gp[3] = {0, 0, 0};
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        const int pt = line_pt<N1>(d, a, t0, t1);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const T val = GR[(j * NSP + gr_slot<T, N1, NE>(pt)) * NE + el];
          gm[j] += K.lm[a] * val;
          gp[j] += K.lp[a] * val;
        }
      }
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        // stored only where a neighbour will read it
        const bool keep = side_mode == 0 || (side_mode > 0 ? !left[d][sd] : left[d][sd]);
        if (!keep) continue;
        const int f = (2 * d + sd) * NF + l;
#pragma unroll
        for (int j = 0; j < 3; ++j) gradf[((int64_t)f * 15 + v * 3 + j) * E + e] = sd ? gp[j] : gm[j];
      }
    }
    __syncthreads();
  }
}

// Variant for p = 4: the state is read from global memory (L2) per line and variable
// instead of being staged, which keeps the LDS and registers of the 125-point element
// within an occupancy of 3-4 waves per SIMD.
template <typename T, int P, int NE, bool CUR = false>
__global__ void __launch_bounds__(NE*(P + 1)*(P + 1)) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1))) hex_grad_lines(
    const T* __restrict__ u, const T* __restrict__ uf, const T* __restrict__ geo, const T* __restrict__ cm,
    Conn C, T* __restrict__ grad, T* __restrict__ gradf, int64_t E, HexK<T> K, T beta, int side_mode) {
  constexpr int N1 = P + 1, NSP = N1 * N1 * N1, NF = N1 * N1, NT = NE * N1 * N1;
  // the physical gradient's contributions of the three line directions, one slot per
  // direction ([d][j][pt][el]): every value has one writer, so the three directions of a
  // variable run without a barrier between them, and the output phase adds the slots
  __shared__ T GR[9 * NSP * NE];
  __shared__ T G[CUR ? 1 : 24 * NE];
  const int el = threadIdx.x % NE, l = threadIdx.x / NE;
  const int64_t e0 = xcd_block() * NE, e = e0 + el;
  const int t0 = l % N1, t1 = l / N1;
  if constexpr (!CUR) stage_geo<T, NE, NT>(geo, E, e0, G);
  // connectivity of this thread's 6 line ends
  NbrSlot ns[3][2];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) ns[d][sd] = nbr_slot<NF>(C, E, e, 2 * d + sd, l);
  __syncthreads();
  // metric of this thread's line points, once for all five variables: row d of S over J
  T sJ[3][N1][3];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int a = 0; a < N1; ++a) {
      T s[3], iJ;
      if constexpr (CUR) {
        const int pt = line_pt<N1>(d, a, t0, t1);
        cm_srow<T, NSP>(cm, E, e, pt, d, s);
        iJ = cm_rjac<T, NSP>(cm, E, e, pt);
      } else {
        T xi[3], g[3][3];
        line_xi(K, d, a, t0, t1, xi);
        hex_cols(G + el, NE, xi[0], xi[1], xi[2], g);
        srow(g, d, s);
        iJ = rcp(det_cols(g));
      }
#pragma unroll
      for (int j = 0; j < 3; ++j) sJ[d][a][j] = s[j] * iJ;
    }
  // the line values (and the partner traces the common value needs) of the next
  // (variable, direction) are loaded before the current one is worked on, so the loads
  // of one step overlap the arithmetic and the barrier of the previous one
  bool need[3][2];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
      // the common value equals the own trace when the switch points at this side
      need[d][sd] = side_mode == 0 || (side_mode > 0 ? !ns[d][sd].left : ns[d][sd].left);
  T nuv[N1], nun[2];
  auto load_line = [&](int v, int d) {
#pragma unroll
    for (int a = 0; a < N1; ++a) nuv[a] = u[((int64_t)line_pt<N1>(d, a, t0, t1) * 5 + v) * E + e];
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
      nun[sd] = need[d][sd] ? uf[((int64_t)ns[d][sd].fp * 5 + v) * E + ns[d][sd].elem] : T(0);
  };
  load_line(0, 0);
  for (int v = 0; v < 5; ++v) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T uv[N1], unb[2], tm = 0, tp = 0;
#pragma unroll
      for (int a = 0; a < N1; ++a) uv[a] = nuv[a];
      unb[0] = nun[0];
      unb[1] = nun[1];
      if (d < 2) load_line(v, d + 1);
      else if (v < 4) load_line(v + 1, 0);
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        tm += K.lm[a] * uv[a];
        tp += K.lp[a] * uv[a];
      }
      T uh[2];
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        const NbrSlot& s = ns[d][sd];
        const T own = sd ? tp : tm;
        const T un = need[d][sd] ? unb[sd] : own;
        const T uL = s.left ? own : un, uR = s.left ? un : own;
        uh[sd] = need[d][sd] ? T(0.5) * (uL + uR) + beta * (uL - uR) : own;
      }
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        T gt = K.cp[a] * uh[1] - K.cm[a] * uh[0];
#pragma unroll
        for (int b = 0; b < N1; ++b) gt += K.Dh[a][b] * uv[b];
        const int pt = line_pt<N1>(d, a, t0, t1);
        T* Gp = GR + d * 3 * NSP * NE + (gr_slot<T, N1, NE>(pt) * NE + el);
#pragma unroll
        for (int j = 0; j < 3; ++j) Gp[j * NSP * NE] = sJ[d][a][j] * gt;
      }
    }
    __syncthreads();
    auto gsum = [&](int j, int pt) {
      const int o = (j * NSP + gr_slot<T, N1, NE>(pt)) * NE + el;
      return (GR[o] + GR[3 * NSP * NE + o]) + GR[6 * NSP * NE + o];
    };
#pragma unroll
    for (int a = 0; a < N1; ++a) {
      const int pt = line_pt<N1>(2, a, t0, t1);
#pragma unroll
      for (int j = 0; j < 3; ++j)
        grad[((int64_t)pt * 15 + v * 3 + j) * E + e] = gsum(j, pt);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T gm[3] = {0, 0, 0}, gp[3] = {0, 0, 0};
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        const int pt = line_pt<N1>(d, a, t0, t1);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const T val = gsum(j, pt);
          gm[j] += K.lm[a] * val;
          gp[j] += K.lp[a] * val;
        }
      }
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        // stored only where a neighbour will read it
        if (!need[d][sd]) continue;
        const int f = (2 * d + sd) * NF + l;
#pragma unroll
        for (int j = 0; j < 3; ++j) gradf[((int64_t)f * 15 + v * 3 + j) * E + e] = sd ? gp[j] : gm[j];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Navier--Stokes phase 2a: the LDG common flux at every flux-point pair (eq:comm_flux
// with the viscous terms): inviscid Riemann flux along the left side's normal, minus
// the switched viscous flux, plus the penalty.  Threads over (element, flux point),
// lanes over elements; the left side of each pair computes it once and writes
// +|S^T n~| times it into its own slot and the negative into the right side's slot
// (conservative by construction).  With a one-sided switch only the contributing
// side's gradient trace is read (stored by hex_grad in that side's slot).
template <typename T, bool DEV, int P, bool CUR = false>
__global__ void __launch_bounds__(256) hex_face_ns(const T* __restrict__ uf, const T* __restrict__ gradf,
                                                   const T* __restrict__ geo, const T* __restrict__ cm, Conn C,
                                                   T* __restrict__ fc, int64_t E,
                                                   int64_t n, HexK<T> K, T gamma, T mu, T pr, T beta, T tau,
                                                   int riemann, int side_mode, RefState<T> R) {
  constexpr int N1 = P + 1, NF = N1 * N1, NFP = 6 * NF, NSP = N1 * N1 * N1;
  const int64_t gtid = xcd_block() * 256 + threadIdx.x;
  const int64_t wave = gtid >> 6;
  const int lane = (int)(gtid & 63);
  const int64_t tile = wave / NFP;
  const int fp = (int)(wave % NFP);
  const int64_t e = tile * 64 + lane;
  if (e >= n) return;
  const int face = fp / NF, q = fp % NF, d = face / 2, sd = face % 2, t0 = q % N1, t1 = q / N1;
  const NbrSlot ns = nbr_slot<NF>(C, E, e, face, q);
  // each flux-point pair once: the left side computes it and writes both slots (decided
  // before the geometry is read: which side is left is a property of the face, so the
  // waves of the right sides' faces leave at once)
  if (!ns.left) return;
  T nv[3];
  if constexpr (CUR) {
    cm_fnrm<T, NSP>(cm, E, e, fp, nv);
  } else {
    T c[24];
#pragma unroll
    for (int g = 0; g < 24; ++g) c[g] = geo[(int64_t)g * E + e];
    T xi[3], g[3][3];
    end_xi(K, d, sd, t0, t1, xi);
    hex_cols(c, 1, xi[0], xi[1], xi[2], g);
    srow(g, d, nv);
  }
  const T mag = fsqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
  T own[5], un[5], uL[5], uR[5], nL[3], F[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    own[v] = uf[((int64_t)fp * 5 + v) * E + e];
    un[v] = uf[((int64_t)ns.fp * 5 + v) * E + ns.elem];
  }
  const T sg = sd ? T(1) : T(-1);
  const T sl = fdiv(ns.left ? sg : -sg, mag);
#pragma unroll
  for (int k = 0; k < 3; ++k) nL[k] = nv[k] * sl;
#pragma unroll
  for (int v = 0; v < 5; ++v) { uL[v] = ns.left ? own[v] : un[v]; uR[v] = ns.left ? un[v] : own[v]; }
  common_inviscid<T, DEV>(riemann, uL, uR, nL, gamma, R, F);
  const T wL = T(0.5) - beta, wR = T(0.5) + beta;
  const T w_own = ns.left ? wL : wR, w_nbr = ns.left ? wR : wL;
  T fvc[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const T wgt = side == 0 ? w_own : w_nbr;
    if (side_mode != 0 && wgt == T(0)) continue;
    const int64_t gs = side == 0 ? (int64_t)fp : (int64_t)ns.fp;
    const int64_t ge = side == 0 ? e : ns.elem;
    T gk[15], fv[5];
#pragma unroll
    for (int k = 0; k < 15; ++k) gk[k] = gradf[(gs * 15 + k) * E + ge];
    viscous<T, DEV>(side == 0 ? own : un, gk, nL[0], nL[1], nL[2], gamma, mu, pr, R, fv);
#pragma unroll
    for (int v = 0; v < 5; ++v) fvc[v] += wgt * fv[v];
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const T fn = mag * (F[v] - fvc[v] + tau * (uL[v] - uR[v]));
    fc[((int64_t)fp * 5 + v) * E + e] = fn;
    fc[((int64_t)ns.fp * 5 + v) * E + ns.elem] = -fn;
  }
}

// ---------------------------------------------------------------------------
// Navier--Stokes phase 2b: f = f_inv - f_v at the solution points and the
// corrected divergence with the common fluxes of hex_face_ns at the line ends.
// Each thread owns one column (i, j) of one element: it evaluates the transformed
// flux of all three directions at its column's points once (every u and grad u
// value is read once) into LDS, then gathers, for each of its points, the three
// line contractions through that point from LDS.
template <typename T, bool DEV, int P, int NE, bool CUR = false>
__global__ void __launch_bounds__(NE*(P + 1)*(P + 1)) hex_div_ns(
    const T* __restrict__ u, const T* __restrict__ grad, const T* __restrict__ fc, const T* __restrict__ geo,
    const T* __restrict__ cm, T* __restrict__ r, int64_t E, int64_t n, HexK<T> K, T gamma, T mu, T pr, RefState<T> R) {
  constexpr int N1 = P + 1, NSP = N1 * N1 * N1, NF = N1 * N1, NT = NE * N1 * N1;
  // f~ along xi_1 and xi_2 go through LDS ([d][v][pt][el]); along xi_3 the line is the
  // thread's own column, so f~_3 and its common fluxes stay in registers
  __shared__ T FT[2 * 5 * NSP * NE];
  __shared__ T G[CUR ? 1 : 24 * NE];
  const int el = threadIdx.x % NE, l = threadIdx.x / NE;
  const int64_t e0 = xcd_block() * NE, e = e0 + el;
  const int ci = l % N1, cj = l / N1;
  if constexpr (!CUR) stage_geo<T, NE, NT>(geo, E, e0, G);
  __syncthreads();
  const T gm1 = gamma - T(1);
  T iJ[N1], f3[N1][5];
  // the state and gradient of the column's next point are loaded while the current
  // point's fluxes are formed (two buffers), so a wave keeps loads in flight
  T ub[2][5], gb[2][15];
  auto load_pt = [&](int k, T* uu, T* gg) {
    const int pt = ci + N1 * (cj + N1 * k);
#pragma unroll
    for (int v = 0; v < 5; ++v) uu[v] = u[((int64_t)pt * 5 + v) * E + e];
#pragma unroll
    for (int q = 0; q < 15; ++q) gg[q] = grad[((int64_t)pt * 15 + q) * E + e];
  };
  load_pt(0, ub[0], gb[0]);
#pragma unroll
  for (int k = 0; k < N1; ++k) {
    const int pt = ci + N1 * (cj + N1 * k);
    if (k + 1 < N1) load_pt(k + 1, ub[(k + 1) & 1], gb[(k + 1) & 1]);
    const T* uu = ub[k & 1];
    const T* gg = gb[k & 1];
    T g[3][3];
    if constexpr (CUR) {
      iJ[k] = -cm_rjac<T, NSP>(cm, E, e, pt);
    } else {
      hex_cols(G + el, NE, K.x[ci], K.x[cj], K.x[k], g);
      iJ[k] = -rcp(det_cols(g));
    }
    const PointFluxNS<T, DEV> pf(uu, gg, gamma, mu, pr, R);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T s[3], f[5];
      if constexpr (CUR) cm_srow<T, NSP>(cm, E, e, pt, d, s);
      else srow(g, d, s);
      pf.dir(s[0], s[1], s[2], f);
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        if (d < 2) FT[((d * 5 + v) * NSP + pt) * NE + el] = f[v];
        else f3[k][v] = f[v];
      }
    }
  }
  // own column: common fluxes at its two xi_3 ends
  const int q2 = ci + N1 * cj;
  T F4[5], F5[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    F4[v] = fc[(((int64_t)4 * NF + q2) * 5 + v) * E + e];
    F5[v] = fc[(((int64_t)5 * NF + q2) * 5 + v) * E + e];
  }
  // common fluxes at the xi_1 and xi_2 ends of the lines through point k, all five
  // variables at once; the next point's are loaded while the current one is summed
  T fb[2][4][5];
  auto load_ends = [&](int k, T (&F)[4][5]) {
    const int q0 = cj + N1 * k, q1 = ci + N1 * k;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      F[0][v] = fc[(((int64_t)0 * NF + q0) * 5 + v) * E + e];
      F[1][v] = fc[(((int64_t)1 * NF + q0) * 5 + v) * E + e];
      F[2][v] = fc[(((int64_t)2 * NF + q1) * 5 + v) * E + e];
      F[3][v] = fc[(((int64_t)3 * NF + q1) * 5 + v) * E + e];
    }
  };
  load_ends(0, fb[0]);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < N1; ++k) {
    const int pt = ci + N1 * (cj + N1 * k);
    if (k + 1 < N1) load_ends(k + 1, fb[(k + 1) & 1]);
    const T (&F)[4][5] = fb[k & 1];
    // line coordinates of this point in each direction: position a
    const int a0 = ci, a1 = cj;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      T acc = K.cp[k] * F5[v] + K.cm[k] * F4[v];
#pragma unroll
      for (int b = 0; b < N1; ++b) {
        acc += K.Dh[a0][b] * FT[((0 * 5 + v) * NSP + (b + N1 * (cj + N1 * k))) * NE + el];
        acc += K.Dh[a1][b] * FT[((1 * 5 + v) * NSP + (ci + N1 * (b + N1 * k))) * NE + el];
        acc += K.Dh[k][b] * f3[b][v];
      }
      acc += K.cp[a0] * F[1][v] + K.cm[a0] * F[0][v];
      acc += K.cp[a1] * F[3][v] + K.cm[a1] * F[2][v];
      if (e < n) r[((int64_t)pt * 5 + v) * E + e] = acc * iJ[k];
    }
  }
}

// Variant with all three directions' f~ in LDS, for FP64 at p = 4, where f~_3 of a
// whole column in registers does not fit beside the rest.  (In FP32 it does, at 166
// VGPRs: 3 waves per SIMD and 40 KB of LDS per 8 elements, three blocks per CU, where
// this variant's 60 KB allow two; bounding the register kernel to 128 VGPRs for a
// fourth block spills and is slower.)
template <typename T, bool DEV, int P, int NE, bool CUR = false>
__global__ void __launch_bounds__(NE*(P + 1)*(P + 1)) hex_div_ns_lds(
    const T* __restrict__ u, const T* __restrict__ grad, const T* __restrict__ fc, const T* __restrict__ geo,
    const T* __restrict__ cm, T* __restrict__ r, int64_t E, int64_t n, HexK<T> K, T gamma, T mu, T pr, RefState<T> R) {
  constexpr int N1 = P + 1, NSP = N1 * N1 * N1, NF = N1 * N1, NT = NE * N1 * N1;
  __shared__ T FT[3 * 5 * NSP * NE];       // [d][v][pt][el]
  __shared__ T G[CUR ? 1 : 24 * NE];
  const int el = threadIdx.x % NE, l = threadIdx.x / NE;
  const int64_t e0 = xcd_block() * NE, e = e0 + el;
  const int ci = l % N1, cj = l / N1;
  if constexpr (!CUR) stage_geo<T, NE, NT>(geo, E, e0, G);
  __syncthreads();
  const T gm1 = gamma - T(1);
  T iJ[N1];
  // as in hex_div_ns: the next point's state and gradient load while the current
  // point's fluxes are formed (this variant is held to 1-2 waves per SIMD by its LDS,
  // so registers are not what limits it)
  T ub[2][5], gb[2][15];
  auto load_pt = [&](int k, T* uu, T* gg) {
    const int pt = ci + N1 * (cj + N1 * k);
#pragma unroll
    for (int v = 0; v < 5; ++v) uu[v] = u[((int64_t)pt * 5 + v) * E + e];
#pragma unroll
    for (int q = 0; q < 15; ++q) gg[q] = grad[((int64_t)pt * 15 + q) * E + e];
  };
  load_pt(0, ub[0], gb[0]);
#pragma unroll
  for (int k = 0; k < N1; ++k) {
    const int pt = ci + N1 * (cj + N1 * k);
    if (k + 1 < N1) load_pt(k + 1, ub[(k + 1) & 1], gb[(k + 1) & 1]);
    const T* uu = ub[k & 1];
    const T* gg = gb[k & 1];
    T g[3][3];
    if constexpr (CUR) {
      iJ[k] = -cm_rjac<T, NSP>(cm, E, e, pt);
    } else {
      hex_cols(G + el, NE, K.x[ci], K.x[cj], K.x[k], g);
      iJ[k] = -rcp(det_cols(g));
    }
    const PointFluxNS<T, DEV> pf(uu, gg, gamma, mu, pr, R);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T s[3], f[5];
      if constexpr (CUR) cm_srow<T, NSP>(cm, E, e, pt, d, s);
      else srow(g, d, s);
      pf.dir(s[0], s[1], s[2], f);
#pragma unroll
      for (int v = 0; v < 5; ++v) FT[((d * 5 + v) * NSP + pt) * NE + el] = f[v];
    }
  }
  // common fluxes at the six line ends through point k (the xi_3 ends are the same
  // for every k), all variables at once, the next point's loaded during the sums
  const int q2 = ci + N1 * cj;
  T F4[5], F5[5], fb[2][4][5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    F4[v] = fc[(((int64_t)4 * NF + q2) * 5 + v) * E + e];
    F5[v] = fc[(((int64_t)5 * NF + q2) * 5 + v) * E + e];
  }
  auto load_ends = [&](int k, T (&F)[4][5]) {
    const int q0 = cj + N1 * k, q1 = ci + N1 * k;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      F[0][v] = fc[(((int64_t)0 * NF + q0) * 5 + v) * E + e];
      F[1][v] = fc[(((int64_t)1 * NF + q0) * 5 + v) * E + e];
      F[2][v] = fc[(((int64_t)2 * NF + q1) * 5 + v) * E + e];
      F[3][v] = fc[(((int64_t)3 * NF + q1) * 5 + v) * E + e];
    }
  };
  load_ends(0, fb[0]);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < N1; ++k) {
    const int pt = ci + N1 * (cj + N1 * k);
    if (k + 1 < N1) load_ends(k + 1, fb[(k + 1) & 1]);
    const T (&F)[4][5] = fb[k & 1];
    // line coordinates of this point in each direction: position a
    const int a0 = ci, a1 = cj, a2 = k;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      T acc = T(0);
#pragma unroll
      for (int b = 0; b < N1; ++b) {
        acc += K.Dh[a0][b] * FT[((0 * 5 + v) * NSP + (b + N1 * (cj + N1 * k))) * NE + el];
        acc += K.Dh[a1][b] * FT[((1 * 5 + v) * NSP + (ci + N1 * (b + N1 * k))) * NE + el];
        acc += K.Dh[a2][b] * FT[((2 * 5 + v) * NSP + (ci + N1 * (cj + N1 * b))) * NE + el];
      }
      acc += K.cp[a0] * F[1][v] + K.cm[a0] * F[0][v];
      acc += K.cp[a1] * F[3][v] + K.cm[a1] * F[2][v];
      acc += K.cp[a2] * F5[v] + K.cm[a2] * F4[v];
      if (e < n) r[((int64_t)pt * 5 + v) * E + e] = acc * iJ[k];
    }
  }
}

}  // namespace frmi
