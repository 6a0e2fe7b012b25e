// Order-4 pyramids with an affine base (Sec. "Mixed elements and domain decomposition":
// the transition element, supported with an affine base), meshes of pyramids only.
//
// The rational pyramid space has no tensor structure and its 55 x 55 operators are
// dense, so these kernels apply them as plain matrix-vector products over a block of
// elements: a thread per (element, solution point or flux point), elements fastest so
// that global loads and stores are coalesced, the elements' states, transformed fluxes,
// interface jumps and gradients staged in LDS, the operators shared by all threads
// through the caches.  The steps are those of
// the other element types: traces at the flux points (eq:disu), the common flux
// along the left side's normal (eq:comm_flux), the transformed flux S f and its normal
// trace, and the corrected divergence D_i f~_i + lift (F^C - f~perp) (eq:FRfinal),
// R = -div / J; Navier--Stokes adds the LDG gradient (corrected by the lifted jump of
// the common solution) and the viscous parts of both fluxes.
//
// Layouts (element fastest): u, r [(pt*5 + v) E + e]; uf [(fp*5 + v) E + e];
// grad [(pt*15 + 3v + j) E + e]; gradf [(fp*15 + 3v + j) E + e]; geo rows 3i + j
// = S_ij (S = J G^{-1}), row 9 = J.  Operators: It[j][fp] = l_j(x_fp),
// Dt[i][j][pt] = d l_j / d xi_i (x_pt), Lt[fp][pt] = lift[pt][fp].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hex.hpp"

namespace frmi {

constexpr int PY_NSP = 55, PY_NFP = 85;

template <typename T>
struct PyrK {
  int face_off[6];
  T nref[5][3];
};

template <typename T>
struct PyrOpsDev {
  const T* It;   // [55][85]
  const T* Dt;   // [3][55][55]
  const T* Lt;   // [85][55]
};

__device__ __forceinline__ int pyr_face_of(const int* off, int fp) {
  int f = 0;
#pragma unroll
  for (int k = 1; k < 5; ++k) f += fp >= off[k];
  return f;
}

// Partner of flux point fp of element e: neighbour element, its flux point, and whether
// e is the left side.
template <typename T>
__device__ __forceinline__ void pyr_partner(const Conn& C, const PyrK<T>& K, int64_t E, int64_t e, int fp, int& f,
                                            int64_t& en, int& fpn, bool& left) {
  f = pyr_face_of(K.face_off, fp);
  const int q = fp - K.face_off[f];
  const int info = C.nbr_info[(int64_t)f * E + e];
  en = C.nbr_elem[(int64_t)f * E + e];
  const int fb = info & 7, orient = (info >> 3) & 511;
  left = (info >> 12) & 1;
  fpn = K.face_off[fb] + C.perm[orient * C.perm_stride + q];
}

template <typename T>
__device__ __forceinline__ void pyr_metric(const T* __restrict__ geo, int64_t E, int64_t e, T S[9], T& J) {
#pragma unroll
  for (int k = 0; k < 9; ++k) S[k] = geo[(int64_t)k * E + e];
  J = geo[(int64_t)9 * E + e];
}

// Threads of a block work on NE elements at once, element fastest: thread t takes
// element t % NE and point (t / NE) + k (PY_NT / NE), so that each load or store of a
// point's values covers NE consecutive elements of a row (32 bytes: 8 FP32 or 4 FP64
// elements, which keeps the LDS tiles of the gradient kernel under 50 KB), and the
// tiles staged in LDS serve the dense products with the same mapping.
constexpr int PY_NT = 256;
template <typename T>
constexpr int py_ne() { return sizeof(T) == 8 ? 4 : 8; }
// threads per block of the trace and divergence kernels: FP64 takes 128 (two solution
// points and three flux points per thread, as FP32 at 256: measured faster for FP64,
// slower for FP32); the gradient kernel takes PY_NT for both
template <typename T>
constexpr int py_nt() { return sizeof(T) == 8 ? 128 : PY_NT; }

// Step 1 (eq:disu): traces of u at the flux points.
template <typename T>
__global__ void __launch_bounds__(py_nt<T>()) pyr_trace(const T* __restrict__ u, T* __restrict__ uf, int64_t E,
                                                   const T* __restrict__ It) {
  constexpr int NE = py_ne<T>(), ROWS = py_nt<T>() / NE;
  __shared__ T U_s[NE][5][PY_NSP];
  const int el = threadIdx.x % NE, r0 = threadIdx.x / NE;
  const int64_t e = xcd_block() * NE + el;
  for (int pt = r0; pt < PY_NSP; pt += ROWS)
#pragma unroll
    for (int v = 0; v < 5; ++v) U_s[el][v][pt] = u[((int64_t)pt * 5 + v) * E + e];
  __syncthreads();
  // each thread's flux points at once, so that every LDS value serves all of them
  constexpr int NF = (PY_NFP + ROWS - 1) / ROWS;
  int fps[NF];
#pragma unroll
  for (int k = 0; k < NF; ++k) fps[k] = min(r0 + k * ROWS, PY_NFP - 1);
  T acc[NF][5];
#pragma unroll
  for (int k = 0; k < NF; ++k)
#pragma unroll
    for (int v = 0; v < 5; ++v) acc[k][v] = 0;
#pragma unroll 5
  for (int j = 0; j < PY_NSP; ++j) {
    T x[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) x[v] = U_s[el][v][j];
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      const T l = It[j * PY_NFP + fps[k]];
#pragma unroll
      for (int v = 0; v < 5; ++v) acc[k][v] += l * x[v];
    }
  }
#pragma unroll
  for (int k = 0; k < NF; ++k)
    if (r0 + k * ROWS < PY_NFP)
#pragma unroll
      for (int v = 0; v < 5; ++v) uf[((int64_t)fps[k] * 5 + v) * E + e] = acc[k][v];
}

// Navier--Stokes gradient (LDG): grad~u = D_i u + lift (n~_i (u^ - u_f)), u^ = (uL + uR)/2
// + beta (uL - uR); physical grad_j = sum_i S_ij / J grad~_i u.  Writes grad at the
// solution points and its traces at the flux points whose viscous common flux reads
// this side: all of them for side_mode 0, where this element is the right side for
// side_mode +1 (beta = +1/2: the common viscous flux is the right side's), the left
// side for -1 (beta = -1/2).
template <typename T>
__global__ void __launch_bounds__(PY_NT) pyr_grad(const T* __restrict__ u, const T* __restrict__ uf,
                                                  const T* __restrict__ geo, Conn C, PyrOpsDev<T> O, PyrK<T> K,
                                                  T* __restrict__ grad, T* __restrict__ gradf, int64_t E, T beta,
                                                  int side_mode) {
  constexpr int NE = py_ne<T>(), ROWS = PY_NT / NE;
  // one LDS tile per element: u (5 x 55) and the LDG jumps (5 x 85), and the physical
  // gradient (15 x 55).  FP32 overlays the gradient on the first two once every thread has
  // read them (26 KB per block instead of 49: four waves per SIMD instead of three); FP64,
  // held to three waves per SIMD by its registers, keeps them apart and saves the barrier.
  constexpr bool OVERLAY = sizeof(T) == 4;
  constexpr int GOFF = OVERLAY ? 0 : 5 * PY_NSP + 5 * PY_NFP;
  __shared__ T W_s[NE][GOFF + 15 * PY_NSP];
  static_assert(5 * PY_NSP + 5 * PY_NFP <= 15 * PY_NSP, "state and jumps fit in the gradient's tile");
  T* Wl = W_s[threadIdx.x % NE];
  auto U_at = [&](int v, int pt) -> T& { return Wl[v * PY_NSP + pt]; };
  auto JM_at = [&](int v, int fp) -> T& { return Wl[5 * PY_NSP + v * PY_NFP + fp]; };
  auto G_at = [&](int q, int pt) -> T& { return Wl[GOFF + q * PY_NSP + pt]; };
  const int el = threadIdx.x % NE, r0 = threadIdx.x / NE;
  const int64_t e = xcd_block() * NE + el;
  for (int pt = r0; pt < PY_NSP; pt += ROWS)
#pragma unroll
    for (int v = 0; v < 5; ++v) U_at(v, pt) = u[((int64_t)pt * 5 + v) * E + e];
  for (int fp = r0; fp < PY_NFP; fp += ROWS) {
    int f, fpn;
    int64_t en;
    bool left;
    pyr_partner(C, K, E, e, fp, f, en, fpn, left);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const T uo = uf[((int64_t)fp * 5 + v) * E + e];
      const T un = uf[((int64_t)fpn * 5 + v) * E + en];
      const T uL = left ? uo : un, uR = left ? un : uo;
      JM_at(v, fp) = T(0.5) * (uL + uR) + beta * (uL - uR) - uo;
    }
  }
  T S[9], J;
  pyr_metric(geo, E, e, S, J);
  const T iJ = rcp(J);
  __syncthreads();
  // each thread's solution points at once (every LDS value serves all of them)
  constexpr int NP = (PY_NSP + ROWS - 1) / ROWS, NF = (PY_NFP + ROWS - 1) / ROWS;
  int pts[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) pts[k] = min(r0 + k * ROWS, PY_NSP - 1);
  T gt[NP][3][5];
#pragma unroll
  for (int k = 0; k < NP; ++k)
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int v = 0; v < 5; ++v) gt[k][i][v] = 0;
  // unrolled by 5: the operator loads of five steps in flight together (measured: FP32
  // 0.84 -> 0.70 ms per launch; the same in the divergence was slower)
#pragma unroll 5
  for (int j = 0; j < PY_NSP; ++j) {
    T x[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) x[v] = U_at(v, j);
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const T d0 = O.Dt[(0 * PY_NSP + j) * PY_NSP + pts[k]];
      const T d1 = O.Dt[(1 * PY_NSP + j) * PY_NSP + pts[k]];
      const T d2 = O.Dt[(2 * PY_NSP + j) * PY_NSP + pts[k]];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        gt[k][0][v] += d0 * x[v];
        gt[k][1][v] += d1 * x[v];
        gt[k][2][v] += d2 * x[v];
      }
    }
  }
  // the reference normal is constant over a face: lift the face's jumps, then scale
#pragma unroll 1
  for (int f = 0; f < 5; ++f) {
    T sf[NP][5];
#pragma unroll
    for (int k = 0; k < NP; ++k)
#pragma unroll
      for (int v = 0; v < 5; ++v) sf[k][v] = 0;
    for (int fp = K.face_off[f]; fp < K.face_off[f + 1]; ++fp) {
      T y[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) y[v] = JM_at(v, fp);
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        const T l = O.Lt[fp * PY_NSP + pts[k]];
#pragma unroll
        for (int v = 0; v < 5; ++v) sf[k][v] += l * y[v];
      }
    }
    const T n0 = K.nref[f][0], n1 = K.nref[f][1], n2 = K.nref[f][2];
#pragma unroll
    for (int k = 0; k < NP; ++k)
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        gt[k][0][v] += n0 * sf[k][v];
        gt[k][1][v] += n1 * sf[k][v];
        gt[k][2][v] += n2 * sf[k][v];
      }
  }
  if constexpr (OVERLAY) __syncthreads();            // u and the jumps are read: the tile takes grad
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    if (r0 + k * ROWS >= PY_NSP) continue;
    const int pt = pts[k];
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const T g = (S[0 * 3 + j] * gt[k][0][v] + S[1 * 3 + j] * gt[k][1][v] + S[2 * 3 + j] * gt[k][2][v]) * iJ;
        G_at(v * 3 + j, pt) = g;
        grad[((int64_t)pt * 15 + v * 3 + j) * E + e] = g;
      }
  }
  __syncthreads();
  int fps[NF];
#pragma unroll
  for (int k = 0; k < NF; ++k) fps[k] = min(r0 + k * ROWS, PY_NFP - 1);
  T acc[NF][15];
#pragma unroll
  for (int k = 0; k < NF; ++k)
#pragma unroll
    for (int q = 0; q < 15; ++q) acc[k][q] = 0;
  for (int j = 0; j < PY_NSP; ++j) {
    T x[15];
#pragma unroll
    for (int q = 0; q < 15; ++q) x[q] = G_at(q, j);
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      const T l = O.It[j * PY_NFP + fps[k]];
#pragma unroll
      for (int q = 0; q < 15; ++q) acc[k][q] += l * x[q];
    }
  }
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    if (r0 + k * ROWS >= PY_NFP) continue;
    const int f = pyr_face_of(K.face_off, fps[k]);
    const bool left = (C.nbr_info[(int64_t)f * E + e] >> 12) & 1;
    if (side_mode != 0 && (side_mode > 0) == left) continue;      // the partner's trace is the one read
#pragma unroll
    for (int q = 0; q < 15; ++q) gradf[((int64_t)fps[k] * 15 + q) * E + e] = acc[k][q];
  }
}

// Corrected divergence (Euler, or Navier--Stokes with NS = true), R = -div / J.
template <typename T, bool DEV, bool NS>
__global__ void __launch_bounds__(py_nt<T>()) pyr_div(const T* __restrict__ u, const T* __restrict__ uf,
                                                 const T* __restrict__ grad, const T* __restrict__ gradf,
                                                 const T* __restrict__ geo, Conn C, PyrOpsDev<T> O, PyrK<T> K,
                                                 T* __restrict__ r, int64_t E, T gamma, T mu, T pr, T beta, T tau,
                                                 int riemann, int side_mode, RefState<T> R) {
  constexpr int NE = py_ne<T>(), ROWS = py_nt<T>() / NE;
  __shared__ T F_s[NE][3][5][PY_NSP];
  __shared__ T JM_s[NE][5][PY_NFP];
  const int el = threadIdx.x % NE, r0 = threadIdx.x / NE;
  const int64_t e = xcd_block() * NE + el;
  const T gm1 = gamma - T(1);
  T S[9], J;
  pyr_metric(geo, E, e, S, J);
  // transformed flux f~_i = (S f)_i at the solution points
  for (int pt = r0; pt < PY_NSP; pt += ROWS) {
    T wv[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) wv[v] = u[((int64_t)pt * 5 + v) * E + e];
    T g[15];
    if constexpr (NS) {
#pragma unroll
      for (int k = 0; k < 15; ++k) g[k] = grad[((int64_t)pt * 15 + k) * E + e];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      T f[5], vs, ps;
      Flux<T, DEV>::eval(wv, S[i * 3], S[i * 3 + 1], S[i * 3 + 2], gm1, R, f, vs, ps);
      if constexpr (NS) {
        T fv[5];
        viscous<T, DEV>(wv, g, S[i * 3], S[i * 3 + 1], S[i * 3 + 2], gamma, mu, pr, R, fv);
#pragma unroll
        for (int v = 0; v < 5; ++v) f[v] -= fv[v];
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) F_s[el][i][v][pt] = f[v];
    }
  }
  __syncthreads();
  // normal trace of f~ at each of the thread's flux points (every LDS value serves all)
  constexpr int NP = (PY_NSP + ROWS - 1) / ROWS, NF = (PY_NFP + ROWS - 1) / ROWS;
  int fps[NF];
  T nrk[NF][3];
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    fps[k] = min(r0 + k * ROWS, PY_NFP - 1);
    const int f = pyr_face_of(K.face_off, fps[k]);
#pragma unroll
    for (int q = 0; q < 3; ++q) nrk[k][q] = K.nref[0][q];
#pragma unroll
    for (int ff = 1; ff < 5; ++ff)
      if (f == ff)
#pragma unroll
        for (int q = 0; q < 3; ++q) nrk[k][q] = K.nref[ff][q];
  }
  T fperp[NF][5];
#pragma unroll
  for (int k = 0; k < NF; ++k)
#pragma unroll
    for (int v = 0; v < 5; ++v) fperp[k][v] = 0;
  for (int j = 0; j < PY_NSP; ++j) {
    T x[3][5];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int v = 0; v < 5; ++v) x[i][v] = F_s[el][i][v][j];
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      const T l = O.It[j * PY_NFP + fps[k]];
#pragma unroll
      for (int v = 0; v < 5; ++v) fperp[k][v] += l * (nrk[k][0] * x[0][v] + nrk[k][1] * x[1][v] + nrk[k][2] * x[2][v]);
    }
  }
  // common flux along the left side's normal, minus the normal trace
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    if (r0 + k * ROWS >= PY_NFP) continue;
    const int fp = fps[k];
    int f, fpn;
    int64_t en;
    bool left;
    pyr_partner(C, K, E, e, fp, f, en, fpn, left);
    const T* nr = nrk[k];
    T sn[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) sn[j] = S[0 * 3 + j] * nr[0] + S[1 * 3 + j] * nr[1] + S[2 * 3 + j] * nr[2];
    const T mag = fsqrt(sn[0] * sn[0] + sn[1] * sn[1] + sn[2] * sn[2]);
    const T im = rcp(mag);
    const T sg = left ? T(1) : T(-1);
    const T nL[3] = {sg * sn[0] * im, sg * sn[1] * im, sg * sn[2] * im};
    T uo[5], un[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      uo[v] = uf[((int64_t)fp * 5 + v) * E + e];
      un[v] = uf[((int64_t)fpn * 5 + v) * E + en];
    }
    T uL[5], uR[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) { uL[v] = left ? uo[v] : un[v]; uR[v] = left ? un[v] : uo[v]; }
    T Fc[5];
    common_inviscid<T, DEV>(riemann, uL, uR, nL, gamma, R, Fc);
    if constexpr (NS) {
      // viscous common flux (1/2 - beta) f_v(L) + (1/2 + beta) f_v(R); with beta = +-1/2
      // one side's weight is zero and its gradient trace is neither stored nor read
      const T wL = T(0.5) - beta, wR = T(0.5) + beta;
      T fvc[5] = {0, 0, 0, 0, 0};
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const bool is_left = side == 0;
        const T wgt = is_left ? wL : wR;
        if (side_mode != 0 && wgt == T(0)) continue;
        const bool own = is_left == left;
        const int64_t gs = own ? (int64_t)fp : (int64_t)fpn, ge = own ? e : en;
        T g[15], fv[5];
#pragma unroll
        for (int q = 0; q < 15; ++q) g[q] = gradf[(gs * 15 + q) * E + ge];
        viscous<T, DEV>(is_left ? uL : uR, g, nL[0], nL[1], nL[2], gamma, mu, pr, R, fv);
#pragma unroll
        for (int v = 0; v < 5; ++v) fvc[v] += wgt * fv[v];
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) Fc[v] += tau * (uL[v] - uR[v]) - fvc[v];
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) JM_s[el][v][fp] = mag * sg * Fc[v] - fperp[k][v];
  }
  __syncthreads();
  // corrected divergence at each of the thread's solution points
  int pts[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) pts[k] = min(r0 + k * ROWS, PY_NSP - 1);
  T div[NP][5];
#pragma unroll
  for (int k = 0; k < NP; ++k)
#pragma unroll
    for (int v = 0; v < 5; ++v) div[k][v] = 0;
  for (int j = 0; j < PY_NSP; ++j) {
    T x[3][5];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int v = 0; v < 5; ++v) x[i][v] = F_s[el][i][v][j];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const T d0 = O.Dt[(0 * PY_NSP + j) * PY_NSP + pts[k]];
      const T d1 = O.Dt[(1 * PY_NSP + j) * PY_NSP + pts[k]];
      const T d2 = O.Dt[(2 * PY_NSP + j) * PY_NSP + pts[k]];
#pragma unroll
      for (int v = 0; v < 5; ++v) div[k][v] += d0 * x[0][v] + d1 * x[1][v] + d2 * x[2][v];
    }
  }
  for (int fp = 0; fp < PY_NFP; ++fp) {
    T y[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) y[v] = JM_s[el][v][fp];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const T l = O.Lt[fp * PY_NSP + pts[k]];
#pragma unroll
      for (int v = 0; v < 5; ++v) div[k][v] += l * y[v];
    }
  }
  const T iJ = -rcp(J);
#pragma unroll
  for (int k = 0; k < NP; ++k)
    if (r0 + k * ROWS < PY_NSP)
#pragma unroll
      for (int v = 0; v < 5; ++v) r[((int64_t)pts[k] * 5 + v) * E + e] = div[k][v] * iJ;
}

}  // namespace frmi
