// Tetrahedral FR kernels at p = 4 (the alpha-optimised point set of Fig. mesh).
//
// The 60 flux points are the surface solution points (Fig. mesh(b)), so step 1
// (eq:disu) is a gather of the collocated solution-point value, and the normal
// trace of the transformed flux at a flux point is n~ . f~ at that solution point.
// Folding that trace into the derivative gives (eq:FRfinal, DG lifting L = M^{-1}E)
//     div = sum_i Dh_i f~_i + L F^C,   Dh_i = D_i - L diag(n~_i) (scattered to sources),
// and the LDG corrected reference gradient is gt_i = Dh_i u + L diag(n~_i) u^.
// Affine elements: S = J G^{-1} and J are constant per element (geo[10][E]).
//
// Work mapping: lane = element (NE per block), point groups over the block's waves.
// For each variable the block stages the panel B = [f~_0; f~_1; f~_2; F^C] (165
// rows, or [u; u^] for the gradient) in LDS and contracts it with the dense
// operator rows; flux and Riemann evaluations are redone per variable, which costs
// flops but keeps the per-thread state small.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hex.hpp"
#include "physics.hpp"

namespace frmi {

constexpr int TET_NSP = 35, TET_NFP = 60, TET_NFPF = 15;

template <typename T>
struct TetDev {
  const T* Dh;          // [3][35][35]
  const T* L;           // [35][60]
  const int32_t* src;   // [60] collocated solution point of each flux point
  T nref[4][3];         // unit outward reference normals of the faces
};

template <typename T>
__device__ __forceinline__ void tet_geo(const T* __restrict__ geo, int64_t E, int64_t e, T S[9], T& J) {
#pragma unroll
  for (int k = 0; k < 9; ++k) S[k] = geo[(int64_t)k * E + e];
  J = geo[(int64_t)9 * E + e];
}

// Physical scaled normal S^T n~ of face f.
template <typename T>
__device__ __forceinline__ void tet_normal(const T S[9], const TetDev<T>& O, int f, T nv[3]) {
#pragma unroll
  for (int j = 0; j < 3; ++j) nv[j] = O.nref[f][0] * S[j] + O.nref[f][1] * S[3 + j] + O.nref[f][2] * S[6 + j];
}

template <typename T>
__device__ __forceinline__ void tet_load(const T* __restrict__ u, int64_t E, int64_t e, int pt, T w[5]) {
#pragma unroll
  for (int v = 0; v < 5; ++v) w[v] = u[((int64_t)pt * 5 + v) * E + e];
}

// One row of the contraction: sum_k A[row][k] B[k][el] over nk rows of the panel.
template <typename T, int NE>
__device__ __forceinline__ T tet_dot(const T* __restrict__ A, int nk, const T* B, int el) {
  T acc = T(0);
  for (int k = 0; k < nk; ++k) acc += A[k] * B[k * NE + el];
  return acc;
}

// ---------------------------------------------------------------------------
// Euler: R = -(sum_i Dh_i f~_i + L F^C) / J.
template <typename T, bool DEV, int NE, int NG>
__global__ void __launch_bounds__(NE * NG) tet_div_euler(const T* __restrict__ u, const T* __restrict__ geo,
                                                         Conn C, TetDev<T> O, T* __restrict__ r, int64_t E,
                                                         int64_t n, T gamma, int riemann, RefState<T> R) {
  __shared__ T B[(3 * TET_NSP + TET_NFP) * NE];
  const int el = threadIdx.x % NE, g = threadIdx.x / NE;
  const int64_t e = xcd_block() * NE + el;
  T S[9], J;
  tet_geo(geo, E, e, S, J);
  const T gm1 = gamma - T(1);
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    for (int pt = g; pt < TET_NSP; pt += NG) {
      T w[5], f[5], vs, pr;
      tet_load(u, E, e, pt, w);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        Flux<T, DEV>::eval(w, S[3 * i], S[3 * i + 1], S[3 * i + 2], gm1, R, f, vs, pr);
        B[(i * TET_NSP + pt) * NE + el] = f[v];
      }
    }
    for (int sg = g; sg < TET_NFP; sg += NG) {
      const int face = sg / TET_NFPF, q = sg % TET_NFPF;
      const NbrSlot ns = nbr_slot<TET_NFPF>(C, E, e, face, q);
      T own[5], un[5], nv[3], nL[3], uL[5], uR[5], F[5];
      tet_load(u, E, e, O.src[sg], own);
      tet_load(u, E, ns.elem, O.src[ns.fp], un);
      tet_normal(S, O, face, nv);
      const T mag = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
      const T sl = (ns.left ? T(1) : T(-1)) / mag;
#pragma unroll
      for (int k = 0; k < 3; ++k) nL[k] = nv[k] * sl;
#pragma unroll
      for (int c = 0; c < 5; ++c) { uL[c] = ns.left ? own[c] : un[c]; uR[c] = ns.left ? un[c] : own[c]; }
      common_inviscid<T, DEV>(riemann, uL, uR, nL, gamma, R, F);
      B[(3 * TET_NSP + sg) * NE + el] = (ns.left ? mag : -mag) * F[v];
    }
    __syncthreads();
    const T iJ = T(-1) / J;
    for (int pt = g; pt < TET_NSP; pt += NG) {
      T acc = T(0);
#pragma unroll
      for (int i = 0; i < 3; ++i) acc += tet_dot<T, NE>(O.Dh + (i * TET_NSP + pt) * TET_NSP, TET_NSP, B + i * TET_NSP * NE, el);
      acc += tet_dot<T, NE>(O.L + pt * TET_NFP, TET_NFP, B + 3 * TET_NSP * NE, el);
      if (e < n) r[((int64_t)pt * 5 + v) * E + e] = acc * iJ;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Navier--Stokes phase 1: physical gradient at the solution points,
// grad = G^{-T} (Dh u + L n~ u^)   (G^{-T} = S^T / J).  Flux-point gradients are
// the collocated solution-point values, so no trace array is needed.
template <typename T, int NE, int NG>
__global__ void __launch_bounds__(NE * NG) tet_grad(const T* __restrict__ u, const T* __restrict__ geo, Conn C,
                                                    TetDev<T> O, T* __restrict__ grad, int64_t E, T beta) {
  __shared__ T B[(TET_NSP + TET_NFP) * NE];
  const int el = threadIdx.x % NE, g = threadIdx.x / NE;
  const int64_t e = xcd_block() * NE + el;
  T S[9], J;
  tet_geo(geo, E, e, S, J);
  for (int v = 0; v < 5; ++v) {
    for (int pt = g; pt < TET_NSP; pt += NG) B[pt * NE + el] = u[((int64_t)pt * 5 + v) * E + e];
    for (int sg = g; sg < TET_NFP; sg += NG) {
      const int face = sg / TET_NFPF, q = sg % TET_NFPF;
      const NbrSlot ns = nbr_slot<TET_NFPF>(C, E, e, face, q);
      const T own = u[((int64_t)O.src[sg] * 5 + v) * E + e];
      const T un = u[((int64_t)O.src[ns.fp] * 5 + v) * E + ns.elem];
      const T uL = ns.left ? own : un, uR = ns.left ? un : own;
      B[(TET_NSP + sg) * NE + el] = T(0.5) * (uL + uR) + beta * (uL - uR);
    }
    __syncthreads();
    const T iJ = T(1) / J;
    for (int pt = g; pt < TET_NSP; pt += NG) {
      T gt[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        T acc = tet_dot<T, NE>(O.Dh + (i * TET_NSP + pt) * TET_NSP, TET_NSP, B, el);
        const T* Lr = O.L + pt * TET_NFP;
        for (int sg = 0; sg < TET_NFP; ++sg) acc += Lr[sg] * O.nref[sg / TET_NFPF][i] * B[(TET_NSP + sg) * NE + el];
        gt[i] = acc;
      }
#pragma unroll
      for (int j = 0; j < 3; ++j)
        grad[((int64_t)pt * 15 + v * 3 + j) * E + e] = (S[j] * gt[0] + S[3 + j] * gt[1] + S[6 + j] * gt[2]) * iJ;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Navier--Stokes phase 2: f = f_inv - f_v at the solution points, LDG common flux
// at the flux points from the collocated values of both sides, corrected divergence.
template <typename T, bool DEV, int NE, int NG>
__global__ void __launch_bounds__(NE * NG) tet_div_ns(const T* __restrict__ u, const T* __restrict__ grad,
                                                      const T* __restrict__ geo, Conn C, TetDev<T> O,
                                                      T* __restrict__ r, int64_t E, int64_t n, T gamma, T mu, T pr,
                                                      T beta, T tau, int riemann, RefState<T> R) {
  __shared__ T B[(3 * TET_NSP + TET_NFP) * NE];
  const int el = threadIdx.x % NE, g = threadIdx.x / NE;
  const int64_t e = xcd_block() * NE + el;
  T S[9], J;
  tet_geo(geo, E, e, S, J);
  const T gm1 = gamma - T(1);
  const T wL = T(0.5) - beta, wR = T(0.5) + beta;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    for (int pt = g; pt < TET_NSP; pt += NG) {
      T w[5], gg[15], f[5], fv[5], vs, prs;
      tet_load(u, E, e, pt, w);
#pragma unroll
      for (int k = 0; k < 15; ++k) gg[k] = grad[((int64_t)pt * 15 + k) * E + e];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        Flux<T, DEV>::eval(w, S[3 * i], S[3 * i + 1], S[3 * i + 2], gm1, R, f, vs, prs);
        viscous<T, DEV>(w, gg, S[3 * i], S[3 * i + 1], S[3 * i + 2], gamma, mu, pr, R, fv);
        B[(i * TET_NSP + pt) * NE + el] = f[v] - fv[v];
      }
    }
    for (int sg = g; sg < TET_NFP; sg += NG) {
      const int face = sg / TET_NFPF, q = sg % TET_NFPF;
      const NbrSlot ns = nbr_slot<TET_NFPF>(C, E, e, face, q);
      const int so = O.src[sg], sn = O.src[ns.fp];
      T own[5], un[5], nv[3], nL[3], uL[5], uR[5], F[5], go[15], gn[15], fvo[5], fvn[5];
      tet_load(u, E, e, so, own);
      tet_load(u, E, ns.elem, sn, un);
#pragma unroll
      for (int k = 0; k < 15; ++k) {
        go[k] = grad[((int64_t)so * 15 + k) * E + e];
        gn[k] = grad[((int64_t)sn * 15 + k) * E + ns.elem];
      }
      tet_normal(S, O, face, nv);
      const T mag = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
      const T sl = (ns.left ? T(1) : T(-1)) / mag;
#pragma unroll
      for (int k = 0; k < 3; ++k) nL[k] = nv[k] * sl;
#pragma unroll
      for (int c = 0; c < 5; ++c) { uL[c] = ns.left ? own[c] : un[c]; uR[c] = ns.left ? un[c] : own[c]; }
      common_inviscid<T, DEV>(riemann, uL, uR, nL, gamma, R, F);
      viscous<T, DEV>(own, go, nL[0], nL[1], nL[2], gamma, mu, pr, R, fvo);
      viscous<T, DEV>(un, gn, nL[0], nL[1], nL[2], gamma, mu, pr, R, fvn);
      const T w_own = ns.left ? wL : wR, w_nbr = ns.left ? wR : wL;
      const T fvc = w_own * fvo[v] + w_nbr * fvn[v];
      B[(3 * TET_NSP + sg) * NE + el] = (ns.left ? mag : -mag) * (F[v] - fvc + tau * (uL[v] - uR[v]));
    }
    __syncthreads();
    const T iJ = T(-1) / J;
    for (int pt = g; pt < TET_NSP; pt += NG) {
      T acc = T(0);
#pragma unroll
      for (int i = 0; i < 3; ++i) acc += tet_dot<T, NE>(O.Dh + (i * TET_NSP + pt) * TET_NSP, TET_NSP, B + i * TET_NSP * NE, el);
      acc += tet_dot<T, NE>(O.L + pt * TET_NFP, TET_NFP, B + 3 * TET_NSP * NE, el);
      if (e < n) r[((int64_t)pt * 5 + v) * E + e] = acc * iJ;
    }
    __syncthreads();
  }
}

}  // namespace frmi
