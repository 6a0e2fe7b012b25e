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
// Kernels: the gradient and the divergence, each one dense contraction per block of
// 16 elements on the matrix cores, with the panel ([u; u^], or the transformed and
// common fluxes) evaluated into LDS by the same block.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hex.hpp"
#include "physics.hpp"

namespace frmi {

constexpr int TET_NSP = 35, TET_NFP = 60, TET_NFPF = 15;

template <typename T>
struct TetDev {
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

// ---------------------------------------------------------------------------
// Common normal flux at flux point sg of element e (eq:comm_flux, with the LDG viscous
// part for Navier--Stokes), times +-|S^T n~| (the sign of the element's side).  Both
// sides' states are collocated solution-point values; with a one-sided switch only
// the contributing side's gradient is read.
template <typename T, bool DEV, bool NS>
__device__ __forceinline__ void tet_common_flux(const T* __restrict__ u, const T* __restrict__ grad, const T S[9],
                                                const Conn& C, const TetDev<T>& O, int64_t E, int64_t e, int sg,
                                                T gamma, T mu, T pr, T beta, T tau, int riemann, int side_mode,
                                                const RefState<T>& R, T out[5]) {
  const int face = sg / TET_NFPF, q = sg % TET_NFPF;
  const NbrSlot ns = nbr_slot<TET_NFPF>(C, E, e, face, q);
  const int so = O.src[sg], sn = O.src[ns.fp];
  T own[5], un[5], nv[3], nL[3], uL[5], uR[5];
  tet_load(u, E, e, so, own);
  tet_load(u, E, ns.elem, sn, un);
  tet_normal(S, O, face, nv);
  const T mag = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
  const T sl = (ns.left ? T(1) : T(-1)) / mag;
#pragma unroll
  for (int k = 0; k < 3; ++k) nL[k] = nv[k] * sl;
#pragma unroll
  for (int c = 0; c < 5; ++c) { uL[c] = ns.left ? own[c] : un[c]; uR[c] = ns.left ? un[c] : own[c]; }
  common_inviscid<T, DEV>(riemann, uL, uR, nL, gamma, R, out);
  if constexpr (NS) {
    const T wL = T(0.5) - beta, wR = T(0.5) + beta;
    const T w_own = ns.left ? wL : wR, w_nbr = ns.left ? wR : wL;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const T wgt = side == 0 ? w_own : w_nbr;
      if (side_mode != 0 && wgt == T(0)) continue;
      const int64_t gp = side == 0 ? so : sn, ge = side == 0 ? e : ns.elem;
      T gk[15], fv[5];
#pragma unroll
      for (int k = 0; k < 15; ++k) gk[k] = grad[(gp * 15 + k) * E + ge];
      viscous<T, DEV>(side == 0 ? own : un, gk, nL[0], nL[1], nL[2], gamma, mu, pr, R, fv);
#pragma unroll
      for (int c = 0; c < 5; ++c) out[c] -= wgt * fv[c];
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) out[c] += tau * (uL[c] - uR[c]);
  }
  const T fs = ns.left ? mag : -mag;
#pragma unroll
  for (int c = 0; c < 5; ++c) out[c] *= fs;
}

// 16x16x4 matrix-core products: D = A B + C with A 16x4 (lane l: A[l % 16][l / 16]),
// B 4x16 (lane l: B[l / 16][l % 16]) and D 16x16, lane l holding column l % 16 in four
// registers q: rows 4 (l / 16) + q for FP32, rows l / 16 + 4 q for FP64 (both checked
// on gfx950 by a one-wave product of known matrices).
typedef float tet_f4 __attribute__((ext_vector_type(4)));
typedef double tet_d4 __attribute__((ext_vector_type(4)));
template <typename T>
struct Mma16;
template <>
struct Mma16<float> {
  using V = tet_f4;
  __device__ __forceinline__ static V run(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int q) { return 4 * (lane / 16) + q; }
};
template <>
struct Mma16<double> {
  using V = tet_d4;
  __device__ __forceinline__ static V run(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int q) { return lane / 16 + 4 * q; }
};

// BF16x3 split products: x = hi + lo with hi = bf16(x), lo = bf16(x - hi) (round to
// nearest even), a b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi accumulated in FP32 by the
// 16x16x16 bf16 matrix-core product (lane l holds 4 consecutive k of row / column
// l % 16; output layout as the FP32 product, checked on gfx950 like it).
typedef short tet_s4 __attribute__((ext_vector_type(4)));
typedef __bf16 tet_b4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void bf16_split4(const float x[4], tet_s4& hi, tet_s4& lo) {
  tet_b4 h, l;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    h[t] = (__bf16)x[t];
    l[t] = (__bf16)(x[t] - (float)h[t]);
  }
  hi = __builtin_bit_cast(tet_s4, h);
  lo = __builtin_bit_cast(tet_s4, l);
}

// acc[m] += Op[16 m .. 16 m + 15][k] P[k][v][col] over nk rows of the LDS panel starting at
// panel row pk, operator rows starting at column ko.  FP path: opT[k][ldm] (k-major, FP32 or
// FP64), steps of 4.  BF16x3 path: opH / opL [M][ldk] bf16 (k contiguous), steps of 16.
template <typename T, bool BF3, int NM, int NE>
__device__ __forceinline__ void tet_contract(typename Mma16<T>::V (&acc)[NM], const T* PAN, int pk, int nk, int v,
                                             int lane, const T* __restrict__ opT, int ko, int ldm,
                                             const tet_s4* __restrict__ opH, const tet_s4* __restrict__ opL, int ldk) {
  const int kr = lane / 16, col = lane % 16;
  if constexpr (!BF3) {
#pragma unroll 2
    for (int k0 = 0; k0 < nk; k0 += 4) {
      const T bop = PAN[((pk + k0 + kr) * 5 + v) * NE + col];
      const T* arow = opT + (ko + k0 + kr) * ldm + col;
#pragma unroll
      for (int m = 0; m < NM; ++m) acc[m] = Mma16<T>::run(arow[m * 16], bop, acc[m]);
    }
  } else {
    for (int k0 = 0; k0 < nk; k0 += 16) {
      float x[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) x[t] = PAN[((pk + k0 + 4 * kr + t) * 5 + v) * NE + col];
      tet_s4 bh, bl;
      bf16_split4(x, bh, bl);
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        const int a = ((m * 16 + col) * ldk + ko + k0 + 4 * kr) / 4;
        const tet_s4 ah = opH[a], al = opL[a];
        acc[m] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc[m], 0, 0, 0);
        acc[m] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc[m], 0, 0, 0);
        acc[m] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc[m], 0, 0, 0);
      }
    }
  }
}

// Contraction layout: K rows 0..104 are the transformed fluxes f~_i at the solution
// points (k = 35 i + point), 105..107 zero, 108..167 the common fluxes at the flux
// points; output rows are the 35 solution points padded to 48.  opT[k][pt] holds
// Op = [Dh_0 Dh_1 Dh_2 L] transposed and zero-padded.
constexpr int TET_KA = 108, TET_KB = 60, TET_KP = TET_KA + TET_KB, TET_MP = 48;
// the BF16x3 path pads both K chunks to multiples of 16: [0, 112) and [112, 176)
constexpr int TET_KA16 = 112, TET_KB16 = 64, TET_KP16 = TET_KA16 + TET_KB16;
constexpr int TDIV_NE = 16, TDIV_NT = 5 * 64;

// Corrected divergence (eq:FRfinal) on the matrix cores: per block of 16 elements,
// R^T = -(1/J) Op P with the panel P = [f~_0; f~_1; f~_2; F^C] (K x 5*16).  A block
// takes one tile of elements: its 5 waves evaluate the transformed fluxes at the
// solution points, then the common fluxes at the flux points, into the panel (two K
// chunks through LDS), and wave v multiplies the 16 columns of variable v by the
// three 16-row tiles of Op (read through the caches).
template <typename T, bool DEV, bool NS, bool BF3>
__global__ void __launch_bounds__(TDIV_NT) tet_div(const T* __restrict__ u, const T* __restrict__ grad,
                                                   const T* __restrict__ geo, Conn C, TetDev<T> O,
                                                   const T* __restrict__ opT, const tet_s4* __restrict__ opH,
                                                   const tet_s4* __restrict__ opL, T* __restrict__ r, int64_t E,
                                                   int64_t n, T gamma, T mu, T pr, T beta, T tau, int riemann,
                                                   int side_mode, RefState<T> R) {
  constexpr int NE = TDIV_NE, NT = TDIV_NT;
  constexpr int KA = BF3 ? TET_KA16 : TET_KA, KB = BF3 ? TET_KB16 : TET_KB;
  __shared__ T PAN[KA * 5 * NE];          // [k][v][el]; the second K chunk reuses it
  __shared__ T SJ[10 * NE];
  const int t = threadIdx.x;
  const int v = t / 64, lane = t % 64, col = lane % 16;
  const T gm1 = gamma - T(1);
  const int64_t e0 = xcd_block() * NE;
  {
    for (int i = t; i < 10 * NE; i += NT) SJ[i] = geo[(int64_t)(i / NE) * E + e0 + i % NE];
    for (int i = t; i < (KA - 105) * 5 * NE; i += NT) PAN[105 * 5 * NE + i] = T(0);
    __syncthreads();
    // K chunk 1: transformed fluxes at the solution points
    for (int it = t; it < NE * TET_NSP; it += NT) {
      const int el = it % NE, pt = it / NE;
      const int64_t e = e0 + el;
      T w[5], gg[15];
      tet_load(u, E, e, pt, w);
      if constexpr (NS) {
#pragma unroll
        for (int k = 0; k < 15; ++k) gg[k] = grad[((int64_t)pt * 15 + k) * E + e];
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const T sx = SJ[(3 * i) * NE + el], sy = SJ[(3 * i + 1) * NE + el], sz = SJ[(3 * i + 2) * NE + el];
        T f[5], vs, prs;
        Flux<T, DEV>::eval(w, sx, sy, sz, gm1, R, f, vs, prs);
        if constexpr (NS) {
          T fv[5];
          viscous<T, DEV>(w, gg, sx, sy, sz, gamma, mu, pr, R, fv);
#pragma unroll
          for (int c = 0; c < 5; ++c) f[c] -= fv[c];
        }
#pragma unroll
        for (int c = 0; c < 5; ++c) PAN[((i * TET_NSP + pt) * 5 + c) * NE + el] = f[c];
      }
    }
    __syncthreads();
    typename Mma16<T>::V acc[3];
#pragma unroll
    for (int mt = 0; mt < 3; ++mt) acc[mt] = typename Mma16<T>::V{0, 0, 0, 0};
    tet_contract<T, BF3, 3, NE>(acc, PAN, 0, KA, v, lane, opT, 0, TET_MP, opH, opL, TET_KP16);
    __syncthreads();
    // K chunk 2: common fluxes at the flux points (rows past 60 zero)
    if constexpr (KB > TET_NFP)
      for (int i = t; i < (KB - TET_NFP) * 5 * NE; i += NT) PAN[TET_NFP * 5 * NE + i] = T(0);
    for (int it = t; it < NE * TET_NFP; it += NT) {
      const int el = it % NE, sg = it / NE;
      T S[9], F[5];
#pragma unroll
      for (int k = 0; k < 9; ++k) S[k] = SJ[k * NE + el];
      tet_common_flux<T, DEV, NS>(u, grad, S, C, O, E, e0 + el, sg, gamma, mu, pr, beta, tau, riemann, side_mode, R, F);
#pragma unroll
      for (int c = 0; c < 5; ++c) PAN[(sg * 5 + c) * NE + el] = F[c];
    }
    __syncthreads();
    tet_contract<T, BF3, 3, NE>(acc, PAN, 0, KB, v, lane, opT, BF3 ? TET_KA16 : TET_KA, TET_MP, opH, opL, TET_KP16);
    const int64_t e = e0 + col;
    const T iJ = T(-1) / SJ[9 * NE + col];
    if (e < n) {
#pragma unroll
      for (int mt = 0; mt < 3; ++mt)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int pt = mt * 16 + Mma16<T>::row(lane, q);
          if (pt < TET_NSP) r[((int64_t)pt * 5 + v) * E + e] = acc[mt][q] * iJ;
        }
    }
  }
}

// ---------------------------------------------------------------------------
// Navier--Stokes gradient on the matrix cores.  Per element and variable the
// reference gradient is gt_i = Dh_i u + L diag(n~_i) u^ (i = 0, 1, 2): one product of
// the stacked operator G = [[Dh_0, L n~_0], [Dh_1, L n~_1], [Dh_2, L n~_2]] (3 x 35 rows
// padded to 3 x 48, K = 35 + 60 padded to 96; stored transposed, ogT[k][48 i + pt])
// with the panel [u; u^] of a block of 16 elements.  Wave v holds the nine 16x16
// output tiles of variable v, so the three gt_i of a point meet in one lane, where
// the physical gradient S^T gt / J is formed and stored.
constexpr int TGR_K = 96, TGR_M = 3 * TET_MP;

template <typename T, bool BF3>
__global__ void __launch_bounds__(TDIV_NT) tet_grad_mma(const T* __restrict__ u, const T* __restrict__ geo, Conn C,
                                                        TetDev<T> O, const T* __restrict__ ogT,
                                                        const tet_s4* __restrict__ ogH, const tet_s4* __restrict__ ogL,
                                                        T* __restrict__ grad, int64_t E, int64_t n, T beta) {
  constexpr int NE = TDIV_NE, NT = TDIV_NT;
  __shared__ T PAN[TGR_K * 5 * NE];      // [k][v][el]: u at the 35 points, u^ at the 60 flux points, 0
  __shared__ T SJ[10 * NE];
  const int t = threadIdx.x;
  const int v = t / 64, lane = t % 64, col = lane % 16;
  const int64_t e0 = xcd_block() * NE;
  {
    for (int i = t; i < 10 * NE; i += NT) SJ[i] = geo[(int64_t)(i / NE) * E + e0 + i % NE];
    for (int i = t; i < 5 * NE; i += NT) PAN[(TGR_K - 1) * 5 * NE + i] = T(0);
    for (int i = t; i < TET_NSP * 5 * NE; i += NT) PAN[i] = u[(int64_t)(i / NE) * E + e0 + i % NE];
    __syncthreads();
    for (int it = t; it < TET_NFP * NE; it += NT) {
      const int el = it % NE, sg = it / NE;
      const int64_t e = e0 + el;
      const int face = sg / TET_NFPF, q = sg % TET_NFPF;
      const NbrSlot ns = nbr_slot<TET_NFPF>(C, E, e, face, q);
      const int so = O.src[sg];
      T un[5];
      tet_load(u, E, ns.elem, O.src[ns.fp], un);
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        const T own = PAN[(so * 5 + c) * NE + el];
        const T uL = ns.left ? own : un[c], uR = ns.left ? un[c] : own;
        PAN[((TET_NSP + sg) * 5 + c) * NE + el] = T(0.5) * (uL + uR) + beta * (uL - uR);
      }
    }
    __syncthreads();
    typename Mma16<T>::V acc[9];
#pragma unroll
    for (int m = 0; m < 9; ++m) acc[m] = typename Mma16<T>::V{0, 0, 0, 0};
    tet_contract<T, BF3, 9, NE>(acc, PAN, 0, TGR_K, v, lane, ogT, 0, TGR_M, ogH, ogL, TGR_K);
    const int64_t e = e0 + col;
    if (e < n) {
      T S[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) S[k] = SJ[k * NE + col];
      const T iJ = T(1) / SJ[9 * NE + col];
#pragma unroll
      for (int mt = 0; mt < 3; ++mt)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int pt = mt * 16 + Mma16<T>::row(lane, q);
          if (pt >= TET_NSP) continue;
          const T g0 = acc[mt][q], g1 = acc[3 + mt][q], g2 = acc[6 + mt][q];
#pragma unroll
          for (int j = 0; j < 3; ++j)
            grad[((int64_t)pt * 15 + v * 3 + j) * E + e] = (S[j] * g0 + S[3 + j] * g1 + S[6 + j] * g2) * iJ;
        }
    }
  }
}

}  // namespace frmi
