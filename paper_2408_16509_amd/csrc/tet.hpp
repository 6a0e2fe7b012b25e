// Tetrahedral FR kernels at p = 4 (the alpha-optimised point set of Fig. mesh).
//
// The 60 flux points are the surface solution points (Fig. mesh(b)), so step 1
// (eq:disu) is a gather of the collocated solution-point value, and the normal
// trace of the transformed flux at a flux point is n~ . f~ at that solution point.
// Folding that trace into the derivative gives (eq:FRfinal, DG lifting L = M^{-1}E)
//     div = sum_i Dh_i f~_i + L F^C,   Dh_i = D_i - L diag(n~_i) (scattered to sources),
// and the LDG corrected reference gradient is gt_i = Dh_i u + L diag(n~_i) u^.
// Affine elements: S = J G^{-1} and J are constant per element (geo[10][E]).  Curved
// elements (CUR, Sec. "Curved elements"): S and J stored per solution point
// (geo[pt * 10 + k][E]), and at each flux point the scaled normal S^T n~ of its face at
// the collocated solution point (geo[350 + fp * 3 + j][E]).
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
  const int32_t* pfp;   // [35][4]: number of flux points at solution point z (0..3), then their indices
  const int32_t* slot;  // [48]: solution point of each output row of the gradient product (-1: padding)
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

// Curved elements: the stored scaled normal S^T n~ at flux point sg.
template <typename T>
__device__ __forceinline__ void tet_cur_normal(const T* __restrict__ geo, int64_t E, int64_t e, int sg, T nv[3]) {
#pragma unroll
  for (int j = 0; j < 3; ++j) nv[j] = geo[((int64_t)10 * TET_NSP + sg * 3 + j) * E + e];
}

// ... and the unit normal there, oriented from the left to the right side (`left`: the
// element is the left side).
template <typename T>
__device__ __forceinline__ void tet_cur_unit_normal(const T* __restrict__ geo, int64_t E, int64_t e, int sg,
                                                    bool left, T nL[3]) {
  T nv[3];
  tet_cur_normal(geo, E, e, sg, nv);
  const T sl = fdiv(left ? T(1) : T(-1), fsqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]));
#pragma unroll
  for (int k = 0; k < 3; ++k) nL[k] = nv[k] * sl;
}

template <typename T>
__device__ __forceinline__ void tet_load(const T* __restrict__ u, int64_t E, int64_t e, int pt, T w[5]) {
#pragma unroll
  for (int v = 0; v < 5; ++v) w[v] = u[((int64_t)pt * 5 + v) * E + e];
}

// ---------------------------------------------------------------------------
// Common normal flux at flux point sg of element e (eq:comm_flux, with the LDG viscous
// part for Navier--Stokes), times +-|S^T n~| (the sign of the element's side; nv is the
// element's scaled normal S^T n~ there).  Both
// sides' states are collocated solution-point values; with a one-sided switch only
// the contributing side's gradient is read.
template <typename T, bool DEV, bool NS>
__device__ __forceinline__ void tet_common_flux(const T* __restrict__ u, const T* __restrict__ grad, const T nv[3],
                                                const Conn& C, const TetDev<T>& O, int64_t E, int64_t e, int sg,
                                                T gamma, T mu, T pr, T beta, T tau, int riemann, int side_mode,
                                                const RefState<T>& R, T out[5]) {
  const int face = sg / TET_NFPF, q = sg % TET_NFPF;
  const NbrSlot ns = nbr_slot<TET_NFPF>(C, E, e, face, q);
  const int so = O.src[sg], sn = O.src[ns.fp];
  T own[5], un[5], nL[3], uL[5], uR[5];
  tet_load(u, E, e, so, own);
  tet_load(u, E, ns.elem, sn, un);
  const T mag = fsqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
  const T sl = fdiv(ns.left ? T(1) : T(-1), mag);
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

// acc[i][v] += Op[16 mt[i] .. 16 mt[i] + 15][k] P[k][v][col] over the nk rows of the LDS
// panel, operator rows starting at column ko, for all five variables v: each operator
// value the wave loads serves five products.  FP path: opT[k][ldm] (k-major, FP32 or
// FP64), steps of 4.  BF16x3 path: opH / opL [M][ldk] bf16 (k contiguous), steps of 16.
template <typename T, bool BF3, int NW, int NE>
__device__ __forceinline__ void tet_contract(typename Mma16<T>::V (&acc)[NW][5], const T* PAN, int nk, int lane,
                                             const T* __restrict__ opT, int ko, int ldm, const int (&mt)[NW],
                                             const tet_s4* __restrict__ opH, const tet_s4* __restrict__ opL, int ldk) {
  const int kr = lane / 16, col = lane % 16;
  if constexpr (!BF3) {
#pragma unroll 2
    for (int k0 = 0; k0 < nk; k0 += 4) {
      T b[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) b[v] = PAN[((k0 + kr) * 5 + v) * NE + col];
      const T* arow = opT + (ko + k0 + kr) * ldm + col;
#pragma unroll
      for (int i = 0; i < NW; ++i) {
        const T a = arow[mt[i] * 16];
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[i][v] = Mma16<T>::run(a, b[v], acc[i][v]);
      }
    }
  } else {
    for (int k0 = 0; k0 < nk; k0 += 16) {
      tet_s4 bh[5], bl[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        float x[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) x[t] = PAN[((k0 + 4 * kr + t) * 5 + v) * NE + col];
        bf16_split4(x, bh[v], bl[v]);
      }
#pragma unroll
      for (int i = 0; i < NW; ++i) {
        const int a = ((mt[i] * 16 + col) * ldk + ko + k0 + 4 * kr) / 4;
        const tet_s4 ah = opH[a], al = opL[a];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          acc[i][v] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh[v], acc[i][v], 0, 0, 0);
          acc[i][v] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl[v], acc[i][v], 0, 0, 0);
          acc[i][v] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh[v], acc[i][v], 0, 0, 0);
        }
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
// 16 elements per block.  The divergence runs one wave per point tile (three), which
// also share the gathers (3.0 -> 2.65 ms per FP32 launch on the mixed workload against
// five waves of which two only gather); in FP32 a fourth wave joins the gathers and the
// flux evaluation (four blocks per CU either way, set by LDS: 1.286 -> 1.246 ms).  The
// gradient gathers more (the common solution at all 60 flux points): four waves in
// FP32 (three multiply; 2.95 -> 2.47 ms per launch against five), five in FP64 (four:
// 5.7 ms against 3.85).
constexpr int TDIV_NE = 16;
// Layout of the transformed viscous fluxes S_i . f_v that the FP32 gradient kernel stores
// for the divergence kernel (12 rows per solution point): tile by tile of NE elements,
// [tile][pt * 12 + k][el], so the rows of one tile are contiguous and the two halves of
// every 128-byte line are written by the same wave in consecutive stores (in the
// element-fastest layout of the state each 16-element row is half a line, whose other
// half another block writes).  Both kernels walk the same tiles.
template <int NE>
__device__ __forceinline__ int64_t tet_fv_index(int64_t e0, int row, int el) {
  return e0 * (12 * TET_NSP) + (int64_t)row * NE + el;
}
// The same for the pair-once common fluxes of the FP32 one-sided form (5 rows per flux
// point, [tile][sg * 5 + c][el]); the divergence kernel also reads the partner's slot,
// at element e of any tile.
template <int NE>
__device__ __forceinline__ int64_t tet_fc_index(int64_t e, int row) {
  return (e / NE) * (NE * 5 * TET_NFP) + (int64_t)row * NE + e % NE;
}
template <typename T>
constexpr int tdiv_nt() { return sizeof(T) == 4 ? 4 * 64 : 3 * 64; }
template <typename T>
constexpr int tgr_nt() { return sizeof(T) == 4 ? 4 * 64 : 5 * 64; }

// Corrected divergence (eq:FRfinal) on the matrix cores: per block of 16 elements,
// R^T = -(1/J) Op P with the panel P = [f~_0; f~_1; f~_2; F^C] (K x 5*16).  A block
// takes one tile of elements: its 5 waves evaluate the transformed fluxes at the
// solution points, then the common fluxes at the flux points, into the panel (two K
// chunks through LDS), and waves 0..2 each multiply one 16-row tile of Op (read
// through the caches, once per block) by the panel columns of all five variables.
// FCIN: the common fluxes (unit normal, left-to-right orientation) were already
// formed once per flux-point pair by the gradient kernel and stored in the slot of the
// side that formed them; here each flux point reads its pair's value and scales it by
// the element's own +-|S^T n~|.
template <typename T, bool DEV, bool NS, bool BF3, bool FCIN, bool CUR = false>
__global__ void __launch_bounds__(tdiv_nt<T>()) tet_div(const T* __restrict__ u, const T* __restrict__ grad,
                                                   const T* __restrict__ fcin,
                                                   const T* __restrict__ geo, Conn C, TetDev<T> O,
                                                   const T* __restrict__ opT, const tet_s4* __restrict__ opH,
                                                   const tet_s4* __restrict__ opL, T* __restrict__ r, int64_t E,
                                                   int64_t n, T gamma, T mu, T pr, T beta, T tau, int riemann,
                                                   int side_mode, RefState<T> R) {
  constexpr int NE = TDIV_NE, NT = tdiv_nt<T>();
  constexpr int KA = BF3 ? TET_KA16 : TET_KA, KB = BF3 ? TET_KB16 : TET_KB;
  __shared__ T PAN[KA * 5 * NE];          // [k][v][el]; the second K chunk reuses it
  __shared__ T SJ[CUR ? 1 : 10 * NE];
  const int t = threadIdx.x;
  const int w = t / 64, lane = t % 64, col = lane % 16;
  const int mt[1] = {w};
  const T gm1 = gamma - T(1);
  const int64_t e0 = xcd_block() * NE;
  // S of tile element el at solution point pt: the element's (staged in LDS) or, for
  // curved elements, the point's
  auto metric_at = [&](int pt, int el, T S[9]) {
    if constexpr (CUR) {
#pragma unroll
      for (int k = 0; k < 9; ++k) S[k] = geo[((int64_t)pt * 10 + k) * E + e0 + el];
    } else {
#pragma unroll
      for (int k = 0; k < 9; ++k) S[k] = SJ[k * NE + el];
    }
  };
  // the scaled normal S^T n~ at flux point sg: formed from the element's S, or stored (CUR)
  auto normal_at = [&](int sg, int el, T nv[3]) {
    if constexpr (CUR) {
      tet_cur_normal(geo, E, e0 + el, sg, nv);
    } else {
      T S[9];
      metric_at(0, el, S);
      tet_normal(S, O, sg / TET_NFPF, nv);
    }
  };
  {
    // The connectivity of this thread's flux points (FCIN) is read before anything
    // waits, the stored common fluxes right after chunk 1 is evaluated (both ahead of
    // their use in chunk 2, so their latency overlaps chunk 1's products).
    constexpr int NI2 = (NE * TET_NFP + NT - 1) / NT;
    // item it = t + j NT is row t / NE + j NT / NE of element t % NE (NT a multiple of NE)
    static_assert(NT % NE == 0, "rows per pass");
    const int tr = t / NE, tel = t % NE;
    int inf[FCIN ? NI2 : 1], nel[FCIN ? NI2 : 1];
    if constexpr (FCIN) {
#pragma unroll
      for (int j = 0; j < NI2; ++j) {
        const int face = (tr + j * (NT / NE)) / TET_NFPF;
        const int64_t o = (int64_t)face * E + e0 + tel;
        const bool ok = j + 1 < NI2 || t + j * NT < NE * TET_NFP;
        inf[j] = ok ? C.nbr_info[o] : 0;
        nel[j] = ok ? C.nbr_elem[o] : 0;
      }
    }
    if constexpr (!CUR)
      for (int i = t; i < 10 * NE; i += NT) SJ[i] = geo[(int64_t)(i / NE) * E + e0 + i % NE];
    for (int i = t; i < (KA - 105) * 5 * NE; i += NT) PAN[105 * 5 * NE + i] = T(0);
    __syncthreads();
    // K chunk 1: transformed fluxes at the solution points
    for (int pt = tr; pt < TET_NSP; pt += NT / NE) {
      const int el = tel;
      const int64_t e = e0 + el;
      T wv[5], gg[15];
      tet_load(u, E, e, pt, wv);
      T Sp[9];
      metric_at(pt, el, Sp);
      if constexpr (NS && FCIN) {
        // the gradient kernel stored S_i . f_v (12 values) instead of the gradient, tile by
        // tile (tet_fv_index)
        T fvs[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) fvs[k] = grad[tet_fv_index<NE>(e0, pt * 12 + k, el)];
        const PointInv<T, DEV> pin(wv, gamma, R);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          T f[5];
          pin.dir(Sp[3 * i], Sp[3 * i + 1], Sp[3 * i + 2], f);
#pragma unroll
          for (int c = 0; c < 5; ++c) PAN[((i * TET_NSP + pt) * 5 + c) * NE + el] = c == 0 ? f[0] : f[c] - fvs[4 * i + c - 1];
        }
        continue;
      }
      if constexpr (NS) {
#pragma unroll
        for (int k = 0; k < 15; ++k) gg[k] = grad[((int64_t)pt * 15 + k) * E + e];
      }
      if constexpr (NS) {
        const PointFluxNS<T, DEV> pf(wv, gg, gamma, mu, pr, R);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          T f[5];
          pf.dir(Sp[3 * i], Sp[3 * i + 1], Sp[3 * i + 2], f);
#pragma unroll
          for (int c = 0; c < 5; ++c) PAN[((i * TET_NSP + pt) * 5 + c) * NE + el] = f[c];
        }
      } else {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const T sx = Sp[3 * i], sy = Sp[3 * i + 1], sz = Sp[3 * i + 2];
          T f[5], vs, prs;
          Flux<T, DEV>::eval(wv, sx, sy, sz, gm1, R, f, vs, prs);
#pragma unroll
          for (int c = 0; c < 5; ++c) PAN[((i * TET_NSP + pt) * 5 + c) * NE + el] = f[c];
        }
      }
    }
    // the common fluxes formed by the gradient kernel, read from the slot of the side
    // that formed each (own or the partner's) ahead of chunk 1's products
    T fcv[FCIN ? NI2 : 1][5];
    bool lft[FCIN ? NI2 : 1];
    if constexpr (FCIN) {
#pragma unroll
      for (int j = 0; j < NI2; ++j) {
        const int it = t + j * NT;
        const int sg = tr + j * (NT / NE);
        const int nf = inf[j] & 7, orient = (inf[j] >> 3) & 511;
        lft[j] = (inf[j] >> 12) & 1;
        const bool own = lft[j] != (side_mode > 0);
        const bool ok = it < NE * TET_NFP;      // invalid items keep in-bounds addresses
        const int64_t fe = !ok ? e0 : (own ? e0 + tel : (int64_t)nel[j]);
        const int fp = !ok ? 0 : (own ? sg : nf * TET_NFPF + C.perm[orient * C.perm_stride + sg % TET_NFPF]);
#pragma unroll
        for (int c = 0; c < 5; ++c) fcv[j][c] = it < NE * TET_NFP ? fcin[tet_fc_index<NE>(fe, fp * 5 + c)] : T(0);
      }
    }
    __syncthreads();
    typename Mma16<T>::V acc[1][5];
#pragma unroll
    for (int v = 0; v < 5; ++v) acc[0][v] = typename Mma16<T>::V{0, 0, 0, 0};
    if (w < 3) tet_contract<T, BF3, 1, NE>(acc, PAN, KA, lane, opT, 0, TET_MP, mt, opH, opL, TET_KP16);
    __syncthreads();
    // K chunk 2: common fluxes at the flux points (rows past 60 zero)
    if constexpr (KB > TET_NFP)
      for (int i = t; i < (KB - TET_NFP) * 5 * NE; i += NT) PAN[TET_NFP * 5 * NE + i] = T(0);
    if constexpr (FCIN) {
#pragma unroll
      for (int j = 0; j < NI2; ++j) {
        if (t + j * NT >= NE * TET_NFP) continue;
        const int el = tel, sg = tr + j * (NT / NE);
        T nv[3];
        normal_at(sg, el, nv);
        const T mag = fsqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
        const T fs = lft[j] ? mag : -mag;
#pragma unroll
        for (int c = 0; c < 5; ++c) PAN[(sg * 5 + c) * NE + el] = fcv[j][c] * fs;
      }
    } else {
      for (int it = t; it < NE * TET_NFP; it += NT) {
        const int el = it % NE, sg = it / NE;
        T nv[3], F[5];
        normal_at(sg, el, nv);
        tet_common_flux<T, DEV, NS>(u, grad, nv, C, O, E, e0 + el, sg, gamma, mu, pr, beta, tau, riemann, side_mode,
                                    R, F);
#pragma unroll
        for (int c = 0; c < 5; ++c) PAN[(sg * 5 + c) * NE + el] = F[c];
      }
    }
    __syncthreads();
    if (w >= 3) return;
    tet_contract<T, BF3, 1, NE>(acc, PAN, KB, lane, opT, BF3 ? TET_KA16 : TET_KA, TET_MP, mt, opH, opL, TET_KP16);
    const int64_t e = e0 + col;
    T iJe = T(0);                          // -1/J of the element (straight elements)
    if constexpr (!CUR) iJe = -rcp(SJ[9 * NE + col]);
    if (e < n) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int pt = w * 16 + Mma16<T>::row(lane, q);
        if (pt < TET_NSP) {
          T iJ = iJe;
          if constexpr (CUR) iJ = -rcp(geo[((int64_t)pt * 10 + 9) * E + e]);
#pragma unroll
          for (int v = 0; v < 5; ++v) r[((int64_t)pt * 5 + v) * E + e] = acc[0][v][q] * iJ;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Output rows of the gradient product (per direction 48 = 3 point tiles of 16) hold the
// solution points in an order chosen at setup (TetDev::slot): the points that carry the
// same number of flux points share the rows a wave's lanes visit together, so the
// common-flux loop of the one-sided form diverges less.
//
// Navier--Stokes gradient on the matrix cores.  Per element and variable the
// reference gradient is gt_i = Dh_i u + L diag(n~_i) u^ (i = 0, 1, 2): one product of
// the stacked operator G = [[Dh_0, L n~_0], [Dh_1, L n~_1], [Dh_2, L n~_2]] (3 x 35 rows
// padded to 3 x 48, K = 35 + 60 padded to 96; stored transposed, ogT[k][48 i + pt])
// with the panel [u; u^] of a block of 16 elements.  Wave w (0..2) holds the output
// tiles of point tile w in the three directions for all five variables, so the three
// gt_i of a point meet in one lane, where the physical gradient S^T gt / J is formed
// and stored; each operator value the wave loads serves five products.
//
// FC (one-sided LDG, beta = +-1/2, side_mode = sign of beta): the common flux of
// every flux-point pair is formed here, once, by the element whose gradient the
// viscous part takes (the right side for beta = 1/2), and stored in that element's
// slot of fc; the divergence kernel reads it from there for both sides and scales it
// by its own +-|S^T n~|.  The lane that holds the gradient at a solution point stages
// the viscous flux along the left-to-right unit normal of each collocated flux point
// in LDS (over the flux-point rows of the panel, free once the products are done).
// Whether an element forms the fluxes of a face is a property of the face, so the
// formed (flux point, element) pairs of the block -- about half of them -- are then
// listed face by face and spread over all waves of the block, which evaluate
// eq:comm_flux (inviscid solver, staged viscous part, penalty) with the partner's
// state read again from memory (still in cache).  Evaluated per solution point
// instead, a wave would run the flux once for every flux point any of its lanes has,
// formed or not.
constexpr int TGR_K = 96, TGR_M = 3 * TET_MP;
// Panel rows of the FP32 / FP64 gradient: u at the 35 points (row 35 zero), then u^ face
// by face, 16 rows per face (its 15 flux points and a zero row).  The lift part of
// direction i is non-zero only on the faces whose reference normal has an i component,
// face 2 - i (normal -e_i) and face 3 ((1, 1, 1) / sqrt 3), so direction i contracts
// 36 + 16 + 16 of the 100 rows (255 products per wave and variable tile set, not 360).
constexpr int TGS_U = 36, TGS_K = TGS_U + 4 * 16;
__device__ __forceinline__ int tgs_row(int sg) { return TGS_U + 16 * (sg / TET_NFPF) + sg % TET_NFPF; }

// The face-sparse gradient contraction of wave w (point tile w, directions 0..2, all five
// variables); ogS[k][48 i + pt] in the row order above.
template <typename T, int NE>
__device__ __forceinline__ void tet_grad_contract(typename Mma16<T>::V (&acc)[3][5], const T* PAN, int lane,
                                                  const T* __restrict__ ogS, int w) {
  const int kr = lane / 16, col = lane % 16;
  const int mcol[3] = {16 * w + col, 16 * (3 + w) + col, 16 * (6 + w) + col};
  // rows shared by the three directions: the solution points, then face 3
#pragma unroll 3
  for (int s = 0; s < TGS_U / 4 + 4; ++s) {
    const int k = (s < TGS_U / 4 ? 4 * s : TGS_U + 48 + 4 * (s - TGS_U / 4)) + kr;
    T b[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) b[v] = PAN[(k * 5 + v) * NE + col];
    const T* arow = ogS + k * TGR_M;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const T a = arow[mcol[i]];
#pragma unroll
      for (int v = 0; v < 5; ++v) acc[i][v] = Mma16<T>::run(a, b[v], acc[i][v]);
    }
  }
  // face 2 - i: direction i only
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll 2
    for (int s = 0; s < 4; ++s) {
      const int k = TGS_U + 16 * (2 - i) + 4 * s + kr;
      T b[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) b[v] = PAN[(k * 5 + v) * NE + col];
      const T a = ogS[k * TGR_M + mcol[i]];
#pragma unroll
      for (int v = 0; v < 5; ++v) acc[i][v] = Mma16<T>::run(a, b[v], acc[i][v]);
    }
  }
}

template <typename T, bool DEV, bool BF3, bool FC, bool CUR = false>
__global__ void __launch_bounds__(tgr_nt<T>()) __attribute__((amdgpu_waves_per_eu(4))) tet_grad_mma(const T* __restrict__ u, const T* __restrict__ geo, Conn C,
                                                        TetDev<T> O, const T* __restrict__ ogT,
                                                        const tet_s4* __restrict__ ogH, const tet_s4* __restrict__ ogL,
                                                        T* __restrict__ grad, T* __restrict__ fc, int64_t E, int64_t n,
                                                        T beta, int side_mode, T gamma, T mu, T pr, T tau, int riemann,
                                                        RefState<T> R) {
  constexpr int NE = TDIV_NE, NT = tgr_nt<T>();
  constexpr int KR = BF3 ? TGR_K : TGS_K;
  // [k][v][el]: u at the 35 points, u^ at the 60 flux points (BF16x3: rows 35..94; else
  // face by face, tgs_row), zero rows
  __shared__ T PAN[KR * 5 * NE];
  __shared__ T SJ[CUR ? 1 : 10 * NE];
  // FC: per (face, element) the partner element and connectivity word and the unit
  // normal from the left to the right side; per formed (flux point, element) the
  // solution point of the partner's collocated value; per face the formed elements in
  // ascending order (FEL) and, bit 16 f + el, the block's formed mask (FMASK)
  static_assert(!FC || (NE == 16 && NT >= 4 * NE), "face tables assume 16-element tiles");
  __shared__ int32_t NBE[FC ? 4 * NE : 1], NBF[FC ? 4 * NE : 1];
  __shared__ T NRM[FC && !CUR ? 12 * NE : 1];    // straight elements: one normal per face
  __shared__ uint8_t PSRC[FC ? TET_NFP * NE : 1];
  __shared__ uint8_t FEL[FC ? 4 * NE : 1];
  __shared__ uint32_t FMASK[2];
  __shared__ int32_t PFP[FC ? TET_NSP * 4 : 1];
  __shared__ uint8_t SRCT[FC ? TET_NFP : 1];        // FC: collocated solution point of each flux point
  __shared__ int32_t SLOT[TET_MP];
  const int t = threadIdx.x;
  const int w = t / 64, lane = t % 64, col = lane % 16;
  const int64_t e0 = xcd_block() * NE;
  {
    if constexpr (!CUR)
      for (int i = t; i < 10 * NE; i += NT) SJ[i] = geo[(int64_t)(i / NE) * E + e0 + i % NE];
    if constexpr (BF3) {
      for (int i = t; i < 5 * NE; i += NT) PAN[(TGR_K - 1) * 5 * NE + i] = T(0);
    } else {
      for (int i = t; i < 5 * 5 * NE; i += NT) {
        const int zr = i / (5 * NE);            // zero rows 35, 51, 67, 83, 99
        PAN[(zr == 0 ? TET_NSP : TGS_U + 16 * zr - 1) * 5 * NE + i % (5 * NE)] = T(0);
      }
    }
    // Every global read of the gather is issued before the first wait: the block's state
    // (NU values per thread) and the connectivity of this thread's flux points (NI items
    // (el, sg) per thread), then the partners' states, so each block waits on about two
    // memory latencies instead of one per loop trip.
    constexpr int NU = (TET_NSP * 5 * NE + NT - 1) / NT, NI = (TET_NFP * NE + NT - 1) / NT;
    // item i = t + j NT is row i / NE, element i % NE = t % NE (NT a multiple of NE): one
    // base address per thread and a uniform stride of NT / NE rows
    static_assert(NT % NE == 0, "rows per pass");
    const int tr = t / NE, tel = t % NE;
    T ur[NU];
    {
      const T* ub = u + (int64_t)tr * E + e0 + tel;
      const int64_t us = (int64_t)(NT / NE) * E;
#pragma unroll
      for (int j = 0; j < NU; ++j)
        ur[j] = (j + 1 < NU || t + j * NT < TET_NSP * 5 * NE) ? ub[j * us] : T(0);
    }
    int inf[NI], nel[NI];
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const int it = t + j * NT;
      const int face = (tr + j * (NT / NE)) / TET_NFPF;
      const int64_t o = (int64_t)face * E + e0 + tel;
      const bool ok = j + 1 < NI || it < TET_NFP * NE;
      inf[j] = ok ? C.nbr_info[o] : 0;
      nel[j] = ok ? C.nbr_elem[o] : 0;
    }
    if constexpr (FC)
      for (int i = t; i < TET_NSP * 4; i += NT) PFP[i] = O.pfp[i];
    if constexpr (FC)
      for (int i = t; i < TET_NFP; i += NT) SRCT[i] = (uint8_t)O.src[i];
    for (int i = t; i < TET_MP; i += NT) SLOT[i] = O.slot[i];
#pragma unroll
    for (int j = 0; j < NU; ++j) {
      const int i = t + j * NT;
      if (i < TET_NSP * 5 * NE) PAN[i] = ur[j];
    }
    // partners' states where the common solution needs them
    T un[NI][5];
    bool lft[NI], fromn[NI];
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const int it = t + j * NT;
      const int sg = tr + j * (NT / NE);
      const int nf = inf[j] & 7, orient = (inf[j] >> 3) & 511;
      lft[j] = (inf[j] >> 12) & 1;
      fromn[j] = it < TET_NFP * NE && (side_mode == 0 || (side_mode > 0) != lft[j]);
      const int nfp = nf * TET_NFPF + C.perm[orient * C.perm_stride + sg % TET_NFPF];
      const int src = O.src[fromn[j] ? nfp : 0];
      const T* pb = u + (int64_t)src * 5 * E + (fromn[j] ? (int64_t)nel[j] : e0);
#pragma unroll
      for (int c = 0; c < 5; ++c) un[j][c] = fromn[j] ? pb[(int64_t)c * E] : T(0);
      if constexpr (FC) {
        if (it < TET_NFP * NE) {
          const int el = tel;
          if (fromn[j]) PSRC[sg * NE + el] = (uint8_t)src;
          if (sg % TET_NFPF == 0) {
            NBF[(sg / TET_NFPF) * NE + el] = inf[j];
            NBE[(sg / TET_NFPF) * NE + el] = nel[j];
          }
        }
      }
    }
    __syncthreads();
    if constexpr (FC) {
      // wave 0, lane = 16 f + el: the face tables (after the wait: SJ and NBF are in LDS)
      if (w == 0) {
        const int f = lane / NE, el = lane % NE;
        const bool left = (NBF[f * NE + el] >> 12) & 1;
        const bool formed = left != (side_mode > 0) && e0 + el < n;
        if constexpr (!CUR) {
          T S[9], nv[3];
#pragma unroll
          for (int k = 0; k < 9; ++k) S[k] = SJ[k * NE + el];
          tet_normal(S, O, f, nv);
          const T sl = fdiv(left ? T(1) : T(-1), fsqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]));
#pragma unroll
          for (int k = 0; k < 3; ++k) NRM[(f * 3 + k) * NE + el] = nv[k] * sl;
        }
        const uint64_t m = __ballot(formed);
        const uint32_t mf = (uint32_t)(m >> (16 * f)) & 0xffffu;
        if (formed) FEL[f * NE + __popc(mf & ((1u << el) - 1u))] = (uint8_t)el;
        if (lane == 0) {
          FMASK[0] = (uint32_t)m;
          FMASK[1] = (uint32_t)(m >> 32);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < NI; ++j) {
      const int it = t + j * NT;
      if (it >= TET_NFP * NE) continue;
      const int el = it % NE, sg = it / NE;
      const int so = O.src[sg];
      const int row = BF3 ? TET_NSP + sg : tgs_row(sg);
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        const T own = PAN[(so * 5 + c) * NE + el];
        T val;
        if (side_mode != 0) {
          // one-sided: u^ is exactly the state of the side named by beta, so the partner's
          // state was read only where that side is the partner (half of the flux points)
          val = fromn[j] ? un[j][c] : own;
        } else {
          const T uL = lft[j] ? own : un[j][c], uR = lft[j] ? un[j][c] : own;
          val = T(0.5) * (uL + uR) + beta * (uL - uR);
        }
        PAN[(row * 5 + c) * NE + el] = val;
      }
    }
    __syncthreads();
    // the formed pairs of the one-sided common flux, face by face (15 flux points x the
    // face's formed elements in ascending order): item i -> face f, flux point sg, element el
    [[maybe_unused]] int c0 = 0, c1 = 0, c2 = 0, c3 = 0, o1 = 0, o2 = 0, o3 = 0, total = 0;
    if constexpr (FC) {
      const uint64_t m = ((uint64_t)FMASK[1] << 32) | FMASK[0];
      c0 = __popcll(m & 0xffffull);
      c1 = __popcll((m >> 16) & 0xffffull);
      c2 = __popcll((m >> 32) & 0xffffull);
      c3 = __popcll(m >> 48);
      o1 = TET_NFPF * c0;
      o2 = o1 + TET_NFPF * c1;
      o3 = o2 + TET_NFPF * c2;
      total = o3 + TET_NFPF * c3;
    }
    [[maybe_unused]] auto decode = [&](int i, int& f, int& sg, int& el) {
      f = (i >= o1) + (i >= o2) + (i >= o3);
      const int of = f == 0 ? 0 : f == 1 ? o1 : f == 2 ? o2 : o3;
      const int cf = f == 0 ? c0 : f == 1 ? c1 : f == 2 ? c2 : c3;
      const int r = i - of;
      // r = 15 k + position among the face's formed elements; k = floor((r + 1/2) / cf),
      // whose fraction lies in [1/32, 31/32], far from the reciprocal's rounding
      const int k = (int)((float(r) + 0.5f) * __builtin_amdgcn_rcpf((float)cf));
      el = FEL[f * NE + (r - k * cf)];
      sg = f * TET_NFPF + k;
    };
    // formed pairs have the element on the side that beta does not name
    [[maybe_unused]] const bool left = side_mode < 0;
    constexpr int FVB = (BF3 ? TET_NSP : TGS_U) * 5 * NE;   // FVN[(sg * 4 + c) * NE + el] at PAN + FVB
    static_assert(!FC || FVB + TET_NFP * 4 * NE <= KR * 5 * NE, "staged viscous fluxes exceed the panel");
    if constexpr (!FC) {
      if (w >= 3) return;
    }
    static_assert(!FC || NT == 4 * 64, "the FC roles assume waves 0-2 multiplying and wave 3");
    constexpr int JW = 10;                           // FC: pairs per lane of wave 3
    if (FC && w == 3) {
      // wave 3, idle during the products: the inviscid flux and the penalty of the first
      // 64 JW pairs from the panel (read-only until barrier 1), kept in registers until
      // the viscous part is staged.  The two wave roles pass the same two block barriers,
      // (1) and (2), each in its own branch; a barrier counts the waves of the block
      // that reach one.
      T fw[JW][4];
      int iw[JW];
#pragma unroll
      for (int j = 0; j < JW; ++j) {
        const int i = lane + 64 * j;
        iw[j] = -1;
        if (i >= total) continue;
        int f, sg, el;
        decode(i, f, sg, el);
        const int so = SRCT[sg], row = BF3 ? TET_NSP + sg : tgs_row(sg);
        T uL[5], uR[5], nL[3], F[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          const T own = PAN[(so * 5 + c) * NE + el], nb = PAN[(row * 5 + c) * NE + el];
          uL[c] = left ? own : nb;
          uR[c] = left ? nb : own;
        }
        if constexpr (CUR) {
          tet_cur_unit_normal(geo, E, e0 + el, sg, left, nL);
        } else {
#pragma unroll
          for (int k = 0; k < 3; ++k) nL[k] = NRM[(f * 3 + k) * NE + el];
        }
        common_inviscid<T, DEV>(riemann, uL, uR, nL, gamma, R, F);
        fc[tet_fc_index<NE>(e0 + el, sg * 5)] = F[0] + tau * (uL[0] - uR[0]);
#pragma unroll
        for (int c = 1; c < 5; ++c) fw[j][c - 1] = F[c] + tau * (uL[c] - uR[c]);
        iw[j] = sg * NE + el;
      }
      __syncthreads();                             // (1)
      __syncthreads();                             // (2)
#pragma unroll
      for (int j = 0; j < JW; ++j) {
        if (iw[j] < 0) continue;
        const int sg = iw[j] / NE, el = iw[j] % NE;
#pragma unroll
        for (int c = 1; c < 5; ++c)
          fc[tet_fc_index<NE>(e0 + el, sg * 5 + c)] = fw[j][c - 1] - PAN[FVB + (sg * 4 + c - 1) * NE + el];
      }
    } else {
      // waves 0-2: the products, then the gradient epilogue (FC: with the staged viscous
      // normal fluxes, written over the panel's trace rows once all products are done)
      typename Mma16<T>::V acc[3][5];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[i][v] = typename Mma16<T>::V{0, 0, 0, 0};
      if constexpr (BF3) {
        const int mt[3] = {w, 3 + w, 6 + w};
        tet_contract<T, BF3, 3, NE>(acc, PAN, TGR_K, lane, ogT, 0, TGR_M, mt, ogH, ogL, TGR_K);
      } else {
        tet_grad_contract<T, NE>(acc, PAN, lane, ogT, w);
      }
      if constexpr (FC) __syncthreads();           // (1) every wave's products are done
      const int64_t e = e0 + col;
      if (e < n) {
        T S[9], iJ = T(0);
        if constexpr (!CUR) {
#pragma unroll
          for (int k = 0; k < 9; ++k) S[k] = SJ[k * NE + col];
          iJ = rcp(SJ[9 * NE + col]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int pt = SLOT[w * 16 + Mma16<T>::row(lane, q)];
          if (pt < 0) continue;
          if constexpr (CUR) {
#pragma unroll
            for (int k = 0; k < 9; ++k) S[k] = geo[((int64_t)pt * 10 + k) * E + e];
            iJ = rcp(geo[((int64_t)pt * 10 + 9) * E + e]);
          }
          T gp[15];
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            const T g0 = acc[0][v][q], g1 = acc[1][v][q], g2 = acc[2][v][q];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              gp[v * 3 + j] = (S[j] * g0 + S[3 + j] * g1 + S[6 + j] * g2) * iJ;
              if constexpr (!FC) grad[((int64_t)pt * 15 + v * 3 + j) * E + e] = gp[v * 3 + j];
            }
          }
          if constexpr (FC) {
            // the divergence kernel needs the gradient only through the transformed viscous
            // flux at the solution points: S_i . f_v for i = 0, 1, 2 (momentum and energy,
            // the mass component is zero), 12 values instead of 15
            T own[5];
#pragma unroll
            for (int c = 0; c < 5; ++c) own[c] = PAN[(pt * 5 + c) * NE + col];
            const PointFluxNS<T, DEV> pf(own, gp, gamma, mu, pr, R);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
              T fv[4];
              pf.visc(S[3 * i], S[3 * i + 1], S[3 * i + 2], fv);
#pragma unroll
              for (int c = 0; c < 4; ++c) grad[tet_fv_index<NE>(e0, pt * 12 + i * 4 + c, col)] = fv[c];
            }
            // the viscous flux along the left-to-right unit normal at each collocated flux
            // point (the flux phase reads only those of formed faces)
            const int nf = PFP[pt * 4];
            for (int i = 0; i < nf; ++i) {
              const int sg = PFP[pt * 4 + 1 + i];
              const int f = sg / TET_NFPF;
              T fv[4];
              if constexpr (CUR) {
                // the unit normal from this point's own metric, oriented left to right
                T nv[3];
                tet_normal(S, O, f, nv);
                const bool lf = (NBF[f * NE + col] >> 12) & 1;
                const T sl = fdiv(lf ? T(1) : T(-1), fsqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]));
                pf.visc(nv[0] * sl, nv[1] * sl, nv[2] * sl, fv);
              } else {
                pf.visc(NRM[(f * 3) * NE + col], NRM[(f * 3 + 1) * NE + col], NRM[(f * 3 + 2) * NE + col], fv);
              }
#pragma unroll
              for (int c = 0; c < 4; ++c) PAN[FVB + (sg * 4 + c) * NE + col] = fv[c];
            }
          }
        }
      }
      if constexpr (FC) __syncthreads();           // (2) the viscous normal fluxes are staged
    }
    if constexpr (FC) {
      // pairs past 64 JW (more than 640 formed pairs in the block, rare): all waves, the
      // partner's state read again from memory (the panel's trace rows hold the staged
      // viscous fluxes by now)
      for (int i = 64 * JW + t; i < total; i += NT) {
        int f, sg, el;
        decode(i, f, sg, el);
        const int so = SRCT[sg], src = PSRC[sg * NE + el];
        const int64_t ne = NBE[f * NE + el];
        T uL[5], uR[5], nL[3], F[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          const T own = PAN[(so * 5 + c) * NE + el], nb = u[((int64_t)src * 5 + c) * E + ne];
          uL[c] = left ? own : nb;
          uR[c] = left ? nb : own;
        }
        if constexpr (CUR) {
          tet_cur_unit_normal(geo, E, e0 + el, sg, left, nL);
        } else {
#pragma unroll
          for (int k = 0; k < 3; ++k) nL[k] = NRM[(f * 3 + k) * NE + el];
        }
        common_inviscid<T, DEV>(riemann, uL, uR, nL, gamma, R, F);
        fc[tet_fc_index<NE>(e0 + el, sg * 5)] = F[0] + tau * (uL[0] - uR[0]);
#pragma unroll
        for (int c = 1; c < 5; ++c)
          fc[tet_fc_index<NE>(e0 + el, sg * 5 + c)] =
              (F[c] + tau * (uL[c] - uR[c])) - PAN[FVB + (sg * 4 + c - 1) * NE + el];
      }
    }
  }
}

}  // namespace frmi
