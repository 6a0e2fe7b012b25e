// Order-4 pyramids with an affine base (Sec. "Mixed elements and domain decomposition":
// the transition element, supported with an affine base), meshes of pyramids only.
//
// The rational pyramid space has no tensor structure and its 55 x 55 operators are
// dense, so these kernels apply them as plain matrix-vector products: one wave per
// element, a lane per solution point or flux point, the element's transformed fluxes
// and interface jumps staged in LDS, the operators (transposed so that lanes read
// consecutive entries) shared by all waves through the caches.  The steps are those of
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
constexpr int PY_WAVES = 4;                 // elements (waves) per block

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

// Step 1 (eq:disu): traces of u at the flux points.  Thread = (element, flux point):
// lanes are 64 consecutive elements, a wave one flux point of a 64-element tile.
template <typename T>
__global__ void __launch_bounds__(256) pyr_trace(const T* __restrict__ u, T* __restrict__ uf, int64_t E,
                                                 const T* __restrict__ It) {
  const int64_t gtid = xcd_block() * 256 + threadIdx.x;
  const int64_t wave = gtid >> 6;
  const int64_t tile = wave / PY_NFP;
  const int fp = (int)(wave % PY_NFP);
  const int64_t e = tile * 64 + (gtid & 63);
  if (e >= E) return;
  T acc[5] = {0, 0, 0, 0, 0};
  for (int j = 0; j < PY_NSP; ++j) {
    const T w = It[j * PY_NFP + fp];
#pragma unroll
    for (int v = 0; v < 5; ++v) acc[v] += w * u[((int64_t)j * 5 + v) * E + e];
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) uf[((int64_t)fp * 5 + v) * E + e] = acc[v];
}

// Navier--Stokes gradient (LDG): grad~u = D_i u + lift (n~_i (u^ - u_f)), u^ = (uL + uR)/2
// + beta (uL - uR); physical grad_j = sum_i S_ij / J grad~_i u.  Writes grad at the
// solution points and its traces at the flux points.
template <typename T>
__global__ void __launch_bounds__(64 * PY_WAVES) pyr_grad(const T* __restrict__ u, const T* __restrict__ uf,
                                                          const T* __restrict__ geo, Conn C, PyrOpsDev<T> O, PyrK<T> K,
                                                          T* __restrict__ grad, T* __restrict__ gradf, int64_t E, T beta) {
  __shared__ T U_s[PY_WAVES][5][PY_NSP];
  __shared__ T JM_s[PY_WAVES][5][PY_NFP];
  __shared__ T G_s[PY_WAVES][15][PY_NSP];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t e = xcd_block() * PY_WAVES + w;
  T S[9], J;
  pyr_metric(geo, E, e, S, J);
  if (lane < PY_NSP)
#pragma unroll
    for (int v = 0; v < 5; ++v) U_s[w][v][lane] = u[((int64_t)lane * 5 + v) * E + e];
  for (int fp = lane; fp < PY_NFP; fp += 64) {
    int f, fpn;
    int64_t en;
    bool left;
    pyr_partner(C, K, E, e, fp, f, en, fpn, left);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const T uo = uf[((int64_t)fp * 5 + v) * E + e];
      const T un = uf[((int64_t)fpn * 5 + v) * E + en];
      const T uL = left ? uo : un, uR = left ? un : uo;
      JM_s[w][v][fp] = T(0.5) * (uL + uR) + beta * (uL - uR) - uo;
    }
  }
  __syncthreads();
  if (lane < PY_NSP) {
    T gt[3][5];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int v = 0; v < 5; ++v) gt[i][v] = 0;
    for (int j = 0; j < PY_NSP; ++j) {
      const T d0 = O.Dt[(0 * PY_NSP + j) * PY_NSP + lane];
      const T d1 = O.Dt[(1 * PY_NSP + j) * PY_NSP + lane];
      const T d2 = O.Dt[(2 * PY_NSP + j) * PY_NSP + lane];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const T x = U_s[w][v][j];
        gt[0][v] += d0 * x;
        gt[1][v] += d1 * x;
        gt[2][v] += d2 * x;
      }
    }
    for (int fp = 0; fp < PY_NFP; ++fp) {
      const T l = O.Lt[fp * PY_NSP + lane];
      const int f = pyr_face_of(K.face_off, fp);
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const T x = l * JM_s[w][v][fp];
        gt[0][v] += x * K.nref[f][0];
        gt[1][v] += x * K.nref[f][1];
        gt[2][v] += x * K.nref[f][2];
      }
    }
    const T iJ = rcp(J);
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const T g = (S[0 * 3 + j] * gt[0][v] + S[1 * 3 + j] * gt[1][v] + S[2 * 3 + j] * gt[2][v]) * iJ;
        G_s[w][v * 3 + j][lane] = g;
        grad[((int64_t)lane * 15 + v * 3 + j) * E + e] = g;
      }
  }
  __syncthreads();
  for (int fp = lane; fp < PY_NFP; fp += 64) {
    T acc[15];
#pragma unroll
    for (int k = 0; k < 15; ++k) acc[k] = 0;
    for (int j = 0; j < PY_NSP; ++j) {
      const T l = O.It[j * PY_NFP + fp];
#pragma unroll
      for (int k = 0; k < 15; ++k) acc[k] += l * G_s[w][k][j];
    }
#pragma unroll
    for (int k = 0; k < 15; ++k) gradf[((int64_t)fp * 15 + k) * E + e] = acc[k];
  }
}

// Corrected divergence (Euler, or Navier--Stokes with NS = true), R = -div / J.
template <typename T, bool DEV, bool NS>
__global__ void __launch_bounds__(64 * PY_WAVES) pyr_div(const T* __restrict__ u, const T* __restrict__ uf,
                                                         const T* __restrict__ grad, const T* __restrict__ gradf,
                                                         const T* __restrict__ geo, Conn C, PyrOpsDev<T> O, PyrK<T> K,
                                                         T* __restrict__ r, int64_t E, T gamma, T mu, T pr, T beta,
                                                         T tau, int riemann, RefState<T> R) {
  __shared__ T F_s[PY_WAVES][3][5][PY_NSP];
  __shared__ T JM_s[PY_WAVES][5][PY_NFP];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t e = xcd_block() * PY_WAVES + w;
  const T gm1 = gamma - T(1);
  T S[9], J;
  pyr_metric(geo, E, e, S, J);
  // transformed flux f~_i = (S f)_i at the solution points
  if (lane < PY_NSP) {
    T wv[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) wv[v] = u[((int64_t)lane * 5 + v) * E + e];
    T g[15];
    if constexpr (NS) {
#pragma unroll
      for (int k = 0; k < 15; ++k) g[k] = grad[((int64_t)lane * 15 + k) * E + e];
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
      for (int v = 0; v < 5; ++v) F_s[w][i][v][lane] = f[v];
    }
  }
  __syncthreads();
  // common flux minus the normal trace of f~ at the flux points
  for (int fp = lane; fp < PY_NFP; fp += 64) {
    int f, fpn;
    int64_t en;
    bool left;
    pyr_partner(C, K, E, e, fp, f, en, fpn, left);
    const T* nr = K.nref[f];
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
      T go[15], gn[15];
#pragma unroll
      for (int k = 0; k < 15; ++k) {
        go[k] = gradf[((int64_t)fp * 15 + k) * E + e];
        gn[k] = gradf[((int64_t)fpn * 15 + k) * E + en];
      }
      T fvL[5], fvR[5];
      viscous<T, DEV>(uL, left ? go : gn, nL[0], nL[1], nL[2], gamma, mu, pr, R, fvL);
      viscous<T, DEV>(uR, left ? gn : go, nL[0], nL[1], nL[2], gamma, mu, pr, R, fvR);
#pragma unroll
      for (int v = 0; v < 5; ++v)
        Fc[v] -= T(0.5) * (fvL[v] + fvR[v]) - beta * (fvL[v] - fvR[v]) - tau * (uL[v] - uR[v]);
    }
    T fperp[5] = {0, 0, 0, 0, 0};
    for (int j = 0; j < PY_NSP; ++j) {
      const T l = O.It[j * PY_NFP + fp];
#pragma unroll
      for (int v = 0; v < 5; ++v)
        fperp[v] += l * (nr[0] * F_s[w][0][v][j] + nr[1] * F_s[w][1][v][j] + nr[2] * F_s[w][2][v][j]);
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) JM_s[w][v][fp] = mag * sg * Fc[v] - fperp[v];
  }
  __syncthreads();
  if (lane < PY_NSP) {
    T div[5] = {0, 0, 0, 0, 0};
    for (int j = 0; j < PY_NSP; ++j) {
      const T d0 = O.Dt[(0 * PY_NSP + j) * PY_NSP + lane];
      const T d1 = O.Dt[(1 * PY_NSP + j) * PY_NSP + lane];
      const T d2 = O.Dt[(2 * PY_NSP + j) * PY_NSP + lane];
#pragma unroll
      for (int v = 0; v < 5; ++v) div[v] += d0 * F_s[w][0][v][j] + d1 * F_s[w][1][v][j] + d2 * F_s[w][2][v][j];
    }
    for (int fp = 0; fp < PY_NFP; ++fp) {
      const T l = O.Lt[fp * PY_NSP + lane];
#pragma unroll
      for (int v = 0; v < 5; ++v) div[v] += l * JM_s[w][v][fp];
    }
    const T iJ = -rcp(J);
#pragma unroll
    for (int v = 0; v < 5; ++v) r[((int64_t)lane * 5 + v) * E + e] = div[v] * iJ;
  }
}

}  // namespace frmi
