// Device-side compressible-flow physics: Euler flux along a direction, Rusanov
// and HLLC common fluxes (the paper's 𝔉 "e.g. an appropriate Riemann solver"),
// and the Navier--Stokes viscous flux (Newtonian stress, Fourier heat flux with
// constant mu and Prandtl number).
#pragma once
#include <hip/hip_runtime.h>

namespace frmi {

// Reciprocal and square root as the right-hand side kernels take them: in FP32 the
// hardware instructions (within 1 ulp, against about ten instructions for the
// correctly rounded division and several for the square root), in FP64 IEEE division
// and sqrt.  The FP32 form's error is set by its FP32 products and storage, far above
// an ulp per operation.
template <typename T>
__device__ __forceinline__ T fdiv(T a, T b) { return a / b; }
template <>
__device__ __forceinline__ float fdiv<float>(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
template <typename T>
__device__ __forceinline__ T rcp(T x) { return fdiv(T(1), x); }
template <typename T>
__device__ __forceinline__ T fsqrt(T x) { return sqrt(x); }
template <>
__device__ __forceinline__ float fsqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }

struct Phys {
  double gamma, mu, prandtl, beta, tau;
  int riemann;     // 0 Rusanov, 1 HLLC
};

// f(u).s for a (not necessarily unit) direction s; also returns v.s and p.
template <typename T>
__device__ __forceinline__ void flux_dir(const T u[5], T sx, T sy, T sz, T gm1, T f[5], T& vs, T& p) {
  T ir = T(1) / u[0];
  T vx = u[1] * ir, vy = u[2] * ir, vz = u[3] * ir;
  p = gm1 * (u[4] - T(0.5) * (u[1] * vx + u[2] * vy + u[3] * vz));
  vs = vx * sx + vy * sy + vz * sz;
  f[0] = u[0] * vs;
  f[1] = u[1] * vs + p * sx;
  f[2] = u[2] * vs + p * sy;
  f[3] = u[3] * vs + p * sz;
  f[4] = (u[4] + p) * vs;
}

template <typename T>
__device__ __forceinline__ void rusanov(const T uL[5], const T uR[5], const T n[3], T gamma, T F[5]) {
  T fL[5], fR[5], vnL, vnR, pL, pR;
  flux_dir(uL, n[0], n[1], n[2], gamma - T(1), fL, vnL, pL);
  flux_dir(uR, n[0], n[1], n[2], gamma - T(1), fR, vnR, pR);
  T cL = sqrt(gamma * pL / uL[0]), cR = sqrt(gamma * pR / uR[0]);
  T lam = fmax(fabs(vnL) + cL, fabs(vnR) + cR);
#pragma unroll
  for (int v = 0; v < 5; ++v) F[v] = T(0.5) * (fL[v] + fR[v]) - T(0.5) * lam * (uR[v] - uL[v]);
}

template <typename T>
__device__ __forceinline__ void hllc(const T uL[5], const T uR[5], const T n[3], T gamma, T F[5]) {
  T fL[5], fR[5], vnL, vnR, pL, pR;
  flux_dir(uL, n[0], n[1], n[2], gamma - T(1), fL, vnL, pL);
  flux_dir(uR, n[0], n[1], n[2], gamma - T(1), fR, vnR, pR);
  T rL = uL[0], rR = uR[0];
  T cL = sqrt(gamma * pL / rL), cR = sqrt(gamma * pR / rR);
  T SL = fmin(vnL - cL, vnR - cR);
  T SR = fmax(vnL + cL, vnR + cR);
  T Ss = (pR - pL + rL * vnL * (SL - vnL) - rR * vnR * (SR - vnR)) / (rL * (SL - vnL) - rR * (SR - vnR));
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
  const T* uK = left ? uL : uR;
  const T* fK = left ? fL : fR;
  T S = left ? SL : SR, vn = left ? vnL : vnR, p = left ? pL : pR, r = uK[0];
  T ir = T(1) / r;
  T fac = r * (S - vn) / (S - Ss);
  T us[5];
  us[0] = fac;
  us[1] = fac * (uK[1] * ir + (Ss - vn) * n[0]);
  us[2] = fac * (uK[2] * ir + (Ss - vn) * n[1]);
  us[3] = fac * (uK[3] * ir + (Ss - vn) * n[2]);
  us[4] = fac * (uK[4] * ir + (Ss - vn) * (Ss + p / (r * (S - vn))));
#pragma unroll
  for (int v = 0; v < 5; ++v) F[v] = fK[v] + S * (us[v] - uK[v]);
}

template <typename T>
__device__ __forceinline__ void riemann(int kind, const T uL[5], const T uR[5], const T n[3], T gamma, T F[5]) {
  if (kind == 1) hllc(uL, uR, n, gamma, F);
  else rusanov(uL, uR, n, gamma, F);
}

// Viscous flux along direction s: fv(u, grad u).s, with g[v*3 + j] = d u_v / d x_j.
template <typename T>
__device__ __forceinline__ void viscous_dir(const T u[5], const T g[15], T sx, T sy, T sz,
                                            T gamma, T mu, T prandtl, T fv[5]) {
  T ir = rcp(u[0]);
  T v[3] = {u[1] * ir, u[2] * ir, u[3] * ir};
  T gv[3][3];                                    // gv[i][j] = d v_i / d x_j
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) gv[i][j] = (g[(1 + i) * 3 + j] - v[i] * g[j]) * ir;
  // grad e = (grad E - (E/rho) grad rho - (rho v).grad v) / rho
  T Er = u[4] * ir;
  T ge[3];
#pragma unroll
  for (int j = 0; j < 3; ++j)
    ge[j] = (g[12 + j] - Er * g[j] - (u[1] * gv[0][j] + u[2] * gv[1][j] + u[3] * gv[2][j])) * ir;
  T div = gv[0][0] + gv[1][1] + gv[2][2];
  T s[3] = {sx, sy, sz};
  T ts[3];                                        // (tau s)_i = sum_j tau_ij s_j
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T acc = T(0);
#pragma unroll
    for (int j = 0; j < 3; ++j) acc += (gv[i][j] + gv[j][i]) * s[j];
    ts[i] = mu * (acc - T(2.0 / 3.0) * div * s[i]);
  }
  T kappa = fdiv(mu * gamma, prandtl);
  fv[0] = T(0);
  fv[1] = ts[0];
  fv[2] = ts[1];
  fv[3] = ts[2];
  fv[4] = ts[0] * v[0] + ts[1] * v[1] + ts[2] * v[2] + kappa * (ge[0] * sx + ge[1] * sy + ge[2] * sz);
}

}  // namespace frmi
