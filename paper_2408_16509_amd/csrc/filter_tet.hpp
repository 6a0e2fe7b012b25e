// Entropy-bounded modal filter for the order-4 tetrahedra (Sec. "Numerical Stability":
// modal filtering of the elements that violate positivity or the minimum-entropy
// bound, with the strength found iteratively so as to filter as little as possible).
// FP64 throughout; the same checks, s_min, search and features as the hexahedral
// filter, with these element-specific parts:
//
//   modes      u^ = V^{-1} u, V the orthonormal basis graded by total degree d
//              (mode m has degree 0 for m = 0, 1 for m < 4, 2 for m < 10, 3 for m < 20,
//              else 4)
//   filter     u^_m <- exp(-zeta (d_m / p)^2) u^_m
//   checks     the flux points of these elements coincide with solution points, so
//              the check points reduce to the 35 solution points (each flux point
//              repeats a value already checked; the violation fraction among the
//              features counts every repeat)
//
// One wave per element, lane z = solution point z (lanes 35..63 idle in the checks),
// no LDS and no block barriers: values move between lanes with readlane, decisions are
// wave votes.  The filtered state is linear in the five per-degree factors, so after
// one modal transform each lane keeps the per-degree parts of its point,
//     Q[d][v](z) = sum over the modes m of degree d of V[z][m] u^[v][m],
// and a constraint evaluation costs 25 FMAs per lane: u_F[v](z) = sum_d sigma_d Q[d][v](z).
// The check at zeta = 0 uses the nodal values themselves.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "filter.hpp"

namespace frmi {

constexpr int TF_NSP = 35, TF_P = 4;
// Device table (FP64): V^T [m][z], V^{-1} transposed [q][m], normalised quadrature
// weights [z], check-point multiplicity [z] (1 + number of flux points at z).
constexpr int TF_VT = 0, TF_VIT = TF_NSP * TF_NSP, TF_W = 2 * TF_NSP * TF_NSP, TF_MULT = TF_W + TF_NSP,
              TF_LEN = TF_MULT + TF_NSP;

__host__ __device__ constexpr int tet_mode_deg(int m) { return m < 1 ? 0 : (m < 4 ? 1 : (m < 10 ? 2 : (m < 20 ? 3 : 4))); }
// First mode of degree d (d = 5: the mode count).
__host__ __device__ constexpr int tet_deg_first(int d) { return d * (d + 1) * (d + 2) / 6; }

// Value of x in lane l (l wave-uniform).
__device__ __forceinline__ double rl_d(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xFFFFFFFFLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
struct TetFiltWave {
  double x[5];      // nodal state at point z = lane (lanes >= 35: point 0, never checked)
  double uh[5];     // modal coefficient m = lane
  double Q[5][5];   // per-degree parts [d][v] at point z = lane
};

// Nodal state and modal coefficients of element e.
__device__ __forceinline__ void tet_wave_load(const double* __restrict__ tab, const double* __restrict__ u, int64_t E,
                                              int64_t e, int lane, TetFiltWave& W) {
  const int z = lane < TF_NSP ? lane : 0;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    W.x[v] = u[((int64_t)z * 5 + v) * E + e];
    W.uh[v] = 0.0;
  }
#pragma unroll 5
  for (int q = 0; q < TF_NSP; ++q) {
    const double vi = tab[TF_VIT + q * TF_NSP + z];
#pragma unroll
    for (int v = 0; v < 5; ++v) W.uh[v] += vi * rl_d(W.x[v], q);
  }
}

// The per-degree parts Q of the lane's point (from the modal coefficients).
__device__ __forceinline__ void tet_wave_parts(const double* __restrict__ tab, int lane, TetFiltWave& W) {
  const int z = lane < TF_NSP ? lane : 0;
#pragma unroll
  for (int d = 0; d < 5; ++d) {
#pragma unroll
    for (int v = 0; v < 5; ++v) W.Q[d][v] = 0.0;
#pragma unroll 1
    for (int m = tet_deg_first(d); m < tet_deg_first(d + 1); ++m) {
      const double vt = tab[TF_VT + m * TF_NSP + z];
#pragma unroll
      for (int v = 0; v < 5; ++v) W.Q[d][v] += vt * rl_d(W.uh[v], m);
    }
  }
}

// Whether every check point is admissible at strength zeta (wave-uniform); w receives
// the lane's filtered values.
__device__ __forceinline__ bool tet_wave_check(const TetFiltWave& W, double zeta, double smin, const FiltPrm& F,
                                               int lane, double w[5]) {
  double s[5];
  s[0] = 1.0;
#pragma unroll
  for (int d = 1; d < 5; ++d) s[d] = exp(-zeta * (double)(d * d) / (double)(TF_P * TF_P));
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    double a = W.Q[0][v];
#pragma unroll
    for (int d = 1; d < 5; ++d) a += s[d] * W.Q[d][v];
    w[v] = a;
  }
  return __all(lane >= TF_NSP || admissible_screened(w, smin, F)) != 0;
}

__device__ __forceinline__ bool tet_wave_ok0(const TetFiltWave& W, double smin, const FiltPrm& F, int lane) {
  return __all(lane >= TF_NSP || admissible(W.x, smin, F)) != 0;
}

// Search and application for an element whose check at zeta = 0 failed.
__device__ void tet_filter_wave(const TetFiltWave& W, double* __restrict__ u, double smin, int64_t E, int64_t e,
                                int lane, const FiltPrm& F, int mode, float kh_in, int32_t* __restrict__ k_out,
                                int32_t* __restrict__ evals_out, const Dev32& s32) {
  int evals = 1;
  const double dz = F.zeta_max / (double)((int64_t)1 << F.n_bits);
  double w[5];
  auto G = [&](int64_t k) {
    ++evals;
    return tet_wave_check(W, (double)k * dz, smin, F, lane, w);
  };
  bool fallback = false;
  const int64_t hi = dyadic_search(F, mode, kh_in, G, fallback);
  const double zeta = fallback ? F.zeta_max : (double)hi * dz;
  (void)tet_wave_check(W, zeta, smin, F, lane, w);
  if (lane < TF_NSP) {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      u[((int64_t)lane * 5 + v) * E + e] = w[v];
      if (s32.p) s32.p[((int64_t)lane * 5 + v) * E + e] = (float)(w[v] - s32.ref[v]);
    }
  }
  if (lane == 0) {
    if (k_out) k_out[e] = fallback ? -1 : (int32_t)hi;
    if (evals_out) evals_out[e] = evals;
  }
}

// Own minimum entropy of each element (thread per element), in ord_bits form; NaN
// values are ignored (as fmin does).
__global__ void __launch_bounds__(256) tet_sown(const double* __restrict__ u, unsigned long long* __restrict__ sown,
                                                int64_t E, int64_t n, double gamma) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  double smin = INFINITY;
  for (int z = 0; z < TF_NSP; ++z) {
    double w[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) w[v] = u[((int64_t)z * 5 + v) * E + e];
    const double p = (gamma - 1.0) * (w[4] - 0.5 * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]) / w[0]);
    smin = fmin(smin, entropy_of(w[0], p, gamma));
  }
  sown[e] = ord_bits(smin);
}

// Detection (thread per element): pessimistic test at every solution point, as the
// hexahedral detection (flag must be cleared before).  With an RK stage source the
// thread also performs the stage update of its element (all E_pad elements), and
// cand64 (if not null) receives the FP64 stage state of a flagged element.
template <typename Src>
__global__ void __launch_bounds__(256) tet_filter_detect(Src src, const double* __restrict__ smin_a, int64_t E,
                                                         int64_t n, FiltPrm F, int32_t* __restrict__ flag,
                                                         double* __restrict__ cand64) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  constexpr bool kUpdate = !std::is_same<Src, PlainSrc>::value;
  if (e >= (kUpdate ? E : n)) return;
  const double smin = e < n ? smin_a[e] : 0.0;
  const double sb = smin - F.eps_s * fabs(smin);
  const double sbm = sb + 1e-10 * fabs(sb);
  const double lsb = sbm > 0 ? log(sbm) : -INFINITY;
  bool bad = false;
  for (int z = 0; z < TF_NSP && (kUpdate || !bad); ++z) {
    double w[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) w[v] = src(((int64_t)z * 5 + v) * E + e, v);
    bad = bad || maybe_violates(w, lsb, F);
  }
  if (!bad || e >= n) return;
  flag[e] = 1;
  if constexpr (kUpdate) {
    if (cand64)
      for (int i = 0; i < TF_NSP * 5; ++i) cand64[(int64_t)i * E + e] = src.stage((int64_t)i * E + e);
  }
}

// The 16 features (same definitions as for hexahedra; the shells are the total
// degrees 1, 2, >= 3 and the element mean comes from the quadrature weights) of an
// element whose check at zeta = 0 failed; wave-uniform result.
__device__ void tet_wave_features(const TetFiltWave& W, const double* __restrict__ tab, double smin,
                                  const FiltPrm& F, int lane, float x[16]) {
  const double g = F.gamma;
  const bool act = lane < TF_NSP;
  const int z = act ? lane : 0;
  const double wz = act ? tab[TF_W + z] : 0.0, mult = act ? tab[TF_MULT + z] : 0.0;
  double mean[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) mean[v] = wave_sum(wz * W.x[v]);
  const double rb = mean[0], vx = mean[1] / rb, vy = mean[2] / rb, vz = mean[3] / rb, Eb = mean[4];
  const double pb = (g - 1.0) * (Eb - 0.5 * rb * (vx * vx + vy * vy + vz * vz));
  const double pbc = fmax(pb, 1e-300);
  const double cb = sqrt(g * pbc / rb);
  const double sb = pbc * pow(rb, -g);
  const double rho = W.x[0];
  const double p = (g - 1.0) * (W.x[4] - 0.5 * (W.x[1] * W.x[1] + W.x[2] * W.x[2] + W.x[3] * W.x[3]) / rho);
  double s = entropy_of(rho, p, g);
  if (!isfinite(s)) s = -1e30;
  const double mrho = wave_min(act ? rho : INFINITY);
  const double mp = wave_min(act ? p : INFINITY);
  const double ms = wave_min(act ? s : INFINITY);
  const double mdr = wave_max(act ? fabs(rho - rb) : 0.0);
  const double nbad = wave_sum(act && !admissible(W.x, smin, F) ? mult : 0.0);
  // modal coefficients of the nodal pressure (lane m)
  double ph = 0.0;
#pragma unroll 5
  for (int q = 0; q < TF_NSP; ++q) ph += tab[TF_VIT + q * TF_NSP + z] * rl_d(p, q);
  const int dm = tet_mode_deg(z);
  double en[3][3];
#pragma unroll
  for (int fi = 0; fi < 3; ++fi) {
    const double c = fi == 0 ? W.uh[0] : (fi == 1 ? W.uh[4] : ph);
    const double c0 = rl_d(c, 0);
    const double e0 = c0 * c0 + 1e-300;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const bool in = act && (q < 2 ? dm == q + 1 : dm >= 3);
      en[fi][q] = wave_sum(in ? c * c : 0.0) / e0;
    }
  }
#pragma unroll
  for (int fi = 0; fi < 3; ++fi)
#pragma unroll
    for (int q = 0; q < 3; ++q) x[3 * fi + q] = (float)log10(fmax(en[fi][q], 1e-30));
  x[9] = (float)(mrho / rb - 1.0);
  x[10] = (float)(mp / pb - 1.0);
  x[11] = (float)fmin(fmax((ms - smin) / fmax(fabs(smin), 1e-300), -10.0), 10.0);
  x[12] = (float)(nbad / (double)(TF_NSP + 60));
  x[13] = (float)(mdr / rb);
  x[14] = (float)log10(fmax(sb / fmax(smin, 1e-300), 1e-30));
  x[15] = (float)(sqrt(vx * vx + vy * vy + vz * vz) / cb);
}

// Candidates list[0 .. *count), one wave per candidate.
__global__ void __launch_bounds__(256) tet_filter(double* __restrict__ u, const double* __restrict__ smin_a, int64_t E,
                                                  const int32_t* __restrict__ list, const int32_t* __restrict__ count,
                                                  const double* __restrict__ tab, FiltPrm F,
                                                  int32_t* __restrict__ k_out, int32_t* __restrict__ evals_out,
                                                  Dev32 s32) {
  const int lane = threadIdx.x & 63;
  const int32_t m = *count;
  for (int32_t i = blockIdx.x * 4 + (threadIdx.x >> 6); i < m; i += gridDim.x * 4) {
    const int32_t e = list[i];
    const double smin = smin_a[e];
    TetFiltWave W;
    tet_wave_load(tab, u, E, e, lane, W);
    if (tet_wave_ok0(W, smin, F, lane)) continue;   // k = 0, one evaluation (set by the reset)
    tet_wave_parts(tab, lane, W);
    tet_filter_wave(W, u, smin, E, e, lane, F, 0, 0.0f, k_out, evals_out, s32);
  }
}

// Features of the candidates list[0 .. *count): flag[e] = 1 and feat[e] for the
// elements failing the check at zeta = 0, flag[e] = 0 for the others.
__global__ void __launch_bounds__(256) tet_features(const double* __restrict__ u, const double* __restrict__ smin_a,
                                                    int64_t E, const int32_t* __restrict__ list,
                                                    const int32_t* __restrict__ count, const double* __restrict__ tab,
                                                    FiltPrm F, int32_t* __restrict__ flag, float* __restrict__ feat) {
  const int lane = threadIdx.x & 63;
  const int32_t m = *count;
  for (int32_t i = blockIdx.x * 4 + (threadIdx.x >> 6); i < m; i += gridDim.x * 4) {
    const int32_t e = list[i];
    const double smin = smin_a[e];
    TetFiltWave W;
    tet_wave_load(tab, u, E, e, lane, W);
    if (tet_wave_ok0(W, smin, F, lane)) {
      if (lane == 0) flag[e] = 0;
      continue;
    }
    float x[16];
    tet_wave_features(W, tab, smin, F, lane, x);
    if (lane < 16) {
      float xv = x[0];
#pragma unroll
      for (int k = 1; k < 16; ++k) xv = lane == k ? x[k] : xv;
      feat[(int64_t)e * 16 + lane] = xv;
    }
    if (lane == 0) flag[e] = 1;
  }
}

// The learned warm start in one pass per candidate: features, the MLP forward
// (mlp_wave_khat), then the search bracketed around the predicted index 2^(n y).
__global__ void __launch_bounds__(256) tet_filter_learned(double* __restrict__ u, const double* __restrict__ smin_a,
                                                          int64_t E, const int32_t* __restrict__ list,
                                                          const int32_t* __restrict__ count,
                                                          const double* __restrict__ tab, FiltPrm F,
                                                          const float* __restrict__ wm, const float* __restrict__ scale,
                                                          int32_t* __restrict__ k_out, int32_t* __restrict__ evals_out,
                                                          Dev32 s32) {
  const int lane = threadIdx.x & 63;
  const int32_t m = *count;
  for (int32_t i = blockIdx.x * 4 + (threadIdx.x >> 6); i < m; i += gridDim.x * 4) {
    const int32_t e = list[i];
    const double smin = smin_a[e];
    TetFiltWave W;
    tet_wave_load(tab, u, E, e, lane, W);
    if (tet_wave_ok0(W, smin, F, lane)) continue;
    float x[16];
    tet_wave_features(W, tab, smin, F, lane, x);
    const float kh = mlp_wave_khat(wm, scale, x, lane, F.n_bits);
    tet_wave_parts(tab, lane, W);
    tet_filter_wave(W, u, smin, E, e, lane, F, 1, kh, k_out, evals_out, s32);
  }
}

}  // namespace frmi
