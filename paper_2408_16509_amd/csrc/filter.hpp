// Entropy-bounded modal filter for hexahedra (Sec. "Numerical Stability": modal
// filtering, applied per element only where density, pressure or a minimum-entropy
// bound is violated, with the strength found iteratively so as to filter as
// little as possible).  FP64 throughout.
//
//   modes      u^ = V^{-1} u, tensor Legendre modes (i, j, k)
//   filter     u^_ijk <- exp(-zeta (i^2 + j^2 + k^2) / p^2) u^_ijk  (separable in i, j, k)
//   checks     at the solution points and the 6 (p+1)^2 face flux points:
//              rho >= eps_rho, p >= eps_p, s = p rho^-gamma >= s_min - eps_s |s_min|
//   s_min      min of s over the check points of the element and of its face
//              neighbours, taken from the state at the start of the step
//   search     k in [0, 2^n], zeta = k zeta_max / 2^n; G(0) -> untouched; not G(2^n)
//              -> zeta_max (fallback, k = -1); else bisection keeping G(lo) false and
//              G(hi) true, result hi.  A predicted k^ (learned warm start) replaces the
//              starting bracket by [floor(k^/2), ceil(2 k^)] and the search continues in
//              whichever bracket keeps that invariant.
//
// One wave per candidate element (several per block, each with its own LDS region; no
// block barriers, decisions are wave votes).  A constraint evaluation at strength zeta
// is three 1-D passes through the wave's LDS with the filtered evaluation matrix
//     W[r][m] = P~_m(x_r) exp(-zeta m^2 / p^2),   r = nodes 0..p, then xi = -1, +1,
// so a check point (r1, r2, r3) with at most one end row covers both solution and
// flux points.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hex.hpp"

namespace frmi {

constexpr int FNT = 256;   // threads of the filter blocks

struct FiltK {
  double Vm[5][5];    // P~_m(x_a) (rows nodes, cols modes)
  double Vmi[5][5];   // inverse: modes from nodal values
  double Pe[2][5];    // P~_m(-1), P~_m(+1)
  double lm[5], lp[5];
};

struct FiltPrm {
  double gamma, eps_rho, eps_p, eps_s, zeta_max;
  int n_bits;
};

// Optional FP32 copy of a filtered state: the deviation (u - ref) in the native layout
// of the FP32 form (p null: none).
struct Dev32 {
  float* p;
  double ref[5];
};

// Where a detection pass takes its FP64 states from (called once per value of the
// pass, in native index i = (pt * 5 + v) * E + e).  PlainSrc: the state itself.
// RkStageSrc: the classical RK4 stage update fused into the pass, so the stage state
// is formed in registers instead of being written and read back:
//   stages 1..3 (mode 0 first, 1 middle): acc = (first ? u : acc) + b k, s = u + c k,
//   optionally s64 = s (the FP64 form, whose right-hand side reads it) and
//   s32 = (float)(s - ref) (the FP32 form's deviation); the pass checks s;
//   last stage (mode 2): u = acc + b k (in place), s32 as above; the pass checks u.
// stage() recomputes s for the candidates' FP64 copy (the same fused multiply-adds).
// Both take a value in two steps, so a caller can issue the loads of several values
// before any of them is used: raw(i) reads what the value needs, value(i, v, raw)
// forms it (and performs the update's stores).
struct PlainSrc {
  const double* __restrict__ u;
  struct Raw { double x; };
  __device__ __forceinline__ Raw raw(int64_t i) const { return Raw{u[i]}; }
  __device__ __forceinline__ double value(int64_t, int, const Raw& r) const { return r.x; }
  __device__ __forceinline__ double operator()(int64_t i, int v) const { return value(i, v, raw(i)); }
  __device__ __forceinline__ double peek(int64_t i) const { return u[i]; }
};
template <typename KT>
struct RkStageSrc {
  double* u;
  const KT* k;
  double* acc;
  double* s64;
  float* s32;
  double b, c;
  int mode;
  double ref[5];
  struct Raw { double x, a; KT k; };
  __device__ __forceinline__ double stage(int64_t i) const { return fma(c, (double)k[i], u[i]); }
  // the value value() forms, read without side effects from what the update leaves
  // unchanged (u_n and k in the stages, the accumulator and k in the last one)
  __device__ __forceinline__ double peek(int64_t i) const {
    return mode == 2 ? fma(b, (double)k[i], acc[i]) : fma(c, (double)k[i], u[i]);
  }
  __device__ __forceinline__ Raw raw(int64_t i) const {
    return Raw{mode == 2 ? 0.0 : u[i], mode == 0 ? 0.0 : acc[i], k[i]};
  }
  __device__ __forceinline__ double value(int64_t i, int v, const Raw& r) const {
    const double rk = (double)r.k;
    if (mode == 2) {
      const double un = fma(b, rk, r.a);
      u[i] = un;
      if (s32) s32[i] = (float)(un - ref[v]);
      return un;
    }
    acc[i] = fma(b, rk, mode == 0 ? r.x : r.a);
    const double si = fma(c, rk, r.x);
    if (s64) s64[i] = si;
    if (s32) s32[i] = (float)(si - ref[v]);
    return si;
  }
  __device__ __forceinline__ double operator()(int64_t i, int v) const { return value(i, v, raw(i)); }
};

__device__ __forceinline__ double entropy_of(double rho, double p, double gamma) {
  return rho > 0 ? p * pow(rho, -gamma) : -INFINITY;
}

__device__ __forceinline__ bool admissible(const double w[5], double smin, const FiltPrm& F) {
  const double rho = w[0];
  const double p = (F.gamma - 1.0) * (w[4] - 0.5 * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]) / rho);
  const double s = entropy_of(rho, p, F.gamma);
  return rho >= F.eps_rho && p >= F.eps_p && s >= smin - F.eps_s * fabs(smin);
}

// The same decision as admissible(), with the entropy test screened in FP32 logarithms:
// log2 p - gamma log2 rho - log2 s_b is formed from FP32 values (each log2f within a few
// ulp, so the computed value is within about 1e-4 of the exact one for the magnitudes
// admitted below); only when it lies within 2^-8 of zero is the exact FP64 power formed.
// Points far from the entropy bound (nearly all of them) skip the FP64 pow.
__device__ __forceinline__ bool admissible_screened(const double w[5], double smin, const FiltPrm& F) {
  const double rho = w[0];
  const double p = (F.gamma - 1.0) * (w[4] - 0.5 * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]) / rho);
  if (!(rho >= F.eps_rho) || !(p >= F.eps_p)) return false;
  const double sb = smin - F.eps_s * fabs(smin);
  if (sb <= 0.0) return true;                   // s > 0 here
  const float pf = (float)p, rf = (float)rho, bf = (float)sb;
  if (pf >= 1e-30f && pf <= 1e30f && rf >= 1e-30f && rf <= 1e30f && bf >= 1e-30f && bf <= 1e30f) {
    const float L = log2f(pf) - (float)F.gamma * log2f(rf) - log2f(bf);
    if (L > 0.00390625f) return true;
    if (L < -0.00390625f) return false;
  }
  return p * pow(rho, -F.gamma) >= sb;
}

// Doubles as unsigned integers with the same order (for an atomic minimum).
__device__ __forceinline__ unsigned long long ord_bits(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ULL);
}
__device__ __forceinline__ double ord_val(unsigned long long o) {
  return __longlong_as_double((long long)((o >> 63) ? (o & 0x7FFFFFFFFFFFFFFFULL) : ~o));
}

__global__ void k_fill_u64(unsigned long long* __restrict__ a, int64_t n, unsigned long long v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

// Check points of a tile of NE elements, each point read from HBM once: a block of
// NE x (p+1)^2 threads stages the tile's states in LDS (U[v][pt][el], 40 KB at p = 3
// and 4), thread (el, column (c0, c1)) then visits the N1 solution points of its own
// column (the line along xi_3 through (c0, c1)), that line's two ends, and the ends of
// the lines along xi_1 through (c0, c1) = (j, k) and along xi_2 through (c0, c1) = (i, k)
// — every solution point once and every face flux point once.  f(w) is called per
// check point with its state w[5].
template <int P>
struct HexTileCfg {
  static constexpr int N1 = P + 1, NE = P == 1 ? 64 : (P == 2 ? 32 : (P == 3 ? 16 : 8)), NT = NE * N1 * N1;
};

template <int P, typename Src, typename Fn>
__device__ __forceinline__ void hex_tile_checks(const Src& src, double* U, int64_t E, int64_t e0, const FiltK& K,
                                                Fn&& f) {
  using C = HexTileCfg<P>;
  constexpr int N1 = C::N1, NE = C::NE, NSP = N1 * N1 * N1;
  const int el = threadIdx.x % NE, l = threadIdx.x / NE, c0 = l % N1, c1 = l / N1;
  const int64_t e = e0 + el;
  double m[5] = {0, 0, 0, 0, 0}, pl[5] = {0, 0, 0, 0, 0};
  // the column's reads are issued point by point ahead of their use: the raw values of
  // the next point load while the current one is formed, stored and checked
  typename Src::Raw rw[5], rn[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) rn[v] = src.raw(((int64_t)(c0 + N1 * c1) * 5 + v) * E + e);
#pragma unroll
  for (int a = 0; a < N1; ++a) {
    const int pt = c0 + N1 * (c1 + N1 * a);
#pragma unroll
    for (int v = 0; v < 5; ++v) rw[v] = rn[v];
    if (a + 1 < N1) {
#pragma unroll
      for (int v = 0; v < 5; ++v) rn[v] = src.raw(((int64_t)(pt + N1 * N1) * 5 + v) * E + e);
    }
    double w[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      w[v] = src.value(((int64_t)pt * 5 + v) * E + e, v, rw[v]);
      U[(v * NSP + pt) * NE + el] = w[v];
      m[v] += K.lm[a] * w[v];
      pl[v] += K.lp[a] * w[v];
    }
    f(w);
  }
  f(m);
  f(pl);
  __syncthreads();
#pragma unroll
  for (int d = 0; d < 2; ++d) {
#pragma unroll
    for (int v = 0; v < 5; ++v) { m[v] = 0; pl[v] = 0; }
#pragma unroll
    for (int a = 0; a < N1; ++a) {
      const int pt = d == 0 ? a + N1 * (c0 + N1 * c1) : c0 + N1 * (a + N1 * c1);
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const double x = U[(v * NSP + pt) * NE + el];
        m[v] += K.lm[a] * x;
        pl[v] += K.lp[a] * x;
      }
    }
    f(m);
    f(pl);
  }
}

// Minimum entropy of each element over its check points (one tile of elements per
// block, hex_tile_checks); NaN values are ignored (as fmin does).  sown holds the
// minimum in ord_bits form and must start at ord_bits(+inf).
template <int P>
__global__ void __launch_bounds__(HexTileCfg<P>::NT) hex_sown(const double* __restrict__ u,
                                                             unsigned long long* __restrict__ sown, int64_t E,
                                                             int64_t n, FiltK K, double gamma) {
  using C = HexTileCfg<P>;
  __shared__ double U[5 * C::N1 * C::N1 * C::N1 * C::NE];
  const int64_t e0 = xcd_block() * C::NE, e = e0 + threadIdx.x % C::NE;
  double smin = INFINITY;
  hex_tile_checks<P>(PlainSrc{u}, U, E, e0, K, [&](const double w[5]) {
    const double p = (gamma - 1.0) * (w[4] - 0.5 * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]) / w[0]);
    smin = fmin(smin, entropy_of(w[0], p, gamma));
  });
  if (e < n && !isnan(smin)) atomicMin(sown + e, ord_bits(smin));
}

// s_min over the element and its face neighbours.
__global__ void __launch_bounds__(256) elem_smin(const unsigned long long* __restrict__ sown,
                                                 const int32_t* __restrict__ nbr_elem, int nfaces,
                                                 double* __restrict__ smin, int64_t E, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  double s = ord_val(sown[e]);
  for (int f = 0; f < nfaces; ++f) s = fmin(s, ord_val(sown[nbr_elem[(int64_t)f * E + e]]));
  smin[e] = s;
}

// Wave-level synchronisation of LDS traffic between the lanes of one wave.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Butterfly reductions over the 64 lanes; every lane receives the same bits.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) v = fmin(v, __shfl_xor(v, s));
  return v;
}
__device__ __forceinline__ double wave_max(double v) { return -wave_min(-v); }
__device__ __forceinline__ float rl_f(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

// Waves (candidates) per filter block: the LDS of one wave grows as (p + 1)^3.
template <int P>
struct HexFW { static constexpr int value = P <= 3 ? 4 : 2; };

template <int P>
struct HexWaveSmem {
  static constexpr int N1 = P + 1, NR = N1 + 2, NSP = N1 * N1 * N1;
  double U[5][NSP];                    // modal coefficients u^[v][i + N1 j + N1^2 k]
  double T1[5][N1 * N1 * NR];          // [v][i + N1 j][r3]
  double T2[5][N1 * NR * NR];          // [v][i][r2][r3]
  double W[NR][N1];                    // filtered evaluation matrix
  double PM[NSP];                      // nodal, then modal pressure (features)
};

// Check point c (solution points, then the 6 faces' flux points) as evaluation rows.
template <int N1>
__device__ __forceinline__ void hex_check_rows(int c, int& r1, int& r2, int& r3) {
  constexpr int NSP = N1 * N1 * N1;
  if (c < NSP) {
    r1 = c % N1; r2 = (c / N1) % N1; r3 = c / (N1 * N1);
  } else {
    const int f = (c - NSP) / (N1 * N1), q = (c - NSP) % (N1 * N1), d = f / 2, s = f % 2;
    const int ta = q % N1, tb = q / N1, end = N1 + s;
    r1 = d == 0 ? end : ta;
    r2 = d == 0 ? ta : (d == 1 ? end : tb);
    r3 = d == 2 ? end : tb;
  }
}

// The first two passes of an evaluation at the strength held in S.W (into T1, T2).
template <int P>
__device__ void hex_wave_passes(HexWaveSmem<P>& S, int lane) {
  constexpr int N1 = P + 1, NR = N1 + 2;
  for (int o = lane; o < 5 * N1 * N1 * NR; o += 64) {      // over k: T1[v][i + N1 j][r3]
    const int v = o / (N1 * N1 * NR), rem = o % (N1 * N1 * NR), ij = rem / NR, r3 = rem % NR;
    double acc = 0;
#pragma unroll
    for (int k = 0; k < N1; ++k) acc += S.W[r3][k] * S.U[v][ij + N1 * N1 * k];
    S.T1[v][rem] = acc;
  }
  wave_sync();
  for (int o = lane; o < 5 * N1 * NR * NR; o += 64) {      // over j: T2[v][i][r2][r3]
    const int v = o / (N1 * NR * NR), rem = o % (N1 * NR * NR);
    const int i = rem / (NR * NR), r2 = (rem / NR) % NR, r3 = rem % NR;
    double acc = 0;
#pragma unroll
    for (int j = 0; j < N1; ++j) acc += S.W[r2][j] * S.T1[v][(i + N1 * j) * NR + r3];
    S.T2[v][rem] = acc;
  }
  wave_sync();
}

// The state at check point (r1, r2, r3) after the passes (the last pass, over i).
template <int P>
__device__ __forceinline__ void hex_wave_point(const HexWaveSmem<P>& S, int r1, int r2, int r3, double w[5]) {
  constexpr int N1 = P + 1, NR = N1 + 2;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    double acc = 0;
#pragma unroll
    for (int i = 0; i < N1; ++i) acc += S.W[r1][i] * S.T2[v][(i * NR + r2) * NR + r3];
    w[v] = acc;
  }
}

// Check-point evaluation at the strength held in S.W: returns (wave-uniformly) whether
// every check point is admissible.  When `store` is non-null the nodal values at the
// solution points are written there ([pt][5][E] layout).
template <int P>
__device__ bool hex_wave_checks(HexWaveSmem<P>& S, int lane, double smin, const FiltPrm& F,
                                double* __restrict__ store, const Dev32& s32, int64_t E, int64_t e) {
  constexpr int N1 = P + 1, NSP = N1 * N1 * N1, NFP = 6 * N1 * N1;
  hex_wave_passes<P>(S, lane);
  bool ok = true;
  for (int c = lane; c < NSP + NFP; c += 64) {
    int r1, r2, r3;
    hex_check_rows<N1>(c, r1, r2, r3);
    double w[5];
    hex_wave_point<P>(S, r1, r2, r3, w);
    ok = ok && admissible_screened(w, smin, F);
    if (store && c < NSP) {
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        store[((int64_t)c * 5 + v) * E + e] = w[v];
        if (s32.p) s32.p[((int64_t)c * 5 + v) * E + e] = (float)(w[v] - s32.ref[v]);
      }
    }
  }
  return __all(ok) != 0;
}

template <int P>
__device__ __forceinline__ void hex_wave_set_w(HexWaveSmem<P>& S, const FiltK& K, double zeta, int lane) {
  constexpr int N1 = P + 1, NR = N1 + 2;
  if (lane < NR * N1) {
    const int r = lane / N1, m = lane % N1;
    const double sig = exp(-zeta * (double)(m * m) / (double)(P * P));
    const double pm = r < N1 ? K.Vm[r][m] : K.Pe[r - N1][m];
    S.W[r][m] = pm * sig;
  }
  wave_sync();
}

// Nodal values of nv variables (X, [v][pt]) -> modal coefficients (into `out`),
// three 1-D passes with V^{-1}; Y is scratch of the same size.
template <int P>
__device__ void hex_wave_to_modal(double* X, double* Y, double* out, int nv, const FiltK& K, int lane) {
  constexpr int N1 = P + 1, NSP = N1 * N1 * N1;
  for (int o = lane; o < nv * NSP; o += 64) {
    const int v = o / NSP, pt = o % NSP, ij = pt % (N1 * N1), m = pt / (N1 * N1);
    double acc = 0;
#pragma unroll
    for (int k = 0; k < N1; ++k) acc += K.Vmi[m][k] * X[v * NSP + ij + N1 * N1 * k];
    Y[o] = acc;
  }
  wave_sync();
  for (int o = lane; o < nv * NSP; o += 64) {
    const int v = o / NSP, pt = o % NSP, i = pt % N1, m = (pt / N1) % N1, kk = pt / (N1 * N1);
    double acc = 0;
#pragma unroll
    for (int j = 0; j < N1; ++j) acc += K.Vmi[m][j] * Y[v * NSP + i + N1 * j + N1 * N1 * kk];
    X[o] = acc;
  }
  wave_sync();
  for (int o = lane; o < nv * NSP; o += 64) {
    const int v = o / NSP, pt = o % NSP, m = pt % N1, rest = pt / N1;
    double acc = 0;
#pragma unroll
    for (int i = 0; i < N1; ++i) acc += K.Vmi[m][i] * X[v * NSP + i + N1 * rest];
    out[o] = acc;
  }
  wave_sync();
}

template <int P>
__device__ void hex_wave_load_modal(HexWaveSmem<P>& S, const double* __restrict__ u, int64_t E, int64_t e,
                                    const FiltK& K, int lane) {
  constexpr int N1 = P + 1, NSP = N1 * N1 * N1;
  double* X = &S.T1[0][0];
  double* Y = &S.T2[0][0];
  for (int o = lane; o < 5 * NSP; o += 64) {
    const int v = o / NSP, pt = o % NSP;
    X[o] = u[((int64_t)pt * 5 + v) * E + e];
  }
  wave_sync();
  hex_wave_to_modal<P>(X, Y, &S.U[0][0], 5, K, lane);
}

// The search shared by the element types, for an element that fails the checks at
// zeta = 0.  G(k) evaluates the checks at zeta = k zeta_max / 2^n (block-uniform).
// Plain (mode 0): G(2^n) false -> fallback, else bisection on [0, 2^n] keeping G(lo)
// false and G(hi) true.  Warm start (mode 1): the predicted index kh gives the bracket
// [floor(kh / 2), ceil(2 kh)]; its ends are evaluated and the bisection continues in
// whichever bracket keeps that invariant.  Returns hi (meaningless with fallback).
template <typename Gf>
__device__ int64_t dyadic_search(const FiltPrm& F, int mode, float kh_in, Gf& G, bool& fallback) {
  const int64_t N = (int64_t)1 << F.n_bits;
  int64_t lo = 0, hi = N;
  fallback = false;
  if (mode == 1) {
    double kh = (double)kh_in;
    kh = fmin(fmax(kh, 1.0), (double)N);
    const int64_t blo = (int64_t)floor(kh / 2), bhi = min((int64_t)ceil(2 * kh), N);
    const bool g_hi = G(bhi);
    if (g_hi) {
      bool g_lo = false;
      if (blo > 0) g_lo = G(blo);
      if (g_lo) { lo = 0; hi = blo; }
      else { lo = blo; hi = bhi; }
    } else {
      lo = bhi; hi = N;
      fallback = bhi >= N ? true : !G(N);
    }
  } else {
    fallback = !G(N);
  }
  if (!fallback) {
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) / 2;
      if (G(mid)) hi = mid;
      else lo = mid;
    }
  }
  return hi;
}

// Search (mode 0 plain, 1 warm start from the predicted index kh) and application of
// the filter for an element whose modal coefficients are in S.U and whose check at
// zeta = 0 has failed.
template <int P>
__device__ void hex_wave_search(HexWaveSmem<P>& S, int lane, double* __restrict__ u, double smin, int64_t E,
                                int64_t e, const FiltK& K, const FiltPrm& F, int mode, float kh_in,
                                int32_t* __restrict__ k_out, int32_t* __restrict__ evals_out, const Dev32& s32) {
  int evals = 1;
  const double dz = F.zeta_max / (double)((int64_t)1 << F.n_bits);
  auto G = [&](int64_t k) {
    hex_wave_set_w<P>(S, K, (double)k * dz, lane);
    ++evals;
    return hex_wave_checks<P>(S, lane, smin, F, nullptr, Dev32{}, E, e);
  };
  bool fallback = false;
  const int64_t hi = dyadic_search(F, mode, kh_in, G, fallback);
  const double zeta = fallback ? F.zeta_max : (double)hi * dz;
  hex_wave_set_w<P>(S, K, zeta, lane);
  (void)hex_wave_checks<P>(S, lane, smin, F, u, s32, E, e);
  if (lane == 0) {
    if (k_out) k_out[e] = fallback ? -1 : (int32_t)hi;
    if (evals_out) evals_out[e] = evals;
  }
}

// The candidates list[0 .. *count) (from the detection), one wave per candidate:
// modal transform, exact check at zeta = 0, then the plain search.
template <int P>
__global__ void __launch_bounds__(64 * HexFW<P>::value) hex_filter(
    double* __restrict__ u, const double* __restrict__ smin_a, int64_t E, const int32_t* __restrict__ list,
    const int32_t* __restrict__ count, FiltK K, FiltPrm F, int32_t* __restrict__ k_out,
    int32_t* __restrict__ evals_out, Dev32 s32) {
  constexpr int FW = HexFW<P>::value;
  __shared__ HexWaveSmem<P> SM[FW];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  HexWaveSmem<P>& S = SM[wv];
  const int32_t m = *count;
  for (int32_t i = blockIdx.x * FW + wv; i < m; i += gridDim.x * FW) {
    const int32_t e = list[i];
    const double smin = smin_a[e];
    hex_wave_load_modal<P>(S, u, E, e, K, lane);
    hex_wave_set_w<P>(S, K, 0.0, lane);
    if (hex_wave_checks<P>(S, lane, smin, F, nullptr, Dev32{}, E, e)) continue;   // k = 0 (set by the reset)
    hex_wave_search<P>(S, lane, u, smin, E, e, K, F, 0, 0.0f, k_out, evals_out, s32);
  }
}

// ---------------------------------------------------------------------------
// Detection: elements that may fail the checks at zeta = 0, every check point of a
// tile staged once (hex_tile_checks).  The test is pessimistic by a relative 1e-10 in rho, E and
// |m|^2 (far above the rounding of either evaluation), so every element the exact
// check of the search rejects is flagged; the search re-checks and leaves false
// positives untouched.  flag must be cleared before.
// lsb = log(bound + dl |bound|) of the entropy bound, or -inf when that is <= 0
// (then any state with positive density and pressure passes the entropy check).
// The entropy part is screened like admissible_screened: log2 plo - gamma log2 rhi -
// lsb / ln 2 in FP32 (within ~1e-5 of the exact value for the magnitudes admitted),
// decided there unless it lies within 2^-8 of zero; only then the FP64 logarithms.
__device__ __forceinline__ bool maybe_violates(const double w[5], double lsb, const FiltPrm& F) {
  constexpr double dl = 1e-10;
  const double rho = w[0];
  const double rlo = rho - dl * fabs(rho), rhi = rho + dl * fabs(rho);
  if (!(rlo >= F.eps_rho)) return true;
  const double m2 = (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]) * (1.0 + dl);
  const double plo = (F.gamma - 1.0) * (w[4] - dl * fabs(w[4]) - 0.5 * m2 / rlo);
  if (!(plo >= F.eps_p)) return true;
  if (lsb == -INFINITY) return false;
  const float pf = (float)plo, rf = (float)rhi;
  if (pf >= 1e-30f && pf <= 1e30f && rf >= 1e-30f && rf <= 1e30f && fabs(lsb) <= 60.0) {
    const float L = log2f(pf) - (float)F.gamma * log2f(rf) - (float)(lsb * 1.4426950408889634);
    if (L > 0.00390625f) return false;
    if (L < -0.00390625f) return true;
  }
  return !(log(plo) - F.gamma * log(rhi) >= lsb);
}

// Detection of the candidates of the exact search: thread (el, column) flags its element
// when one of its check points may violate a bound.  With an RK stage source the pass
// also performs the stage update (every value of the tile once), and cand64 (if not
// null) receives the FP64 stage state of the flagged elements from the tile in LDS.
template <int P, typename Src>
__global__ void __launch_bounds__(HexTileCfg<P>::NT) hex_filter_detect(Src src, const double* __restrict__ smin_a,
                                                                      int64_t E, int64_t n, FiltK K, FiltPrm F,
                                                                      int32_t* __restrict__ flag,
                                                                      double* __restrict__ cand64) {
  using C = HexTileCfg<P>;
  constexpr int NSP = C::N1 * C::N1 * C::N1;
  __shared__ double U[5 * NSP * C::NE];
  __shared__ int BAD[C::NE];
  const int el = threadIdx.x % C::NE;
  const int64_t e0 = xcd_block() * C::NE, e = e0 + el;
  if (threadIdx.x < C::NE) BAD[threadIdx.x] = 0;
  const double smin = smin_a[e];
  const double sb = smin - F.eps_s * fabs(smin);
  const double sbm = sb + 1e-10 * fabs(sb);
  const double lsb = sbm > 0 ? log(sbm) : -INFINITY;
  bool bad = false;
  hex_tile_checks<P>(src, U, E, e0, K, [&](const double w[5]) { bad = bad || maybe_violates(w, lsb, F); });
  bad = bad && e < n;
  if (bad) flag[e] = 1;
  if (cand64 == nullptr) return;
  if (bad) BAD[el] = 1;
  __syncthreads();
  if (!BAD[el]) return;
  const int l = threadIdx.x / C::NE, c0 = l % C::N1, c1 = l / C::N1;
  for (int a = 0; a < C::N1; ++a) {
    const int pt = c0 + C::N1 * (c1 + C::N1 * a);
#pragma unroll
    for (int v = 0; v < 5; ++v) cand64[((int64_t)pt * 5 + v) * E + e] = U[(v * NSP + pt) * C::NE + el];
  }
}

// Detection without LDS staging: one wave per (64-element tile, column (c0, c1)), lanes
// over consecutive elements, so every row the wave touches is a 64-element (512-byte
// FP64) segment.  The thread checks its own column (the line along xi_3: its points and
// both ends, every value once through src, which performs the RK stage update if any)
// and the ends of the lines along xi_1 through (c0, c1) = (j, k) and along xi_2 through
// (i, k) = (c0, c1), whose values it reads through src.peek (no side effects; the
// other lines' owners update them) -- every solution point once and every face flux
// point once per element, as in the tiled detection.  flag[e] = 1 for elements that may
// fail (flag cleared before).
template <int P, typename Src>
__global__ void __launch_bounds__(256) hex_filter_detect_lines(Src src, const double* __restrict__ smin_a,
                                                               int64_t E, int64_t n, FiltK K, FiltPrm F,
                                                               int32_t* __restrict__ flag) {
  constexpr int N1 = P + 1, NC = N1 * N1;
  const int64_t gtid = xcd_block() * 256 + threadIdx.x;
  const int64_t wave = gtid >> 6;
  const int lane = (int)(gtid & 63);
  const int64_t tile = wave / NC;
  const int l = (int)(wave % NC), c0 = l % N1, c1 = l / N1;
  const int64_t e = tile * 64 + lane;
  if (e >= E) return;                   // E is a multiple of 64: whole waves only
  const double smin = e < n ? smin_a[e] : 0.0;
  const double sb = smin - F.eps_s * fabs(smin);
  const double sbm = sb + 1e-10 * fabs(sb);
  const double lsb = sbm > 0 ? log(sbm) : -INFINITY;
  bool bad = false;
  // own column: raw values of the next point in flight while the current one is formed.
  // The xi_1 line through (j, k) = (c0, c1) and the xi_2 line through (i, k) = (c0, c1)
  // both lie at height c1, so they are read in the iteration a = c1, when the waves that
  // own those columns read the same height: the values are then still in L2 (read a
  // column later, most of them had to come from HBM again).
  double m[5] = {0, 0, 0, 0, 0}, pl[5] = {0, 0, 0, 0, 0};
  typename Src::Raw rw[5], rn[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) rn[v] = src.raw(((int64_t)(c0 + N1 * c1) * 5 + v) * E + e);
  // not unrolled: one copy of the lines' block (the height a is wave-uniform)
#pragma unroll 1
  for (int a = 0; a < N1; ++a) {
    const int pt = c0 + N1 * (c1 + N1 * a);
#pragma unroll
    for (int v = 0; v < 5; ++v) rw[v] = rn[v];
    // the next point's loads: issued before this point is formed, except in the
    // iteration of the two lines, where they follow the lines' reads (keeping them
    // apart keeps the registers of the two sets apart)
    if (a + 1 < N1 && a != c1) {        // wave-uniform
#pragma unroll
      for (int v = 0; v < 5; ++v) rn[v] = src.raw(((int64_t)(pt + NC) * 5 + v) * E + e);
    }
    double w[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      w[v] = src.value(((int64_t)pt * 5 + v) * E + e, v, rw[v]);
      m[v] += K.lm[a] * w[v];
      pl[v] += K.lp[a] * w[v];
    }
    bad = bad || maybe_violates(w, lsb, F);
    if (a == c1) {
#pragma unroll 1
      for (int d = 0; d < 2; ++d) {
        // point b of the line: (b, c0, c1) along xi_1, (c0, b, c1) along xi_2
        const int q0 = d == 0 ? N1 * (c0 + N1 * c1) : c0 + N1 * N1 * c1, qs = d == 0 ? 1 : N1;
        double lm[5] = {0, 0, 0, 0, 0}, lp[5] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int b = 0; b < N1; ++b) {
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            const double x = src.peek(((int64_t)(q0 + qs * b) * 5 + v) * E + e);
            lm[v] += K.lm[b] * x;
            lp[v] += K.lp[b] * x;
          }
        }
        bad = bad || maybe_violates(lm, lsb, F) || maybe_violates(lp, lsb, F);
      }
      if (a + 1 < N1) {
#pragma unroll
        for (int v = 0; v < 5; ++v) rn[v] = src.raw(((int64_t)(pt + NC) * 5 + v) * E + e);
      }
    }
  }
  bad = bad || maybe_violates(m, lsb, F) || maybe_violates(pl, lsb, F);
  if (bad && e < n) flag[e] = 1;
}

// FP64 stage state u + c k of the candidates (the search's input in the FP32 form,
// whose detection pass forms the stage state without storing it): one block of 256
// threads per candidate, values in native layout.
template <typename KT>
__global__ void __launch_bounds__(256) k_cand_stage(RkStageSrc<KT> src, const int32_t* __restrict__ list,
                                                    const int32_t* __restrict__ count, int nvals, int64_t E,
                                                    double* __restrict__ cand64) {
  const int cnt = *count;
  for (int i = blockIdx.x; i < cnt; i += gridDim.x) {
    const int64_t e = list[i];
    for (int j = threadIdx.x; j < nvals; j += 256) cand64[(int64_t)j * E + e] = src.stage((int64_t)j * E + e);
  }
}

__global__ void k_fill_i32(int32_t* __restrict__ a, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

// Reset of a filter call: no candidates flagged, k = 0 and one evaluation everywhere.
__global__ void k_filter_reset(int32_t* __restrict__ det, int32_t* __restrict__ k, int32_t* __restrict__ evals,
                               int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    det[i] = 0;
    k[i] = 0;
    evals[i] = 1;
  }
}

// Ordered compaction of the flagged elements into a list: per-256 counts, one
// block scanning the counts (count[nb] receives the total), scatter.
__global__ void __launch_bounds__(256) k_flag_count(const int32_t* __restrict__ flag, int64_t n,
                                                    int32_t* __restrict__ counts) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int c = __syncthreads_count(e < n && flag[e] != 0);
  if (threadIdx.x == 0) counts[blockIdx.x] = c;
}

__global__ void __launch_bounds__(1024) k_scan_counts(int32_t* __restrict__ counts, int nb) {
  __shared__ int32_t part[1024];
  const int t = threadIdx.x;
  const int chunk = (nb + 1023) / 1024, lo = min(t * chunk, nb), hi = min(lo + chunk, nb);
  int32_t s = 0;
  for (int i = lo; i < hi; ++i) s += counts[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {      // inclusive scan (Hillis--Steele)
    const int32_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int32_t run = t > 0 ? part[t - 1] : 0;
  for (int i = lo; i < hi; ++i) {
    const int32_t c = counts[i];
    counts[i] = run;
    run += c;
  }
  if (t == 1023) counts[nb] = part[1023];
}

__global__ void __launch_bounds__(256) k_flag_scatter(const int32_t* __restrict__ flag, int64_t n,
                                                      const int32_t* __restrict__ offsets, int32_t* __restrict__ list) {
  __shared__ int32_t wsum[4];
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool f = e < n && flag[e] != 0;
  const uint64_t mask = __ballot(f);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) wsum[w] = __popcll(mask);
  __syncthreads();
  int32_t base = offsets[blockIdx.x];
  for (int i = 0; i < w; ++i) base += wsum[i];
  if (f) list[base + __popcll(mask & ((1ull << lane) - 1ull))] = (int32_t)e;
}

// The 16 per-element features of the learned warm start, for an element whose modal
// coefficients are in S.U and whose check at zeta = 0 (evaluated with S.W at zeta = 0,
// so T2 holds its passes) has failed:
//   0-8   log10 of the modal energy of rho, E, p in the shells max(i,j,k) = 1, 2, >= 3,
//         relative to the mean mode's energy (floored at 1e-30)
//   9     min rho / rho_mean - 1        10  min p / p_mean - 1
//   11    (min s - s_min) / |s_min| clipped to [-10, 10]
//   12    fraction of violating check points
//   13    max |rho - rho_mean| / rho_mean
//   14    log10(s_mean / s_min)         15  |v_mean| / c_mean
// (mean = element mean state; its pressure, entropy and sound speed.)  The result is
// wave-uniform.
template <int P>
__device__ void hex_wave_features(HexWaveSmem<P>& S, int lane, double smin, const FiltK& K, const FiltPrm& F,
                                  float x[16]) {
  constexpr int N1 = P + 1, NSP = N1 * N1 * N1, NFP = 6 * N1 * N1;
  const double g = F.gamma;
  // mean state from the (0,0,0) mode: mean = u^_000 P~_0^3 = u^_000 / (2 sqrt 2)
  const double c0 = 1.0 / (2.0 * sqrt(2.0));
  const double rb = S.U[0][0] * c0, mx = S.U[1][0] * c0, my = S.U[2][0] * c0, mz = S.U[3][0] * c0;
  const double Eb = S.U[4][0] * c0;
  const double vx = mx / rb, vy = my / rb, vz = mz / rb;
  const double pb = (g - 1.0) * (Eb - 0.5 * rb * (vx * vx + vy * vy + vz * vz));
  const double pbc = fmax(pb, 1e-300);
  const double cb = sqrt(g * pbc / rb);
  const double sb = pbc * pow(rb, -g);
  // check-point statistics at zeta = 0
  // the minimum entropy: each lane ranks its points by an FP32 estimate of log2 s and
  // forms s exactly (FP64 pow) for its lowest one only
  double mrho = INFINITY, mp = INFINITY, mdr = 0, nbad = 0;
  double arho = 1.0, ap = 1.0;
  float al = INFINITY;
  bool nonfinite = false;
  for (int c = lane; c < NSP + NFP; c += 64) {
    int r1, r2, r3;
    hex_check_rows<N1>(c, r1, r2, r3);
    double w[5];
    hex_wave_point<P>(S, r1, r2, r3, w);
    const double p = (g - 1.0) * (w[4] - 0.5 * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]) / w[0]);
    if (!(w[0] > 0.0) || !isfinite(p)) {
      nonfinite = true;
    } else {
      const float l = log2f(fmaxf((float)fabs(p), 1e-37f)) - (float)g * log2f((float)w[0]);
      const bool lower = p < 0.0 ? (ap >= 0.0 || l > al) : (ap >= 0.0 && l < al);
      if (lower) { al = l; arho = w[0]; ap = p; }
    }
    mrho = fmin(mrho, w[0]);
    mp = fmin(mp, p);
    mdr = fmax(mdr, fabs(w[0] - rb));
    nbad += admissible_screened(w, smin, F) ? 0.0 : 1.0;
    if (c < NSP) S.PM[c] = p;
  }
  double ms = al < INFINITY ? entropy_of(arho, ap, g) : INFINITY;
  if (!isfinite(ms)) ms = -1e30;
  if (nonfinite) ms = -1e30;
  mrho = wave_min(mrho);
  mp = wave_min(mp);
  ms = wave_min(ms);
  mdr = wave_max(mdr);
  nbad = wave_sum(nbad);
  wave_sync();
  // modal coefficients of the nodal pressure
  double* X = &S.T1[0][0];
  double* Y = &S.T2[0][0];
  for (int o = lane; o < NSP; o += 64) X[o] = S.PM[o];
  wave_sync();
  hex_wave_to_modal<P>(X, Y, S.PM, 1, K, lane);
  // shell energies of rho (U[0]), E (U[4]), p (PM)
#pragma unroll
  for (int fi = 0; fi < 3; ++fi) {
    const double* c = fi == 0 ? S.U[0] : (fi == 1 ? S.U[4] : S.PM);
    double sh[3] = {0, 0, 0};
    for (int m = lane; m < NSP; m += 64) {
      const int i = m % N1, j = (m / N1) % N1, k = m / (N1 * N1);
      const int shell = max(i, max(j, k));
      if (shell >= 1) sh[min(shell, 3) - 1] += c[m] * c[m];
    }
    const double e0 = c[0] * c[0] + 1e-300;
#pragma unroll
    for (int q = 0; q < 3; ++q) x[3 * fi + q] = (float)log10(fmax(wave_sum(sh[q]) / e0, 1e-30));
  }
  x[9] = (float)(mrho / rb - 1.0);
  x[10] = (float)(mp / pb - 1.0);
  x[11] = (float)fmin(fmax((ms - smin) / fmax(fabs(smin), 1e-300), -10.0), 10.0);
  x[12] = (float)(nbad / (double)(NSP + NFP));
  x[13] = (float)(mdr / rb);
  x[14] = (float)log10(fmax(sb / fmax(smin, 1e-300), 1e-30));
  x[15] = (float)(sqrt(vx * vx + vy * vy + vz * vz) / cb);
}

// Features of the candidates list[0 .. *count), one wave per candidate: flag[e] = 1 and
// feat[e] for the elements failing the check at zeta = 0, flag[e] = 0 for the others.
template <int P>
__global__ void __launch_bounds__(64 * HexFW<P>::value) hex_features(
    const double* __restrict__ u, const double* __restrict__ smin_a, int64_t E, const int32_t* __restrict__ list,
    const int32_t* __restrict__ count, FiltK K, FiltPrm F, int32_t* __restrict__ flag, float* __restrict__ feat) {
  constexpr int FW = HexFW<P>::value;
  __shared__ HexWaveSmem<P> SM[FW];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  HexWaveSmem<P>& S = SM[wv];
  const int32_t m = *count;
  for (int32_t i = blockIdx.x * FW + wv; i < m; i += gridDim.x * FW) {
    const int32_t e = list[i];
    const double smin = smin_a[e];
    hex_wave_load_modal<P>(S, u, E, e, K, lane);
    hex_wave_set_w<P>(S, K, 0.0, lane);
    if (hex_wave_checks<P>(S, lane, smin, F, nullptr, Dev32{}, E, e)) {
      if (lane == 0) flag[e] = 0;
      continue;
    }
    float x[16];
    hex_wave_features<P>(S, lane, smin, K, F, x);
    if (lane < 16) {
      float xv = x[0];
#pragma unroll
      for (int k = 1; k < 16; ++k) xv = lane == k ? x[k] : xv;
      feat[(int64_t)e * 16 + lane] = xv;
    }
    if (lane == 0) flag[e] = 1;
    wave_sync();
  }
}

// The warm-start index 2^(n y) from the MLP forward pass on features x (wave-uniform):
// lane t holds hidden unit t of both layers and reads its rows of the flat weights
// W1[64][16] b1 W2[64][64] b2 w3 b3 (and the input scaling [mean; std]) through the
// caches, 16 bytes at a time.
__device__ __forceinline__ float mlp_wave_khat(const float* __restrict__ wm, const float* __restrict__ scale,
                                               const float x[16], int lane, int n_bits) {
  const float4* r1 = reinterpret_cast<const float4*>(wm + lane * 16);
  float a = wm[64 * 16 + lane];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 c = r1[q];
    a += c.x * ((x[4 * q] - scale[4 * q]) / scale[16 + 4 * q]);
    a += c.y * ((x[4 * q + 1] - scale[4 * q + 1]) / scale[16 + 4 * q + 1]);
    a += c.z * ((x[4 * q + 2] - scale[4 * q + 2]) / scale[16 + 4 * q + 2]);
    a += c.w * ((x[4 * q + 3] - scale[4 * q + 3]) / scale[16 + 4 * q + 3]);
  }
  const float h1 = tanhf(a);
  const float4* r2 = reinterpret_cast<const float4*>(wm + 64 * 16 + 64 + lane * 64);
  float b = wm[64 * 16 + 64 + 64 * 64 + lane];
#pragma unroll 4
  for (int q = 0; q < 16; ++q) {
    const float4 c = r2[q];
    b += c.x * rl_f(h1, 4 * q) + c.y * rl_f(h1, 4 * q + 1) + c.z * rl_f(h1, 4 * q + 2) + c.w * rl_f(h1, 4 * q + 3);
  }
  const double contrib = (double)(wm[64 * 16 + 64 + 64 * 64 + 64 + lane] * tanhf(b));
  const double y = wave_sum(contrib) + (double)wm[64 * 16 + 64 + 64 * 64 + 64 + 64];
  return exp2f((float)n_bits * (float)y);
}

// The learned warm start in one pass per candidate (one wave each): modal transform,
// exact check at zeta = 0, features, the MLP forward, then the search bracketed around
// the predicted index.
template <int P>
__global__ void __launch_bounds__(64 * HexFW<P>::value) hex_filter_learned(
    double* __restrict__ u, const double* __restrict__ smin_a, int64_t E, const int32_t* __restrict__ list,
    const int32_t* __restrict__ count, FiltK K, FiltPrm F, const float* __restrict__ w,
    const float* __restrict__ scale, int32_t* __restrict__ k_out, int32_t* __restrict__ evals_out, Dev32 s32) {
  constexpr int FW = HexFW<P>::value;
  __shared__ HexWaveSmem<P> SM[FW];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  HexWaveSmem<P>& S = SM[wv];
  const int32_t m = *count;
  for (int32_t i = blockIdx.x * FW + wv; i < m; i += gridDim.x * FW) {
    const int32_t e = list[i];
    const double smin = smin_a[e];
    hex_wave_load_modal<P>(S, u, E, e, K, lane);
    hex_wave_set_w<P>(S, K, 0.0, lane);
    if (hex_wave_checks<P>(S, lane, smin, F, nullptr, Dev32{}, E, e)) continue;
    float x[16];
    hex_wave_features<P>(S, lane, smin, K, F, x);
    const float kh = mlp_wave_khat(w, scale, x, lane, F.n_bits);
    hex_wave_search<P>(S, lane, u, smin, E, e, K, F, 1, kh, k_out, evals_out, s32);
  }
}

}  // namespace frmi
