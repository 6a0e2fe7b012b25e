// C ABI of the MI355X-native FR right-hand side (declared in include/frmi.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/frmi.h"
#include "filter.hpp"
#include "filter_tet.hpp"
#include "hex.hpp"
#include "mlp.hpp"
#include "pyr.hpp"
#include "setup.hpp"
#include "tet.hpp"

using namespace frmi;

namespace {

thread_local std::string g_thread_err;

// x rounded to FP32, then split into bf16 hi = rne(x) and lo = rne(x - hi) (bit patterns).
uint16_t bf16_rne(float f) {
  uint32_t b;
  std::memcpy(&b, &f, 4);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}
void bf16_split_host(double x, uint16_t& hi, uint16_t& lo) {
  const float xf = (float)x;
  hi = bf16_rne(xf);
  const uint32_t hb = (uint32_t)hi << 16;
  float hf;
  std::memcpy(&hf, &hb, 4);
  lo = bf16_rne(xf - hf);
}

struct DevBlock {
  int etype = 0;
  int64_t n = 0, E = 0;
  int nsp = 0, nfp = 0, nfaces = 0;
  int64_t canon_off = 0, native_off = 0;
  double* geo = nullptr;    // FP64 geometry
  void* geo_t = nullptr;    // geometry in the kernels' arithmetic type (== geo for FP64)
  int32_t* nbr_elem = nullptr;
  int32_t* nbr_info = nullptr;
  void* uf = nullptr;       // [nfp][5][E]
  void* grad = nullptr;     // [nsp][15][E]
  void* gradf = nullptr;    // [nfp][15][E]
  void* fc = nullptr;       // [nfp][5][E] common fluxes (Navier--Stokes)
  void* cmet = nullptr;     // curved hexahedra: stored metric terms in the kernels' type (else NULL)
  int64_t elem_off = 0;     // offset of the block in the element numbering (both orders)
  int32_t* cpos = nullptr;  // native index -> canonical index within the block [E] (-1: padding)
  int32_t* npos = nullptr;  // canonical index -> native index within the block [n]
  double* sown = nullptr;   // entropy filter: own min entropy [E]
  double* smin = nullptr;   // entropy filter: neighbourhood min entropy [E]
  int32_t* f_det = nullptr;   // entropy filter: detection flags [n]
  int32_t* f_list = nullptr;  // candidates of the search, native ids [n]
  int32_t* f_cnt = nullptr;   // per-256 offsets [nb], then the candidate count
};

struct RefVec {
  double v[5];
};

}  // namespace

struct fr_ctx_s {
  fr_params prm;
  hipStream_t stream = nullptr;
  Setup host;
  std::vector<DevBlock> blocks;
  int32_t* perm = nullptr;
  int32_t* g_npos = nullptr;          // canonical -> native element index, all blocks [n_elem_total]
  std::vector<int32_t> h_cpos;        // native -> canonical element index, all blocks (host)
  int64_t canon_len = 0, native_len = 0;
  // RK workspace: stage state and increment in the native dtype, FP64 accumulator
  void* rk_stage = nullptr;
  double* rk_acc = nullptr;
  void* rk_k = nullptr;
  int* flag = nullptr;
  std::string err;
  // entropy filter / MLP workspace (canonical element order)
  int64_t n_elem_total = 0;
  int32_t* f_k = nullptr;
  int32_t* f_evals = nullptr;
  int32_t* f_flag = nullptr;
  float* f_feat = nullptr;
  float* f_khat = nullptr;
  double* f_copy = nullptr;     // FP64 native state copy (training targets)
  float* m_w = nullptr;         // MLP parameters, Adam moments, gradient, input scaling
  float* m_m = nullptr;
  float* m_v = nullptr;
  float* m_g = nullptr;
  float* m_scale = nullptr;
  float* m_loss = nullptr;
  float* m_scratch = nullptr;
  float* m_sqerr = nullptr;
  int32_t* m_idx = nullptr;
  int m_batch_cap = 0;
  bool mlp_ready = false;
  float* static_scratch = nullptr;  // this device's copy of the library's fixed scratch array
  // tetrahedral operators on the device (arithmetic type of the context)
  void* tet_opT = nullptr;    // [TET_KP][TET_MP] transposed divergence operator
  void* tet_ogT = nullptr;    // [TGS_K][TGR_M] transposed stacked gradient operator, face-sparse row order
  void* tet_opH = nullptr;    // BF16x3 split of the divergence operator: hi [TET_MP][TET_KP16], then lo
  void* tet_ogH = nullptr;    // BF16x3 split of the gradient operator: hi [TGR_M][TGR_K], then lo
  double* rk_x0 = nullptr;    // adaptive stepping: u_n and the error register (FP64)
  double* rk_err = nullptr;
  double* rk_part = nullptr;   // adaptive stepping: per-workgroup partial sums of the norm
  double* rk_s64 = nullptr;   // FP64 stage state of the filtered FP32 form    // [TET_KP][TET_MP] transposed divergence operator
  int32_t* tet_src = nullptr;
  void* pyr_ops = nullptr;    // pyramids: It [55][85], Dt [3][55][55], Lt [85][55] in the context's type
  double* tet_ftab = nullptr; // entropy filter on tetrahedra: modal operators, weights, multiplicities
  // training-data collection during filtered RK steps (fr_mlp_collect)
  bool collecting = false;
  float* col_x = nullptr;
  int32_t* col_k = nullptr;
  int64_t col_cap = 0, col_n = 0, col_seen = 0;
  // per-kernel event timing
  bool prof = false;
  struct ProfEv { int id; hipEvent_t a, b; };
  std::vector<std::string> prof_names;
  std::vector<ProfEv> prof_events;
  int prof_begin(const char* name) {
    if (!prof) return -1;
    int id = -1;
    for (size_t i = 0; i < prof_names.size(); ++i) if (prof_names[i] == name) id = (int)i;
    if (id < 0) { id = (int)prof_names.size(); prof_names.push_back(name); }
    ProfEv ev{id, nullptr, nullptr};
    if (hipEventCreate(&ev.a) != hipSuccess || hipEventCreate(&ev.b) != hipSuccess) return -1;
    (void)hipEventRecord(ev.a, stream);
    prof_events.push_back(ev);
    return (int)prof_events.size() - 1;
  }
  void prof_end(int k) {
    if (k >= 0) (void)hipEventRecord(prof_events[k].b, stream);
  }
  void prof_clear() {
    for (auto& e : prof_events) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
    prof_events.clear();
    prof_names.clear();
  }
};

// Fixed device scratch of fr_mlp_grad_static: per-sample quantities (MLP_SS floats each)
// of up to FR_MLP_STATIC_MAX_BATCH samples, then their squared errors.  Each GPU holds its
// own copy; host code uses only the device address taken once per device at setup.
constexpr int64_t kStaticScratchFloats = (int64_t)FR_MLP_STATIC_MAX_BATCH * (MLP_SS + 1);
static __device__ __align__(256) float scratch[kStaticScratchFloats];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_addr[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

// The current device's address of `scratch` (looked up once per device), or nullptr.
float* static_scratch_address() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_done[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      ptr = nullptr;
    }
    g_scratch_addr[dev] = (float*)ptr;
    g_scratch_done[dev] = true;
  }
  return g_scratch_addr[dev];
}

}  // namespace

namespace {

fr_status fail(fr_ctx c, fr_status s, const std::string& msg) {
  if (c) c->err = msg;
  else g_thread_err = msg;
  return s;
}

#define HIP_TRY(ctx, call)                                                                  \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return fail(ctx, FR_ERR_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
fr_status dalloc(fr_ctx c, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) return fail(c, FR_ERR_ALLOC, std::string("hipMalloc: ") + hipGetErrorString(e));
  return FR_OK;
}

Phys phys_of(const fr_params& p) {
  Phys ph;
  ph.gamma = p.gamma;
  ph.mu = p.mu;
  ph.prandtl = p.prandtl;
  ph.beta = p.ldg_beta;
  ph.tau = p.ldg_tau;
  ph.riemann = p.riemann;
  return ph;
}

// ------------------------------------------------------------ layout kernels
// Canonical [elem][var][pt] (input element order) <-> native [pt][var][E] (native
// element order, cpos / npos map between the two).
__global__ void k_pack(const double* __restrict__ canon, double* __restrict__ nat, const int32_t* __restrict__ cpos,
                       int64_t n, int64_t E, int nsp) {
  const int64_t total = (int64_t)nsp * 5 * E;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i % E;
    const int64_t pv = i / E;
    const int v = (int)(pv % 5), pt = (int)(pv / 5);
    nat[i] = e < n ? canon[((int64_t)cpos[e] * 5 + v) * nsp + pt] : (v == 0 || v == 4 ? 1.0 : 0.0);
  }
}

__global__ void k_unpack(const double* __restrict__ nat, double* __restrict__ canon, const int32_t* __restrict__ npos,
                         int64_t n, int64_t E, int nsp) {
  const int64_t total = n * 5 * nsp;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int pt = (int)(i % nsp);
    const int64_t ev = i / nsp;
    const int v = (int)(ev % 5);
    const int64_t e = ev / 5;
    canon[i] = nat[((int64_t)pt * 5 + v) * E + npos[e]];
  }
}

// Per-element values from native to canonical element order (both global numberings).
__global__ void k_elem_to_canon(const int32_t* __restrict__ src, const int32_t* __restrict__ npos, int64_t n,
                                int32_t* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[npos[i]];
}

// ------------------------------------------------------------ RK4 kernels
// stage 1: acc = u + dt/6 k ; st = u + dt/2 k  (FP64 state; increments FP64 or FP32)
template <typename KT>
__global__ void k_rk_first(const double* __restrict__ u, const KT* __restrict__ k, double* __restrict__ acc,
                           double* __restrict__ st, int64_t n, double b, double c) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double ui = u[i], ki = (double)k[i];
    acc[i] = ui + b * ki;
    st[i] = ui + c * ki;
  }
}
// middle stages: acc += b k ; st = u + c k
template <typename KT>
__global__ void k_rk_mid(const double* __restrict__ u, const KT* __restrict__ k, double* __restrict__ acc,
                         double* __restrict__ st, int64_t n, double b, double c) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double ki = (double)k[i];
    acc[i] += b * ki;
    st[i] = u[i] + c * ki;
  }
}
// last: u = acc + b k
template <typename KT>
__global__ void k_rk_last(double* __restrict__ u, const KT* __restrict__ k, const double* __restrict__ acc,
                          int64_t n, double b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    u[i] = acc[i] + b * (double)k[i];
}

// ------------------------------------------------------------ check kernel
__global__ void k_check(const double* __restrict__ u, int64_t n, int64_t E, int nsp, double gm1, int* flag) {
  const int64_t total = (int64_t)nsp * n;
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i % n;
    const int pt = (int)(i / n);
    double w[5];
    for (int v = 0; v < 5; ++v) w[v] = u[((int64_t)pt * 5 + v) * E + e];
    const double p = gm1 * (w[4] - 0.5 * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]) / w[0]);
    bool ok = true;
    for (int v = 0; v < 5; ++v) ok = ok && isfinite(w[v]);
    ok = ok && w[0] > 0 && p > 0 && isfinite(p);
    bad |= !ok;
  }
  if (bad) atomicOr(flag, 1);
}

int grid_for(int64_t n, int threads) {
  int64_t g = (n + threads - 1) / threads;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

// ------------------------------------------------------------ FP32-form kernels
// Deviation of the FP64 state from the reference state, rounded to FP32.
__global__ void k_to_dev(const double* __restrict__ u, float* __restrict__ w, int64_t n, int64_t E, RefVec ref) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    w[i] = (float)(u[i] - ref.v[(i / E) % 5]);
}
// ------------------------------------------------------------ embedded-pair stages
// One stage of the two-register embedded pair on a block's native values: with
// x = X (= u_n + dt sum_{j<i} b_j k_j) and the stage's increment k,
//   Y = x + dt a_{i+1,i} k  (the next stage state; in the native dtype, FP32 deviation
//   in the FP32 form), X = x + dt b_i k, Err (+)= dt (b_i - b^_i) k; the first stage also
// saves X0 = u_n.
template <typename KT, typename YT>
__global__ void k_lsrk_stage(double* __restrict__ X, double* __restrict__ X0, const KT* __restrict__ K,
                             YT* __restrict__ Y, double* __restrict__ Err, int64_t n, int64_t E, double ya,
                             double xb, double ed, int first, int last, RefVec ref) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double x = X[i], k = (double)K[i];
    if (first) X0[i] = x;
    if (!last) Y[i] = (YT)(x + ya * k - (sizeof(YT) == 4 ? ref.v[(i / E) % 5] : 0.0));
    X[i] = x + xb * k;
    Err[i] = (first ? 0.0 : Err[i]) + ed * k;
  }
}

// Partial sums of (Err / (atol + rtol max(|X0|, |X|)))^2 over a block's real elements
// (native index mod E < n_real): one FP64 sum per workgroup, in a fixed order.
__global__ void __launch_bounds__(256) k_err_sumsq(const double* __restrict__ Err, const double* __restrict__ X0,
                                                    const double* __restrict__ X, int64_t n, int64_t E,
                                                    int64_t n_real, double atol, double rtol,
                                                    double* __restrict__ part) {
  __shared__ double red[256];
  double a = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (i % E >= n_real) continue;
    const double sc = atol + rtol * fmax(fabs(X0[i]), fabs(X[i]));
    const double q = Err[i] / sc;
    a += q * q;
  }
  red[threadIdx.x] = a;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_pack32(const double* __restrict__ canon, float* __restrict__ nat, const int32_t* __restrict__ cpos,
                         int64_t n, int64_t E, int nsp, RefVec ref) {
  const int64_t total = (int64_t)nsp * 5 * E;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i % E;
    const int64_t pv = i / E;
    const int v = (int)(pv % 5), pt = (int)(pv / 5);
    nat[i] = e < n ? (float)(canon[((int64_t)cpos[e] * 5 + v) * nsp + pt] - ref.v[v]) : 0.0f;
  }
}
__global__ void k_unpack32(const float* __restrict__ nat, double* __restrict__ canon, const int32_t* __restrict__ npos,
                           int64_t n, int64_t E, int nsp, RefVec ref, int add_ref) {
  const int64_t total = n * 5 * nsp;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int pt = (int)(i % nsp);
    const int64_t ev = i / nsp;
    const int v = (int)(ev % 5);
    const int64_t e = ev / 5;
    canon[i] = (double)nat[((int64_t)pt * 5 + v) * E + npos[e]] + (add_ref ? ref.v[v] : 0.0);
  }
}
// RK stages of the FP32 form: FP64 state and accumulator, FP32 increments and stage deviations.
__global__ void k_rk32_first(const double* __restrict__ u, const float* __restrict__ k, double* __restrict__ acc,
                             float* __restrict__ st, int64_t n, int64_t E, double b, double c, RefVec ref) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double ui = u[i], ki = (double)k[i];
    acc[i] = ui + b * ki;
    st[i] = (float)(ui + c * ki - ref.v[(i / E) % 5]);
  }
}
__global__ void k_rk32_mid(const double* __restrict__ u, const float* __restrict__ k, double* __restrict__ acc,
                           float* __restrict__ st, int64_t n, int64_t E, double b, double c, RefVec ref) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double ki = (double)k[i];
    acc[i] += b * ki;
    st[i] = (float)(u[i] + c * ki - ref.v[(i / E) % 5]);
  }
}
__global__ void k_rk32_last(double* __restrict__ u, const float* __restrict__ k, const double* __restrict__ acc,
                            float* __restrict__ st, int64_t n, int64_t E, double b, RefVec ref) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double un = acc[i] + b * (double)k[i];
    u[i] = un;
    st[i] = (float)(un - ref.v[(i / E) % 5]);
  }
}

// Filtered FP32 form: the stage state in FP64 (for the filter) and its FP32 deviation
// (for the right-hand side) in one pass; acc = (first ? u : acc) + b k.
__global__ void k_rk32f_stage(const double* __restrict__ u, const float* __restrict__ k, double* __restrict__ acc,
                              double* __restrict__ s64, float* __restrict__ s32, int64_t n, int64_t E, double b,
                              double c, RefVec ref, int first) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double ui = u[i], ki = (double)k[i];
    acc[i] = (first ? ui : acc[i]) + b * ki;
    const double si = ui + c * ki;
    s64[i] = si;
    s32[i] = (float)(si - ref.v[(i / E) % 5]);
  }
}

// ------------------------------------------------------------ hex dispatch
template <int P>
struct HexCfg;
template <> struct HexCfg<1> { static constexpr int NE = 64; };
template <> struct HexCfg<2> { static constexpr int NE = 32; };
template <> struct HexCfg<3> { static constexpr int NE = 16; };
template <> struct HexCfg<4> { static constexpr int NE = 8; };
// element tile of the NS divergence (its LDS holds 10 or 15 values per point and element)
template <typename T, int P>
struct DivNsCfg { static constexpr int NE = (sizeof(T) == 8 ? 8 : 16) / (P == 4 ? 2 : 1) * (P <= 2 ? 2 : 1); };

template <typename T>
HexK<T> hexk_of(const HexOps& H) {
  HexK<T> k;
  for (int a = 0; a < 5; ++a) {
    k.x[a] = (T)H.x[a]; k.lm[a] = (T)H.lm[a]; k.lp[a] = (T)H.lp[a];
    k.cp[a] = (T)H.cp[a]; k.cm[a] = (T)H.cm[a];
    for (int b = 0; b < 5; ++b) k.Dh[a][b] = (T)H.Dh[a][b];
  }
  return k;
}

template <typename T>
RefState<T> ref_of(const fr_params& p) {
  RefState<T> R;
  R.rho0 = (T)p.u_ref[0];
  R.E0 = (T)p.u_ref[4];
  R.p0 = (T)((p.gamma - 1.0) * p.u_ref[4]);
  R.H0 = (T)(p.u_ref[4] + (p.gamma - 1.0) * p.u_ref[4]);
  return R;
}

int side_mode_of(double beta) { return beta == 0.5 ? 1 : (beta == -0.5 ? -1 : 0); }

template <typename T, bool DEV, int P, bool CUR>
fr_status hex_rhs_p(fr_ctx c, DevBlock& b, const T* u, T* r) {
  constexpr int N1 = P + 1, NE = HexCfg<P>::NE, NT = NE * N1 * N1;
  Conn C{b.nbr_elem, b.nbr_info, c->perm, c->host.perm_stride};
  const fr_params& p = c->prm;
  const HexK<T> K = hexk_of<T>(c->host.hex);
  const RefState<T> R = ref_of<T>(p);
  const T* geo = (const T*)b.geo_t;
  const T* cm = (const T*)b.cmet;
  T* uf = (T*)b.uf;
  T* grad = (T*)b.grad;
  T* gradf = (T*)b.gradf;
  const int sm = side_mode_of(p.ldg_beta);
  const int64_t trace_threads = b.E * 3 * N1 * N1;
  static const std::string sfx =
      std::string(CUR ? "_cur" : "") + (sizeof(T) == 8 ? "" : "_f32") + "_p" + std::to_string(P);
  int pk = c->prof_begin(("hex_trace" + sfx).c_str());
  hex_trace<T, P><<<(unsigned)((trace_threads + 255) / 256), 256, 0, c->stream>>>(u, uf, b.E, K);
  c->prof_end(pk);
  const unsigned nblk = (unsigned)(b.E / NE);
  if (p.system == FR_EULER) {
    pk = c->prof_begin(("hex_div_euler" + sfx).c_str());
    hex_div_euler<T, DEV, P, NE, CUR><<<nblk, NT, 0, c->stream>>>(u, uf, geo, cm, C, r, b.E, b.n, K, (T)p.gamma,
                                                                   p.riemann, R);
    c->prof_end(pk);
  } else {
    pk = c->prof_begin(("hex_grad" + sfx).c_str());
    if constexpr (P <= 3)
      hex_grad<T, P, NE, CUR><<<nblk, NT, 0, c->stream>>>(u, uf, geo, cm, C, grad, gradf, b.E, K, (T)p.ldg_beta, sm);
    else {
      // 16 FP32 elements per tile (64-byte rows); FP64 keeps 8 (64-byte rows as well)
      constexpr int NEg = sizeof(T) == 4 ? 16 : NE;
      hex_grad_lines<T, P, NEg, CUR><<<(unsigned)(b.E / NEg), NEg * N1 * N1, 0, c->stream>>>(
          u, uf, geo, cm, C, grad, gradf, b.E, K, (T)p.ldg_beta, sm);
    }
    c->prof_end(pk);
    T* fc = (T*)b.fc;
    const int64_t face_threads = b.E * 6 * N1 * N1;
    pk = c->prof_begin(("hex_face_ns" + sfx).c_str());
    hex_face_ns<T, DEV, P, CUR><<<(unsigned)((face_threads + 255) / 256), 256, 0, c->stream>>>(
        uf, gradf, geo, cm, C, fc, b.E, b.n, K, (T)p.gamma, (T)p.mu, (T)p.prandtl, (T)p.ldg_beta, (T)p.ldg_tau,
        p.riemann, sm, R);
    c->prof_end(pk);
    constexpr int NE2 = DivNsCfg<T, P>::NE;
    pk = c->prof_begin(("hex_div_ns" + sfx).c_str());
    // f~_3 of a column in registers except for FP64 at p = 4 (all of f~ in LDS there)
    if constexpr (P <= 3 || sizeof(T) == 4)
      hex_div_ns<T, DEV, P, NE2, CUR><<<(unsigned)(b.E / NE2), NE2 * N1 * N1, 0, c->stream>>>(
          u, grad, fc, geo, cm, r, b.E, b.n, K, (T)p.gamma, (T)p.mu, (T)p.prandtl, R);
    else
      hex_div_ns_lds<T, DEV, P, NE2, CUR><<<(unsigned)(b.E / NE2), NE2 * N1 * N1, 0, c->stream>>>(
          u, grad, fc, geo, cm, r, b.E, b.n, K, (T)p.gamma, (T)p.mu, (T)p.prandtl, R);
    c->prof_end(pk);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, FR_ERR_DEVICE, std::string("hex kernel launch: ") + hipGetErrorString(e));
  return FR_OK;
}

// CUR: curved tetrahedra, the metric stored per solution point (b.cmet) in place of the
// per-element terms.
template <typename T, bool DEV, bool CUR>
fr_status tet_rhs(fr_ctx c, DevBlock& b, const T* u, T* r) {
  Conn C{b.nbr_elem, b.nbr_info, c->perm, c->host.perm_stride};
  const fr_params& p = c->prm;
  TetDev<T> O;
  O.src = c->tet_src;
  O.pfp = c->tet_src + 60;
  O.slot = c->tet_src + 60 + 35 * 4;
  for (int f = 0; f < 4; ++f)
    for (int k = 0; k < 3; ++k) O.nref[f][k] = (T)c->host.tet.nref[f][k];
  const RefState<T> R = ref_of<T>(p);
  const T* geo = (const T*)(CUR ? b.cmet : b.geo_t);
  static const std::string sfx = std::string(CUR ? "_cur" : "") + (sizeof(T) == 8 ? "" : "_f32");
  const int sm = side_mode_of(p.ldg_beta);
  const unsigned div_grid = (unsigned)(b.E / TDIV_NE);   // one 16-element tile per block
  const T* opT = (const T*)c->tet_opT;
  const tet_s4 *opH = (const tet_s4*)c->tet_opH, *opL = opH ? opH + TET_MP * TET_KP16 / 4 : nullptr;
  const tet_s4 *ogH = (const tet_s4*)c->tet_ogH, *ogL = ogH ? ogH + TGR_M * TGR_K / 4 : nullptr;
  // BF16x3 contractions: only in the FP32 form (T = float) when asked for
  constexpr bool can_bf3 = sizeof(T) == 4;
  const bool bf3 = can_bf3 && c->prm.precision == FR_FP32_BF16X3;
  int pk;
  const T zero = T(0);
  if (p.system == FR_EULER) {
    pk = c->prof_begin(("tet_div_euler" + sfx).c_str());
    if (bf3)
      tet_div<T, DEV, false, can_bf3, false, CUR><<<div_grid, tdiv_nt<T>(), 0, c->stream>>>(
          u, nullptr, nullptr, geo, C, O, opT, opH, opL, r, b.E, b.n, (T)p.gamma, zero, zero, zero, zero, p.riemann, 0,
          R);
    else
      tet_div<T, DEV, false, false, false, CUR><<<div_grid, tdiv_nt<T>(), 0, c->stream>>>(
          u, nullptr, nullptr, geo, C, O, opT, opH, opL, r, b.E, b.n, (T)p.gamma, zero, zero, zero, zero, p.riemann, 0,
          R);
    c->prof_end(pk);
  } else {
    // one-sided LDG (beta = +-1/2), FP32 form: the gradient kernel also forms the common
    // fluxes (in FP64 the extra registers cost that kernel more than the divergence saves)
    constexpr bool can_fc = sizeof(T) == 4;
    const bool fc = sm != 0 && can_fc;
    T* fcb = (T*)b.fc;
    const T gam = (T)p.gamma, mu = (T)p.mu, pr = (T)p.prandtl, beta = (T)p.ldg_beta, tau = (T)p.ldg_tau;
    const T* ogT = (const T*)c->tet_ogT;
    pk = c->prof_begin(("tet_grad" + sfx).c_str());
#define FR_TET_GRAD(BF, FCX)                                                                                   \
  tet_grad_mma<T, DEV, BF, FCX, CUR><<<div_grid, tgr_nt<T>(), 0, c->stream>>>(u, geo, C, O, ogT, ogH, ogL, (T*)b.grad, fcb, \
                                                                    b.E, b.n, beta, sm, gam, mu, pr, tau,       \
                                                                    p.riemann, R)
    if (bf3) {
      if (fc) FR_TET_GRAD(can_bf3, can_fc); else FR_TET_GRAD(can_bf3, false);
    } else {
      if (fc) FR_TET_GRAD(false, can_fc); else FR_TET_GRAD(false, false);
    }
#undef FR_TET_GRAD
    c->prof_end(pk);
    pk = c->prof_begin(("tet_div_ns" + sfx).c_str());
#define FR_TET_DIV(BF, FCX)                                                                                     \
  tet_div<T, DEV, true, BF, FCX, CUR><<<div_grid, tdiv_nt<T>(), 0, c->stream>>>(u, (const T*)b.grad, fcb, geo, C, O, opT, opH, \
                                                                     opL, r, b.E, b.n, gam, mu, pr, beta, tau,   \
                                                                     p.riemann, sm, R)
    if (bf3) {
      if (fc) FR_TET_DIV(can_bf3, can_fc); else FR_TET_DIV(can_bf3, false);
    } else {
      if (fc) FR_TET_DIV(false, can_fc); else FR_TET_DIV(false, false);
    }
#undef FR_TET_DIV
    c->prof_end(pk);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, FR_ERR_DEVICE, std::string("tet kernel launch: ") + hipGetErrorString(e));
  return FR_OK;
}

// Pyramids: traces, then (Navier--Stokes) the LDG gradient, then the corrected divergence.
template <typename T, bool DEV>
fr_status pyr_rhs(fr_ctx c, DevBlock& b, const T* u, T* r) {
  Conn C{b.nbr_elem, b.nbr_info, c->perm, c->host.perm_stride};
  const fr_params& p = c->prm;
  const PyrOps& Y = c->host.pyr;
  PyrK<T> K;
  for (int f = 0; f <= 5; ++f) K.face_off[f] = Y.face_off[f];
  for (int f = 0; f < 5; ++f) for (int k = 0; k < 3; ++k) K.nref[f][k] = (T)Y.nref[f][k];
  const T* ops = (const T*)c->pyr_ops;
  PyrOpsDev<T> O{ops, ops + PY_NSP * PY_NFP, ops + PY_NSP * PY_NFP + 3 * PY_NSP * PY_NSP};
  const RefState<T> R = ref_of<T>(p);
  const T* geo = (const T*)b.geo_t;
  T* uf = (T*)b.uf;
  static const std::string sfx = sizeof(T) == 8 ? "" : "_f32";
  if (b.E % 64 != 0) return fail(c, FR_ERR_STATE, "pyramid block not padded to 64 elements");
  const unsigned nblk = (unsigned)(b.E / py_ne<T>());
  int pk = c->prof_begin(("pyr_trace" + sfx).c_str());
  pyr_trace<T><<<nblk, py_nt<T>(), 0, c->stream>>>(u, uf, b.E, O.It);
  c->prof_end(pk);
  const T gam = (T)p.gamma, mu = (T)p.mu, pr = (T)p.prandtl, beta = (T)p.ldg_beta, tau = (T)p.ldg_tau;
  const int sm = side_mode_of(p.ldg_beta);
  if (p.system == FR_EULER) {
    pk = c->prof_begin(("pyr_div_euler" + sfx).c_str());
    pyr_div<T, DEV, false><<<nblk, py_nt<T>(), 0, c->stream>>>(u, uf, nullptr, nullptr, geo, C, O, K, r, b.E, gam,
                                                                    mu, pr, beta, tau, p.riemann, 0, R);
    c->prof_end(pk);
  } else {
    T* grad = (T*)b.grad;
    T* gradf = (T*)b.gradf;
    pk = c->prof_begin(("pyr_grad" + sfx).c_str());
    pyr_grad<T><<<nblk, PY_NT, 0, c->stream>>>(u, uf, geo, C, O, K, grad, gradf, b.E, beta, sm);
    c->prof_end(pk);
    pk = c->prof_begin(("pyr_div_ns" + sfx).c_str());
    pyr_div<T, DEV, true><<<nblk, py_nt<T>(), 0, c->stream>>>(u, uf, grad, gradf, geo, C, O, K, r, b.E, gam, mu,
                                                                   pr, beta, tau, p.riemann, sm, R);
    c->prof_end(pk);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, FR_ERR_DEVICE, std::string("pyramid kernel launch: ") + hipGetErrorString(e));
  return FR_OK;
}

template <typename T, bool DEV>
fr_status rhs_t(fr_ctx c, const T* u, T* r) {
  for (auto& b : c->blocks) {
    const T* ub = u + b.native_off;
    T* rb = r + b.native_off;
    fr_status s = FR_OK;
    if (b.etype == FR_HEX) {
      switch (c->prm.order) {
        case 1: s = b.cmet ? hex_rhs_p<T, DEV, 1, true>(c, b, ub, rb) : hex_rhs_p<T, DEV, 1, false>(c, b, ub, rb); break;
        case 2: s = b.cmet ? hex_rhs_p<T, DEV, 2, true>(c, b, ub, rb) : hex_rhs_p<T, DEV, 2, false>(c, b, ub, rb); break;
        case 3: s = b.cmet ? hex_rhs_p<T, DEV, 3, true>(c, b, ub, rb) : hex_rhs_p<T, DEV, 3, false>(c, b, ub, rb); break;
        case 4: s = b.cmet ? hex_rhs_p<T, DEV, 4, true>(c, b, ub, rb) : hex_rhs_p<T, DEV, 4, false>(c, b, ub, rb); break;
        default: s = fail(c, FR_ERR_UNSUPPORTED, "order");
      }
    } else if (b.etype == FR_PYR) {
      s = pyr_rhs<T, DEV>(c, b, ub, rb);
    } else {
      s = b.cmet ? tet_rhs<T, DEV, true>(c, b, ub, rb) : tet_rhs<T, DEV, false>(c, b, ub, rb);
    }
    if (s != FR_OK) return s;
  }
  return FR_OK;
}

// RHS of the context's precision on its native state.
fr_status rhs_native(fr_ctx c, const void* u, void* r) {
  if (c->prm.precision != FR_FP64) return rhs_t<float, true>(c, (const float*)u, (float*)r);
  return rhs_t<double, false>(c, (const double*)u, (double*)r);
}

RefVec refvec(const fr_params& p) {
  RefVec r;
  for (int i = 0; i < 5; ++i) r.v[i] = p.u_ref[i];
  return r;
}


// ------------------------------------------------------------ entropy filter
FiltK filtk_of(const HexOps& H) {
  FiltK k;
  std::memset(&k, 0, sizeof(k));
  for (int a = 0; a < 5; ++a) {
    k.lm[a] = H.lm[a];
    k.lp[a] = H.lp[a];
    for (int m = 0; m < 5; ++m) { k.Vm[a][m] = H.Vm[a][m]; k.Vmi[a][m] = H.Vmi[a][m]; }
  }
  for (int m = 0; m < H.n1; ++m) {
    const double nm = std::sqrt((2.0 * m + 1.0) / 2.0);
    k.Pe[0][m] = nm * ((m % 2) ? -1.0 : 1.0);
    k.Pe[1][m] = nm;
  }
  return k;
}

FiltPrm filtprm_of(const fr_params& p, int order) {
  FiltPrm f;
  f.gamma = p.gamma;
  f.eps_rho = p.filt_eps_rho;
  f.eps_p = p.filt_eps_p;
  f.eps_s = p.filt_eps_s;
  f.zeta_max = p.filt_zeta_max_coef * order * order;
  f.n_bits = p.filt_bits;
  return f;
}

fr_status filter_alloc(fr_ctx c) {
  for (auto& b : c->blocks)
    if (b.etype == FR_PYR)
      return fail(c, FR_ERR_UNSUPPORTED, "the entropy filter and its learned warm start have no pyramid form");
  if (c->f_k) return FR_OK;
  bool has_tet = false;
  for (auto& b : c->blocks) has_tet = has_tet || b.etype == FR_TET;
  if (has_tet && !c->tet_ftab) {
    // V^T, V^{-1} transposed, normalised weights, check-point multiplicities
    const TetOps& T = c->host.tet;
    std::vector<double> tab(TF_LEN);
    double wsum = 0;
    for (int z = 0; z < TF_NSP; ++z) wsum += T.weights[z];
    for (int m = 0; m < TF_NSP; ++m) {
      if (T.deg[m] != tet_mode_deg(m)) return fail(c, FR_ERR_STATE, "tetrahedral modes not graded by degree");
      for (int z = 0; z < TF_NSP; ++z) {
        tab[TF_VT + m * TF_NSP + z] = T.V[z][m];
        tab[TF_VIT + z * TF_NSP + m] = T.Vinv[m][z];
      }
    }
    for (int z = 0; z < TF_NSP; ++z) {
      tab[TF_W + z] = T.weights[z] / wsum;
      tab[TF_MULT + z] = 1.0;
    }
    for (int f = 0; f < TetOps::nfp; ++f) tab[TF_MULT + T.fp_src[f]] += 1.0;
    if (dalloc(c, &c->tet_ftab, TF_LEN)) return FR_ERR_ALLOC;
    HIP_TRY(c, hipMemcpy(c->tet_ftab, tab.data(), TF_LEN * sizeof(double), hipMemcpyHostToDevice));
  }
  const int64_t n = c->n_elem_total;
  for (auto& b : c->blocks)
    if (dalloc(c, &b.sown, b.E) || dalloc(c, &b.smin, b.E) || dalloc(c, &b.f_det, b.n) ||
        dalloc(c, &b.f_list, b.n) || dalloc(c, &b.f_cnt, (b.n + 255) / 256 + 1))
      return FR_ERR_ALLOC;
  if (dalloc(c, &c->f_k, n) || dalloc(c, &c->f_evals, n) || dalloc(c, &c->f_flag, n) ||
      dalloc(c, &c->f_feat, n * 16) || dalloc(c, &c->f_khat, n))
    return FR_ERR_ALLOC;
  return FR_OK;
}

// An RK4 stage update fused into the filter's detection pass (see RkStageSrc): the
// pass forms the stage state (or the new state) while checking it.
struct StageFuse {
  int mode = 0;                 // 0 first stage, 1 middle stages, 2 last (new state in place)
  double b = 0, c = 0;          // accumulator and stage coefficients (times dt)
  const void* k = nullptr;      // the stage's right-hand side, native dtype
  bool k32 = false;             // k (and s32) FP32: the FP32 form
  double* u = nullptr;          // u_n, or the state updated in place (last stage)
  double* acc = nullptr;        // FP64 accumulator
  double* s64 = nullptr;        // FP64 stage state written in full (FP64 form) or null
  float* s32 = nullptr;         // FP32 deviation of the stage state (FP32 form) or null
  double* cand64 = nullptr;     // FP64 stage state of the candidates only (FP32 form) or null
};

template <typename KT>
RkStageSrc<KT> stage_src(const StageFuse& z, const DevBlock& b, const fr_params& prm) {
  const int64_t o = b.native_off;
  RkStageSrc<KT> s{z.u + o, (const KT*)z.k + o, z.acc + o, z.s64 ? z.s64 + o : nullptr,
                   z.s32 ? z.s32 + o : nullptr, z.b, z.c, z.mode, {0, 0, 0, 0, 0}};
  for (int v = 0; v < 5; ++v) s.ref[v] = prm.u_ref[v];
  return s;
}

template <int P>
void hex_smin_p(fr_ctx c, DevBlock& b, const double* uprev) {
  const FiltK K = filtk_of(c->host.hex);
  const int g = (int)((b.n + 255) / 256);
  unsigned long long* sown = (unsigned long long*)b.sown;
  int pk = c->prof_begin("filter_smin");
  k_fill_u64<<<grid_for(b.n, 256), 256, 0, c->stream>>>(sown, b.n, 0xFFF0000000000000ULL);   // ord_bits(+inf)
  hex_sown<P><<<(unsigned)(b.E / HexTileCfg<P>::NE), HexTileCfg<P>::NT, 0, c->stream>>>(
      uprev + b.native_off, sown, b.E, b.n, K, c->prm.gamma);
  elem_smin<<<g, 256, 0, c->stream>>>(sown, b.nbr_elem, b.nfaces, b.smin, b.E, b.n);
  c->prof_end(pk);
}

// Candidates of the search: detection at zeta = 0 and ordered compaction into
// b.f_list / count b.f_cnt[nb]; untouched elements get k = 0 and one evaluation.
template <int P>
void hex_candidates_p(fr_ctx c, DevBlock& b, const double* u, const StageFuse* fz = nullptr) {
  const FiltK K = filtk_of(c->host.hex);
  const FiltPrm F = filtprm_of(c->prm, P);
  const int64_t o = b.elem_off;
  const int nb = (int)((b.n + 255) / 256);
  const int gf = grid_for(b.n, 256);
  int pk = c->prof_begin(fz ? "rk4_stage_filter_detect_hex" : "filter_detect");
  k_filter_reset<<<gf, 256, 0, c->stream>>>(b.f_det, c->f_k + o, c->f_evals + o, b.n);
  if constexpr (P == 4) {
    // p = 4: a tile holds only 8 elements, so the tiled pass would move its rows in
    // 64-byte segments; one wave per (64-element tile, column) reads whole 512-byte rows
    // and the line ends through L2 (0.78 -> 0.72 ms per stage on the mixed workload).
    // At p <= 3 (16-64 elements a tile) the tiled pass is faster (1.43 against 1.63 ms
    // per step on the 48^3 p = 3 shock).
    const unsigned g = (unsigned)((b.E / 64 * (P + 1) * (P + 1) + 3) / 4);
    if (!fz)
      hex_filter_detect_lines<P, PlainSrc><<<g, 256, 0, c->stream>>>(PlainSrc{u + b.native_off}, b.smin, b.E,
                                                                     b.n, K, F, b.f_det);
    else if (fz->k32)
      hex_filter_detect_lines<P, RkStageSrc<float>><<<g, 256, 0, c->stream>>>(stage_src<float>(*fz, b, c->prm),
                                                                              b.smin, b.E, b.n, K, F, b.f_det);
    else
      hex_filter_detect_lines<P, RkStageSrc<double>><<<g, 256, 0, c->stream>>>(stage_src<double>(*fz, b, c->prm),
                                                                               b.smin, b.E, b.n, K, F, b.f_det);
  } else {
    const unsigned g = (unsigned)(b.E / HexTileCfg<P>::NE);
    if (!fz)
      hex_filter_detect<P, PlainSrc><<<g, HexTileCfg<P>::NT, 0, c->stream>>>(PlainSrc{u + b.native_off}, b.smin,
                                                                             b.E, b.n, K, F, b.f_det, nullptr);
    else if (fz->k32)
      hex_filter_detect<P, RkStageSrc<float>><<<g, HexTileCfg<P>::NT, 0, c->stream>>>(
          stage_src<float>(*fz, b, c->prm), b.smin, b.E, b.n, K, F, b.f_det,
          fz->cand64 ? fz->cand64 + b.native_off : nullptr);
    else
      hex_filter_detect<P, RkStageSrc<double>><<<g, HexTileCfg<P>::NT, 0, c->stream>>>(
          stage_src<double>(*fz, b, c->prm), b.smin, b.E, b.n, K, F, b.f_det,
          fz->cand64 ? fz->cand64 + b.native_off : nullptr);
  }
  k_flag_count<<<nb, 256, 0, c->stream>>>(b.f_det, b.n, b.f_cnt);
  k_scan_counts<<<1, 1024, 0, c->stream>>>(b.f_cnt, nb);
  k_flag_scatter<<<nb, 256, 0, c->stream>>>(b.f_det, b.n, b.f_cnt, b.f_list);
  if (P == 4 && fz && fz->cand64 && fz->k32)
    k_cand_stage<float><<<(unsigned)std::max<int64_t>(1, std::min<int64_t>(b.n, 4096)), 256, 0, c->stream>>>(
        stage_src<float>(*fz, b, c->prm), b.f_list, b.f_cnt + nb, b.nsp * 5, b.E, fz->cand64 + b.native_off);
  c->prof_end(pk);
}

// Grid of the per-candidate filter kernels: FW candidates (waves) per block.
inline unsigned list_grid(const DevBlock& b, int fw) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((b.n + fw - 1) / fw, 2048));
}

// Features (and the exact troubled flag) of the candidates of b.
template <int P>
void hex_features_p(fr_ctx c, DevBlock& b, const double* u) {
  const FiltK K = filtk_of(c->host.hex);
  const FiltPrm F = filtprm_of(c->prm, P);
  const int64_t o = b.elem_off;
  const int nb = (int)((b.n + 255) / 256);
  k_fill_i32<<<grid_for(b.n, 256), 256, 0, c->stream>>>(c->f_flag + o, b.n, 0);
  constexpr int FW = HexFW<P>::value;
  hex_features<P><<<list_grid(b, FW), 64 * FW, 0, c->stream>>>(u + b.native_off, b.smin, b.E, b.f_list, b.f_cnt + nb, K, F,
                                                       c->f_flag + o, c->f_feat + o * 16);
}

template <int P>
void hex_filter_p(fr_ctx c, DevBlock& b, double* u, int mode, float* u32, const StageFuse* fz) {
  constexpr int FW = HexFW<P>::value;
  const FiltK K = filtk_of(c->host.hex);
  const FiltPrm F = filtprm_of(c->prm, P);
  const int64_t o = b.elem_off;
  const int nb = (int)((b.n + 255) / 256);
  Dev32 s32{u32 ? u32 + b.native_off : nullptr, {0, 0, 0, 0, 0}};
  for (int v = 0; v < 5; ++v) s32.ref[v] = c->prm.u_ref[v];
  hex_candidates_p<P>(c, b, u, fz);
  int pk;
  if (mode == 1) {
    pk = c->prof_begin("filter_search_learned");
    hex_filter_learned<P><<<list_grid(b, FW), 64 * FW, 0, c->stream>>>(
        u + b.native_off, b.smin, b.E, b.f_list, b.f_cnt + nb, K, F, c->m_w, c->m_scale, c->f_k + o,
        c->f_evals + o, s32);
  } else {
    pk = c->prof_begin("filter_search_plain");
    hex_filter<P><<<list_grid(b, FW), 64 * FW, 0, c->stream>>>(u + b.native_off, b.smin, b.E, b.f_list,
                                                               b.f_cnt + nb, K, F, c->f_k + o, c->f_evals + o, s32);
  }
  c->prof_end(pk);
}


void tet_smin(fr_ctx c, DevBlock& b, const double* uprev) {
  const int g = (int)((b.n + 255) / 256);
  unsigned long long* sown = (unsigned long long*)b.sown;
  int pk = c->prof_begin("filter_smin");
  tet_sown<<<g, 256, 0, c->stream>>>(uprev + b.native_off, sown, b.E, b.n, c->prm.gamma);
  elem_smin<<<g, 256, 0, c->stream>>>(sown, b.nbr_elem, b.nfaces, b.smin, b.E, b.n);
  c->prof_end(pk);
}

void tet_candidates(fr_ctx c, DevBlock& b, const double* u, const StageFuse* fz = nullptr) {
  const FiltPrm F = filtprm_of(c->prm, c->prm.order);
  const int64_t o = b.elem_off;
  const int nb = (int)((b.n + 255) / 256);
  int pk = c->prof_begin(fz ? "rk4_stage_filter_detect_tet" : "filter_detect");
  k_filter_reset<<<grid_for(b.n, 256), 256, 0, c->stream>>>(b.f_det, c->f_k + o, c->f_evals + o, b.n);
  const unsigned gE = (unsigned)((b.E + 255) / 256);
  if (!fz)
    tet_filter_detect<PlainSrc><<<nb, 256, 0, c->stream>>>(PlainSrc{u + b.native_off}, b.smin, b.E, b.n, F, b.f_det,
                                                           nullptr);
  else if (fz->k32)
    tet_filter_detect<RkStageSrc<float>><<<gE, 256, 0, c->stream>>>(
        stage_src<float>(*fz, b, c->prm), b.smin, b.E, b.n, F, b.f_det,
        fz->cand64 ? fz->cand64 + b.native_off : nullptr);
  else
    tet_filter_detect<RkStageSrc<double>><<<gE, 256, 0, c->stream>>>(
        stage_src<double>(*fz, b, c->prm), b.smin, b.E, b.n, F, b.f_det,
        fz->cand64 ? fz->cand64 + b.native_off : nullptr);
  k_flag_count<<<nb, 256, 0, c->stream>>>(b.f_det, b.n, b.f_cnt);
  k_scan_counts<<<1, 1024, 0, c->stream>>>(b.f_cnt, nb);
  k_flag_scatter<<<nb, 256, 0, c->stream>>>(b.f_det, b.n, b.f_cnt, b.f_list);
  c->prof_end(pk);
}

void tet_features_b(fr_ctx c, DevBlock& b, const double* u) {
  const FiltPrm F = filtprm_of(c->prm, c->prm.order);
  const int64_t o = b.elem_off;
  const int nb = (int)((b.n + 255) / 256);
  k_fill_i32<<<grid_for(b.n, 256), 256, 0, c->stream>>>(c->f_flag + o, b.n, 0);
  tet_features<<<list_grid(b, 4), 256, 0, c->stream>>>(u + b.native_off, b.smin, b.E, b.f_list, b.f_cnt + nb,
                                                         c->tet_ftab, F, c->f_flag + o, c->f_feat + o * 16);
}

void tet_filter_b(fr_ctx c, DevBlock& b, double* u, int mode, float* u32, const StageFuse* fz) {
  const FiltPrm F = filtprm_of(c->prm, c->prm.order);
  const int64_t o = b.elem_off;
  const int nb = (int)((b.n + 255) / 256);
  Dev32 s32{u32 ? u32 + b.native_off : nullptr, {0, 0, 0, 0, 0}};
  for (int v = 0; v < 5; ++v) s32.ref[v] = c->prm.u_ref[v];
  tet_candidates(c, b, u, fz);
  int pk;
  if (mode == 1) {
    pk = c->prof_begin("filter_search_learned");
    tet_filter_learned<<<list_grid(b, 4), 256, 0, c->stream>>>(u + b.native_off, b.smin, b.E, b.f_list,
                                                                 b.f_cnt + nb, c->tet_ftab, F, c->m_w, c->m_scale,
                                                                 c->f_k + o, c->f_evals + o, s32);
  } else {
    pk = c->prof_begin("filter_search_plain");
    tet_filter<<<list_grid(b, 4), 256, 0, c->stream>>>(u + b.native_off, b.smin, b.E, b.f_list, b.f_cnt + nb,
                                                         c->tet_ftab, F, c->f_k + o, c->f_evals + o, s32);
  }
  c->prof_end(pk);
}

fr_status compute_smin(fr_ctx c, const double* uprev) {
  for (auto& b : c->blocks) {
    if (b.etype == FR_TET) {
      tet_smin(c, b, uprev);
      continue;
    }
    switch (c->prm.order) {
      case 1: hex_smin_p<1>(c, b, uprev); break;
      case 2: hex_smin_p<2>(c, b, uprev); break;
      case 3: hex_smin_p<3>(c, b, uprev); break;
      case 4: hex_smin_p<4>(c, b, uprev); break;
    }
  }
  HIP_TRY(c, hipGetLastError());
  return FR_OK;
}

fr_status collect_rows(fr_ctx c, const double* u);
fr_status apply_filter(fr_ctx c, double* u, int mode, float* u32 = nullptr, const StageFuse* fz = nullptr);

// Filter the FP64 native state u in place; with u32 (the FP32 form's stage buffer) the
// filtered elements' FP32 deviations are rewritten there as well.  With fz the
// detection pass first performs that RK stage update (u is then the buffer the search
// works on: the full FP64 stage state, the candidates' copy, or the new state).
fr_status apply_filter(fr_ctx c, double* u, int mode, float* u32, const StageFuse* fz) {
  if (c->collecting) {
    if (fz) return fail(c, FR_ERR_STATE, "training-data collection needs the stage state before the filter");
    fr_status st = collect_rows(c, u);
    if (st) return st;
  }
  for (auto& b : c->blocks) {
    if (b.etype == FR_TET) {
      tet_filter_b(c, b, u, mode, u32, fz);
      continue;
    }
    switch (c->prm.order) {
      case 1: hex_filter_p<1>(c, b, u, mode, u32, fz); break;
      case 2: hex_filter_p<2>(c, b, u, mode, u32, fz); break;
      case 3: hex_filter_p<3>(c, b, u, mode, u32, fz); break;
      case 4: hex_filter_p<4>(c, b, u, mode, u32, fz); break;
    }
  }
  HIP_TRY(c, hipGetLastError());
  return FR_OK;
}

__global__ void k_gather_features(const float* __restrict__ feat, const int32_t* __restrict__ kk,
                                  const int32_t* __restrict__ idx, int64_t n, float* __restrict__ x,
                                  int32_t* __restrict__ elem, int32_t* __restrict__ kout) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t e = idx[i];
  for (int f = 0; f < 16; ++f) x[i * 16 + f] = feat[(int64_t)e * 16 + f];
  if (elem) elem[i] = e;
  if (kout) kout[i] = kk[e];
}

// Features and plain-search targets of the troubled elements of u (entropy bound
// from the current s_min), appended to the collection buffers.
template <int P>
void hex_candidate_features_p(fr_ctx c, DevBlock& b, const double* u) {
  hex_candidates_p<P>(c, b, u);
  hex_features_p<P>(c, b, u);
}

fr_status candidate_features(fr_ctx c, const double* u) {
  for (auto& b : c->blocks) {
    if (b.etype == FR_TET) {
      tet_candidates(c, b, u);
      tet_features_b(c, b, u);
      continue;
    }
    switch (c->prm.order) {
      case 1: hex_candidate_features_p<1>(c, b, u); break;
      case 2: hex_candidate_features_p<2>(c, b, u); break;
      case 3: hex_candidate_features_p<3>(c, b, u); break;
      case 4: hex_candidate_features_p<4>(c, b, u); break;
    }
  }
  HIP_TRY(c, hipGetLastError());
  return FR_OK;
}

fr_status collect_rows(fr_ctx c, const double* u) {
  fr_status cs = candidate_features(c, u);
  if (cs) return cs;
  HIP_TRY(c, hipMemcpyAsync(c->f_copy, u, c->native_len * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  c->collecting = false;
  fr_status st = apply_filter(c, c->f_copy, 0);
  c->collecting = true;
  if (st) return st;
  std::vector<int32_t> flag(c->n_elem_total);
  HIP_TRY(c, hipMemcpyAsync(flag.data(), c->f_flag, flag.size() * 4, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  std::vector<int32_t> idx;
  for (size_t i = 0; i < flag.size(); ++i) if (flag[i]) idx.push_back((int32_t)i);
  c->col_seen += (int64_t)idx.size();
  const int64_t m = std::min<int64_t>((int64_t)idx.size(), c->col_cap - c->col_n);
  if (m > 0) {
    int32_t* didx = nullptr;
    if (dalloc(c, &didx, m)) return FR_ERR_ALLOC;
    HIP_TRY(c, hipMemcpyAsync(didx, idx.data(), m * 4, hipMemcpyHostToDevice, c->stream));
    k_gather_features<<<(unsigned)((m + 255) / 256), 256, 0, c->stream>>>(c->f_feat, c->f_k, didx, m,
                                                                          c->col_x + c->col_n * 16, nullptr,
                                                                          c->col_k + c->col_n);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    (void)hipFree(didx);
    c->col_n += m;
  }
  return FR_OK;
}

fr_status mlp_alloc(fr_ctx c, int batch) {
  if (!c->m_w) {
    if (dalloc(c, &c->m_w, MLP_NP) || dalloc(c, &c->m_m, MLP_NP) || dalloc(c, &c->m_v, MLP_NP) ||
        dalloc(c, &c->m_g, MLP_NP) || dalloc(c, &c->m_scale, 2 * MLP_IN) || dalloc(c, &c->m_loss, 1))
      return FR_ERR_ALLOC;
  }
  if (batch > c->m_batch_cap) {
    (void)hipFree(c->m_scratch);
    (void)hipFree(c->m_sqerr);
    if (dalloc(c, &c->m_scratch, (size_t)batch * MLP_SS) || dalloc(c, &c->m_sqerr, batch)) return FR_ERR_ALLOC;
    c->m_batch_cap = batch;
  }
  return FR_OK;
}

}  // namespace

// =============================================================================
extern "C" {

void fr_default_params(fr_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->struct_size = sizeof(fr_params);
  p->system = FR_EULER;
  p->order = 3;
  p->riemann = FR_RUSANOV;
  p->precision = FR_FP64;
  p->gamma = 1.4;
  p->mu = 1.0 / 1600.0;
  p->prandtl = 0.71;
  p->ldg_beta = 0.5;
  p->ldg_tau = 0.1;
  p->u_ref[0] = 1.0;
  p->u_ref[4] = 1.0 / (0.4 * 1.4 * 0.01);
  p->filt_eps_rho = 1e-8;
  p->filt_eps_p = 1e-8;
  p->filt_eps_s = 1e-4;
  p->filt_zeta_max_coef = 40.0;
  p->filt_bits = 20;
}

const char* fr_last_error(fr_ctx ctx) { return ctx ? ctx->err.c_str() : g_thread_err.c_str(); }

void fr_destroy(fr_ctx c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (auto& b : c->blocks) {
    if (b.geo_t && b.geo_t != b.geo) (void)hipFree(b.geo_t);
    (void)hipFree(b.geo); (void)hipFree(b.nbr_elem); (void)hipFree(b.nbr_info);
    (void)hipFree(b.uf); (void)hipFree(b.grad); (void)hipFree(b.gradf); (void)hipFree(b.fc);
    (void)hipFree(b.cmet);
    (void)hipFree(b.cpos); (void)hipFree(b.npos);
  }
  (void)hipFree(c->perm);
  (void)hipFree(c->g_npos);
  (void)hipFree(c->rk_stage); (void)hipFree(c->rk_acc); (void)hipFree(c->rk_k); (void)hipFree(c->rk_s64);
  (void)hipFree(c->rk_x0); (void)hipFree(c->rk_err); (void)hipFree(c->rk_part);
  (void)hipFree(c->flag);
  (void)hipFree(c->tet_src); (void)hipFree(c->tet_opT); (void)hipFree(c->tet_ogT); (void)hipFree(c->pyr_ops);
  (void)hipFree(c->tet_opH); (void)hipFree(c->tet_ogH); (void)hipFree(c->tet_ftab);
  for (auto& b : c->blocks) {
    (void)hipFree(b.sown); (void)hipFree(b.smin);
    (void)hipFree(b.f_det); (void)hipFree(b.f_list); (void)hipFree(b.f_cnt);
  }
  for (void* q : {(void*)c->f_k, (void*)c->f_evals, (void*)c->f_flag, (void*)c->f_feat, (void*)c->f_khat,
                  (void*)c->f_copy, (void*)c->m_w, (void*)c->m_m, (void*)c->m_v, (void*)c->m_g, (void*)c->m_scale,
                  (void*)c->m_loss, (void*)c->m_scratch, (void*)c->m_sqerr, (void*)c->m_idx})
    (void)hipFree(q);
  c->prof_clear();
  delete c;
}

namespace {
fr_status setup_impl(const fr_params* p, int64_t n_vert, const double* xyz, const double* period,
                     int64_t n_elem, const int32_t* etype, const int64_t* enodes, int geo_order,
                     const int64_t* ho_nodes, void* stream, fr_ctx* out) {
  if (!out) return fail(nullptr, FR_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!p || p->struct_size != sizeof(fr_params)) return fail(nullptr, FR_ERR_ARG, "fr_params missing or struct_size mismatch");
  if (!xyz || !period || !etype || !enodes || n_vert <= 0 || n_elem <= 0) return fail(nullptr, FR_ERR_ARG, "empty mesh or NULL array");
  if (p->system != FR_EULER && p->system != FR_NAVIER_STOKES) return fail(nullptr, FR_ERR_ARG, "system");
  if (p->riemann != FR_RUSANOV && p->riemann != FR_HLLC) return fail(nullptr, FR_ERR_ARG, "riemann");
  if (p->precision != FR_FP64 && p->precision != FR_FP32 && p->precision != FR_FP32_BF16X3)
    return fail(nullptr, FR_ERR_ARG, "precision");
  if (p->precision == FR_FP32_BF16X3 && std::none_of(etype, etype + n_elem, [](int32_t t) { return t == FR_TET; }))
    return fail(nullptr, FR_ERR_UNSUPPORTED,
                "FR_FP32_BF16X3 splits the dense tetrahedral operator products; a mesh without tetrahedra has "
                "none (hexahedra contract 1-D lines on the vector units): use FR_FP32");
  if (p->precision != FR_FP64 && (p->u_ref[1] != 0 || p->u_ref[2] != 0 || p->u_ref[3] != 0 ||
                                  !(p->u_ref[0] > 0) || !(p->u_ref[4] > 0)))
    return fail(nullptr, FR_ERR_ARG, "the FP32 form needs a reference state at rest with rho > 0, E > 0");
  if (!(p->gamma > 1.0)) return fail(nullptr, FR_ERR_ARG, "gamma must exceed 1");
  if (p->filt_bits < 1 || p->filt_bits > 30) return fail(nullptr, FR_ERR_ARG, "filt_bits must be in 1..30");
  if (!(p->filt_zeta_max_coef > 0) || !std::isfinite(p->filt_zeta_max_coef))
    return fail(nullptr, FR_ERR_ARG, "filt_zeta_max_coef must be positive and finite");
  if (!(p->filt_eps_rho >= 0) || !(p->filt_eps_p >= 0) || !(p->filt_eps_s >= 0))
    return fail(nullptr, FR_ERR_ARG, "filter floors and entropy tolerance must be >= 0");
  if (p->elem_order < 0 || p->elem_order > 2) return fail(nullptr, FR_ERR_ARG, "elem_order must be 0, 1 or 2");
  if (p->hex_metric != FR_METRIC_CONSERVATIVE && p->hex_metric != FR_METRIC_CROSS)
    return fail(nullptr, FR_ERR_ARG, "hex_metric must be FR_METRIC_CONSERVATIVE or FR_METRIC_CROSS");
  fr_ctx c = new (std::nothrow) fr_ctx_s();
  if (!c) return fail(nullptr, FR_ERR_ALLOC, "context allocation");
  c->prm = *p;
  c->stream = (hipStream_t)stream;
  c->static_scratch = static_scratch_address();
  int code = 0;
  std::string msg;
  try {
    msg = build_setup(p->order, n_vert, xyz, period, n_elem, etype, enodes, 64, p->elem_order, c->host, code);
    if (msg.empty() && ho_nodes) {
      const bool tets = !c->host.blocks.empty() && c->host.blocks[0].etype == kTet;
      msg = tets ? build_curved_tet(geo_order, p->hex_metric, xyz, ho_nodes, c->host, code)
                 : build_curved_hex(geo_order, p->hex_metric, xyz, ho_nodes, c->host, code);
    }
  } catch (const std::exception& ex) {
    msg = ex.what();
    code = 3;
  }
  if (!msg.empty()) {
    fr_status s = code == 2 ? FR_ERR_MESH : (code == 3 ? FR_ERR_UNSUPPORTED : FR_ERR_ARG);
    delete c;
    return fail(nullptr, s, msg);
  }
  const size_t tsz = p->precision != FR_FP64 ? sizeof(float) : sizeof(double);
  int64_t canon = 0, native = 0;
  auto bail = [&](fr_status s) { std::string m = c->err; fr_destroy(c); return fail(nullptr, s, m); };
  for (auto& hb : c->host.blocks) {
    DevBlock b;
    b.etype = hb.etype; b.n = hb.n; b.E = hb.e_pad; b.nsp = hb.nsp; b.nfp = hb.nfp; b.nfaces = hb.nfaces;
    b.canon_off = canon; b.native_off = native;
    b.elem_off = c->n_elem_total;
    c->n_elem_total += b.n;
    canon += b.n * 5 * b.nsp;
    native += b.E * 5 * b.nsp;
    c->blocks.push_back(b);
    DevBlock& d = c->blocks.back();
    {
      std::vector<int32_t> cp((size_t)d.E, -1), np_((size_t)d.n);
      for (int64_t i = 0; i < d.n; ++i) { cp[i] = hb.canon_pos[i]; np_[hb.canon_pos[i]] = (int32_t)i; }
      if (dalloc(c, &d.cpos, cp.size()) || dalloc(c, &d.npos, np_.size())) return bail(FR_ERR_ALLOC);
      if (hipMemcpy(d.cpos, cp.data(), cp.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(d.npos, np_.data(), np_.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
        c->err = "upload failed";
        return bail(FR_ERR_DEVICE);
      }
    }
    if (dalloc(c, &d.geo, hb.geo.size()) || dalloc(c, &d.nbr_elem, hb.nbr_elem.size()) ||
        dalloc(c, &d.nbr_info, hb.nbr_info.size()) || dalloc(c, (char**)&d.uf, (size_t)d.nfp * 5 * d.E * tsz))
      return bail(FR_ERR_ALLOC);
    const bool is_tet = d.etype == FR_TET;
    if (p->system == FR_NAVIER_STOKES &&
        (dalloc(c, (char**)&d.grad, (size_t)d.nsp * 15 * d.E * tsz) ||
         (!is_tet && dalloc(c, (char**)&d.gradf, (size_t)d.nfp * 15 * d.E * tsz))))
      return bail(FR_ERR_ALLOC);
    if (p->system == FR_NAVIER_STOKES && dalloc(c, (char**)&d.fc, (size_t)d.nfp * 5 * d.E * tsz))
      return bail(FR_ERR_ALLOC);
    d.geo_t = d.geo;
    if (tsz == sizeof(float)) {
      std::vector<float> g32(hb.geo.begin(), hb.geo.end());
      if (dalloc(c, (float**)&d.geo_t, g32.size())) return bail(FR_ERR_ALLOC);
      if (hipMemcpy(d.geo_t, g32.data(), g32.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
        c->err = "upload failed";
        return bail(FR_ERR_DEVICE);
      }
    }
    if (!hb.cmet.empty()) {
      if (tsz == sizeof(float)) {
        std::vector<float> m32(hb.cmet.begin(), hb.cmet.end());
        if (dalloc(c, (float**)&d.cmet, m32.size())) return bail(FR_ERR_ALLOC);
        if (hipMemcpy(d.cmet, m32.data(), m32.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
          c->err = "upload failed";
          return bail(FR_ERR_DEVICE);
        }
      } else {
        if (dalloc(c, (double**)&d.cmet, hb.cmet.size())) return bail(FR_ERR_ALLOC);
        if (hipMemcpy(d.cmet, hb.cmet.data(), hb.cmet.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
          c->err = "upload failed";
          return bail(FR_ERR_DEVICE);
        }
      }
    }
    if (hipMemcpy(d.geo, hb.geo.data(), hb.geo.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d.nbr_elem, hb.nbr_elem.data(), hb.nbr_elem.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d.nbr_info, hb.nbr_info.data(), hb.nbr_info.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
      c->err = "upload failed";
      return bail(FR_ERR_DEVICE);
    }
  }
  c->canon_len = canon;
  c->native_len = native;
  {
    std::vector<int32_t> gn((size_t)c->n_elem_total);
    c->h_cpos.assign((size_t)c->n_elem_total, 0);
    for (size_t bi = 0; bi < c->blocks.size(); ++bi) {
      const Block& hb = c->host.blocks[bi];
      const int64_t o = c->blocks[bi].elem_off;
      for (int64_t i = 0; i < hb.n; ++i) {
        c->h_cpos[o + i] = (int32_t)(o + hb.canon_pos[i]);
        gn[o + hb.canon_pos[i]] = (int32_t)(o + i);
      }
    }
    if (dalloc(c, &c->g_npos, gn.size())) return bail(FR_ERR_ALLOC);
    if (hipMemcpy(c->g_npos, gn.data(), gn.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
      c->err = "upload failed";
      return bail(FR_ERR_DEVICE);
    }
  }
  if (dalloc(c, &c->perm, c->host.orient_perm.size()) || dalloc(c, &c->flag, 1)) return bail(FR_ERR_ALLOC);
  if (hipMemcpy(c->perm, c->host.orient_perm.data(), c->host.orient_perm.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
    c->err = "upload failed";
    return bail(FR_ERR_DEVICE);
  }
  bool has_tet = false;
  for (auto& b : c->blocks) has_tet = has_tet || b.etype == FR_TET;
  if (has_tet) {
    const TetOps& T = c->host.tet;
    // flux point -> collocated solution point, then per solution point its flux points
    std::vector<int32_t> src(T.fp_src, T.fp_src + 60);
    src.resize(60 + 35 * 4, 0);
    for (int sg = 0; sg < 60; ++sg) {
      int32_t* row = &src[60 + 4 * T.fp_src[sg]];
      if (row[0] >= 3) { c->err = "a solution point collocated with more than 3 flux points"; return bail(FR_ERR_STATE); }
      row[1 + row[0]++] = sg;
    }
    // transposed, zero-padded divergence operator [Dh_0 Dh_1 Dh_2 L] of the matrix-core contraction
    std::vector<double> opT((size_t)TET_KP * TET_MP, 0.0);
    for (int k = 0; k < 105; ++k)
      for (int pt = 0; pt < 35; ++pt) opT[(size_t)k * TET_MP + pt] = T.Dh[k / 35][pt][k % 35];
    for (int sg = 0; sg < 60; ++sg)
      for (int pt = 0; pt < 35; ++pt) opT[(size_t)(TET_KA + sg) * TET_MP + pt] = T.lift[pt][sg];
    std::vector<char> bop(opT.size() * tsz);
    if (tsz == sizeof(float)) for (size_t i = 0; i < opT.size(); ++i) ((float*)bop.data())[i] = (float)opT[i];
    else std::memcpy(bop.data(), opT.data(), bop.size());
    // stacked, transposed gradient operator [[Dh_i, L diag(n~_i)]] (i = 0, 1, 2)
    std::vector<double> ogT((size_t)TGR_K * TGR_M, 0.0);
    for (int i = 0; i < 3; ++i)
      for (int pt = 0; pt < 35; ++pt) {
        for (int k = 0; k < 35; ++k) ogT[(size_t)k * TGR_M + TET_MP * i + pt] = T.Dh[i][pt][k];
        for (int sg = 0; sg < 60; ++sg)
          ogT[(size_t)(35 + sg) * TGR_M + TET_MP * i + pt] = T.lift[pt][sg] * T.nref[T.fp_face[sg]][i];
      }
    // Output-row order of the gradient product: rows {16 w + 4 g + q : g = 0..3} are the
    // ones the lanes of wave w visit together at step q of the common-flux loop, so points
    // are grouped by their number of flux points (3, 2, 1, 0) into such quadruples, and
    // the quadruples are dealt to the three waves so their loop trips balance.
    std::vector<int> slot_pt(TET_MP, -1);
    {
      std::vector<int> order(35);
      for (int z = 0; z < 35; ++z) order[z] = z;
      auto nfp_of = [&](int z) { return src[60 + 4 * z]; };
      std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nfp_of(a) > nfp_of(b); });
      order.resize(TET_MP, -1);
      // 12 quadruples, costs = the largest flux-point count in each
      std::vector<int> cost(12, 0);
      for (int g = 0; g < 12; ++g)
        for (int j = 0; j < 4; ++j) if (order[4 * g + j] >= 0) cost[g] = std::max(cost[g], nfp_of(order[4 * g + j]));
      int load[3] = {0, 0, 0}, used[3] = {0, 0, 0};
      for (int g = 0; g < 12; ++g) {            // costs are non-increasing in g
        int wbest = -1;
        for (int w = 0; w < 3; ++w)
          if (used[w] < 4 && (wbest < 0 || load[w] < load[wbest])) wbest = w;
        const int q = used[wbest]++;
        load[wbest] += cost[g];
        for (int j = 0; j < 4; ++j) slot_pt[16 * wbest + 4 * j + q] = order[4 * g + j];
      }
    }
    std::vector<int> pt_slot(35, -1);
    for (int r = 0; r < TET_MP; ++r) if (slot_pt[r] >= 0) pt_slot[slot_pt[r]] = r;
    for (int r = 0; r < TET_MP; ++r) src.push_back(slot_pt[r]);
    // the same operator in the face-sparse row order of the FP32 / FP64 kernels (tgs_row):
    // direction i reads only the rows of faces 2 - i and 3, whose normals have an i component
    std::vector<double> ogS((size_t)TGS_K * TGR_M, 0.0);
    for (int i = 0; i < 3; ++i)
      for (int pt = 0; pt < 35; ++pt) {
        for (int k = 0; k < 35; ++k) ogS[(size_t)k * TGR_M + TET_MP * i + pt_slot[pt]] = T.Dh[i][pt][k];
        for (int sg = 0; sg < 60; ++sg) {
          const int f = T.fp_face[sg];
          if (f != sg / TET_NFPF || ((f != 2 - i && f != 3) && T.nref[f][i] != 0.0)) {
            c->err = "tetrahedral flux points not ordered by face, or a face normal off the expected axes";
            return bail(FR_ERR_STATE);
          }
          ogS[(size_t)(TGS_U + 16 * f + sg % TET_NFPF) * TGR_M + TET_MP * i + pt_slot[pt]] =
              T.lift[pt][sg] * T.nref[f][i];
        }
      }
    std::vector<char> bog(ogS.size() * tsz);
    if (tsz == sizeof(float)) for (size_t i = 0; i < ogS.size(); ++i) ((float*)bog.data())[i] = (float)ogS[i];
    else std::memcpy(bog.data(), ogS.data(), bog.size());
    if (p->precision == FR_FP32_BF16X3) {
      // [M][K] row-major (k contiguous), hi then lo, K padded to multiples of 16
      std::vector<uint16_t> dh((size_t)2 * TET_MP * TET_KP16, 0), gh((size_t)2 * TGR_M * TGR_K, 0);
      const size_t dlo = (size_t)TET_MP * TET_KP16, glo = (size_t)TGR_M * TGR_K;
      for (int m = 0; m < TET_MP; ++m) {
        for (int k = 0; k < 105; ++k) bf16_split_host(opT[(size_t)k * TET_MP + m], dh[(size_t)m * TET_KP16 + k],
                                                      dh[dlo + (size_t)m * TET_KP16 + k]);
        for (int s2 = 0; s2 < 60; ++s2)
          bf16_split_host(opT[(size_t)(TET_KA + s2) * TET_MP + m], dh[(size_t)m * TET_KP16 + TET_KA16 + s2],
                          dh[dlo + (size_t)m * TET_KP16 + TET_KA16 + s2]);
      }
      for (int i = 0; i < 3; ++i)
        for (int r = 0; r < TET_MP; ++r) {
          const int m = TET_MP * i + r, pt = slot_pt[r];
          if (pt < 0) continue;
          for (int k = 0; k < TGR_K; ++k)
            bf16_split_host(ogT[(size_t)k * TGR_M + TET_MP * i + pt], gh[(size_t)m * TGR_K + k],
                            gh[glo + (size_t)m * TGR_K + k]);
        }
      if (dalloc(c, (char**)&c->tet_opH, dh.size() * 2) || dalloc(c, (char**)&c->tet_ogH, gh.size() * 2) ||
          hipMemcpy(c->tet_opH, dh.data(), dh.size() * 2, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(c->tet_ogH, gh.data(), gh.size() * 2, hipMemcpyHostToDevice) != hipSuccess) {
        c->err = "tet operator upload failed";
        return bail(FR_ERR_DEVICE);
      }
    }
    if (dalloc(c, (char**)&c->tet_opT, bop.size()) || dalloc(c, (char**)&c->tet_ogT, bog.size()) ||
        hipMemcpy(c->tet_opT, bop.data(), bop.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->tet_ogT, bog.data(), bog.size(), hipMemcpyHostToDevice) != hipSuccess) {
      c->err = "tet operator upload failed";
      return bail(FR_ERR_DEVICE);
    }
    if (dalloc(c, &c->tet_src, src.size())) return bail(FR_ERR_ALLOC);
    if (hipMemcpy(c->tet_src, src.data(), src.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
      c->err = "upload failed";
      return bail(FR_ERR_DEVICE);
    }
  }
  if (std::any_of(c->blocks.begin(), c->blocks.end(), [](const DevBlock& b) { return b.etype == FR_PYR; })) {
    const PyrOps& Y = c->host.pyr;
    std::vector<double> ops((size_t)PY_NSP * PY_NFP * 2 + 3 * PY_NSP * PY_NSP);
    double* It = ops.data();
    double* Dt = It + PY_NSP * PY_NFP;
    double* Lt = Dt + 3 * PY_NSP * PY_NSP;
    for (int j = 0; j < PY_NSP; ++j)
      for (int fp = 0; fp < PY_NFP; ++fp) It[j * PY_NFP + fp] = Y.interp[fp][j];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < PY_NSP; ++j)
        for (int pt = 0; pt < PY_NSP; ++pt) Dt[(i * PY_NSP + j) * PY_NSP + pt] = Y.D[i][pt][j];
    for (int fp = 0; fp < PY_NFP; ++fp)
      for (int pt = 0; pt < PY_NSP; ++pt) Lt[fp * PY_NSP + pt] = Y.lift[pt][fp];
    std::vector<char> bo(ops.size() * tsz);
    if (tsz == sizeof(float)) for (size_t i = 0; i < ops.size(); ++i) ((float*)bo.data())[i] = (float)ops[i];
    else std::memcpy(bo.data(), ops.data(), bo.size());
    if (dalloc(c, (char**)&c->pyr_ops, bo.size()) ||
        hipMemcpy(c->pyr_ops, bo.data(), bo.size(), hipMemcpyHostToDevice) != hipSuccess) {
      c->err = "pyramid operator upload failed";
      return bail(FR_ERR_DEVICE);
    }
  }
  *out = c;
  return FR_OK;
}
}  // namespace

fr_status fr_setup_mesh(const fr_params* p, int64_t n_vert, const double* xyz, const double* period,
                        int64_t n_elem, const int32_t* etype, const int64_t* enodes, void* stream,
                        fr_ctx* out) {
  return setup_impl(p, n_vert, xyz, period, n_elem, etype, enodes, 0, nullptr, stream, out);
}

fr_status fr_setup_mesh_curved(const fr_params* p, int32_t geo_order, int64_t n_vert, const double* xyz,
                               const double* period, int64_t n_elem, const int64_t* ho_nodes, void* stream,
                               fr_ctx* out) {
  if (!out) return fail(nullptr, FR_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!p || p->struct_size != sizeof(fr_params)) return fail(nullptr, FR_ERR_ARG, "fr_params missing or struct_size mismatch");
  if (!xyz || !period || !ho_nodes || n_vert <= 0 || n_elem <= 0) return fail(nullptr, FR_ERR_ARG, "empty mesh or NULL array");
  if (geo_order < 1 || geo_order > 4) return fail(nullptr, FR_ERR_UNSUPPORTED, "geometry order must be in 1..4");
  if (geo_order > p->order)
    return fail(nullptr, FR_ERR_UNSUPPORTED, "geometry order above the solution order (periodic faces would not be watertight)");
  const int nq = geo_order + 1, NQ = nq * nq * nq;
  for (int64_t i = 0; i < n_elem * NQ; ++i)
    if (ho_nodes[i] < 0 || ho_nodes[i] >= n_vert) return fail(nullptr, FR_ERR_ARG, "node index out of range");
  // the 8 corners in VTK order: tensor nodes with each index 0 or q
  static const int kc[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0}, {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};
  std::vector<int64_t> corners((size_t)n_elem * 8);
  for (int64_t e = 0; e < n_elem; ++e)
    for (int c = 0; c < 8; ++c) {
      const int i = kc[c][0] * geo_order, j = kc[c][1] * geo_order, k = kc[c][2] * geo_order;
      corners[(size_t)e * 8 + c] = ho_nodes[e * NQ + i + nq * (j + nq * k)];
    }
  std::vector<int32_t> et((size_t)n_elem, FR_HEX);
  return setup_impl(p, n_vert, xyz, period, n_elem, et.data(), corners.data(), geo_order, ho_nodes, stream, out);
}

fr_status fr_setup_mesh_curved_tet(const fr_params* p, int32_t geo_order, int64_t n_vert, const double* xyz,
                                   const double* period, int64_t n_elem, const int64_t* ho_nodes, void* stream,
                                   fr_ctx* out) {
  if (!out) return fail(nullptr, FR_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!p || p->struct_size != sizeof(fr_params)) return fail(nullptr, FR_ERR_ARG, "fr_params missing or struct_size mismatch");
  if (!xyz || !period || !ho_nodes || n_vert <= 0 || n_elem <= 0) return fail(nullptr, FR_ERR_ARG, "empty mesh or NULL array");
  if (geo_order < 1 || geo_order > 4) return fail(nullptr, FR_ERR_UNSUPPORTED, "geometry order must be in 1..4");
  const int q = geo_order, NQ = (q + 1) * (q + 2) * (q + 3) / 6;
  for (int64_t i = 0; i < n_elem * NQ; ++i)
    if (ho_nodes[i] < 0 || ho_nodes[i] >= n_vert) return fail(nullptr, FR_ERR_ARG, "node index out of range");
  // node (i, j, k) has index k-outer, j, i-inner among i + j + k <= q; the corners in
  // reference order are the nodes (0,0,0), (q,0,0), (0,0,q), (0,q,0)
  auto node_id = [q](int i, int j, int k) {
    int id = 0;
    for (int kk = 0; kk < k; ++kk) id += (q + 1 - kk) * (q + 2 - kk) / 2;
    for (int jj = 0; jj < j; ++jj) id += q + 1 - k - jj;
    return id + i;
  };
  const int cid[4] = {node_id(0, 0, 0), node_id(q, 0, 0), node_id(0, 0, q), node_id(0, q, 0)};
  std::vector<int64_t> corners((size_t)n_elem * 8, -1);
  for (int64_t e = 0; e < n_elem; ++e)
    for (int c = 0; c < 4; ++c) corners[(size_t)e * 8 + c] = ho_nodes[e * NQ + cid[c]];
  std::vector<int32_t> et((size_t)n_elem, FR_TET);
  return setup_impl(p, n_vert, xyz, period, n_elem, et.data(), corners.data(), geo_order, ho_nodes, stream, out);
}

fr_status fr_layout(fr_ctx c, fr_layout_t* o) {
  if (!c || !o) return fail(c, FR_ERR_ARG, "NULL argument");
  std::memset(o, 0, sizeof(*o));
  o->n_types = (int32_t)c->blocks.size();
  for (size_t i = 0; i < c->blocks.size(); ++i) {
    const DevBlock& b = c->blocks[i];
    o->etype[i] = b.etype; o->n_elem[i] = b.n; o->e_pad[i] = b.E; o->n_sp[i] = b.nsp; o->n_fp[i] = b.nfp;
    o->canon_offset[i] = b.canon_off; o->native_offset[i] = b.native_off;
  }
  o->canon_len = c->canon_len;
  o->native_len = c->native_len;
  o->native_dtype = c->prm.precision == FR_FP64 ? FR_FP64 : FR_FP32;
  return FR_OK;
}

fr_status fr_sol_points(fr_ctx c, double* xyz) {
  if (!c || !xyz) return fail(c, FR_ERR_ARG, "NULL argument");
  size_t off = 0;
  for (auto& hb : c->host.blocks) {
    std::memcpy(xyz + off, hb.sol_xyz.data(), hb.sol_xyz.size() * sizeof(double));
    off += hb.sol_xyz.size();
  }
  return FR_OK;
}

static fr_status pack64(fr_ctx c, const double* canon, double* native) {
  for (auto& b : c->blocks) {
    const int64_t tot = (int64_t)b.nsp * 5 * b.E;
    k_pack<<<grid_for(tot, 256), 256, 0, c->stream>>>(canon + b.canon_off, native + b.native_off, b.cpos, b.n, b.E,
                                                      b.nsp);
  }
  HIP_TRY(c, hipGetLastError());
  return FR_OK;
}

static fr_status unpack64(fr_ctx c, const double* native, double* canon) {
  for (auto& b : c->blocks) {
    const int64_t tot = b.n * 5 * b.nsp;
    k_unpack<<<grid_for(tot, 256), 256, 0, c->stream>>>(native + b.native_off, canon + b.canon_off, b.npos, b.n, b.E,
                                                        b.nsp);
  }
  HIP_TRY(c, hipGetLastError());
  return FR_OK;
}

fr_status fr_pack(fr_ctx c, const double* canon, void* native) {
  if (!c || !canon || !native) return fail(c, FR_ERR_ARG, "NULL argument");
  if (c->prm.precision == FR_FP64) return pack64(c, canon, (double*)native);
  const RefVec ref = refvec(c->prm);
  for (auto& b : c->blocks) {
    const int64_t tot = (int64_t)b.nsp * 5 * b.E;
    k_pack32<<<grid_for(tot, 256), 256, 0, c->stream>>>(canon + b.canon_off, (float*)native + b.native_off, b.cpos,
                                                        b.n, b.E, b.nsp, ref);
  }
  HIP_TRY(c, hipGetLastError());
  return FR_OK;
}

fr_status fr_unpack(fr_ctx c, const void* native, double* canon) {
  if (!c || !canon || !native) return fail(c, FR_ERR_ARG, "NULL argument");
  if (c->prm.precision == FR_FP64) return unpack64(c, (const double*)native, canon);
  const RefVec ref = refvec(c->prm);
  for (auto& b : c->blocks) {
    const int64_t tot = b.n * 5 * b.nsp;
    k_unpack32<<<grid_for(tot, 256), 256, 0, c->stream>>>((const float*)native + b.native_off, canon + b.canon_off,
                                                          b.npos, b.n, b.E, b.nsp, ref, 1);
  }
  HIP_TRY(c, hipGetLastError());
  return FR_OK;
}

fr_status fr_unpack_rhs(fr_ctx c, const void* r, double* canon) {
  if (!c || !canon || !r) return fail(c, FR_ERR_ARG, "NULL argument");
  if (c->prm.precision == FR_FP64) return unpack64(c, (const double*)r, canon);
  const RefVec ref = refvec(c->prm);
  for (auto& b : c->blocks) {
    const int64_t tot = b.n * 5 * b.nsp;
    k_unpack32<<<grid_for(tot, 256), 256, 0, c->stream>>>((const float*)r + b.native_off, canon + b.canon_off,
                                                          b.npos, b.n, b.E, b.nsp, ref, 0);
  }
  HIP_TRY(c, hipGetLastError());
  return FR_OK;
}

fr_status fr_pack64(fr_ctx c, const double* canon, double* native) {
  if (!c || !canon || !native) return fail(c, FR_ERR_ARG, "NULL argument");
  return pack64(c, canon, native);
}

fr_status fr_unpack64(fr_ctx c, const double* native, double* canon) {
  if (!c || !canon || !native) return fail(c, FR_ERR_ARG, "NULL argument");
  return unpack64(c, native, canon);
}

fr_status fr_rhs(fr_ctx c, const void* u, void* r) {
  if (!c || !u || !r) return fail(c, FR_ERR_ARG, "NULL argument");
  if (u == r) return fail(c, FR_ERR_ARG, "u and r must not alias");
  return rhs_native(c, u, r);
}

}  // extern "C"

namespace {
// RK workspace: stage state and increment in the native dtype, FP64 accumulator.
fr_status rk_alloc(fr_ctx c) {
  if (c->rk_stage) return FR_OK;
  const int64_t n = c->native_len;
  const size_t tsz = c->prm.precision != FR_FP64 ? sizeof(float) : sizeof(double);
  if (dalloc(c, (char**)&c->rk_stage, n * tsz) || dalloc(c, &c->rk_acc, n) || dalloc(c, (char**)&c->rk_k, n * tsz))
    return FR_ERR_ALLOC;
  // padding lanes are never written by the RHS: keep them defined (zero increments)
  HIP_TRY(c, hipMemsetAsync(c->rk_k, 0, n * tsz, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->rk_stage, 0, n * tsz, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->rk_acc, 0, n * sizeof(double), c->stream));
  return FR_OK;
}

// RK3(2)4[2R+]C (Kennedy, Carpenter & Lewis 2000): subdiagonal, weights, embedded weights.
constexpr double kLsA[3][2] = {{11847461282814.0, 36547543011857.0}, {3943225443063.0, 7078155732230.0},
                               {-346793006927.0, 4029903576067.0}};
constexpr double kLsB[4][2] = {{1017324711453.0, 9774461848756.0}, {8237718856693.0, 13685301971492.0},
                               {57731312506979.0, 19404895981398.0}, {-101169746363290.0, 37734290219643.0}};
constexpr double kLsBh[4][2] = {{15763415370699.0, 46270243929542.0}, {514528521746.0, 5659431552419.0},
                                {27030193851939.0, 9429696342944.0}, {-69544964788955.0, 30262026368149.0}};
constexpr int kNormGrid = 1024;
}  // namespace

extern "C" {

void fr_default_adaptive_params(fr_adaptive_params* p) {
  if (!p) return;
  p->atol = 1e-6;
  p->rtol = 1e-6;
  p->safety = 0.9;
  p->fac_min = 0.3;
  p->fac_max = 2.5;
  p->max_attempts = 100000;
  p->reserved = 0;
}

fr_status fr_rk_adaptive(fr_ctx c, void* u_, double t_end, double dt0, const fr_adaptive_params* ap,
                         fr_adaptive_stats* stats) {
  if (!c || !u_ || !ap) return fail(c, FR_ERR_ARG, "NULL argument");
  if (!(t_end > 0) || !std::isfinite(t_end) || !(dt0 > 0) || !std::isfinite(dt0))
    return fail(c, FR_ERR_ARG, "t_end and dt0 must be positive and finite");
  if (!(ap->atol > 0) || !(ap->rtol >= 0) || !(ap->safety > 0) || !(ap->safety <= 1) || !(ap->fac_min > 0) ||
      !(ap->fac_min <= 1) || !(ap->fac_max >= 1) || !std::isfinite(ap->fac_max) || ap->max_attempts < 1)
    return fail(c, FR_ERR_ARG, "adaptive parameters out of range");
  fr_status st;
  if ((st = rk_alloc(c))) return st;
  const int64_t n = c->native_len;
  if (!c->rk_x0) {
    if (dalloc(c, &c->rk_x0, n) || dalloc(c, &c->rk_err, n) ||
        dalloc(c, &c->rk_part, (int64_t)kNormGrid * (int64_t)c->blocks.size()))
      return FR_ERR_ALLOC;
  }
  double* X = (double*)u_;
  const bool f32 = c->prm.precision != FR_FP64;
  const RefVec ref = refvec(c->prm);
  int64_t count = 0;
  for (auto& b : c->blocks) count += b.n * b.nsp * 5;
  std::vector<double> part(c->blocks.size() * kNormGrid);
  // one stage update on every block
  auto stage = [&](int i, double h) {
    const double ya = i < 3 ? h * (kLsA[i][0] / kLsA[i][1]) : 0.0;
    const double xb = h * (kLsB[i][0] / kLsB[i][1]);
    const double ed = h * (kLsB[i][0] / kLsB[i][1] - kLsBh[i][0] / kLsBh[i][1]);
    for (auto& b : c->blocks) {
      const int64_t nb = (int64_t)b.nsp * 5 * b.E, o = b.native_off;
      const int gb = grid_for(nb, 256);
      if (f32)
        k_lsrk_stage<float, float><<<gb, 256, 0, c->stream>>>(X + o, c->rk_x0 + o, (const float*)c->rk_k + o,
                                                              (float*)c->rk_stage + o, c->rk_err + o, nb, b.E, ya,
                                                              xb, ed, i == 0, i == 3, ref);
      else
        k_lsrk_stage<double, double><<<gb, 256, 0, c->stream>>>(X + o, c->rk_x0 + o, (const double*)c->rk_k + o,
                                                                (double*)c->rk_stage + o, c->rk_err + o, nb, b.E,
                                                                ya, xb, ed, i == 0, i == 3, ref);
    }
  };
  fr_adaptive_stats s{};
  double t = 0.0, dt = dt0, nrm = 0.0;
  while (t < t_end && s.accepted + s.rejected < ap->max_attempts) {
    const bool last = dt >= t_end - t;
    const double h = last ? t_end - t : dt;
    for (int i = 0; i < 4; ++i) {
      void* in = c->rk_stage;
      if (i == 0) {
        if (f32) {
          for (auto& b : c->blocks) {
            const int64_t nb = (int64_t)b.nsp * 5 * b.E, o = b.native_off;
            k_to_dev<<<grid_for(nb, 256), 256, 0, c->stream>>>(X + o, (float*)c->rk_stage + o, nb, b.E, ref);
          }
        } else {
          in = X;
        }
      }
      if ((st = rhs_native(c, in, c->rk_k))) return st;
      stage(i, h);
    }
    for (size_t bi = 0; bi < c->blocks.size(); ++bi) {
      const DevBlock& b = c->blocks[bi];
      const int64_t nb = (int64_t)b.nsp * 5 * b.E, o = b.native_off;
      k_err_sumsq<<<kNormGrid, 256, 0, c->stream>>>(c->rk_err + o, c->rk_x0 + o, X + o, nb, b.E, b.n, ap->atol,
                                                     ap->rtol, c->rk_part + bi * kNormGrid);
    }
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipMemcpyAsync(part.data(), c->rk_part, part.size() * sizeof(double), hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    double sum = 0.0;
    for (double v : part) sum += v;
    nrm = std::sqrt(sum / (double)count);
    s.n_rhs += 4;
    if (nrm <= 1.0) {
      t = last ? t_end : t + h;
      ++s.accepted;
    } else {
      HIP_TRY(c, hipMemcpyAsync(X, c->rk_x0, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      ++s.rejected;
    }
    double fac;
    if (!std::isfinite(nrm)) fac = ap->fac_min;
    else if (nrm == 0.0) fac = ap->fac_max;
    else fac = std::min(ap->fac_max, std::max(ap->fac_min, ap->safety * std::pow(nrm, -1.0 / 3.0)));
    dt = h * fac;
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  s.t = t;
  s.dt_next = dt;
  s.last_norm = nrm;
  if (stats) *stats = s;
  return FR_OK;
}

fr_status fr_rk_step(fr_ctx c, void* u_, double dt, int32_t n_steps, int32_t filter_mode) {
  if (!c || !u_) return fail(c, FR_ERR_ARG, "NULL argument");
  if (n_steps < 0 || !std::isfinite(dt)) return fail(c, FR_ERR_ARG, "n_steps or dt");
  if (filter_mode < -1 || filter_mode > 1) return fail(c, FR_ERR_ARG, "filter_mode must be -1, 0 or 1");
  if (filter_mode == 1 && !c->mlp_ready) return fail(c, FR_ERR_STATE, "MLP weights not set");
  if (filter_mode >= 0) {
    fr_status fs = filter_alloc(c);
    if (fs) return fs;
  }
  double* u = (double*)u_;
  const int64_t n = c->native_len;
  const bool f32 = c->prm.precision != FR_FP64;
  fr_status st;
  if ((st = rk_alloc(c))) return st;
  const int g = grid_for(n, 256);
  const double b1 = dt / 6.0, b2 = dt / 3.0, c2 = dt / 2.0;
  int pk;
  if (!f32) {
    double *K = (double*)c->rk_k, *S = (double*)c->rk_stage;
    const bool filt = filter_mode >= 0;
    if (filt && !c->collecting) {
      // each stage update runs inside the filter's detection pass (the stage state is
      // checked as it is formed instead of being read back)
      for (int s = 0; s < n_steps; ++s) {
        if ((st = compute_smin(c, u))) return st;
        for (int stage = 0; stage < 4; ++stage) {
          if ((st = rhs_native(c, stage == 0 ? u : S, K))) return st;
          StageFuse fz;
          fz.mode = stage == 0 ? 0 : (stage < 3 ? 1 : 2);
          fz.b = stage == 0 || stage == 3 ? b1 : b2;
          fz.c = stage == 2 ? dt : c2;
          fz.k = K;
          fz.u = u;
          fz.acc = c->rk_acc;
          fz.s64 = stage < 3 ? S : nullptr;
          if ((st = apply_filter(c, stage < 3 ? S : u, filter_mode, nullptr, &fz))) return st;
        }
      }
      HIP_TRY(c, hipGetLastError());
      return FR_OK;
    }
    for (int s = 0; s < n_steps; ++s) {
      // entropy bound of this step from u_n; every later stage state and u_{n+1} is filtered
      if (filt && (st = compute_smin(c, u))) return st;
      if ((st = rhs_native(c, u, K))) return st;
      pk = c->prof_begin("rk4_update");
      k_rk_first<double><<<g, 256, 0, c->stream>>>(u, K, c->rk_acc, S, n, b1, c2);
      c->prof_end(pk);
      if (filt && (st = apply_filter(c, S, filter_mode))) return st;
      if ((st = rhs_native(c, S, K))) return st;
      pk = c->prof_begin("rk4_update");
      k_rk_mid<double><<<g, 256, 0, c->stream>>>(u, K, c->rk_acc, S, n, b2, c2);
      c->prof_end(pk);
      if (filt && (st = apply_filter(c, S, filter_mode))) return st;
      if ((st = rhs_native(c, S, K))) return st;
      pk = c->prof_begin("rk4_update");
      k_rk_mid<double><<<g, 256, 0, c->stream>>>(u, K, c->rk_acc, S, n, b2, dt);
      c->prof_end(pk);
      if (filt && (st = apply_filter(c, S, filter_mode))) return st;
      if ((st = rhs_native(c, S, K))) return st;
      pk = c->prof_begin("rk4_update");
      k_rk_last<double><<<g, 256, 0, c->stream>>>(u, K, c->rk_acc, n, b1);
      c->prof_end(pk);
      if (filt && (st = apply_filter(c, u, filter_mode))) return st;
    }
  } else {
    float *K = (float*)c->rk_k, *S = (float*)c->rk_stage;
    const RefVec ref = refvec(c->prm);
    // the FP32 deviation of u_n; later steps get it from the previous step's last update
    for (auto& b : c->blocks) {
      const int64_t nb = (int64_t)b.nsp * 5 * b.E;
      k_to_dev<<<grid_for(nb, 256), 256, 0, c->stream>>>(u + b.native_off, S + b.native_off, nb, b.E, ref);
    }
    if (filter_mode >= 0) {
      // filtered: every stage state is formed in FP64 (for the filter and its FP64
      // checks) together with the FP32 deviation the kernels read
      if (!c->rk_s64 && dalloc(c, &c->rk_s64, n)) return FR_ERR_ALLOC;
      double* S64 = c->rk_s64;
      if (!c->collecting) {
        // each stage update runs inside the filter's detection pass: the FP64 stage state
        // is formed in registers and checked there, its FP32 deviation written for the
        // next right-hand side, and only the candidates' FP64 states written for the search
        for (int s = 0; s < n_steps; ++s) {
          if ((st = compute_smin(c, u))) return st;
          for (int stage = 0; stage < 4; ++stage) {
            if ((st = rhs_native(c, S, K))) return st;
            StageFuse fz;
            fz.mode = stage == 0 ? 0 : (stage < 3 ? 1 : 2);
            fz.b = stage == 0 || stage == 3 ? b1 : b2;
            fz.c = stage == 2 ? dt : c2;
            fz.k = K;
            fz.k32 = true;
            fz.u = u;
            fz.acc = c->rk_acc;
            fz.s32 = S;
            fz.cand64 = stage < 3 ? S64 : nullptr;
            if ((st = apply_filter(c, stage < 3 ? S64 : u, filter_mode, S, &fz))) return st;
          }
        }
        HIP_TRY(c, hipGetLastError());
        return FR_OK;
      }
      for (int s = 0; s < n_steps; ++s) {
        if ((st = compute_smin(c, u))) return st;
        for (int stage = 0; stage < 4; ++stage) {
          if ((st = rhs_native(c, S, K))) return st;
          pk = c->prof_begin("rk4_update_f32");
          for (auto& b : c->blocks) {
            const int64_t nb = (int64_t)b.nsp * 5 * b.E, o = b.native_off;
            const int gb = grid_for(nb, 256);
            if (stage < 3)
              k_rk32f_stage<<<gb, 256, 0, c->stream>>>(u + o, K + o, c->rk_acc + o, S64 + o, S + o, nb, b.E,
                                                        stage == 0 ? b1 : b2, stage == 2 ? dt : c2, ref, stage == 0);
            else
              k_rk32_last<<<gb, 256, 0, c->stream>>>(u + o, K + o, c->rk_acc + o, S + o, nb, b.E, b1, ref);
          }
          c->prof_end(pk);
          // the filter rewrites the FP32 deviation of every element it changes
          if ((st = apply_filter(c, stage < 3 ? S64 : u, filter_mode, S))) return st;
        }
      }
    } else {
      for (int s = 0; s < n_steps; ++s) {
        for (int stage = 0; stage < 4; ++stage) {
          if ((st = rhs_native(c, S, K))) return st;
          pk = c->prof_begin("rk4_update_f32");
          for (auto& b : c->blocks) {
            const int64_t nb = (int64_t)b.nsp * 5 * b.E, o = b.native_off;
            const int gb = grid_for(nb, 256);
            if (stage == 0)
              k_rk32_first<<<gb, 256, 0, c->stream>>>(u + o, K + o, c->rk_acc + o, S + o, nb, b.E, b1, c2, ref);
            else if (stage < 3)
              k_rk32_mid<<<gb, 256, 0, c->stream>>>(u + o, K + o, c->rk_acc + o, S + o, nb, b.E, b2,
                                                    stage == 1 ? c2 : dt, ref);
            else
              k_rk32_last<<<gb, 256, 0, c->stream>>>(u + o, K + o, c->rk_acc + o, S + o, nb, b.E, b1, ref);
          }
          c->prof_end(pk);
        }
      }
    }
  }
  HIP_TRY(c, hipGetLastError());
  return FR_OK;
}

fr_status fr_check(fr_ctx c, const void* u) {
  if (!c || !u) return fail(c, FR_ERR_ARG, "NULL argument");
  HIP_TRY(c, hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
  for (auto& b : c->blocks) {
    k_check<<<grid_for(b.n * b.nsp, 256), 256, 0, c->stream>>>((const double*)u + b.native_off, b.n, b.E, b.nsp,
                                                              c->prm.gamma - 1.0, c->flag);
  }
  int h = 0;
  HIP_TRY(c, hipMemcpyAsync(&h, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return h ? fail(c, FR_ERR_NONFINITE, "non-finite value or non-positive density/pressure") : FR_OK;
}

fr_status fr_profile(fr_ctx c, int32_t enable) {
  if (!c) return fail(c, FR_ERR_ARG, "NULL context");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (enable) c->prof_clear();
  c->prof = enable != 0;
  return FR_OK;
}

fr_status fr_profile_read(fr_ctx c, fr_kernel_time* out, int32_t cap, int32_t* n) {
  if (!c || !n || (cap > 0 && !out)) return fail(c, FR_ERR_ARG, "NULL argument");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  std::vector<fr_kernel_time> acc(c->prof_names.size());
  for (size_t i = 0; i < acc.size(); ++i) {
    std::memset(&acc[i], 0, sizeof(fr_kernel_time));
    std::strncpy(acc[i].name, c->prof_names[i].c_str(), sizeof(acc[i].name) - 1);
  }
  for (auto& e : c->prof_events) {
    float ms = 0;
    HIP_TRY(c, hipEventElapsedTime(&ms, e.a, e.b));
    acc[e.id].launches += 1;
    acc[e.id].total_ms += ms;
  }
  *n = (int32_t)acc.size();
  for (int32_t i = 0; i < cap && i < (int32_t)acc.size(); ++i) out[i] = acc[i];
  return FR_OK;
}

fr_status fr_sync(fr_ctx c) {
  if (!c) return fail(c, FR_ERR_ARG, "NULL context");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return FR_OK;
}

fr_status fr_filter(fr_ctx c, void* u_, const void* uprev_, int32_t mode, int32_t* k_dev, fr_filter_stats* stats) {
  if (!c || !u_ || !uprev_) return fail(c, FR_ERR_ARG, "NULL argument");
  if (mode != 0 && mode != 1) return fail(c, FR_ERR_ARG, "mode must be 0 (plain) or 1 (MLP warm start)");
  if (mode == 1 && !c->mlp_ready) return fail(c, FR_ERR_STATE, "MLP weights not set");
  fr_status st;
  if ((st = filter_alloc(c))) return st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (stats) {
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    HIP_TRY(c, hipEventRecord(e0, c->stream));
  }
  if ((st = compute_smin(c, (const double*)uprev_))) return st;
  if ((st = apply_filter(c, (double*)u_, mode))) return st;
  if (k_dev)
    k_elem_to_canon<<<grid_for(c->n_elem_total, 256), 256, 0, c->stream>>>(c->f_k, c->g_npos, c->n_elem_total, k_dev);
  if (stats) {
    HIP_TRY(c, hipEventRecord(e1, c->stream));
    std::vector<int32_t> k(c->n_elem_total), ev(c->n_elem_total);
    HIP_TRY(c, hipMemcpyAsync(k.data(), c->f_k, k.size() * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(ev.data(), c->f_evals, ev.size() * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    float ms = 0;
    HIP_TRY(c, hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::memset(stats, 0, sizeof(*stats));
    for (size_t i = 0; i < k.size(); ++i) {
      if (k[i] != 0) { stats->n_troubled++; stats->n_evals += ev[i]; }
      if (k[i] < 0) stats->n_fallback++;
    }
    stats->seconds = ms * 1e-3;
    for (auto& b : c->blocks) {
      int32_t m = 0;
      HIP_TRY(c, hipMemcpy(&m, b.f_cnt + (b.n + 255) / 256, 4, hipMemcpyDeviceToHost));
      stats->n_candidates += m;
    }
  }
  return FR_OK;
}

fr_status fr_mlp_set_weights(fr_ctx c, const float* w, const float* xm, const float* xs) {
  if (!c || !w || !xm || !xs) return fail(c, FR_ERR_ARG, "NULL argument");
  for (int i = 0; i < MLP_IN; ++i)
    if (!(xs[i] > 0)) return fail(c, FR_ERR_ARG, "x_std must be positive");
  fr_status st;
  if ((st = mlp_alloc(c, 1))) return st;
  std::vector<float> sc(2 * MLP_IN);
  for (int i = 0; i < MLP_IN; ++i) { sc[i] = xm[i]; sc[MLP_IN + i] = xs[i]; }
  HIP_TRY(c, hipMemcpyAsync(c->m_w, w, MLP_NP * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->m_scale, sc.data(), sc.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->mlp_ready = true;
  return FR_OK;
}

fr_status fr_mlp_get_weights(fr_ctx c, float* w) {
  if (!c || !w) return fail(c, FR_ERR_ARG, "NULL argument");
  if (!c->mlp_ready) return fail(c, FR_ERR_STATE, "MLP weights not set");
  HIP_TRY(c, hipMemcpyAsync(w, c->m_w, MLP_NP * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return FR_OK;
}

fr_status fr_mlp_features(fr_ctx c, const void* u_, const void* uprev_, float* x, int32_t* elem, int32_t* kout,
                          int64_t cap, int64_t* n) {
  if (!c || !u_ || !uprev_ || !n || (cap > 0 && !x)) return fail(c, FR_ERR_ARG, "NULL argument");
  fr_status st;
  if ((st = filter_alloc(c))) return st;
  if (!c->f_copy && dalloc(c, &c->f_copy, c->native_len)) return FR_ERR_ALLOC;
  if ((st = compute_smin(c, (const double*)uprev_))) return st;
  if ((st = candidate_features(c, (const double*)u_))) return st;
  // training targets: the plain search on a copy of the state
  HIP_TRY(c, hipMemcpyAsync(c->f_copy, u_, c->native_len * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if ((st = apply_filter(c, c->f_copy, 0))) return st;
  std::vector<int32_t> flag(c->n_elem_total);
  HIP_TRY(c, hipMemcpyAsync(flag.data(), c->f_flag, flag.size() * 4, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  // rows in canonical element order
  std::vector<std::pair<int32_t, int32_t>> sel;
  for (size_t i = 0; i < flag.size(); ++i) if (flag[i]) sel.push_back({c->h_cpos[i], (int32_t)i});
  std::sort(sel.begin(), sel.end());
  std::vector<int32_t> idx(sel.size()), cid(sel.size());
  for (size_t i = 0; i < sel.size(); ++i) { cid[i] = sel[i].first; idx[i] = sel[i].second; }
  *n = (int64_t)idx.size();
  const int64_t m = std::min<int64_t>(cap, *n);
  if (m > 0) {
    int32_t* didx = nullptr;
    if (dalloc(c, &didx, m)) return FR_ERR_ALLOC;
    HIP_TRY(c, hipMemcpyAsync(didx, idx.data(), m * 4, hipMemcpyHostToDevice, c->stream));
    k_gather_features<<<(unsigned)((m + 255) / 256), 256, 0, c->stream>>>(c->f_feat, c->f_k, didx, m, x, nullptr,
                                                                          kout);
    if (elem) HIP_TRY(c, hipMemcpyAsync(elem, cid.data(), m * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    (void)hipFree(didx);
  }
  return FR_OK;
}

fr_status fr_mlp_collect(fr_ctx c, void* u, double dt, int32_t n_steps, float* x, int32_t* k, int64_t cap,
                         int64_t* n) {
  if (!c || !u || !n || cap < 0 || (cap > 0 && (!x || !k))) return fail(c, FR_ERR_ARG, "bad argument");
  fr_status st;
  if ((st = filter_alloc(c))) return st;
  if (!c->f_copy && dalloc(c, &c->f_copy, c->native_len)) return FR_ERR_ALLOC;
  c->collecting = true;
  c->col_x = x;
  c->col_k = k;
  c->col_cap = cap;
  c->col_n = 0;
  c->col_seen = 0;
  st = fr_rk_step(c, u, dt, n_steps, 0);
  c->collecting = false;
  *n = c->col_n;
  return st;
}

fr_status fr_mlp_forward(fr_ctx c, const float* x, int64_t n, float* y) {
  if (!c || (n > 0 && (!x || !y)) || n < 0) return fail(c, FR_ERR_ARG, "bad argument");
  if (!c->mlp_ready) return fail(c, FR_ERR_STATE, "MLP weights not set");
  if (n == 0) return FR_OK;
  mlp_forward<<<(unsigned)((n + 255) / 256), 256, 0, c->stream>>>(c->m_w, c->m_scale, x, nullptr, n, 0, y);
  HIP_TRY(c, hipGetLastError());
  return FR_OK;
}

fr_status fr_mlp_grad(fr_ctx c, const float* x, const float* y, int64_t n, float* grad, float* loss) {
  if (!c || !x || !y || !grad || !loss || n <= 0 || n > (1 << 20)) return fail(c, FR_ERR_ARG, "bad argument");
  if (!c->mlp_ready) return fail(c, FR_ERR_STATE, "MLP weights not set");
  fr_status st;
  if ((st = mlp_alloc(c, (int)n))) return st;
  mlp_fwd_bwd<<<(unsigned)((n + MLP_FB_WAVES - 1) / MLP_FB_WAVES), 64 * MLP_FB_WAVES, 0, c->stream>>>(
      c->m_w, c->m_scale, x, y, nullptr, (int)n, c->m_scratch, c->m_sqerr);
  mlp_grad_reduce<<<(MLP_NP + 1 + MLP_GR_NT - 1) / MLP_GR_NT, MLP_GR_NT, 0, c->stream>>>(c->m_scratch, (int)n,
                                                                                        c->m_sqerr, grad, loss);
  HIP_TRY(c, hipGetLastError());
  return FR_OK;
}

fr_status fr_mlp_grad_static(fr_ctx c, const float* x, const float* y, int64_t n, float* grad, float* loss) {
  if (!c || !x || !y || !grad || !loss) return fail(c, FR_ERR_ARG, "NULL argument");
  if (n <= 0 || n > FR_MLP_STATIC_MAX_BATCH)
    return fail(c, FR_ERR_ARG, "batch size must be in 1..FR_MLP_STATIC_MAX_BATCH (4096)");
  if (!c->mlp_ready) return fail(c, FR_ERR_STATE, "MLP weights not set");
  if (!c->static_scratch) return fail(c, FR_ERR_DEVICE, "address of the static scratch array not available");
  float* S = c->static_scratch;
  float* sq = S + (int64_t)FR_MLP_STATIC_MAX_BATCH * MLP_SS;
  mlp_fwd_bwd<<<(unsigned)((n + MLP_FB_WAVES - 1) / MLP_FB_WAVES), 64 * MLP_FB_WAVES, 0, c->stream>>>(
      c->m_w, c->m_scale, x, y, nullptr, (int)n, S, sq);
  mlp_grad_reduce<<<(MLP_NP + 1 + MLP_GR_NT - 1) / MLP_GR_NT, MLP_GR_NT, 0, c->stream>>>(S, (int)n, sq, grad,
                                                                                        loss);
  HIP_TRY(c, hipGetLastError());
  return FR_OK;
}

fr_status fr_mlp_train(fr_ctx c, const float* x, const float* y, int64_t n, const int32_t* perm, int32_t n_steps,
                       int32_t batch, float lr, float b1, float b2, float eps, float* loss_hist) {
  if (!c || !x || !y || !perm || n <= 0 || n_steps < 0 || batch <= 0 || batch > (1 << 16))
    return fail(c, FR_ERR_ARG, "bad argument");
  if (!c->mlp_ready) return fail(c, FR_ERR_STATE, "MLP weights not set");
  fr_status st;
  if ((st = mlp_alloc(c, batch))) return st;
  HIP_TRY(c, hipMemsetAsync(c->m_m, 0, MLP_NP * sizeof(float), c->stream));
  HIP_TRY(c, hipMemsetAsync(c->m_v, 0, MLP_NP * sizeof(float), c->stream));
  for (int t = 1; t <= n_steps; ++t) {
    mlp_fwd_bwd<<<(unsigned)((batch + MLP_FB_WAVES - 1) / MLP_FB_WAVES), 64 * MLP_FB_WAVES, 0, c->stream>>>(
        c->m_w, c->m_scale, x, y, perm + (int64_t)(t - 1) * batch, batch, c->m_scratch, c->m_sqerr);
    mlp_grad_reduce<<<(MLP_NP + 1 + MLP_GR_NT - 1) / MLP_GR_NT, MLP_GR_NT, 0, c->stream>>>(
        c->m_scratch, batch, c->m_sqerr, c->m_g, loss_hist ? loss_hist + (t - 1) : c->m_loss);
    mlp_adam<<<(MLP_NP + 255) / 256, 256, 0, c->stream>>>(c->m_w, c->m_g, c->m_m, c->m_v, t, lr, b1, b2, eps);
  }
  HIP_TRY(c, hipGetLastError());
  return FR_OK;
}

}  // extern "C"
