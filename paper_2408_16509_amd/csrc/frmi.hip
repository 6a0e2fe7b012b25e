// C ABI of the MI355X-native FR right-hand side (declared in include/frmi.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/frmi.h"
#include "hex.hpp"
#include "setup.hpp"

using namespace frmi;

namespace {

thread_local std::string g_thread_err;

struct DevBlock {
  int etype = 0;
  int64_t n = 0, E = 0;
  int nsp = 0, nfp = 0, nfaces = 0;
  int64_t canon_off = 0, native_off = 0;
  double* geo = nullptr;
  int32_t* nbr_elem = nullptr;
  int32_t* nbr_info = nullptr;
  double* uf = nullptr;     // [nfp][5][E]
  double* grad = nullptr;   // [nsp][15][E]
  double* gradf = nullptr;  // [nfp][15][E]
};

}  // namespace

struct fr_ctx_s {
  fr_params prm;
  hipStream_t stream = nullptr;
  Setup host;
  std::vector<DevBlock> blocks;
  int32_t* perm = nullptr;
  HexK hexk;
  int64_t canon_len = 0, native_len = 0;
  // RK workspace (FP64 native states)
  double* rk_stage = nullptr;
  double* rk_acc = nullptr;
  double* rk_k = nullptr;
  int* flag = nullptr;
  std::string err;
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
__global__ void k_pack(const double* __restrict__ canon, double* __restrict__ nat, int64_t n, int64_t E, int nsp) {
  const int64_t total = (int64_t)nsp * 5 * E;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i % E;
    const int64_t pv = i / E;
    const int v = (int)(pv % 5), pt = (int)(pv / 5);
    nat[i] = e < n ? canon[(e * 5 + v) * nsp + pt] : (v == 0 || v == 4 ? 1.0 : 0.0);
  }
}

__global__ void k_unpack(const double* __restrict__ nat, double* __restrict__ canon, int64_t n, int64_t E, int nsp) {
  const int64_t total = n * 5 * nsp;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int pt = (int)(i % nsp);
    const int64_t ev = i / nsp;
    const int v = (int)(ev % 5);
    const int64_t e = ev / 5;
    canon[i] = nat[((int64_t)pt * 5 + v) * E + e];
  }
}

// ------------------------------------------------------------ RK4 kernels
// stage 1: acc = u + dt/6 k ; st = u + dt/2 k
__global__ void k_rk_first(const double* __restrict__ u, const double* __restrict__ k, double* __restrict__ acc,
                           double* __restrict__ st, int64_t n, double b, double c) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double ui = u[i], ki = k[i];
    acc[i] = ui + b * ki;
    st[i] = ui + c * ki;
  }
}
// middle stages: acc += b k ; st = u + c k
__global__ void k_rk_mid(const double* __restrict__ u, const double* __restrict__ k, double* __restrict__ acc,
                         double* __restrict__ st, int64_t n, double b, double c) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double ki = k[i];
    acc[i] += b * ki;
    st[i] = u[i] + c * ki;
  }
}
// last: u = acc + b k
__global__ void k_rk_last(double* __restrict__ u, const double* __restrict__ k, const double* __restrict__ acc,
                          int64_t n, double b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    u[i] = acc[i] + b * k[i];
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

// ------------------------------------------------------------ hex dispatch
template <int P>
struct HexCfg;
template <> struct HexCfg<1> { static constexpr int NE = 64; };
template <> struct HexCfg<2> { static constexpr int NE = 32; };
template <> struct HexCfg<3> { static constexpr int NE = 16; };
template <> struct HexCfg<4> { static constexpr int NE = 8; };

template <int P>
fr_status hex_rhs_p(fr_ctx c, DevBlock& b, const double* u, double* r) {
  constexpr int N1 = P + 1, NE = HexCfg<P>::NE, NT = NE * N1 * N1;
  Conn C{b.nbr_elem, b.nbr_info, c->perm, c->host.perm_stride};
  const Phys ph = phys_of(c->prm);
  const int64_t trace_threads = b.E * 3 * N1 * N1;
  static const std::string sfx = "_p" + std::to_string(P);
  int pk = c->prof_begin(("hex_trace" + sfx).c_str());
  hex_trace<P><<<(unsigned)((trace_threads + 255) / 256), 256, 0, c->stream>>>(u, b.uf, b.E, c->hexk);
  c->prof_end(pk);
  const unsigned nblk = (unsigned)(b.E / NE);
  if (c->prm.system == FR_EULER) {
    pk = c->prof_begin(("hex_div_euler" + sfx).c_str());
    hex_div_euler<P, NE><<<nblk, NT, 0, c->stream>>>(u, b.uf, b.geo, C, r, b.E, b.n, c->hexk, ph);
    c->prof_end(pk);
  } else {
    pk = c->prof_begin(("hex_grad" + sfx).c_str());
    hex_grad<P, NE><<<nblk, NT, 0, c->stream>>>(u, b.uf, b.geo, C, b.grad, b.gradf, b.E, c->hexk, ph);
    c->prof_end(pk);
    pk = c->prof_begin(("hex_div_ns" + sfx).c_str());
    hex_div_ns<P, NE><<<nblk, NT, 0, c->stream>>>(u, b.uf, b.grad, b.gradf, b.geo, C, r, b.E, b.n, c->hexk, ph);
    c->prof_end(pk);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, FR_ERR_DEVICE, std::string("hex kernel launch: ") + hipGetErrorString(e));
  return FR_OK;
}

fr_status rhs_fp64(fr_ctx c, const double* u, double* r) {
  for (auto& b : c->blocks) {
    const double* ub = u + b.native_off;
    double* rb = r + b.native_off;
    fr_status s = FR_OK;
    if (b.etype == FR_HEX) {
      switch (c->prm.order) {
        case 1: s = hex_rhs_p<1>(c, b, ub, rb); break;
        case 2: s = hex_rhs_p<2>(c, b, ub, rb); break;
        case 3: s = hex_rhs_p<3>(c, b, ub, rb); break;
        case 4: s = hex_rhs_p<4>(c, b, ub, rb); break;
        default: s = fail(c, FR_ERR_UNSUPPORTED, "order");
      }
    } else {
      s = fail(c, FR_ERR_UNSUPPORTED, "tetrahedra not yet available");
    }
    if (s != FR_OK) return s;
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
    (void)hipFree(b.geo); (void)hipFree(b.nbr_elem); (void)hipFree(b.nbr_info);
    (void)hipFree(b.uf); (void)hipFree(b.grad); (void)hipFree(b.gradf);
  }
  (void)hipFree(c->perm);
  (void)hipFree(c->rk_stage); (void)hipFree(c->rk_acc); (void)hipFree(c->rk_k);
  (void)hipFree(c->flag);
  c->prof_clear();
  delete c;
}

fr_status fr_setup_mesh(const fr_params* p, int64_t n_vert, const double* xyz, const double* period,
                        int64_t n_elem, const int32_t* etype, const int64_t* enodes, void* stream,
                        fr_ctx* out) {
  if (!out) return fail(nullptr, FR_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!p || p->struct_size != sizeof(fr_params)) return fail(nullptr, FR_ERR_ARG, "fr_params missing or struct_size mismatch");
  if (!xyz || !period || !etype || !enodes || n_vert <= 0 || n_elem <= 0) return fail(nullptr, FR_ERR_ARG, "empty mesh or NULL array");
  if (p->system != FR_EULER && p->system != FR_NAVIER_STOKES) return fail(nullptr, FR_ERR_ARG, "system");
  if (p->riemann != FR_RUSANOV && p->riemann != FR_HLLC) return fail(nullptr, FR_ERR_ARG, "riemann");
  if (p->precision != FR_FP64) return fail(nullptr, FR_ERR_UNSUPPORTED, "precision");
  if (!(p->gamma > 1.0)) return fail(nullptr, FR_ERR_ARG, "gamma must exceed 1");
  if (p->filt_bits < 1 || p->filt_bits > 30) return fail(nullptr, FR_ERR_ARG, "filt_bits must be in 1..30");
  fr_ctx c = new (std::nothrow) fr_ctx_s();
  if (!c) return fail(nullptr, FR_ERR_ALLOC, "context allocation");
  c->prm = *p;
  c->stream = (hipStream_t)stream;
  int code = 0;
  std::string msg;
  try {
    msg = build_setup(p->order, n_vert, xyz, period, n_elem, etype, enodes, 64, c->host, code);
  } catch (const std::exception& ex) {
    msg = ex.what();
    code = 3;
  }
  if (!msg.empty()) {
    fr_status s = code == 2 ? FR_ERR_MESH : (code == 3 ? FR_ERR_UNSUPPORTED : FR_ERR_ARG);
    delete c;
    return fail(nullptr, s, msg);
  }
  const HexOps& H = c->host.hex;
  for (int a = 0; a < 5; ++a) {
    c->hexk.x[a] = H.x[a]; c->hexk.lm[a] = H.lm[a]; c->hexk.lp[a] = H.lp[a];
    c->hexk.cp[a] = H.cp[a]; c->hexk.cm[a] = H.cm[a];
    for (int b = 0; b < 5; ++b) c->hexk.Dh[a][b] = H.Dh[a][b];
  }
  int64_t canon = 0, native = 0;
  auto bail = [&](fr_status s) { std::string m = c->err; fr_destroy(c); return fail(nullptr, s, m); };
  for (auto& hb : c->host.blocks) {
    DevBlock b;
    b.etype = hb.etype; b.n = hb.n; b.E = hb.e_pad; b.nsp = hb.nsp; b.nfp = hb.nfp; b.nfaces = hb.nfaces;
    b.canon_off = canon; b.native_off = native;
    canon += b.n * 5 * b.nsp;
    native += b.E * 5 * b.nsp;
    c->blocks.push_back(b);
    DevBlock& d = c->blocks.back();
    if (dalloc(c, &d.geo, hb.geo.size()) || dalloc(c, &d.nbr_elem, hb.nbr_elem.size()) ||
        dalloc(c, &d.nbr_info, hb.nbr_info.size()) || dalloc(c, &d.uf, (size_t)d.nfp * 5 * d.E))
      return bail(FR_ERR_ALLOC);
    if (p->system == FR_NAVIER_STOKES &&
        (dalloc(c, &d.grad, (size_t)d.nsp * 15 * d.E) || dalloc(c, &d.gradf, (size_t)d.nfp * 15 * d.E)))
      return bail(FR_ERR_ALLOC);
    if (hipMemcpy(d.geo, hb.geo.data(), hb.geo.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d.nbr_elem, hb.nbr_elem.data(), hb.nbr_elem.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d.nbr_info, hb.nbr_info.data(), hb.nbr_info.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
      c->err = "upload failed";
      return bail(FR_ERR_DEVICE);
    }
  }
  c->canon_len = canon;
  c->native_len = native;
  if (dalloc(c, &c->perm, c->host.orient_perm.size()) || dalloc(c, &c->flag, 1)) return bail(FR_ERR_ALLOC);
  if (hipMemcpy(c->perm, c->host.orient_perm.data(), c->host.orient_perm.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
    c->err = "upload failed";
    return bail(FR_ERR_DEVICE);
  }
  *out = c;
  return FR_OK;
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
  o->native_dtype = c->prm.precision;
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

fr_status fr_pack(fr_ctx c, const double* canon, void* native) {
  if (!c || !canon || !native) return fail(c, FR_ERR_ARG, "NULL argument");
  for (auto& b : c->blocks) {
    const int64_t tot = (int64_t)b.nsp * 5 * b.E;
    k_pack<<<grid_for(tot, 256), 256, 0, c->stream>>>(canon + b.canon_off, (double*)native + b.native_off, b.n, b.E, b.nsp);
  }
  HIP_TRY(c, hipGetLastError());
  return FR_OK;
}

fr_status fr_unpack(fr_ctx c, const void* native, double* canon) {
  if (!c || !canon || !native) return fail(c, FR_ERR_ARG, "NULL argument");
  for (auto& b : c->blocks) {
    const int64_t tot = b.n * 5 * b.nsp;
    k_unpack<<<grid_for(tot, 256), 256, 0, c->stream>>>((const double*)native + b.native_off, canon + b.canon_off, b.n, b.E, b.nsp);
  }
  HIP_TRY(c, hipGetLastError());
  return FR_OK;
}

fr_status fr_rhs(fr_ctx c, const void* u, void* r) {
  if (!c || !u || !r) return fail(c, FR_ERR_ARG, "NULL argument");
  if (u == r) return fail(c, FR_ERR_ARG, "u and r must not alias");
  return rhs_fp64(c, (const double*)u, (double*)r);
}

fr_status fr_rk_step(fr_ctx c, void* u_, double dt, int32_t n_steps, int32_t filter_mode) {
  if (!c || !u_) return fail(c, FR_ERR_ARG, "NULL argument");
  if (n_steps < 0 || !std::isfinite(dt)) return fail(c, FR_ERR_ARG, "n_steps or dt");
  if (filter_mode != -1) return fail(c, FR_ERR_UNSUPPORTED, "filter not yet available");
  double* u = (double*)u_;
  const int64_t n = c->native_len;
  if (!c->rk_stage) {
    if (dalloc(c, &c->rk_stage, n) || dalloc(c, &c->rk_acc, n) || dalloc(c, &c->rk_k, n)) return FR_ERR_ALLOC;
    // padding lanes are never written by the RHS: keep them defined (zero increments)
    HIP_TRY(c, hipMemsetAsync(c->rk_k, 0, n * sizeof(double), c->stream));
    HIP_TRY(c, hipMemsetAsync(c->rk_stage, 0, n * sizeof(double), c->stream));
    HIP_TRY(c, hipMemsetAsync(c->rk_acc, 0, n * sizeof(double), c->stream));
  }
  const int g = grid_for(n, 256);
  for (int s = 0; s < n_steps; ++s) {
    fr_status st;
    int pk;
    if ((st = rhs_fp64(c, u, c->rk_k))) return st;
    pk = c->prof_begin("rk4_update");
    k_rk_first<<<g, 256, 0, c->stream>>>(u, c->rk_k, c->rk_acc, c->rk_stage, n, dt / 6.0, dt / 2.0);
    c->prof_end(pk);
    if ((st = rhs_fp64(c, c->rk_stage, c->rk_k))) return st;
    pk = c->prof_begin("rk4_update");
    k_rk_mid<<<g, 256, 0, c->stream>>>(u, c->rk_k, c->rk_acc, c->rk_stage, n, dt / 3.0, dt / 2.0);
    c->prof_end(pk);
    if ((st = rhs_fp64(c, c->rk_stage, c->rk_k))) return st;
    pk = c->prof_begin("rk4_update");
    k_rk_mid<<<g, 256, 0, c->stream>>>(u, c->rk_k, c->rk_acc, c->rk_stage, n, dt / 3.0, dt);
    c->prof_end(pk);
    if ((st = rhs_fp64(c, c->rk_stage, c->rk_k))) return st;
    pk = c->prof_begin("rk4_update");
    k_rk_last<<<g, 256, 0, c->stream>>>(u, c->rk_k, c->rk_acc, n, dt / 6.0);
    c->prof_end(pk);
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

fr_status fr_filter(fr_ctx c, void*, const void*, int32_t, int32_t*, fr_filter_stats*) {
  return fail(c, FR_ERR_UNSUPPORTED, "filter not yet available");
}
fr_status fr_mlp_set_weights(fr_ctx c, const float*, const float*, const float*) { return fail(c, FR_ERR_UNSUPPORTED, "mlp"); }
fr_status fr_mlp_get_weights(fr_ctx c, float*) { return fail(c, FR_ERR_UNSUPPORTED, "mlp"); }
fr_status fr_mlp_features(fr_ctx c, const void*, const void*, float*, int32_t*, int32_t*, int64_t, int64_t*) {
  return fail(c, FR_ERR_UNSUPPORTED, "mlp");
}
fr_status fr_mlp_forward(fr_ctx c, const float*, int64_t, float*) { return fail(c, FR_ERR_UNSUPPORTED, "mlp"); }
fr_status fr_mlp_grad(fr_ctx c, const float*, const float*, int64_t, float*, float*) { return fail(c, FR_ERR_UNSUPPORTED, "mlp"); }
fr_status fr_mlp_train(fr_ctx c, const float*, const float*, int64_t, const int32_t*, int32_t, int32_t, float, float,
                       float, float, float*) {
  return fail(c, FR_ERR_UNSUPPORTED, "mlp");
}

}  // extern "C"
