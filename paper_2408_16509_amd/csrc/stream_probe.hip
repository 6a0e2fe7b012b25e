// Streaming-bandwidth probe of the HBM ceiling the FR kernels are measured against:
// read-only, write-only, copy (1:1) and 2:1 read:write passes over device buffers, each
// a grid-stride loop of 16-byte vector accesses, timed with HIP events on one stream.
// Measurement infrastructure of the benchmark; not part of the FR library.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_read(const f4* __restrict__ a, int64_t n, float* __restrict__ sink) {
  f4 s = {0, 0, 0, 0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += a[i];
  // keep the loads: one store per thread whose value depends on all of them, never taken
  // for finite data (the sum is compared with a value it cannot reach)
  const float t = s.x + s.y + s.z + s.w;
  if (t == 1.2345e38f) sink[blockIdx.x] = t;
}

__global__ void __launch_bounds__(256) k_write(f4* __restrict__ b, int64_t n, float v) {
  const f4 x = {v, v, v, v};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = x;
}

__global__ void __launch_bounds__(256) k_copy(const f4* __restrict__ a, f4* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

__global__ void __launch_bounds__(256) k_add(const f4* __restrict__ a, const f4* __restrict__ b,
                                             f4* __restrict__ c, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    c[i] = a[i] + b[i];
}

}  // namespace

extern "C" {

// Bandwidth of the four passes over buffers of `bytes` each (a multiple of 16): out[0..3]
// = GB/s of read-only, write-only, copy and 2:1 (bytes moved / best of `reps` timed
// launches after one untimed one), out[4] = the grid size used.  Returns 0, or a
// non-zero HIP error code (nothing is left allocated).
int frprobe_stream(int64_t bytes, int reps, int grid, double* out) {
  if (bytes <= 0 || bytes % 16 || reps < 1 || grid < 1 || !out) return -1;
  const int64_t n = bytes / 16;
  f4 *a = nullptr, *b = nullptr, *c = nullptr;
  float* sink = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t err = hipSuccess;
  auto check = [&](hipError_t r) { if (err == hipSuccess && r != hipSuccess) err = r; };
  check(hipMalloc((void**)&a, bytes));
  check(hipMalloc((void**)&b, bytes));
  check(hipMalloc((void**)&c, bytes));
  check(hipMalloc((void**)&sink, (size_t)grid * sizeof(float)));
  check(hipEventCreate(&e0));
  check(hipEventCreate(&e1));
  if (err == hipSuccess) {
    k_write<<<grid, 256>>>(a, n, 1.0f);
    k_write<<<grid, 256>>>(b, n, 2.0f);
    check(hipGetLastError());
    check(hipDeviceSynchronize());
  }
  for (int pass = 0; pass < 4 && err == hipSuccess; ++pass) {
    double best = 0.0;
    for (int r = 0; r <= reps && err == hipSuccess; ++r) {
      check(hipEventRecord(e0, nullptr));
      if (pass == 0) k_read<<<grid, 256>>>(a, n, sink);
      else if (pass == 1) k_write<<<grid, 256>>>(c, n, 3.0f);
      else if (pass == 2) k_copy<<<grid, 256>>>(a, c, n);
      else k_add<<<grid, 256>>>(a, b, c, n);
      check(hipGetLastError());
      check(hipEventRecord(e1, nullptr));
      check(hipEventSynchronize(e1));
      float ms = 0;
      check(hipEventElapsedTime(&ms, e0, e1));
      const double moved = (double)bytes * (pass == 0 || pass == 1 ? 1 : (pass == 2 ? 2 : 3));
      if (r > 0 && ms > 0) best = best > moved / (ms * 1e6) ? best : moved / (ms * 1e6);
    }
    out[pass] = best;
  }
  out[4] = grid;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(a);
  (void)hipFree(b);
  (void)hipFree(c);
  (void)hipFree(sink);
  return err == hipSuccess ? 0 : (int)err;
}

}  // extern "C"
