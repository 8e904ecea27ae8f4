// probe.hip -- streaming kernels of the HBM bandwidth probe (include/probe.h).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "probe.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

typedef float v4f __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_copy(const v4f* __restrict__ a, v4f* __restrict__ b, size_t n4) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i < n4) b[i] = a[i];
}

__global__ __launch_bounds__(256) void k_copy_nt(const v4f* __restrict__ a, v4f* __restrict__ b, size_t n4) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i < n4) __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
}

__global__ __launch_bounds__(256) void k_read(const v4f* __restrict__ a, float* __restrict__ out, size_t n4) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= n4) return;
  const v4f v = a[i];
  const float s = v.x + v.y + v.z + v.w;
  if (s == -1.2345e-30f) out[blockIdx.x] = s;  // keeps the load; never true for the probe's data
}

// 16-bit arrays: one value per lane (2-byte accesses) or two adjacent values
// per lane (4-byte accesses), same bytes per pass
template <int Q, typename T>
__global__ __launch_bounds__(512) void k_soa_t(T* __restrict__ f, size_t m) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= m) return;
  T v[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) v[q] = f[q * m + i];
#pragma unroll
  for (int q = 0; q < Q; ++q) f[(Q - 1 - q) * m + i] = v[q];
}

// q arrays read, one float per lane each, their sum written to one array
// (the phase-field pass's pattern: 19 reads, one write per node)
template <int Q>
__global__ __launch_bounds__(512) void k_soa_sum(const float* __restrict__ f, float* __restrict__ out, size_t m) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= m) return;
  float s = 0.0f;
#pragma unroll
  for (int q = 0; q < Q; ++q) s += f[q * m + i];
  out[i] = s;
}

template <typename T>
void launch_soa(int q, void* src, size_t m, hipStream_t st) {
  const unsigned gm = (unsigned)((m + 511) / 512);
  if (q == 19)
    hipLaunchKernelGGL((k_soa_t<19, T>), dim3(gm), dim3(512), 0, st, (T*)src, m);
  else
    hipLaunchKernelGGL((k_soa_t<38, T>), dim3(gm), dim3(512), 0, st, (T*)src, m);
}

void launch(int kind, void* src, void* dst, size_t n, int q, hipStream_t st) {
  const size_t n4 = n / 4;
  const unsigned g4 = (unsigned)((n4 + 255) / 256);
  if (kind == 0)
    hipLaunchKernelGGL(k_copy, dim3(g4), dim3(256), 0, st, (const v4f*)src, (v4f*)dst, n4);
  else if (kind == 1)
    hipLaunchKernelGGL(k_copy_nt, dim3(g4), dim3(256), 0, st, (const v4f*)src, (v4f*)dst, n4);
  else if (kind == 2)
    hipLaunchKernelGGL(k_read, dim3(g4), dim3(256), 0, st, (const v4f*)src, (float*)dst, n4);
  else if (kind == 3)
    launch_soa<float>(q, src, n / (size_t)q, st);
  else if (kind == 4)
    launch_soa<uint16_t>(q, src, 2 * n / (size_t)q, st);
  else if (kind == 5)
    launch_soa<uint32_t>(q, src, n / (size_t)q, st);
  else {
    const size_t m = n / (size_t)q;
    const unsigned gm = (unsigned)((m + 511) / 512);
    if (q == 19)
      hipLaunchKernelGGL(k_soa_sum<19>, dim3(gm), dim3(512), 0, st, (const float*)src, (float*)dst, m);
    else
      hipLaunchKernelGGL(k_soa_sum<38>, dim3(gm), dim3(512), 0, st, (const float*)src, (float*)dst, m);
  }
}

}  // namespace

extern "C" {

int pb_stream(int kind, void* src, void* dst, size_t n, int q, int reps, void* stream, double* ms_out) {
  if (kind < 0 || kind > 6 || !src || !ms_out || reps < 1 || n == 0 || n % 4 || n >= ((size_t)1 << 33))
    return fail(-1, "pb_stream: bad argument");
  if ((kind <= 2 || kind == 6) && !dst) return fail(-1, "pb_stream: dst is required for kinds 0-2 and 6");
  if (kind >= 3 && ((q != 19 && q != 38) || n % (size_t)q))
    return fail(-1, "pb_stream: q must be 19 or 38 and divide n");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(-3, "pb_stream: hipEventCreate failed");
  }
  launch(kind, src, dst, n, q, st);
  hipError_t e = hipEventRecord(e0, st);
  for (int r = 0; r < reps && e == hipSuccess; ++r) launch(kind, src, dst, n, q, st);
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(-3, std::string("pb_stream: ") + hipGetErrorString(e));
  *ms_out = (double)ms / reps;
  return 0;
}

const char* pb_last_error(void) { return g_err.c_str(); }

}  // extern "C"
