// Streaming-bandwidth probes: the attainable HBM rates the step kernels are
// measured against, beside the chip's nameplate peak.  Not part of the
// method: nothing in libtgv.so calls these, and they live in their own
// library (libtgv_probe.so).
//
//   tgv_probe_copy         plain copy, 16 bytes per lane, nontemporal loads
//                          and stores, one 4 KiB chunk per 256-thread block;
//   tgv_probe_stage_stream the fused stage's memory traffic and order without
//                          its arithmetic or halo: 64 x 4 column tiles
//                          marching kz planes along z, per point reading 5
//                          fields of Q_in and of Q~ and writing 5 fields of
//                          Q_out and of Q~ (layout [5][n][n][n], x fastest),
//                          tiles x fastest in contiguous runs per XCD;
//   tgv_probe_stage_flat   the same per-point traffic (FP64) in plain element
//                          order, two points (16 bytes) per lane and array.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

typedef double d2 __attribute__((ext_vector_type(2)));

__global__ void __launch_bounds__(256) probe_copy_kernel(const d2* __restrict__ x, d2* __restrict__ y, long long n2) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n2) __builtin_nontemporal_store(__builtin_nontemporal_load(x + i), y + i);
}

template <class T>
__device__ __forceinline__ void stage_point(T a, T t, T& t2, T& q2) {
  t2 = T(-0.5) * t + T(1e-3) * a;
  q2 = a + T(0.3) * t2;
}
__device__ __forceinline__ void stage_point(uint16_t a, uint16_t t, uint16_t& t2, uint16_t& q2) {
  t2 = (uint16_t)(t + 1);
  q2 = a;
}

template <class T>
__global__ void __launch_bounds__(256) probe_stage_kernel(const T* __restrict__ qin, T* __restrict__ qt,
                                                          T* __restrict__ qout, int n, int kz, int tiles_x,
                                                          int tiles_y) {
  const int nb = gridDim.x;
  int b = blockIdx.x;
  if (nb % 8 == 0) b = (b % 8) * (nb / 8) + b / 8;
  const int x = (b % tiles_x) * 64 + (int)threadIdx.x % 64;
  const int y = ((b / tiles_x) % tiles_y) * 4 + (int)threadIdx.x / 64;
  const int z0 = (b / (tiles_x * tiles_y)) * kz;
  if (x >= n || y >= n) return;
  const long long N = (long long)n * n * n, plane = (long long)n * n;
  for (int z = z0; z < z0 + kz && z < n; ++z) {
    const long long o = z * plane + (long long)y * n + x;
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      const T a = __builtin_nontemporal_load(qin + f * N + o);
      const T t = __builtin_nontemporal_load(qt + f * N + o);
      T t2, q2;
      stage_point(a, t, t2, q2);
      __builtin_nontemporal_store(t2, qt + f * N + o);
      __builtin_nontemporal_store(q2, qout + f * N + o);
    }
  }
}

__global__ void __launch_bounds__(256) probe_stage_flat_kernel(const double* __restrict__ qin, double* __restrict__ qt,
                                                              double* __restrict__ qout, long long N) {
  const long long i = ((long long)blockIdx.x * 256 + threadIdx.x) * 2;
  if (i >= N) return;
  d2 a[5], t[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    a[f] = __builtin_nontemporal_load(reinterpret_cast<const d2*>(qin + f * N + i));
    t[f] = __builtin_nontemporal_load(reinterpret_cast<const d2*>(qt + f * N + i));
  }
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    const d2 t2 = -0.5 * t[f] + 1e-3 * a[f];
    const d2 q2 = a[f] + 0.3 * t2;
    __builtin_nontemporal_store(t2, reinterpret_cast<d2*>(qt + f * N + i));
    __builtin_nontemporal_store(q2, reinterpret_cast<d2*>(qout + f * N + i));
  }
}

template <class T>
int launch_stage(int n, int kz, const void* qin, void* qt, void* qout, hipStream_t st) {
  const int tiles_x = (n + 63) / 64, tiles_y = (n + 3) / 4;
  const long long nb = (long long)tiles_x * tiles_y * ((n + kz - 1) / kz);
  if (nb > 0x7fffffffLL) return -3;
  hipLaunchKernelGGL((probe_stage_kernel<T>), dim3((unsigned)nb), dim3(256), 0, st, static_cast<const T*>(qin),
                     static_cast<T*>(qt), static_cast<T*>(qout), n, kz, tiles_x, tiles_y);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

}  // namespace

extern "C" {

// Copies `bytes` bytes (a multiple of 16; both pointers 16-byte aligned
// device memory, not overlapping) on `stream`.  Returns 0, -1 for a bad
// argument, -5 for a launch error.
int tgv_probe_copy(const void* src, void* dst, unsigned long long bytes, void* stream) {
  if (!src || !dst || bytes % 16 || (reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16)
    return -1;
  const long long n2 = (long long)(bytes / 16);
  if (n2 == 0) return 0;
  const long long nb = (n2 + 255) / 256;
  if (nb > 0x7fffffffLL) return -1;
  hipLaunchKernelGGL(probe_copy_kernel, dim3((unsigned)nb), dim3(256), 0, static_cast<hipStream_t>(stream),
                     static_cast<const d2*>(src), static_cast<d2*>(dst), n2);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

// One pass of the fused stage's traffic over an n^3 grid: q_in, q_t, q_out
// each hold 5 n^3 elements of `elem_bytes` bytes (8, 4 or 2), element
// (f, z, y, x) at f n^3 + (z n + y) n + x.  kz >= 1 planes per block.
// Returns 0, -1 for a bad argument, -3 for a grid too large, -5 for a
// launch error.
int tgv_probe_stage_stream(int n, int kz, int elem_bytes, const void* q_in, void* q_t, void* q_out, void* stream) {
  if (n < 1 || kz < 1 || !q_in || !q_t || !q_out) return -1;
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (elem_bytes) {
    case 8: return launch_stage<double>(n, kz, q_in, q_t, q_out, st);
    case 4: return launch_stage<float>(n, kz, q_in, q_t, q_out, st);
    case 2: return launch_stage<uint16_t>(n, kz, q_in, q_t, q_out, st);
    default: return -1;
  }
}

// The same traffic as tgv_probe_stage_stream with 8-byte elements over N
// points (N even, every array 16-byte aligned), in element order.  Returns 0,
// -1 for a bad argument, -3 for a grid too large, -5 for a launch error.
int tgv_probe_stage_flat(long long N, const void* q_in, void* q_t, void* q_out, void* stream) {
  if (N < 2 || N % 2 || !q_in || !q_t || !q_out ||
      (reinterpret_cast<uintptr_t>(q_in) | reinterpret_cast<uintptr_t>(q_t) | reinterpret_cast<uintptr_t>(q_out)) % 16)
    return -1;
  const long long nb = (N / 2 + 255) / 256;
  if (nb > 0x7fffffffLL) return -3;
  hipLaunchKernelGGL(probe_stage_flat_kernel, dim3((unsigned)nb), dim3(256), 0, static_cast<hipStream_t>(stream),
                     static_cast<const double*>(q_in), static_cast<double*>(q_t), static_cast<double*>(q_out), N);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

}  // extern "C"
