// Flow integrals of paper Sec. 4.1 (volume-averaged kinetic energy K and
// solenoidal dissipation eps^S), plus K_rho and the means of the conserved
// fields.  Everything -- loads, the 4th-order velocity gradient and the
// accumulation -- is FP64 whatever the storage type of Q.  Deterministic
// two-pass reduction: pass 1 gives one row of 8 partial sums per block (fixed
// point-to-thread mapping, wavefront shuffles then LDS across waves); pass 2
// sums the rows in a fixed order in a single block.
#include "tgv_device.h"
#include "tgv_kernels.h"

namespace tgv {

namespace {

constexpr int kThreads = 256;
constexpr int kPointsPerThread = 8;

__device__ __forceinline__ long long wrap_shift(const Grid& g, long long id, int i, int j, int k, int d, int s) {
  if (d == 0) {
    int t = i + s;
    t += (t < 0) ? g.nx : 0;
    t -= (t >= g.nx) ? g.nx : 0;
    return id + (t - i);
  } else if (d == 1) {
    int t = j + s;
    t += (t < 0) ? g.ny : 0;
    t -= (t >= g.ny) ? g.ny : 0;
    return id + (long long)(t - j) * g.nx;
  }
  int t = k + s;
  t += (t < 0) ? g.nz : 0;
  t -= (t >= g.nz) ? g.nz : 0;
  return id + (long long)(t - k) * g.plane;
}

// Sum of v over the 256 threads of the block; valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* lds) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) t = (lds[0] + lds[1]) + (lds[2] + lds[3]);
  return t;
}

template <class Tq>
__device__ __forceinline__ void vel(const Tq* __restrict__ q, long long N, long long id, double u[3]) {
  const double ir = 1.0 / load_as<double>(q[id]);
#pragma unroll
  for (int a = 0; a < 3; ++a) u[a] = load_as<double>(q[(a + 1) * N + id]) * ir;
}

template <class Tq>
__global__ void __launch_bounds__(kThreads) integrals_pass1(Grid g, Coef<double> c, const Tq* __restrict__ q,
                                                            double* __restrict__ work) {
  __shared__ double lds[4];
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const long long per_block = (long long)kThreads * kPointsPerThread;
  const long long start = (long long)blockIdx.x * per_block;
  for (int e = 0; e < kPointsPerThread; ++e) {
    const long long id = start + (long long)e * kThreads + threadIdx.x;
    if (id >= g.N) break;
    const int i = (int)(id % g.nx), j = (int)((id / g.nx) % g.ny), k = (int)(id / g.plane);
    double u0[3];
    vel(q, g.N, id, u0);
    const double rho = load_as<double>(q[id]);
    const double uu = u0[0] * u0[0] + u0[1] * u0[1] + u0[2] * u0[2];
    double G[3][3];  // G[a][d] = D_d u_a
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double um2[3], um1[3], up1[3], up2[3];
      vel(q, g.N, wrap_shift(g, id, i, j, k, d, -2), um2);
      vel(q, g.N, wrap_shift(g, id, i, j, k, d, -1), um1);
      vel(q, g.N, wrap_shift(g, id, i, j, k, d, +1), up1);
      vel(q, g.N, wrap_shift(g, id, i, j, k, d, +2), up2);
#pragma unroll
      for (int a = 0; a < 3; ++a) G[a][d] = c.c1[d] * (8.0 * (up1[a] - um1[a]) - (up2[a] - um2[a]));
    }
    const double w1 = G[2][1] - G[1][2], w2 = G[0][2] - G[2][0], w3 = G[1][0] - G[0][1];
    acc[0] += 0.5 * uu;
    acc[1] += 0.5 * rho * uu;
    acc[2] += w1 * w1 + w2 * w2 + w3 * w3;
#pragma unroll
    for (int f = 0; f < 5; ++f) acc[3 + f] += load_as<double>(q[f * g.N + id]);
  }
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const double s = block_sum(acc[m], lds);
    if (threadIdx.x == 0) work[(long long)blockIdx.x * 8 + m] = s;
  }
}

__global__ void __launch_bounds__(kThreads) integrals_pass2(long long rows, double invN, double ire,
                                                            const double* __restrict__ work,
                                                            double* __restrict__ out8) {
  __shared__ double lds[4];
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (long long row = threadIdx.x; row < rows; row += kThreads)
#pragma unroll
    for (int m = 0; m < 8; ++m) acc[m] += work[row * 8 + m];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const double s = block_sum(acc[m], lds);
    if (threadIdx.x == 0) out8[m] = (m == 2 ? s * ire : s) * invN;
  }
}

}  // namespace

long long integrals_blocks(const Grid& g) {
  const long long per_block = (long long)kThreads * kPointsPerThread;
  return (g.N + per_block - 1) / per_block;
}

template <class Tq>
hipError_t launch_integrals(const Grid& g, const Coef<double>& c, const void* q, double* work, double* out8,
                            hipStream_t st) {
  const long long rows = integrals_blocks(g);
  hipLaunchKernelGGL((integrals_pass1<Tq>), dim3((unsigned)rows), dim3(kThreads), 0, st, g, c,
                     static_cast<const Tq*>(q), work);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(integrals_pass2, dim3(1), dim3(kThreads), 0, st, rows, 1.0 / (double)g.N, c.ire, work, out8);
  return hipGetLastError();
}

template hipError_t launch_integrals<double>(const Grid&, const Coef<double>&, const void*, double*, double*, hipStream_t);
template hipError_t launch_integrals<float>(const Grid&, const Coef<double>&, const void*, double*, double*, hipStream_t);
template hipError_t launch_integrals<f16>(const Grid&, const Coef<double>&, const void*, double*, double*, hipStream_t);

}  // namespace tgv
