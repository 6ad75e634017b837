// Flow integrals of paper Sec. 4.1 (volume-averaged kinetic energy K and
// solenoidal dissipation eps^S), plus K_rho and the means of the conserved
// fields.  Everything -- loads, the 4th-order velocity gradient and the
// accumulation -- is FP64 whatever the storage type of Q.
//
// Pass 1 marches a 64 x 4 tile of (x, y) columns along z, as the residual
// kernel: each plane of the tile plus a 2-point halo is loaded once (rho and
// the momenta, coalesced along x), turned into velocities in LDS, and each
// thread takes the in-plane parts of the vorticity at its own column from
// LDS and the z-parts from a 5-plane register window of u and v.  Only the
// components the vorticity needs are differentiated:
//   w1 = D_y w - D_z v,  w2 = D_z u - D_x w,  w3 = D_x v - D_y u.
// Deterministic two-pass reduction: pass 1 gives one row of 8 partial sums
// per block (fixed point-to-thread mapping, wavefront shuffles then LDS
// across waves); pass 2 sums the rows in a fixed order in a single block.
#include <mutex>

#include "tgv_device.h"
#include "tgv_kernels.h"

// Partial-sum rows of the allocation-free entry point (flow_integrals_noalloc):
// 8 doubles per first-pass block, for grids of up to kNoAllocRows blocks
// (4 MiB; every cube up to 1024^3).  Each device holds its own copy for the
// life of the process.  In host code this name is not a device address: the
// launcher takes the address from hipGetSymbolAddress, per device.
static __device__ __align__(256) double scratch[tgv::kNoAllocRows * 8];

namespace tgv {

namespace {

constexpr int IX = 64, IY = 4, kThreads = IX * IY;
constexpr int IHX = IX + 4, IHY = IY + 4, IPL = IHX * IHY;  // plane incl. halo
// The plane is loaded in runs of consecutive x-points per lane (the RUN
// parameter of pass 1): two for FP32 and FP16 storage when nx is even (tile
// origins and the halo width are even, so a run never crosses the periodic
// wrap and stays aligned to its length), else one.
template <int V>
struct IRuns {
  static constexpr int VPR = IHX / V, NVS = IPL / V, LOADS = (NVS + kThreads - 1) / kThreads;
};
template <class T, int V>
struct alignas(sizeof(T) * V) IRun {
  T e[V];
};

struct IntLaunch {
  int tiles_x, tiles_y, kz;
  long long blocks;
};

// Planes per block: as long as the grid still fills the chip several times.
IntLaunch int_launch(const Grid& g) {
  IntLaunch L;
  L.tiles_x = (g.nx + IX - 1) / IX;
  L.tiles_y = (g.ny + IY - 1) / IY;
  L.kz = 64;
  while (L.kz > 8 && (long long)L.tiles_x * L.tiles_y * ((g.nz + L.kz - 1) / L.kz) < 4096) L.kz /= 2;
  L.blocks = (long long)L.tiles_x * L.tiles_y * ((g.nz + L.kz - 1) / L.kz);
  return L;
}

// Sum of v over the block; valid in thread 0.
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

// i in [-n, 2n)
__device__ __forceinline__ int wrap(int i, int n) {
  i += (i < 0) ? n : 0;
  i -= (i >= n) ? n : 0;
  return i;
}

template <class Tq, int RUN>
__global__ void __launch_bounds__(kThreads) integrals_pass1(Grid g, Coef<double> c, const Tq* __restrict__ q,
                                                            double* __restrict__ work, int tiles_x, int tiles_y,
                                                            int kz) {
  constexpr int VPR = IRuns<RUN>::VPR, NVS = IRuns<RUN>::NVS, ILOADS = IRuns<RUN>::LOADS;
  __shared__ double vel[2][3][IPL];  // double-buffered velocity plane
  __shared__ double red[4];
  // contiguous runs of tiles per XCD (hardware block b runs on XCD b % 8),
  // x fastest, so that neighbouring tiles' halo rows meet in one L2
  const int nb = gridDim.x;
  int b = blockIdx.x;
  if (nb % 8 == 0) b = (b % 8) * (nb / 8) + b / 8;
  const int x0 = (b % tiles_x) * IX;
  const int y0 = ((b / tiles_x) % tiles_y) * IY;
  const int z0 = (b / (tiles_x * tiles_y)) * kz;
  const int z1 = min(z0 + kz, g.nz);
  const int tid = threadIdx.x;

  // runs this thread loads: wrapped offset of the run's first point within
  // a plane, and whether each point is one of the tile's own (interior,
  // in-grid) points
  long long off[ILOADS];
  bool own[ILOADS][RUN];
#pragma unroll
  for (int l = 0; l < ILOADS; ++l) {
    const int sv = tid + l * kThreads;
    const int lx = (sv % VPR) * RUN, ly = sv / VPR;
    int x = (x0 - 2 + lx) % g.nx, y = (y0 - 2 + ly) % g.ny;  // the halo may wrap more than once
    x += (x < 0) ? g.nx : 0;
    y += (y < 0) ? g.ny : 0;
    off[l] = (long long)y * g.nx + x;
#pragma unroll
    for (int e = 0; e < RUN; ++e)
      own[l][e] = sv < NVS && lx + e >= 2 && lx + e < IX + 2 && ly >= 2 && ly < IY + 2 && x0 - 2 + lx + e < g.nx &&
                  y0 - 2 + ly < g.ny;
  }
  const int tx = tid % IX, ty = tid / IX;
  const bool col_valid = x0 + tx < g.nx && y0 + ty < g.ny;
  const int c0 = (ty + 2) * IHX + tx + 2;  // own column in the LDS plane

  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double uw[5] = {0, 0, 0, 0, 0}, vw[5] = {0, 0, 0, 0, 0};  // u, v at planes p-4 .. p
  double wi[3][3] = {};  // in-plane vorticity parts at planes p-2, p-1, p
  for (int p = z0 - 2, buf = 0; p <= z1 + 1; ++p, buf ^= 1) {
    const long long zo = (long long)wrap(p, g.nz) * g.plane;
    const bool inside = p >= z0 && p < z1;
#pragma unroll
    for (int l = 0; l < ILOADS; ++l) {
      const int sv = tid + l * kThreads;
      if (sv < NVS) {
        const long long id = zo + off[l];
        const int s0 = (sv / VPR) * IHX + (sv % VPR) * RUN;
        const IRun<Tq, RUN> rr = *reinterpret_cast<const IRun<Tq, RUN>*>(q + id);
        const IRun<Tq, RUN> r1 = *reinterpret_cast<const IRun<Tq, RUN>*>(q + g.N + id);
        const IRun<Tq, RUN> r2 = *reinterpret_cast<const IRun<Tq, RUN>*>(q + 2 * g.N + id);
        const IRun<Tq, RUN> r3 = *reinterpret_cast<const IRun<Tq, RUN>*>(q + 3 * g.N + id);
#pragma unroll
        for (int e = 0; e < RUN; ++e) {
          const double rho = load_as<double>(rr.e[e]);
          const double m1 = load_as<double>(r1.e[e]);
          const double m2 = load_as<double>(r2.e[e]);
          const double m3 = load_as<double>(r3.e[e]);
          const double u = m1 / rho, v = m2 / rho, w = m3 / rho;
          vel[buf][0][s0 + e] = u;
          vel[buf][1][s0 + e] = v;
          vel[buf][2][s0 + e] = w;
          if (inside && own[l][e]) {
            const double uu = u * u + v * v + w * w;
            acc[0] += 0.5 * uu;
            acc[1] += 0.5 * rho * uu;
            acc[3] += rho;
            acc[4] += m1;
            acc[5] += m2;
            acc[6] += m3;
            acc[7] += load_as<double>(q[4 * g.N + id + e]);
          }
        }
      }
    }
    __syncthreads();  // one barrier per plane: the other buffer is free again
    const double* U = vel[buf][0];
    const double* V = vel[buf][1];
    const double* W = vel[buf][2];
    const double dxv = c.c1[0] * (8.0 * (V[c0 + 1] - V[c0 - 1]) - (V[c0 + 2] - V[c0 - 2]));
    const double dxw = c.c1[0] * (8.0 * (W[c0 + 1] - W[c0 - 1]) - (W[c0 + 2] - W[c0 - 2]));
    const double dyu = c.c1[1] * (8.0 * (U[c0 + IHX] - U[c0 - IHX]) - (U[c0 + 2 * IHX] - U[c0 - 2 * IHX]));
    const double dyw = c.c1[1] * (8.0 * (W[c0 + IHX] - W[c0 - IHX]) - (W[c0 + 2 * IHX] - W[c0 - 2 * IHX]));
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      uw[i] = uw[i + 1];
      vw[i] = vw[i + 1];
    }
    uw[4] = U[c0];
    vw[4] = V[c0];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      wi[0][k] = wi[1][k];
      wi[1][k] = wi[2][k];
    }
    wi[2][0] = dyw;
    wi[2][1] = -dxw;
    wi[2][2] = dxv - dyu;
    // plane p - 2 has its z-neighbours p - 4 .. p in the window now
    if (p - 2 >= z0 && col_valid) {
      const double dzu = c.c1[2] * (8.0 * (uw[3] - uw[1]) - (uw[4] - uw[0]));
      const double dzv = c.c1[2] * (8.0 * (vw[3] - vw[1]) - (vw[4] - vw[0]));
      const double w1 = wi[0][0] - dzv, w2 = wi[0][1] + dzu, w3 = wi[0][2];
      acc[2] += w1 * w1 + w2 * w2 + w3 * w3;
    }
  }
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const double s = block_sum(acc[m], red);
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

long long integrals_blocks(const Grid& g) { return int_launch(g).blocks; }

long long integrals_work_items(const Grid& g) { return int_launch(g).blocks * kThreads; }

template <class Tq>
hipError_t launch_integrals(const Grid& g, const Coef<double>& c, const void* q, double* work, double* out8,
                            hipStream_t st) {
  const IntLaunch L = int_launch(g);
  // Pairs for FP32 and FP16 storage (9-12 % faster at 512^3); with FP64
  // storage they are no faster and fetch 18 % more from the fabric.
  constexpr bool kPairs = sizeof(Tq) < 8;
  if (kPairs && g.nx % 2 == 0)
    hipLaunchKernelGGL((integrals_pass1<Tq, kPairs ? 2 : 1>), dim3((unsigned)L.blocks), dim3(kThreads), 0, st, g, c,
                       static_cast<const Tq*>(q), work, L.tiles_x, L.tiles_y, L.kz);
  else
    hipLaunchKernelGGL((integrals_pass1<Tq, 1>), dim3((unsigned)L.blocks), dim3(kThreads), 0, st, g, c,
                       static_cast<const Tq*>(q), work, L.tiles_x, L.tiles_y, L.kz);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(integrals_pass2, dim3(1), dim3(kThreads), 0, st, L.blocks, 1.0 / (double)g.N, c.ire, work,
                     out8);
  return hipGetLastError();
}

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the device that runs `st` (the current device
// for the null stream), looked up once per device with that device current.
hipError_t noalloc_scratch(hipStream_t st, double** out) {
  int cur = 0, dev = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  dev = cur;
  if (st != nullptr && (e = hipStreamGetDevice(st, &dev)) != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[dev] == nullptr) {
    if (dev != cur && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (dev != cur) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    g_scratch[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch[dev];
  return hipSuccess;
}
}  // namespace

template <class Tq>
hipError_t launch_integrals_noalloc(const Grid& g, const Coef<double>& c, const void* q, double* out8,
                                    hipStream_t st) {
  if (int_launch(g).blocks > kNoAllocRows) return hipErrorInvalidValue;  // the C-ABI refuses such grids first
  double* work = nullptr;
  const hipError_t e = noalloc_scratch(st, &work);
  if (e != hipSuccess) return e;
  return launch_integrals<Tq>(g, c, q, work, out8, st);
}

template hipError_t launch_integrals_noalloc<double>(const Grid&, const Coef<double>&, const void*, double*, hipStream_t);
template hipError_t launch_integrals_noalloc<float>(const Grid&, const Coef<double>&, const void*, double*, hipStream_t);
template hipError_t launch_integrals_noalloc<f16>(const Grid&, const Coef<double>&, const void*, double*, hipStream_t);

template hipError_t launch_integrals<double>(const Grid&, const Coef<double>&, const void*, double*, double*, hipStream_t);
template hipError_t launch_integrals<float>(const Grid&, const Coef<double>&, const void*, double*, double*, hipStream_t);
template hipError_t launch_integrals<f16>(const Grid&, const Coef<double>&, const void*, double*, double*, hipStream_t);

}  // namespace tgv
