// Taylor-Green initial state (paper Sec. 4.1 initial-condition equations and
// the isothermal density rho = gamma M^2 p), evaluated in FP64 per point and
// rounded once to the storage type of Q; the same fields in primitive form
// (u, rho, p); the conserved vector of a velocity field at fixed density and
// pressure (Sec. 3.1 state vector, E = p / (gamma - 1) + rho |u|^2 / 2) and
// its adjoint; and the trapezoid sum of a dissipation history.
#include "tgv_device.h"
#include "tgv_kernels.h"

namespace tgv {

namespace {

template <class Tq>
__global__ void __launch_bounds__(256) tgv_init_kernel(Grid g, double hx, double hy, double hz,
                                                       double gamma, double gm2, Tq* __restrict__ q) {
  for (long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x; id < g.N;
       id += (long long)gridDim.x * blockDim.x) {
  const int i = (int)(id % g.nx);
  const int j = (int)((id / g.nx) % g.ny);
  const int k = (int)(id / g.plane);
  const double x = i * hx, y = j * hy, z = k * hz;
  const double sx = sin(x), cx = cos(x), sy = sin(y), cy = cos(y), cz = cos(z);
  const double u = sx * cy * cz;
  const double v = -cx * sy * cz;
  const double p = 1.0 / gm2 + (1.0 / 16.0) * (cos(2 * x) + cos(2 * y)) * (2.0 + cos(2 * z));
  const double rho = gm2 * p;
  q[id] = store_as<Tq>(rho);
  q[g.N + id] = store_as<Tq>(rho * u);
  q[2 * g.N + id] = store_as<Tq>(rho * v);
  q[3 * g.N + id] = store_as<Tq>(0.0);
  q[4 * g.N + id] = store_as<Tq>(p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v));
  }
}

template <class T>
__global__ void __launch_bounds__(256) tgv_primitive_kernel(Grid g, double hx, double hy, double hz, double gm2,
                                                            T* __restrict__ u, T* __restrict__ rho,
                                                            T* __restrict__ pr) {
  for (long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x; id < g.N;
       id += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(id % g.nx);
    const int j = (int)((id / g.nx) % g.ny);
    const int k = (int)(id / g.plane);
    const double x = i * hx, y = j * hy, z = k * hz;
    const double sx = sin(x), cx = cos(x), sy = sin(y), cy = cos(y), cz = cos(z);
    const double p = 1.0 / gm2 + (1.0 / 16.0) * (cos(2 * x) + cos(2 * y)) * (2.0 + cos(2 * z));
    u[id] = store_as<T>(sx * cy * cz);
    u[g.N + id] = store_as<T>(-cx * sy * cz);
    u[2 * g.N + id] = store_as<T>(0.0);
    rho[id] = store_as<T>(gm2 * p);
    pr[id] = store_as<T>(p);
  }
}

// Q = (rho, rho u, p / (gamma - 1) + (rho / 2) |u|^2), arithmetic in T.
template <class T>
__global__ void __launch_bounds__(256) state_from_velocity_kernel(long long N, T igm1, const T* __restrict__ u,
                                                                  const T* __restrict__ rho,
                                                                  const T* __restrict__ pr, T* __restrict__ q) {
  for (long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x; id < N;
       id += (long long)gridDim.x * blockDim.x) {
    const T r = rho[id], u0 = u[id], u1 = u[N + id], u2 = u[2 * N + id];
    const T uu = (u0 * u0 + u1 * u1) + u2 * u2;
    q[id] = r;
    q[N + id] = r * u0;
    q[2 * N + id] = r * u1;
    q[3 * N + id] = r * u2;
    q[4 * N + id] = pr[id] * igm1 + (T(0.5) * r) * uu;
  }
}

// Reverse of the map above at fixed rho and p: u_bar_a = rho (q_bar_{m_a} + u_a q_bar_E).
template <class T>
__global__ void __launch_bounds__(256) state_from_velocity_adj_kernel(long long N, const T* __restrict__ u,
                                                                      const T* __restrict__ rho,
                                                                      const T* __restrict__ qbar,
                                                                      T* __restrict__ ubar) {
  for (long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x; id < N;
       id += (long long)gridDim.x * blockDim.x) {
    const T r = rho[id], eb = qbar[4 * N + id];
#pragma unroll
    for (int a = 0; a < 3; ++a) ubar[a * N + id] = r * (qbar[(a + 1) * N + id] + u[a * N + id] * eb);
  }
}

// J = dt sum_n w_n h[n * stride + col], w_0 = w_{rows-1} = 1/2, else 1: one
// block, a fixed order (strided per-thread sums, then a shuffle tree).
__global__ void __launch_bounds__(256) trapezoid_kernel(const double* __restrict__ h, long long rows, int stride,
                                                        int col, double dt, double* __restrict__ out) {
  __shared__ double part[4];
  double acc = 0.0;
  for (long long n = threadIdx.x; n < rows; n += blockDim.x) {
    const double w = (n == 0 || n == rows - 1) ? 0.5 : 1.0;
    acc += w * h[n * stride + col];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = dt * ((part[0] + part[1]) + (part[2] + part[3]));
}

}  // namespace

template <class T>
hipError_t launch_init_primitive(const Grid& g, const double L[3], double gamma, double mach, void* u, void* rho,
                                 void* p, hipStream_t st) {
  (void)gamma;
  hipLaunchKernelGGL((tgv_primitive_kernel<T>), dim3(blocks_1d(g.N, 256)), dim3(256), 0, st, g, L[0] / g.nx,
                     L[1] / g.ny, L[2] / g.nz, gamma * mach * mach, static_cast<T*>(u), static_cast<T*>(rho),
                     static_cast<T*>(p));
  return hipGetLastError();
}

template <class T>
hipError_t launch_state_from_velocity(const Grid& g, double gamma, const void* u, const void* rho, const void* p,
                                      void* q, hipStream_t st) {
  hipLaunchKernelGGL((state_from_velocity_kernel<T>), dim3(blocks_1d(g.N, 256)), dim3(256), 0, st, g.N,
                     (T)(1.0 / (gamma - 1.0)), static_cast<const T*>(u), static_cast<const T*>(rho),
                     static_cast<const T*>(p), static_cast<T*>(q));
  return hipGetLastError();
}

template <class T>
hipError_t launch_state_from_velocity_adjoint(const Grid& g, const void* u, const void* rho, const void* qbar,
                                              void* ubar, hipStream_t st) {
  hipLaunchKernelGGL((state_from_velocity_adj_kernel<T>), dim3(blocks_1d(g.N, 256)), dim3(256), 0, st, g.N,
                     static_cast<const T*>(u), static_cast<const T*>(rho), static_cast<const T*>(qbar),
                     static_cast<T*>(ubar));
  return hipGetLastError();
}

hipError_t launch_trapezoid(const double* h, long long rows, int stride, int col, double dt, double* out,
                            hipStream_t st) {
  hipLaunchKernelGGL(trapezoid_kernel, dim3(1), dim3(256), 0, st, h, rows, stride, col, dt, out);
  return hipGetLastError();
}

template hipError_t launch_init_primitive<double>(const Grid&, const double*, double, double, void*, void*, void*,
                                                  hipStream_t);
template hipError_t launch_init_primitive<float>(const Grid&, const double*, double, double, void*, void*, void*,
                                                 hipStream_t);
template hipError_t launch_state_from_velocity<double>(const Grid&, double, const void*, const void*, const void*,
                                                       void*, hipStream_t);
template hipError_t launch_state_from_velocity<float>(const Grid&, double, const void*, const void*, const void*,
                                                      void*, hipStream_t);
template hipError_t launch_state_from_velocity_adjoint<double>(const Grid&, const void*, const void*, const void*,
                                                               void*, hipStream_t);
template hipError_t launch_state_from_velocity_adjoint<float>(const Grid&, const void*, const void*, const void*,
                                                              void*, hipStream_t);

template <class Tq>
hipError_t launch_init(const Grid& g, const double L[3], double gamma, double mach, void* q,
                       hipStream_t st) {
  const int threads = 256;
  hipLaunchKernelGGL((tgv_init_kernel<Tq>), dim3(blocks_1d(g.N, threads)), dim3(threads), 0, st, g, L[0] / g.nx,
                     L[1] / g.ny, L[2] / g.nz, gamma, gamma * mach * mach, static_cast<Tq*>(q));
  return hipGetLastError();
}

template hipError_t launch_init<double>(const Grid&, const double*, double, double, void*, hipStream_t);
template hipError_t launch_init<float>(const Grid&, const double*, double, double, void*, hipStream_t);
template hipError_t launch_init<f16>(const Grid&, const double*, double, double, void*, hipStream_t);
template hipError_t launch_init<bf16>(const Grid&, const double*, double, double, void*, hipStream_t);

}  // namespace tgv
