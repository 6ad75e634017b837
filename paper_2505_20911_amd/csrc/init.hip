// Taylor-Green initial state (paper Sec. 4.1 initial-condition equations and
// the isothermal density rho = gamma M^2 p), evaluated in FP64 per point and
// rounded once to the storage type of Q.
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

}  // namespace

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
