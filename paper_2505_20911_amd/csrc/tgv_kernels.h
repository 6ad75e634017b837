// Host-side launchers of the libtgv kernels (one translation unit per kernel
// family; the C-ABI layer in abi.hip validates arguments and dispatches here).
#pragma once

#include <hip/hip_runtime.h>

#include "tgv_device.h"

namespace tgv {

// Work-items of the largest dispatch each tiled kernel family makes on grid g
// (a dispatch must hold fewer than 2^32; the C-ABI refuses larger grids).
long long residual_work_items(const Grid& g);
long long integrals_work_items(const Grid& g);
long long adjoint_work_items(const Grid& g);

template <class Tq>
hipError_t launch_init(const Grid& g, const double L[3], double gamma, double mach, void* q,
                       hipStream_t st);

template <class T>
hipError_t launch_init_primitive(const Grid& g, const double L[3], double gamma, double mach, void* u, void* rho,
                                 void* p, hipStream_t st);

template <class T>
hipError_t launch_state_from_velocity(const Grid& g, double gamma, const void* u, const void* rho, const void* p,
                                      void* q, hipStream_t st);

template <class T>
hipError_t launch_state_from_velocity_adjoint(const Grid& g, const void* u, const void* rho, const void* qbar,
                                              void* ubar, hipStream_t st);

hipError_t launch_trapezoid(const double* h, long long rows, int stride, int col, double dt, double* out,
                            hipStream_t st);

template <class Tq, class Tr, class Tc>
hipError_t launch_residual(const Grid& g, const Coef<Tc>& c, int split, const void* q, void* r, hipStream_t st);

template <class Tq, class Tqt, class Tr, class Tc, class Ta>
hipError_t launch_residual_rk(const Grid& g, const Coef<Tc>& c, int split, int stage, double dt, const void* q_in,
                              void* q_out, void* qt, hipStream_t st);

template <class Tq, class Tqt, class Tr, class Ta>
hipError_t launch_rk_stage(const Grid& g, int stage, double dt, void* q, void* qt, const void* r,
                           hipStream_t st);

// Number of first-pass blocks of the integrals reduction (workspace holds
// 8 doubles per block).
long long integrals_blocks(const Grid& g);

template <class Tq>
hipError_t launch_integrals(const Grid& g, const Coef<double>& c, const void* q, double* work,
                            double* out8, hipStream_t st);

// The same two passes with the partial sums in the library's static device
// scratch instead of a caller workspace; grids of more than kNoAllocRows
// first-pass blocks do not fit it.
constexpr long long kNoAllocRows = 1LL << 16;

template <class Tq>
hipError_t launch_integrals_noalloc(const Grid& g, const Coef<double>& c, const void* q, double* out8,
                                    hipStream_t st);

// Fields of N values the residual adjoint's workspace holds.
constexpr int kResidualAdjointWorkFields = 15;

template <class T>
hipError_t launch_residual_adjoint(const Grid& g, const Coef<T>& c, const void* q, const void* rbar,
                                   void* qbar, void* work, hipStream_t st);

template <class T>
hipError_t launch_rk_stage_adjoint(const Grid& g, int stage, double dt, const void* qbar, void* zeta,
                                   void* rbar, hipStream_t st);

template <class T>
hipError_t launch_integrals_adjoint(const Grid& g, const Coef<T>& c, const void* q, double eps_bar,
                                    void* qbar, void* work, hipStream_t st);

}  // namespace tgv
