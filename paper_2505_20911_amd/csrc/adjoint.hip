// Discrete adjoint of the residual, of the RK stage and of eps^S.
//
// For the residual R(Q) the adjoint Q_bar += (dR/dQ)^T R_bar is written in
// gather form.  With D the antisymmetric 4th-order first difference,
// D^T = -D, D2^T = D2 and (D_a D_b)^T = D_a D_b on the periodic grid, every
// stencil term of the forward residual turns into a stencil of R_bar-weighted
// pointwise fields evaluated around the output point, plus pointwise terms.
// Passes, each a z-march over LDS-staged planes, in this order:
//   for the viscous residual, pass A stores in a caller-provided workspace
//     the adjoint of the viscous work sum tau_ad G_ad, the symmetric
//     G_bar_ad = 2 R_bar_E tau_ad (6 components), and the inner derivatives
//     of the mixed second-derivative terms, sigma_a = sum_{b != a} D_b u_b
//     and tau_b = sum_{a != b} D_a V_bar_a, so that D_a D_b u_b and
//     (D_a D_b)^T V_bar_a = D_b D_a V_bar_a become one more first difference
//     each in pass C (D_a and D_b commute on the periodic grid);
//   pass C gathers those workspace terms into u_bar_a and stores it in 3
//     more workspace fields;
//   pass B gathers every transposed-stencil and pointwise contribution that
//     needs only Q and R_bar, re-deriving u_a, V_bar_a = R_bar_{m_a} +
//     R_bar_E u_a and sum_f R_bar_f Q_f at each neighbour, adds pass C's
//     u_bar_a, and chains the sum through the primitive variables into q_bar
//     (the only pass that reads and writes q_bar).
// 1/rho is the hardware reciprocal refined by Newton-Raphson, as in the
// forward residual.
#include "tgv_device.h"
#include "tgv_kernels.h"

namespace tgv {

namespace {

// Threads per block of the element-wise reversed RK stage.
constexpr int kThreads = 256;

// Index of the symmetric pair (a, d) in the 6-component storage.
__device__ __forceinline__ int sym(int a, int d) {
  if (a == d) return a;
  const int lo = a < d ? a : d, hi = a < d ? d : a;
  return lo == 0 ? (hi == 1 ? 3 : 4) : 5;
}

// Workspace layout (viscous residual only), fields of N values each: the
// symmetric G_bar_ad = 2 R_bar_E tau_ad and the inner first differences
// sigma_a = sum_{b != a} D_b u_b and tau_b = sum_{a != b} D_a V_bar_a of the
// mixed second-derivative terms (pass A), and the workspace terms' u_bar_a
// (pass C).
enum { W_GB = 0, W_SIG = 6, W_TAU = 9, W_UB = 12, W_FIELDS = 15 };
static_assert(W_FIELDS == kResidualAdjointWorkFields, "workspace size");

// ---------------------------------------------------------------------------
// Plane march.  A block owns a GTX x GTY tile of (x, y) columns and marches
// along z over a chunk of planes.  Each plane of the operator's fields on the
// tile plus a 2-point halo is staged in LDS, which keeps the three newest
// planes: the x- and y-neighbours of the output plane c come from its LDS
// copy, the z-neighbours c + 1, c + 2 from the own column of the next two LDS
// planes, and c - 1, c - 2 from registers (the own column's values, saved as
// the planes leave LDS).  Every value is loaded from global memory once per
// block (plus the halo), where gathering each stencil neighbour from global
// memory re-read it many times through the caches.  The next plane is
// requested before the current plane's arithmetic.  An operator supplies NL
// values loaded per point (load), the NF fields staged from them (derive), the
// values of the output point it reads from global memory (early: requested
// before the next plane, so their latency overlaps the arithmetic rather than
// being waited for at the end of the step), and the output of one point
// (emit).
// ---------------------------------------------------------------------------
constexpr int GTX = 32, GTY = 8, GNT = GTX * GTY;
constexpr int GHX = GTX + 4, GHY = GTY + 4, GNP = GHX * GHY;
constexpr int GSLOTS = 3;  // LDS planes c, c + 1, c + 2
constexpr int GLOADS = (GNP + GNT - 1) / GNT;

struct PlaneMarch {
  int tiles_x, tiles_y, kz;
  long long blocks;
};

// Planes per block: long marches amortise the 4 halo planes at the ends of a
// chunk; the grid keeps at least 1024 blocks where it can.
PlaneMarch plane_march(const Grid& g) {
  PlaneMarch m;
  m.tiles_x = (g.nx + GTX - 1) / GTX;
  m.tiles_y = (g.ny + GTY - 1) / GTY;
  m.kz = 128;
  while (m.kz > 4 && (long long)m.tiles_x * m.tiles_y * ((g.nz + m.kz - 1) / m.kz) < 1024) m.kz /= 2;
  m.blocks = (long long)m.tiles_x * m.tiles_y * ((g.nz + m.kz - 1) / m.kz);
  return m;
}

// Neighbour accessors handed to an operator's emit: field f at offset index
// s (0..3 = -2, -1, +1, +2 points) along x and y from the LDS plane of the
// output plane, along z from the registers and the next two LDS planes.
template <class T, int NF>
struct Nbrs {
  const T* Pc;
  const T* P1;
  const T* P2;
  const T* wm1;
  const T* wm2;
  int own;
  __device__ __forceinline__ T c(int f) const { return Pc[f * GNP + own]; }
  template <int d>
  __device__ __forceinline__ T at(int f, int s) const {
    if constexpr (d == 2) {
      return s == 0 ? wm2[f] : s == 1 ? wm1[f] : s == 2 ? P1[f * GNP + own] : P2[f * GNP + own];
    } else {
      constexpr int st = d == 0 ? 1 : GHX;
      const int o = (s < 2) ? (s - 2) : (s - 1);
      return Pc[f * GNP + own + o * st];
    }
  }
};

// The tile origin and first plane of this block: hardware block b runs on
// XCD b % 8, and with remap each XCD takes a contiguous range of tiles.
__device__ __forceinline__ void tile_origin(const PlaneMarch& pm, int remap, int& x0, int& y0, int& z0) {
  const int nblk = gridDim.x;
  int b = blockIdx.x;
  if (remap) b = (b % 8) * (nblk / 8) + b / 8;
  x0 = (b % pm.tiles_x) * GTX;
  y0 = ((b / pm.tiles_x) % pm.tiles_y) * GTY;
  z0 = (b / (pm.tiles_x * pm.tiles_y)) * pm.kz;
}

// Offset of plane z (z in [-nz, 2 nz), wrapped periodically).
__device__ __forceinline__ long long plane_off(const Grid& g, int z) {
  z += (z < 0) ? g.nz : 0;
  z -= (z >= g.nz) ? g.nz : 0;
  return (long long)z * g.plane;
}

// The halo-plane runs thread tid of a role stages (one point, or with PAIRS
// two x-points): each run's offset within a plane and LDS index of its first
// point.
template <bool PAIRS, int NSLOT>
__device__ __forceinline__ void halo_runs(const Grid& g, int x0, int y0, int tid, long long (&off)[NSLOT],
                                          int (&sl)[NSLOT]) {
  constexpr int RX = PAIRS ? GHX / 2 : GHX;
#pragma unroll
  for (int l = 0; l < NSLOT; ++l) {
    const int s = tid + l * GNT;
    const int hy = s / RX, hx = (s % RX) * (PAIRS ? 2 : 1);
    int x = (x0 - 2 + hx) % g.nx;
    x += (x < 0) ? g.nx : 0;
    int y = (y0 - 2 + hy) % g.ny;
    y += (y < 0) ? g.ny : 0;
    off[l] = (long long)y * g.nx + x;
    sl[l] = hy * GHX + hx;
  }
}

// The NL values of one point, field f read from op.src(f) at offset i.
template <class T, class Op>
__device__ __forceinline__ void load_point(const Op& op, long long i, T (&v)[Op::NL]) {
#pragma unroll
  for (int f = 0; f < Op::NL; ++f) v[f] = op.src(f)[i];
}

// PAIRS (nx even): the halo plane is loaded in aligned runs of two x-points,
// one 2-element vector load per field for 216 of the 256 threads, instead
// of two single loads (432 points); tile origins and the halo width are even,
// so a run never crosses the periodic wrap and the 16-byte alignment of the
// arrays carries over to every run.
template <class T, class Op, bool PAIRS>
__global__ void __launch_bounds__(GNT, Op::kWavesPerEU) plane_march_kernel(Grid g, PlaneMarch pm, int remap, Op op) {
  constexpr int NF = Op::NF, NL = Op::NL;
  typedef T T2 __attribute__((ext_vector_type(2)));
  constexpr int NSLOT = PAIRS ? 1 : GLOADS;  // load slots per thread
  constexpr int NRUN = PAIRS ? GNP / 2 : GNP;  // runs per plane
  static_assert(!PAIRS || (GHX % 2 == 0 && NRUN <= GNT), "one run per thread");
  __shared__ __align__(16) T lds[GSLOTS][NF * GNP];
  int x0, y0, z0;
  tile_origin(pm, remap, x0, y0, z0);
  const int z1 = min(z0 + pm.kz, g.nz);
  const int tid = threadIdx.x;
  const int lx = tid % GTX, ly = tid / GTX;
  const int cx = x0 + lx, cy = y0 + ly;
  const bool valid = cx < g.nx && cy < g.ny;
  const long long col_off = (long long)cy * g.nx + cx;
  const int own = (ly + 2) * GHX + (lx + 2);

  // the halo-plane runs this thread stages
  long long off[NSLOT];
  int sl[NSLOT];
  halo_runs<PAIRS>(g, x0, y0, tid, off, sl);
  auto zoff = [&](int z) { return plane_off(g, z); };
  T pre[NSLOT][PAIRS ? 2 : 1][NL];
  auto fetch = [&](int z) {
    const long long zo = zoff(z);
#pragma unroll
    for (int l = 0; l < NSLOT; ++l)
      if (tid + l * GNT < NRUN) {
        if constexpr (PAIRS) {
#pragma unroll
          for (int f = 0; f < NL; ++f) {
            const T2 v = *reinterpret_cast<const T2*>(op.src(f) + zo + off[l]);
            pre[l][0][f] = v.x;
            pre[l][PAIRS ? 1 : 0][f] = v.y;
          }
        } else {
          load_point<T>(op, zo + off[l], pre[l][0]);
        }
      }
  };
  auto stash = [&](int z) {
    T* P = lds[(z - z0 + 3) % GSLOTS];
#pragma unroll
    for (int l = 0; l < NSLOT; ++l) {
      if (tid + l * GNT < NRUN) {
        if constexpr (PAIRS) {
          T v0[NF], v1[NF];
          op.derive(pre[l][0], v0);
          op.derive(pre[l][PAIRS ? 1 : 0], v1);
#pragma unroll
          for (int f = 0; f < NF; ++f) *reinterpret_cast<T2*>(&P[f * GNP + sl[l]]) = T2{v0[f], v1[f]};
        } else {
          T v[NF];
          op.derive(pre[l][0], v);
#pragma unroll
          for (int f = 0; f < NF; ++f) P[f * GNP + sl[l]] = v[f];
        }
      }
    }
  };
  // own-column fields of planes c - 2 and c - 1
  T wm2[NF], wm1[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) wm2[f] = wm1[f] = T(0);
  if (valid) {
    T raw[NL];
    load_point<T>(op, zoff(z0 - 2) + col_off, raw);
    op.derive(raw, wm2);
    load_point<T>(op, zoff(z0 - 1) + col_off, raw);
    op.derive(raw, wm1);
  }
  // planes z0 and z0 + 1 into LDS, z0 + 2 requested
  fetch(z0);
  stash(z0);
  fetch(z0 + 1);
  stash(z0 + 1);
  fetch(z0 + 2);

#pragma nounroll
  for (int cz = z0; cz < z1; ++cz) {
    stash(cz + 2);
    __syncthreads();
    const long long id = zoff(cz) + col_off;
    typename Op::Early early;
    if (valid) op.early(id, early);
    if (cz + 3 <= z1 + 1) fetch(cz + 3);
    const T* Pc = lds[(cz - z0 + 3) % GSLOTS];
    if (valid) {
      const Nbrs<T, NF> nbr{Pc, lds[(cz + 1 - z0 + 3) % GSLOTS], lds[(cz + 2 - z0 + 3) % GSLOTS], wm1, wm2, own};
      op.emit(nbr, id, early);
    }
    // the own column of plane c moves to the registers before its slot is
    // overwritten by plane c + 3
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      wm2[f] = wm1[f];
      wm1[f] = Pc[f * GNP + own];
    }
    __syncthreads();
  }
}

template <class T, class Op>
hipError_t launch_march(const Grid& g, const Op& op, hipStream_t st) {
  const PlaneMarch pm = plane_march(g);
  const int remap = pm.blocks % 8 == 0 ? 1 : 0;
  const dim3 grid((unsigned)pm.blocks), block(GNT);
  if (g.nx % 2 == 0)
    hipLaunchKernelGGL((plane_march_kernel<T, Op, true>), grid, block, 0, st, g, pm, remap, op);
  else
    hipLaunchKernelGGL((plane_march_kernel<T, Op, false>), grid, block, 0, st, g, pm, remap, op);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Plane march for operators that difference only a few of their fields along
// z and take no pointwise derivation while staging (the loaded values are the
// staged ones).  LDS holds only the NP fields differenced along x or y, on the
// tile plus halo, double-buffered (planes c and c + 1, one barrier per plane);
// the NZ fields differenced along z come from a register window over the own
// column (planes c - 2 .. c + 2), each loaded by its own thread three planes
// ahead.  Against the three-plane ring this halves the LDS per block for the
// same number of loads per point.
// ---------------------------------------------------------------------------
template <class T, int NP, int NZ>
struct NbrsZ {
  const T* Pc;
  const T (*zw)[NZ];
  int own;
  // plane field f at the output point
  __device__ __forceinline__ T c(int f) const { return Pc[f * GNP + own]; }
  // plane field f at offset index s (0..3 = -2, -1, +1, +2) along x (d = 0) or y
  template <int d>
  __device__ __forceinline__ T at(int f, int s) const {
    static_assert(d < 2, "plane fields are differenced along x and y");
    constexpr int st = d == 0 ? 1 : GHX;
    const int o = (s < 2) ? (s - 2) : (s - 1);
    return Pc[f * GNP + own + o * st];
  }
  // z-field k at offset index s along z
  __device__ __forceinline__ T atz(int k, int s) const { return zw[s < 2 ? s : s + 1][k]; }
};

template <class T, class Op, bool PAIRS>
__global__ void __launch_bounds__(GNT, Op::kWavesPerEU) plane_march_z_kernel(Grid g, PlaneMarch pm, int remap,
                                                                             Op op) {
  constexpr int NP = Op::NP, NZ = Op::NZ;
  typedef T T2 __attribute__((ext_vector_type(2)));
  constexpr int NSLOT = PAIRS ? 1 : GLOADS;
  constexpr int NRUN = PAIRS ? GNP / 2 : GNP;
  static_assert(!PAIRS || (GHX % 2 == 0 && NRUN <= GNT), "one run per thread");
  __shared__ __align__(16) T lds[2][NP * GNP];
  int x0, y0, z0;
  tile_origin(pm, remap, x0, y0, z0);
  const int z1 = min(z0 + pm.kz, g.nz);
  const int tid = threadIdx.x;
  const int lx = tid % GTX, ly = tid / GTX;
  const int cx = x0 + lx, cy = y0 + ly;
  const bool valid = cx < g.nx && cy < g.ny;
  const long long col_off = (long long)cy * g.nx + cx;
  const int own = (ly + 2) * GHX + (lx + 2);

  long long off[NSLOT];
  int sl[NSLOT];
  halo_runs<PAIRS>(g, x0, y0, tid, off, sl);
  auto zoff = [&](int z) { return plane_off(g, z); };
  T pre[NSLOT][PAIRS ? 2 : 1][NP];
  auto fetch = [&](int z) {
    const long long zo = zoff(z);
#pragma unroll
    for (int l = 0; l < NSLOT; ++l)
      if (tid + l * GNT < NRUN) {
#pragma unroll
        for (int f = 0; f < NP; ++f) {
          if constexpr (PAIRS) {
            const T2 v = *reinterpret_cast<const T2*>(op.psrc(f) + zo + off[l]);
            pre[l][0][f] = v.x;
            pre[l][PAIRS ? 1 : 0][f] = v.y;
          } else {
            pre[l][0][f] = op.psrc(f)[zo + off[l]];
          }
        }
      }
  };
  auto stash = [&](int z) {
    T* P = lds[(z - z0) & 1];
#pragma unroll
    for (int l = 0; l < NSLOT; ++l)
      if (tid + l * GNT < NRUN) {
#pragma unroll
        for (int f = 0; f < NP; ++f) {
          if constexpr (PAIRS)
            *reinterpret_cast<T2*>(&P[f * GNP + sl[l]]) = T2{pre[l][0][f], pre[l][PAIRS ? 1 : 0][f]};
          else
            P[f * GNP + sl[l]] = pre[l][0][f];
        }
      }
  };
  auto zload = [&](int z, T (&v)[NZ]) {
    const long long i = zoff(z) + col_off;
#pragma unroll
    for (int k = 0; k < NZ; ++k) v[k] = valid ? op.zsrc(k)[i] : T(0);
  };
  // zw[0..4]: the own column's z-fields of planes c - 2 .. c + 2; zn: plane
  // c + 3, requested one plane before it enters the window
  T zw[5][NZ], zn[NZ];
  zload(z0 - 2, zw[1]);
  zload(z0 - 1, zw[2]);
  zload(z0, zw[3]);
  zload(z0 + 1, zw[4]);
  zload(z0 + 2, zn);
  fetch(z0);

#pragma nounroll
  for (int cz = z0; cz < z1; ++cz) {
    stash(cz);
#pragma unroll
    for (int k = 0; k < NZ; ++k) {
#pragma unroll
      for (int s = 0; s < 4; ++s) zw[s][k] = zw[s + 1][k];
      zw[4][k] = zn[k];
    }
    __syncthreads();
    const long long id = zoff(cz) + col_off;
    typename Op::Early early;
    if (valid) op.early(id, early);
    if (cz + 1 < z1) {
      fetch(cz + 1);
      zload(cz + 3, zn);
    }
    if (valid) {
      const NbrsZ<T, NP, NZ> nbr{lds[(cz - z0) & 1], zw, own};
      op.emit(nbr, id, early);
    }
  }
}

template <class T, class Op>
hipError_t launch_march_z(const Grid& g, const Op& op, hipStream_t st) {
  const PlaneMarch pm = plane_march(g);
  const int remap = pm.blocks % 8 == 0 ? 1 : 0;
  const dim3 grid((unsigned)pm.blocks), block(GNT);
  if (g.nx % 2 == 0)
    hipLaunchKernelGGL((plane_march_z_kernel<T, Op, true>), grid, block, 0, st, g, pm, remap, op);
  else
    hipLaunchKernelGGL((plane_march_z_kernel<T, Op, false>), grid, block, 0, st, g, pm, remap, op);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Plane march with two thread roles per column, for an operator too large in
// registers for two waves of one role per SIMD: a block of 2 x 256 threads
// (one wave of each role per SIMD, at most 256 registers each).  Role 0
// evaluates the x and y terms of the output point and completes it; role 1
// stages the planes, keeps the own column's z-window and evaluates the z
// terms, whose NA partial sums it hands over through LDS.  Two barriers per
// plane: after the staging, and after the hand-over.  In FP32 (73 KB of LDS)
// two blocks share a CU, four waves per SIMD at 128 registers (a few values
// spilled): 10.2 against 11.0 ms for the FP32 residual adjoint at 512^3.
// ---------------------------------------------------------------------------
template <class T, class Op, bool PAIRS>
__global__ void __launch_bounds__(2 * GNT, sizeof(T) == 4 ? 4 : 2) plane_march_split_kernel(Grid g, PlaneMarch pm, int remap, Op op) {
  constexpr int NF = Op::NF, NL = Op::NL, NA = Op::NA;
  typedef T T2 __attribute__((ext_vector_type(2)));
  constexpr int NSLOT = PAIRS ? 1 : GLOADS;
  constexpr int NRUN = PAIRS ? GNP / 2 : GNP;
  static_assert(!PAIRS || (GHX % 2 == 0 && NRUN <= GNT), "one run per thread");
  __shared__ __align__(16) T lds[GSLOTS][NF * GNP];
  __shared__ T xch[NA][GNT];
  int x0, y0, z0;
  tile_origin(pm, remap, x0, y0, z0);
  const int z1 = min(z0 + pm.kz, g.nz);
  const int tid = threadIdx.x % GNT;
  const bool stager = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / GNT)) == 1;  // role 1
  const int lx = tid % GTX, ly = tid / GTX;
  const int cx = x0 + lx, cy = y0 + ly;
  const bool valid = cx < g.nx && cy < g.ny;
  const long long col_off = (long long)cy * g.nx + cx;
  const int own = (ly + 2) * GHX + (lx + 2);

  long long off[NSLOT];
  int sl[NSLOT];
  halo_runs<PAIRS>(g, x0, y0, tid, off, sl);
  auto zoff = [&](int z) { return plane_off(g, z); };
  T pre[NSLOT][PAIRS ? 2 : 1][NL];
  auto fetch = [&](int z) {
    const long long zo = zoff(z);
#pragma unroll
    for (int l = 0; l < NSLOT; ++l)
      if (tid + l * GNT < NRUN) {
        if constexpr (PAIRS) {
#pragma unroll
          for (int f = 0; f < NL; ++f) {
            const T2 v = *reinterpret_cast<const T2*>(op.src(f) + zo + off[l]);
            pre[l][0][f] = v.x;
            pre[l][PAIRS ? 1 : 0][f] = v.y;
          }
        } else {
          load_point<T>(op, zo + off[l], pre[l][0]);
        }
      }
  };
  auto stash = [&](int z) {
    T* P = lds[(z - z0 + 3) % GSLOTS];
#pragma unroll
    for (int l = 0; l < NSLOT; ++l) {
      if (tid + l * GNT < NRUN) {
        if constexpr (PAIRS) {
          T v0[NF], v1[NF];
          op.derive(pre[l][0], v0);
          op.derive(pre[l][PAIRS ? 1 : 0], v1);
#pragma unroll
          for (int f = 0; f < NF; ++f) *reinterpret_cast<T2*>(&P[f * GNP + sl[l]]) = T2{v0[f], v1[f]};
        } else {
          T v[NF];
          op.derive(pre[l][0], v);
#pragma unroll
          for (int f = 0; f < NF; ++f) P[f * GNP + sl[l]] = v[f];
        }
      }
    }
  };
  // Each role runs a loop of its own (the role is wave-uniform and held in a
  // scalar register, so every wave takes one branch), with two barriers per
  // plane in both: the registers one role carries from plane to plane are then
  // not held through the other's code.
  if (stager) {
    T wm2[NF], wm1[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) wm2[f] = wm1[f] = T(0);
    if (valid) {
      T raw[NL];
      load_point<T>(op, zoff(z0 - 2) + col_off, raw);
      op.derive(raw, wm2);
      load_point<T>(op, zoff(z0 - 1) + col_off, raw);
      op.derive(raw, wm1);
    }
    fetch(z0);
    stash(z0);
    fetch(z0 + 1);
    stash(z0 + 1);
    fetch(z0 + 2);
#pragma nounroll
    for (int cz = z0; cz < z1; ++cz) {
      stash(cz + 2);
      __syncthreads();
      const T* Pc = lds[(cz - z0 + 3) % GSLOTS];
      if (cz + 3 <= z1 + 1) fetch(cz + 3);
      if (valid) {
        const Nbrs<T, NF> nbr{Pc, lds[(cz + 1 - z0 + 3) % GSLOTS], lds[(cz + 2 - z0 + 3) % GSLOTS], wm1, wm2, own};
        T h[NA];
        op.along_z(nbr, h);
#pragma unroll
        for (int k = 0; k < NA; ++k) xch[k][tid] = h[k];
      }
      // the own column of plane c moves to the registers before its slot is
      // overwritten by plane c + 3
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        wm2[f] = wm1[f];
        wm1[f] = Pc[f * GNP + own];
      }
      __syncthreads();
    }
  } else {
#pragma nounroll
    for (int cz = z0; cz < z1; ++cz) {
      __syncthreads();
      const long long id = zoff(cz) + col_off;
      typename Op::Early early;
      typename Op::Acc acc;
      if (valid) {
        op.early(id, early);
        const Nbrs<T, NF> nbr{lds[(cz - z0 + 3) % GSLOTS], nullptr, nullptr, nullptr, nullptr, own};
        op.in_plane(nbr, acc);
      }
      __syncthreads();
      if (valid) {
        T h[NA];
#pragma unroll
        for (int k = 0; k < NA; ++k) h[k] = xch[k][tid];
        op.finish(acc, h, id, early);
      }
    }
  }
}

template <class T, class Op>
hipError_t launch_march_split(const Grid& g, const Op& op, hipStream_t st) {
  const PlaneMarch pm = plane_march(g);
  const int remap = pm.blocks % 8 == 0 ? 1 : 0;
  const dim3 grid((unsigned)pm.blocks), block(2 * GNT);
  if (g.nx % 2 == 0)
    hipLaunchKernelGGL((plane_march_split_kernel<T, Op, true>), grid, block, 0, st, g, pm, remap, op);
  else
    hipLaunchKernelGGL((plane_march_split_kernel<T, Op, false>), grid, block, 0, st, g, pm, remap, op);
  return hipGetLastError();
}

// Operators that read nothing at the output point.
struct NoEarly {
  struct Early {};
  __device__ __forceinline__ void early(long long, Early&) const {}
};

template <class T>
__device__ __forceinline__ T first_diff(T m2, T m1, T p1, T p2, T s) {
  return s * (T(8) * (p1 - m1) - (p2 - m2));
}

// ---------------------------------------------------------------------------
// Pass A (viscous only): G_bar_ad, sigma_a and tau_b at every point, from the
// velocity u_a = m_a / rho and V_bar_a = R_bar_{m_a} + R_bar_E u_a, derived
// once per point as it is staged.
// ---------------------------------------------------------------------------
template <class T>
struct StressOp : NoEarly {
  static constexpr int NL = 8, NF = 7, kWavesPerEU = 2;  // (rho, m, R_bar_m, R_bar_E) -> (u, V_bar, R_bar_E)
  Grid g;
  Coef<T> c;
  const T* __restrict__ q;
  const T* __restrict__ rb;
  T* __restrict__ w;
  __device__ __forceinline__ const T* src(int f) const { return f < 4 ? q + f * g.N : rb + (f - 3) * g.N; }
  __device__ __forceinline__ void derive(const T (&v)[NL], T (&o)[NF]) const {
    const T ir = recip(v[0]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const T u = v[a + 1] * ir;
      o[a] = u;
      o[3 + a] = v[4 + a] + v[7] * u;
    }
    o[6] = v[7];
  }
  template <int d>
  __device__ __forceinline__ T D(const Nbrs<T, NF>& n, int f) const {
    return first_diff(n.template at<d>(f, 0), n.template at<d>(f, 1), n.template at<d>(f, 2), n.template at<d>(f, 3),
                      c.c1[d]);
  }
  __device__ __forceinline__ void emit(const Nbrs<T, NF>& n, long long id, const Early&) const {
    const long long N = g.N;
    T G[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      G[a][0] = D<0>(n, a);
      G[a][1] = D<1>(n, a);
      G[a][2] = D<2>(n, a);
    }
    const T dv[3] = {D<0>(n, 3), D<1>(n, 4), D<2>(n, 5)};  // D_a V_bar_a
    stream_store(&w[(W_SIG + 0) * N + id], G[1][1] + G[2][2]);
    stream_store(&w[(W_SIG + 1) * N + id], G[0][0] + G[2][2]);
    stream_store(&w[(W_SIG + 2) * N + id], G[0][0] + G[1][1]);
    stream_store(&w[(W_TAU + 0) * N + id], dv[1] + dv[2]);
    stream_store(&w[(W_TAU + 1) * N + id], dv[0] + dv[2]);
    stream_store(&w[(W_TAU + 2) * N + id], dv[0] + dv[1]);
    const T div = G[0][0] + G[1][1] + G[2][2];
    const T two_rE = T(2) * n.c(6);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int d = a; d < 3; ++d) {
        const T tau = c.ire * (G[a][d] + G[d][a] - (a == d ? T(2.0 / 3.0) * div : T(0)));
        stream_store(&w[(W_GB + sym(a, d)) * N + id], two_rE * tau);
      }
  }
};

// ---------------------------------------------------------------------------
// Pass B: the transposed-stencil and pointwise contributions, everything
// except the viscous-work and mixed-derivative terms that read the workspace
// (pass C).  Along each direction the neighbours are visited in symmetric
// pairs, (-1, +1) and then (-2, +2).  At each neighbour u_a, V_bar_a and
// sum_f R_bar_f Q_f are derived from Q, R_bar and 1/rho, and every first and
// second difference is accumulated pair by pair,
//   8 (f_{+1} - f_{-1}) - (f_{+2} - f_{-2}),
//   16 ((f_{+1} - f_0) + (f_{-1} - f_0)) - ((f_{+2} - f_0) + (f_{-2} - f_0))
// (the factors 8 and 16 are exact), the neighbour differences always taken
// first.  It runs on the two-role march: the x and y directions in one
// thread, the z direction in another, whose sums join before the chain
// through the primitive variables (linear in them).
// ---------------------------------------------------------------------------
enum { G_Q = 0, G_R = 5, G_IR = 10 };

// Difference sums of one direction (before the 1/(12 h) or 1/(12 h^2) factor).
// `ubs` collects the terms that enter u_bar_d through a first difference:
// sum_f (-R_bar_f) D_d q_f + D_d (sum_f R_bar_f Q_f), each difference taken
// from the neighbour values first.
template <class T>
struct DirSums {
  T r[5], rud[5], ud, ubs, rE2, vb2[3], u2[3];
};

template <int K, class T>
__device__ __forceinline__ void d1_add(T& acc, T diff) {
  if (K == 1)
    acc = T(8) * diff;
  else
    acc = acc - diff;
}
template <int K, class T>
__device__ __forceinline__ void d2_add(T& acc, T plus, T minus, T c0) {
  const T sum = (plus - c0) + (minus - c0);
  if (K == 1)
    acc = T(16) * sum;
  else
    acc = acc - sum;
}

// Pair K of direction d: neighbours m at -K and p at +K, whose fields
// (q, R_bar, 1/rho in the G_* order) the accessors M(f) and P(f) read; u_a,
// V_bar_a = R_bar_{m_a} + R_bar_E u_a and sum_f R_bar_f Q_f are derived there.
// Values are read field by field, so that few are live at once.
template <int K, int d, class T, class FM, class FP>
__device__ __forceinline__ void add_pair(DirSums<T>& S, FM M, FP P, bool viscous, const T (&r0)[5],
                                         const T (&vb0)[3], const T (&u0)[3]) {
  const T irm = M(G_IR), irp = P(G_IR);
  T um[3], up[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    um[a] = M(G_Q + 1 + a) * irm;
    up[a] = P(G_Q + 1 + a) * irp;
  }
  const T udm = um[d], udp = up[d];
  T srqm = 0, srqp = 0;
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    const T rm = M(G_R + f), rp = P(G_R + f);
    srqm += rm * M(G_Q + f);
    srqp += rp * P(G_Q + f);
    d1_add<K>(S.r[f], rp - rm);
    const T pu = rp * udp;
    const T mu = rm * udm;
    d1_add<K>(S.rud[f], pu - mu);
  }
  T ubs = srqp - srqm;
#pragma unroll
  for (int f = 0; f < 5; ++f) ubs -= r0[f] * (P(G_Q + f) - M(G_Q + f));
  d1_add<K>(S.ud, udp - udm);
  d1_add<K>(S.ubs, ubs);
  if (viscous) {
    const T r4m = M(G_R + 4), r4p = P(G_R + 4);
    d2_add<K>(S.rE2, r4p, r4m, r0[4]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      d2_add<K>(S.vb2[a], P(G_R + 1 + a) + r4p * up[a], M(G_R + 1 + a) + r4m * um[a], vb0[a]);
      d2_add<K>(S.u2[a], up[a], um[a], u0[a]);
    }
  }
}

// Centre values of the output point and the accumulators of its adjoint.
template <class T>
struct Centre {
  T q0[5], r0[5], ir0, u0[3], vb0[3], p0, T0;
  T qb[5], ub[3], pb, Tb, lap[3], X[3];
};

// Direction d's contributions from its difference sums (terms numbered as
// in the forward residual: (1)-(3) split convection, (4) pressure gradient,
// (5) pressure work, (6) viscous momentum D2 parts, (8) heat flux).
template <int d, class T>
__device__ __forceinline__ void direction_adjoint(const DirSums<T>& S, bool viscous, const Coef<T>& c,
                                                  Centre<T>& C) {
  const T half = T(0.5);
  const T u0d = C.u0[d];
  const T s1 = c.c1[d], s2 = c.c2[d];
  T ubd = 0, Xd = 0;  // contributions to ub[d], X[d]
  const T dud = s1 * S.ud;  // forward D_d u_d at this point
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    const T Dr = s1 * S.r[f];
    // (1) flux term D_d(q_f u_d): F = 1/2 D_d(R_bar_f)
    const T F = half * Dr;
    C.qb[f] += F * u0d;
    ubd += F * C.q0[f];
    // (2) u_d D_d q_f
    C.qb[f] += half * (s1 * S.rud[f]);
    // (3) q_f D_d u_d, pointwise part
    C.qb[f] -= half * C.r0[f] * dud;
    // (4) momentum pressure gradient D_d p
    if (f == d + 1) C.pb += Dr;
    if (f == 4) {
      // (5) pressure work D_d(p u_d)
      C.pb += Dr * u0d;
      ubd += Dr * C.p0;
      // (8) heat flux
      if (viscous) C.Tb += c.kap * (s2 * S.rE2);
    }
  }
  // (2) -R_bar_f D_d q_f and (3) q_f D_d u_d, stencil part summed over f
  ubd += half * (s1 * S.ubs);
  if (viscous) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      // (6) viscous momentum, D2 parts, on V_bar_a = R_bar_{m_a} + R_bar_E u_a
      const T vb = s2 * S.vb2[a];
      C.ub[a] += c.ire * vb;
      if (a == d) ubd += c.ire * (T(1.0 / 3.0)) * vb;
      // forward pieces of V_{m_a} at this point
      const T l = s2 * S.u2[a];
      C.lap[a] += l;
      if (a == d) Xd += l;
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    C.ub[a] += a == d ? ubd : T(0);
    C.X[a] += a == d ? Xd : T(0);
  }
}

template <class T>
struct GatherOp {
  static constexpr int NL = 10, NF = 11;  // (q, R_bar) -> (q, R_bar, 1/rho)
  Grid g;
  Coef<T> c;
  const T* __restrict__ q;
  const T* __restrict__ rb;
  T* __restrict__ qbar;
  const T* __restrict__ ubv;  // pass C's u_bar (3 fields), viscous only
  __device__ __forceinline__ const T* src(int f) const { return f < G_R ? q + f * g.N : rb + (f - G_R) * g.N; }
  __device__ __forceinline__ void derive(const T (&v)[NL], T (&o)[NF]) const {
#pragma unroll
    for (int f = 0; f < NL; ++f) o[f] = v[f];
    o[G_IR] = recip(v[G_Q]);
  }
  template <int d>
  __device__ __forceinline__ void direction(const Nbrs<T, NF>& n, bool viscous, Centre<T>& C) const {
    DirSums<T> S;
    add_pair<1, d>(S, [&](int f) { return n.template at<d>(f, 1); }, [&](int f) { return n.template at<d>(f, 2); },
                   viscous, C.r0, C.vb0, C.u0);
    add_pair<2, d>(S, [&](int f) { return n.template at<d>(f, 0); }, [&](int f) { return n.template at<d>(f, 3); },
                   viscous, C.r0, C.vb0, C.u0);
    direction_adjoint<d>(S, viscous, c, C);
  }
  struct Early {
    T qb[5], ub[3];
  };
  __device__ __forceinline__ void early(long long id, Early& e) const {
#pragma unroll
    for (int f = 0; f < 5; ++f) e.qb[f] = qbar[f * g.N + id];
#pragma unroll
    for (int a = 0; a < 3; ++a) e.ub[a] = ubv ? ubv[a * g.N + id] : T(0);
  }
  // centre values of the output point, accumulators cleared
  __device__ __forceinline__ void centre(const Nbrs<T, NF>& n, Centre<T>& C) const {
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      C.q0[f] = n.c(G_Q + f);
      C.r0[f] = n.c(G_R + f);
      C.qb[f] = 0;
    }
    C.ir0 = n.c(G_IR);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      C.u0[a] = C.q0[a + 1] * C.ir0;
      C.vb0[a] = C.r0[a + 1] + C.r0[4] * C.u0[a];
      C.ub[a] = 0;
      C.lap[a] = 0;
      C.X[a] = 0;
    }
    C.p0 = c.gm1 * (C.q0[4] - T(0.5) * (C.q0[1] * C.u0[0] + C.q0[2] * C.u0[1] + C.q0[3] * C.u0[2]));
    C.T0 = c.gm2 * C.p0 * C.ir0;
    C.pb = 0;
    C.Tb = 0;
  }
  // Accumulators handed from the z role to the in-plane role: q_bar 5, u_bar
  // 3, p_bar, T_bar, the Laplacian pieces 3 and X 3; every direction adds to
  // them, and the chain through the primitive variables is linear in them.
  static constexpr int NA = 16;
  using Acc = Centre<T>;
  __device__ __forceinline__ void in_plane(const Nbrs<T, NF>& n, Centre<T>& C) const {
    const bool viscous = c.viscous != 0;
    centre(n, C);
    direction<0>(n, viscous, C);
    direction<1>(n, viscous, C);
  }
  __device__ __forceinline__ void along_z(const Nbrs<T, NF>& n, T (&h)[NA]) const {
    const bool viscous = c.viscous != 0;
    Centre<T> C;
    centre(n, C);
    direction<2>(n, viscous, C);
#pragma unroll
    for (int f = 0; f < 5; ++f) h[f] = C.qb[f];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      h[5 + a] = C.ub[a];
      h[10 + a] = C.lap[a];
      h[13 + a] = C.X[a];
    }
    h[8] = C.pb;
    h[9] = C.Tb;
  }
  __device__ __forceinline__ void finish(Centre<T>& C, const T (&h)[NA], long long id, const Early& e) const {
    const bool viscous = c.viscous != 0;
#pragma unroll
    for (int f = 0; f < 5; ++f) C.qb[f] += h[f];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      C.ub[a] += h[5 + a];
      C.lap[a] += h[10 + a];
      C.X[a] += h[13 + a];
    }
    C.pb += h[8];
    C.Tb += h[9];
    const T half = T(0.5);
    if (viscous) {
      // pointwise part of sum_a u_a V_{m_a}: the Laplacian and the D2_a u_a
      // part of X_a (its mixed-derivative part comes from pass C)
#pragma unroll
      for (int a = 0; a < 3; ++a) C.ub[a] += C.r0[4] * (c.ire * (C.lap[a] + C.X[a] * T(1.0 / 3.0)));
    }
    // Chain through the primitive variables at this point.
    C.pb += c.gm2 * C.Tb * C.ir0;
    C.qb[0] -= C.T0 * C.Tb * C.ir0;
    C.qb[4] += c.gm1 * C.pb;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      C.qb[a + 1] -= half * c.gm1 * C.pb * C.u0[a];
      C.ub[a] -= half * c.gm1 * C.pb * C.q0[a + 1];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      C.ub[a] += e.ub[a];  // the workspace terms (pass C)
      C.qb[a + 1] += C.ub[a] * C.ir0;
      C.qb[0] -= C.ub[a] * C.u0[a] * C.ir0;
    }
#pragma unroll
    for (int f = 0; f < 5; ++f) stream_store(&qbar[f * g.N + id], e.qb[f] + C.qb[f]);
  }
};

// ---------------------------------------------------------------------------
// Pass C (viscous only): the workspace terms.  u_bar_a gets the viscous-work
// adjoint -sum_d D_d(G_bar_ad) and (1/(3 Re)) D_a tau_a, and the mixed part of
// the forward X_a = D_a sigma_a enters through R_bar_E (1/Re) X_a / 3; the
// result goes to the workspace fields W_UB, which pass B adds to its own u_bar
// before chaining through u = m / rho into q_bar.
// ---------------------------------------------------------------------------
template <class T>
struct ViscOp {
  // workspace fields differenced along x or y (plane fields) and along z
  // (z-fields): G_bar_ad with a or d = x, y; sigma_x, sigma_y, tau_x, tau_y;
  // and G_bar_az, sigma_z, tau_z
  static constexpr int NP = 9, NZ = 5, kWavesPerEU = 2;
  static constexpr int plane_field(int p) { return p < 2 ? W_GB + p : p < 7 ? p + 1 : p + 2; }
  static constexpr int z_field(int k) { return k == 0 ? W_GB + 2 : k < 3 ? W_GB + k + 3 : k == 3 ? W_SIG + 2 : W_TAU + 2; }
  static constexpr int plane_slot(int w) { return w < 2 ? w : w < 8 ? w - 1 : w - 2; }
  static constexpr int z_slot(int w) { return w == W_GB + 2 ? 0 : w < W_SIG ? w - 3 : w == W_SIG + 2 ? 3 : 4; }
  Grid g;
  Coef<T> c;
  const T* __restrict__ rb;
  const T* __restrict__ w;
  T* __restrict__ ubw;  // = w + W_UB N, disjoint from the fields read
  __device__ __forceinline__ const T* psrc(int p) const { return w + plane_field(p) * g.N; }
  __device__ __forceinline__ const T* zsrc(int k) const { return w + z_field(k) * g.N; }
  template <int d>
  __device__ __forceinline__ T D(const NbrsZ<T, NP, NZ>& n, int f) const {
    if constexpr (d == 2) {
      const int k = z_slot(f);
      return first_diff(n.atz(k, 0), n.atz(k, 1), n.atz(k, 2), n.atz(k, 3), c.c1[d]);
    } else {
      const int p = plane_slot(f);
      return first_diff(n.template at<d>(p, 0), n.template at<d>(p, 1), n.template at<d>(p, 2),
                        n.template at<d>(p, 3), c.c1[d]);
    }
  }
  template <int d>
  __device__ __forceinline__ void direction(const NbrsZ<T, NP, NZ>& n, T (&ub)[3], T (&X)[3]) const {
#pragma unroll
    for (int a = 0; a < 3; ++a) ub[a] -= D<d>(n, W_GB + sym(a, d));
    X[d] = D<d>(n, W_SIG + d);
    // (9) mixed second derivatives through the stored inner differences
    ub[d] += c.ire * T(1.0 / 3.0) * D<d>(n, W_TAU + d);
  }
  struct Early {
    T rE;
  };
  __device__ __forceinline__ void early(long long id, Early& e) const { e.rE = rb[4 * g.N + id]; }
  __device__ __forceinline__ void emit(const NbrsZ<T, NP, NZ>& n, long long id, const Early& e) const {
    T ub[3] = {0, 0, 0}, X[3];
    direction<0>(n, ub, X);
    direction<1>(n, ub, X);
    direction<2>(n, ub, X);
#pragma unroll
    for (int a = 0; a < 3; ++a) stream_store(&ubw[a * g.N + id], ub[a] + e.rE * (c.ire * (X[a] * T(1.0 / 3.0))));
  }
};

// Reversed RK stage: zeta += B q_bar ; r_bar = dt zeta ; zeta = A zeta.
template <class T>
__global__ void __launch_bounds__(kThreads) rk_adj(long long n5, T A, T B, T dt, const T* __restrict__ qbar,
                                                   T* __restrict__ zeta, T* __restrict__ rbar) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n5;
       i += (long long)gridDim.x * blockDim.x) {
    const T z = zeta[i] + B * qbar[i];
    rbar[i] = dt * z;
    zeta[i] = A * z;
  }
}

// eps^S adjoint pass A: omega_bar = eps_bar (1/(N Re)) 2 omega, with the
// velocity u_a = m_a / rho derived as each plane is staged.
template <class T>
struct VortOp : NoEarly {
  static constexpr int NL = 4, NF = 3, kWavesPerEU = 2;  // (rho, m) -> u
  Grid g;
  Coef<T> c;
  T scale;
  const T* __restrict__ q;
  T* __restrict__ wbar;
  __device__ __forceinline__ const T* src(int f) const { return q + f * g.N; }
  __device__ __forceinline__ void derive(const T (&v)[NL], T (&o)[NF]) const {
    const T ir = recip(v[0]);
#pragma unroll
    for (int a = 0; a < 3; ++a) o[a] = v[a + 1] * ir;
  }
  template <int d>
  __device__ __forceinline__ T D(const Nbrs<T, NF>& n, int f) const {
    return first_diff(n.template at<d>(f, 0), n.template at<d>(f, 1), n.template at<d>(f, 2), n.template at<d>(f, 3),
                      c.c1[d]);
  }
  __device__ __forceinline__ void emit(const Nbrs<T, NF>& n, long long id, const Early&) const {
    // G[a][d] = D_d u_a, only the off-diagonal ones enter the vorticity
    wbar[id] = scale * (D<1>(n, 2) - D<2>(n, 1));
    wbar[g.N + id] = scale * (D<2>(n, 0) - D<0>(n, 2));
    wbar[2 * g.N + id] = scale * (D<0>(n, 1) - D<1>(n, 0));
  }
};

// eps^S adjoint pass B: u_bar = curl_D(omega_bar) (D^T = -D turns the
// transposed curl back into a curl), then through u = m / rho into q_bar.
template <class T>
struct CurlOp {
  static constexpr int NL = 3, NF = 3, kWavesPerEU = 2;
  Grid g;
  Coef<T> c;
  const T* __restrict__ q;
  const T* __restrict__ wbar;
  T* __restrict__ qbar;
  __device__ __forceinline__ const T* src(int f) const { return wbar + f * g.N; }
  __device__ __forceinline__ void derive(const T (&v)[NL], T (&o)[NF]) const {
#pragma unroll
    for (int f = 0; f < NL; ++f) o[f] = v[f];
  }
  template <int d>
  __device__ __forceinline__ T D(const Nbrs<T, NF>& n, int f) const {
    return first_diff(n.template at<d>(f, 0), n.template at<d>(f, 1), n.template at<d>(f, 2), n.template at<d>(f, 3),
                      c.c1[d]);
  }
  struct Early {
    T q[4], qb[4];
  };
  __device__ __forceinline__ void early(long long id, Early& e) const {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      e.q[f] = q[f * g.N + id];
      e.qb[f] = qbar[f * g.N + id];
    }
  }
  __device__ __forceinline__ void emit(const Nbrs<T, NF>& n, long long id, const Early& e) const {
    const long long N = g.N;
    T ub[3];
    ub[0] = D<1>(n, 2) - D<2>(n, 1);
    ub[1] = D<2>(n, 0) - D<0>(n, 2);
    ub[2] = D<0>(n, 1) - D<1>(n, 0);
    const T ir = recip(e.q[0]);
    T rb = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      qbar[(a + 1) * N + id] = e.qb[a + 1] + ub[a] * ir;
      rb -= ub[a] * e.q[a + 1] * ir * ir;
    }
    qbar[id] = e.qb[0] + rb;
  }
};

inline unsigned blocks_for(long long n) { return blocks_1d(n, kThreads); }

}  // namespace

long long adjoint_work_items(const Grid& g) { return plane_march(g).blocks * GNT; }

template <class T>
hipError_t launch_residual_adjoint(const Grid& g, const Coef<T>& c, const void* q, const void* rbar, void* qbar,
                                   void* work, hipStream_t st) {
  const T* qq = static_cast<const T*>(q);
  const T* rr = static_cast<const T*>(rbar);
  T* w = static_cast<T*>(work);
  T* qb = static_cast<T*>(qbar);
  if (c.viscous) {
    hipError_t e = launch_march<T>(g, StressOp<T>{{}, g, c, qq, rr, w}, st);
    if (e != hipSuccess) return e;
    e = launch_march_z<T>(g, ViscOp<T>{g, c, rr, w, w + W_UB * g.N}, st);
    if (e != hipSuccess) return e;
  }
  return launch_march_split<T>(g, GatherOp<T>{g, c, qq, rr, qb, c.viscous ? w + W_UB * g.N : nullptr}, st);
}

template <class T>
hipError_t launch_rk_stage_adjoint(const Grid& g, int stage, double dt, const void* qbar, void* zeta, void* rbar,
                                   hipStream_t st) {
  static const double kA[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
  static const double kB[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
  const long long n5 = 5 * g.N;
  hipLaunchKernelGGL((rk_adj<T>), dim3(blocks_for(n5)), dim3(kThreads), 0, st, n5, (T)kA[stage], (T)kB[stage],
                     (T)dt, static_cast<const T*>(qbar), static_cast<T*>(zeta), static_cast<T*>(rbar));
  return hipGetLastError();
}

template <class T>
hipError_t launch_integrals_adjoint(const Grid& g, const Coef<T>& c, const void* q, double eps_bar, void* qbar,
                                    void* work, hipStream_t st) {
  const T scale = (T)(eps_bar * 2.0 / ((double)g.N) * (double)c.ire);
  const T* qq = static_cast<const T*>(q);
  T* w = static_cast<T*>(work);
  const hipError_t e = launch_march<T>(g, VortOp<T>{{}, g, c, scale, qq, w}, st);
  if (e != hipSuccess) return e;
  return launch_march<T>(g, CurlOp<T>{g, c, qq, w, static_cast<T*>(qbar)}, st);
}

template hipError_t launch_residual_adjoint<double>(const Grid&, const Coef<double>&, const void*, const void*, void*,
                                                    void*, hipStream_t);
template hipError_t launch_residual_adjoint<float>(const Grid&, const Coef<float>&, const void*, const void*, void*,
                                                   void*, hipStream_t);
template hipError_t launch_rk_stage_adjoint<double>(const Grid&, int, double, const void*, void*, void*, hipStream_t);
template hipError_t launch_rk_stage_adjoint<float>(const Grid&, int, double, const void*, void*, void*, hipStream_t);
template hipError_t launch_integrals_adjoint<double>(const Grid&, const Coef<double>&, const void*, double, void*,
                                                     void*, hipStream_t);
template hipError_t launch_integrals_adjoint<float>(const Grid&, const Coef<float>&, const void*, double, void*,
                                                    void*, hipStream_t);

}  // namespace tgv
