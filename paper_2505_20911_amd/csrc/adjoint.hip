// Discrete adjoint of the residual, of the RK stage and of eps^S.
//
// For the residual R(Q) the adjoint Q_bar += (dR/dQ)^T R_bar is written in
// gather form.  With D the antisymmetric 4th-order first difference,
// D^T = -D, D2^T = D2 and (D_a D_b)^T = D_a D_b on the periodic grid, every
// stencil term of the forward residual turns into a stencil of R_bar-weighted
// pointwise fields evaluated around the output point, plus pointwise terms.
// Three passes over a caller-provided workspace of 19 fields:
//   pass 0 (pointwise) stores the fields the gather needs at stencil
//     neighbours: u_a, V_bar_a = R_bar_{m_a} + R_bar_E u_a and sum_f R_bar_f Q_f;
//   pass A (viscous only) stores the adjoint of the viscous work sum
//     tau_ad G_ad, the symmetric G_bar_ad = 2 R_bar_E tau_ad (6 components),
//     and the inner derivatives of the mixed second-derivative terms,
//     sigma_a = sum_{b != a} D_b u_b and tau_b = sum_{a != b} D_a V_bar_a, so
//     that D_a D_b u_b and (D_a D_b)^T V_bar_a = D_b D_a V_bar_a become one
//     more first difference each in pass B (D_a and D_b commute on the
//     periodic grid);
//   pass B gathers every transposed-stencil and pointwise contribution.
// 1/rho is the hardware reciprocal refined by Newton-Raphson, as in the
// forward residual.
#include "tgv_device.h"
#include "tgv_kernels.h"

namespace tgv {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ long long nb(const Grid& g, long long id, const int ijk[3], int d, int s) {
  if (d == 0) {
    int t = ijk[0] + s;
    t += (t < 0) ? g.nx : 0;
    t -= (t >= g.nx) ? g.nx : 0;
    return id + (t - ijk[0]);
  } else if (d == 1) {
    int t = ijk[1] + s;
    t += (t < 0) ? g.ny : 0;
    t -= (t >= g.ny) ? g.ny : 0;
    return id + (long long)(t - ijk[1]) * g.nx;
  }
  int t = ijk[2] + s;
  t += (t < 0) ? g.nz : 0;
  t -= (t >= g.nz) ? g.nz : 0;
  return id + (long long)(t - ijk[2]) * g.plane;
}

// Gather kernels walk columns: a block owns a CX x CY tile of (x, y) columns
// and a chunk of kz planes, x fastest, and each thread loops over its column's
// planes, so the z-neighbour rows it reads were read by the same block a step
// or two earlier and the tile's x/y neighbours are shared within the block.
// Blocks are spread over the 8 XCDs in contiguous runs (hardware block b runs
// on XCD b mod 8).
constexpr int CX = 64, CY = kThreads / CX;

struct ColMarch {
  int tiles_x, tiles_y, kz;
  long long blocks;
};

ColMarch col_march(const Grid& g) {
  ColMarch m;
  m.tiles_x = (g.nx + CX - 1) / CX;
  m.tiles_y = (g.ny + CY - 1) / CY;
  m.kz = 64;
  while (m.kz > 1 && (long long)m.tiles_x * m.tiles_y * ((g.nz + m.kz - 1) / m.kz) < 2048) m.kz /= 2;
  m.blocks = (long long)m.tiles_x * m.tiles_y * ((g.nz + m.kz - 1) / m.kz);
  return m;
}

struct Column {
  int x, y, z0, z1;
  long long xy;
  bool valid;
};

__device__ __forceinline__ Column column(const Grid& g, const ColMarch& m) {
  const int nb = (int)m.blocks;
  int b = blockIdx.x;
  if (nb % 8 == 0) b = (b % 8) * (nb / 8) + b / 8;
  Column c;
  c.x = (b % m.tiles_x) * CX + threadIdx.x % CX;
  c.y = ((b / m.tiles_x) % m.tiles_y) * CY + threadIdx.x / CX;
  c.z0 = (b / (m.tiles_x * m.tiles_y)) * m.kz;
  c.z1 = min(c.z0 + m.kz, g.nz);
  c.valid = c.x < g.nx && c.y < g.ny;
  c.xy = (long long)c.y * g.nx + c.x;
  return c;
}

template <class T>
__device__ __forceinline__ T D1(T m2, T m1, T p1, T p2, T s) {
  return s * (T(8) * (p1 - m1) - (p2 - m2));
}
template <class T>
__device__ __forceinline__ T D2(T m2, T m1, T c0, T p1, T p2, T s) {
  return s * (T(16) * ((p1 - c0) + (m1 - c0)) - ((p2 - c0) + (m2 - c0)));
}

// Index of the symmetric pair (a, d) in the 6-component storage.
__device__ __forceinline__ int sym(int a, int d) {
  if (a == d) return a;
  const int lo = a < d ? a : d, hi = a < d ? d : a;
  return lo == 0 ? (hi == 1 ? 3 : 4) : 5;
}

// Workspace layout, fields of N values each.
enum { W_U = 0, W_VB = 3, W_SRQ = 6, W_GB = 7, W_SIG = 13, W_TAU = 16, W_FIELDS = 19 };
static_assert(W_FIELDS == kResidualAdjointWorkFields, "workspace size");

// Pass 0: pointwise fields read at stencil neighbours by the later passes.
template <class T>
__global__ void __launch_bounds__(kThreads) adj_prim(Grid g, const T* __restrict__ q, const T* __restrict__ rb,
                                                     T* __restrict__ w) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= g.N) return;
  const long long N = g.N;
  T q0[5], r0[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    q0[f] = q[f * N + id];
    r0[f] = rb[f * N + id];
  }
  const T ir = recip(q0[0]);
  T srq = 0;
#pragma unroll
  for (int f = 0; f < 5; ++f) srq += r0[f] * q0[f];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const T u = q0[a + 1] * ir;
    w[(W_U + a) * N + id] = u;
    w[(W_VB + a) * N + id] = r0[a + 1] + r0[4] * u;
  }
  w[W_SRQ * N + id] = srq;
}

// Pass A: G_bar_ad = 2 R_bar_E tau_ad, sigma_a and tau_b at every point.
template <class T>
__global__ void __launch_bounds__(kThreads) adj_stress(Grid g, ColMarch cm, Coef<T> c, const T* __restrict__ rb,
                                                       T* __restrict__ w) {
  const Column col = column(g, cm);
  if (!col.valid) return;
#pragma nounroll
  for (int z = col.z0; z < col.z1; ++z) {
    const int ijk[3] = {col.x, col.y, z};
    const long long id = (long long)z * g.plane + col.xy;
    const long long N = g.N;
    T G[3][3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T u[4][3];
      const int offs[4] = {-2, -1, 1, 2};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const long long n = nb(g, id, ijk, d, offs[s]);
#pragma unroll
        for (int a = 0; a < 3; ++a) u[s][a] = w[(W_U + a) * N + n];
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) G[a][d] = D1(u[0][a], u[1][a], u[2][a], u[3][a], c.c1[d]);
    }
    T dv[3];  // D_a V_bar_a
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const long long base = (long long)(W_VB + a) * N;
      dv[a] = D1(w[base + nb(g, id, ijk, a, -2)], w[base + nb(g, id, ijk, a, -1)], w[base + nb(g, id, ijk, a, 1)],
                 w[base + nb(g, id, ijk, a, 2)], c.c1[a]);
    }
    w[(W_SIG + 0) * N + id] = G[1][1] + G[2][2];
    w[(W_SIG + 1) * N + id] = G[0][0] + G[2][2];
    w[(W_SIG + 2) * N + id] = G[0][0] + G[1][1];
    w[(W_TAU + 0) * N + id] = dv[1] + dv[2];
    w[(W_TAU + 1) * N + id] = dv[0] + dv[2];
    w[(W_TAU + 2) * N + id] = dv[0] + dv[1];
    const T div = G[0][0] + G[1][1] + G[2][2];
    const T two_rE = T(2) * rb[4 * N + id];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int d = a; d < 3; ++d) {
        const T tau = c.ire * (G[a][d] + G[d][a] - (a == d ? T(2.0 / 3.0) * div : T(0)));
        w[(W_GB + sym(a, d)) * N + id] = two_rE * tau;
      }
  }
}

// Pass B: gather of all transposed-stencil and pointwise contributions.
template <class T>
__global__ void __launch_bounds__(kThreads) adj_gather(Grid g, ColMarch cm, Coef<T> c, const T* __restrict__ q,
                                                       const T* __restrict__ rb, const T* __restrict__ w,
                                                       T* __restrict__ qbar) {
  const Column col = column(g, cm);
  if (!col.valid) return;
#pragma nounroll
  for (int z = col.z0; z < col.z1; ++z) {
    const int ijk[3] = {col.x, col.y, z};
    const long long id = (long long)z * g.plane + col.xy;
    const long long N = g.N;
    const T half = T(0.5);

    T q0[5], r0[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      q0[f] = q[f * N + id];
      r0[f] = rb[f * N + id];
    }
    const T ir0 = recip(q0[0]);
    T u0[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) u0[a] = q0[a + 1] * ir0;
    const T p0 = c.gm1 * (q0[4] - half * (q0[1] * u0[0] + q0[2] * u0[1] + q0[3] * u0[2]));
    const T T0 = c.gm2 * p0 * ir0;

    T qb[5] = {0, 0, 0, 0, 0};
    T ub[3] = {0, 0, 0};
    T pb = 0, Tb = 0;
    T lap[3] = {0, 0, 0}, X[3] = {0, 0, 0};  // forward viscous pieces at this point

    const int offs[4] = {-2, -1, 1, 2};
    // Neighbour values are consumed one field at a time, and the direction
    // loop is not unrolled, so that few of them are live at once; the
    // direction's own components are selected, not indexed.
#pragma unroll 1
    for (int d = 0; d < 3; ++d) {
      const T u0d = d == 0 ? u0[0] : (d == 1 ? u0[1] : u0[2]);
      T ubd = 0, Xd = 0;  // contributions to ub[d], X[d]
      long long n[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) n[s] = nb(g, id, ijk, d, offs[s]);
      auto at = [&](const T* base, int s) { return base[n[s]]; };
      auto D1n = [&](const T* base, T sc) { return D1(at(base, 0), at(base, 1), at(base, 2), at(base, 3), sc); };
      const T s1 = c.c1[d], s2 = c.c2[d];
      T ud[4];  // u_d at the neighbours
#pragma unroll
      for (int s = 0; s < 4; ++s) ud[s] = at(w + (W_U + d) * N, s);
      const T dud = D1(ud[0], ud[1], ud[2], ud[3], s1);  // forward D_d u_d at this point
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        T rn[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) rn[s] = at(rb + f * N, s);
        const T Dr = D1(rn[0], rn[1], rn[2], rn[3], s1);
        // (1) flux term D_d(q_f u_d): F = 1/2 D_d(R_bar_f)
        const T F = half * Dr;
        qb[f] += F * u0d;
        ubd += F * q0[f];
        // (2) u_d D_d q_f
        qb[f] += half * D1(rn[0] * ud[0], rn[1] * ud[1], rn[2] * ud[2], rn[3] * ud[3], s1);
        const T dq = D1n(q + f * N, s1);
        ubd -= half * r0[f] * dq;
        // (3) q_f D_d u_d, pointwise part
        qb[f] -= half * r0[f] * dud;
        // (4) momentum pressure gradient D_d p
        if (f == d + 1) pb += Dr;
        if (f == 4) {
          // (5) pressure work D_d(p u_d)
          pb += Dr * u0d;
          ubd += Dr * p0;
          // (8) heat flux
          if (c.viscous) Tb += c.kap * D2(rn[0], rn[1], r0[4], rn[2], rn[3], s2);
        }
      }
      // (3) q_f D_d u_d, stencil part summed over f
      ubd += half * D1n(w + W_SRQ * N, s1);
      if (c.viscous) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          // (6) viscous momentum, D2 parts, on V_bar_a = R_bar_{m_a} + R_bar_E u_a
          const T* vbase = w + (W_VB + a) * N;
          const T vb = D2(at(vbase, 0), at(vbase, 1), vbase[id], at(vbase, 2), at(vbase, 3), s2);
          ub[a] += c.ire * vb;
          if (a == d) ubd += c.ire * (T(1.0 / 3.0)) * vb;
          // forward pieces of V_{m_a} at this point
          const T* ubase = w + (W_U + a) * N;
          const T l = D2(at(ubase, 0), at(ubase, 1), u0[a], at(ubase, 2), at(ubase, 3), s2);
          lap[a] += l;
          if (a == d) Xd += l;
          // (7) viscous work: u_a += D_d^T(G_bar_ad) = -D_d(G_bar_ad)
          ub[a] -= D1n(w + (W_GB + sym(a, d)) * N, s1);
        }
        // (9) mixed second derivatives through the stored inner differences:
        //   forward X_d += D_d sigma_d ; adjoint u_d += (1/(3 Re)) D_d tau_d
        Xd += D1n(w + (W_SIG + d) * N, s1);
        ubd += c.ire * T(1.0 / 3.0) * D1n(w + (W_TAU + d) * N, s1);
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        ub[a] += a == d ? ubd : T(0);
        X[a] += a == d ? Xd : T(0);
      }
    }

    if (c.viscous) {
      // pointwise part of sum_a u_a V_{m_a}
#pragma unroll
      for (int a = 0; a < 3; ++a) ub[a] += r0[4] * (c.ire * (lap[a] + X[a] * T(1.0 / 3.0)));
    }

    // Chain through the primitive variables at this point.
    pb += c.gm2 * Tb * ir0;
    qb[0] -= T0 * Tb * ir0;
    qb[4] += c.gm1 * pb;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      qb[a + 1] -= half * c.gm1 * pb * u0[a];
      ub[a] -= half * c.gm1 * pb * q0[a + 1];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      qb[a + 1] += ub[a] * ir0;
      qb[0] -= ub[a] * u0[a] * ir0;
    }
#pragma unroll
    for (int f = 0; f < 5; ++f) qbar[f * N + id] += qb[f];
  }
}

// Reversed RK stage: zeta += B q_bar ; r_bar = dt zeta ; zeta = A zeta.
template <class T>
__global__ void __launch_bounds__(kThreads) rk_adj(long long n5, T A, T B, T dt, const T* __restrict__ qbar,
                                                   T* __restrict__ zeta, T* __restrict__ rbar) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n5) return;
  const T z = zeta[i] + B * qbar[i];
  rbar[i] = dt * z;
  zeta[i] = A * z;
}

// eps^S adjoint pass A: omega_bar = eps_bar (1/(N Re)) 2 omega.
template <class T>
__global__ void __launch_bounds__(kThreads) adj_vort(Grid g, ColMarch cm, Coef<T> c, T scale, const T* __restrict__ q,
                                                     T* __restrict__ wbar) {
  const Column col = column(g, cm);
  if (!col.valid) return;
#pragma nounroll
  for (int z = col.z0; z < col.z1; ++z) {
    const int ijk[3] = {col.x, col.y, z};
    const long long id = (long long)z * g.plane + col.xy;
    T G[3][3];
    const int offs[4] = {-2, -1, 1, 2};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T u[4][3];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const long long n = nb(g, id, ijk, d, offs[s]);
        const T ir = recip(q[n]);
#pragma unroll
        for (int a = 0; a < 3; ++a) u[s][a] = q[(a + 1) * g.N + n] * ir;
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) G[a][d] = D1(u[0][a], u[1][a], u[2][a], u[3][a], c.c1[d]);
    }
    wbar[id] = scale * (G[2][1] - G[1][2]);
    wbar[g.N + id] = scale * (G[0][2] - G[2][0]);
    wbar[2 * g.N + id] = scale * (G[1][0] - G[0][1]);
  }
}

// eps^S adjoint pass B: u_bar = curl_D(omega_bar), then through u = m / rho.
template <class T>
__global__ void __launch_bounds__(kThreads) adj_curl(Grid g, ColMarch cm, Coef<T> c, const T* __restrict__ q,
                                                     const T* __restrict__ wbar, T* __restrict__ qbar) {
  const Column col = column(g, cm);
  if (!col.valid) return;
#pragma nounroll
  for (int z = col.z0; z < col.z1; ++z) {
    const int ijk[3] = {col.x, col.y, z};
    const long long id = (long long)z * g.plane + col.xy;
    const long long N = g.N;
    auto d1w = [&](int comp, int d) {
      const T* w = wbar + comp * N;
      return D1(w[nb(g, id, ijk, d, -2)], w[nb(g, id, ijk, d, -1)], w[nb(g, id, ijk, d, 1)],
                w[nb(g, id, ijk, d, 2)], c.c1[d]);
    };
    T ub[3];
    ub[0] = d1w(2, 1) - d1w(1, 2);
    ub[1] = d1w(0, 2) - d1w(2, 0);
    ub[2] = d1w(1, 0) - d1w(0, 1);
    const T ir = recip(q[id]);
    T rb = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      qbar[(a + 1) * N + id] += ub[a] * ir;
      rb -= ub[a] * q[(a + 1) * N + id] * ir * ir;
    }
    qbar[id] += rb;
  }
}

inline unsigned blocks_for(long long n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

template <class T>
hipError_t launch_residual_adjoint(const Grid& g, const Coef<T>& c, const void* q, const void* rbar, void* qbar,
                                   void* work, hipStream_t st) {
  const T* qq = static_cast<const T*>(q);
  const T* rr = static_cast<const T*>(rbar);
  T* w = static_cast<T*>(work);
  const ColMarch cm = col_march(g);
  hipLaunchKernelGGL((adj_prim<T>), dim3(blocks_for(g.N)), dim3(kThreads), 0, st, g, qq, rr, w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (c.viscous) {
    hipLaunchKernelGGL((adj_stress<T>), dim3((unsigned)cm.blocks), dim3(kThreads), 0, st, g, cm, c, rr, w);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((adj_gather<T>), dim3((unsigned)cm.blocks), dim3(kThreads), 0, st, g, cm, c, qq, rr, w,
                     static_cast<T*>(qbar));
  return hipGetLastError();
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
  const ColMarch cm = col_march(g);
  hipLaunchKernelGGL((adj_vort<T>), dim3((unsigned)cm.blocks), dim3(kThreads), 0, st, g, cm, c, scale,
                     static_cast<const T*>(q), static_cast<T*>(work));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((adj_curl<T>), dim3((unsigned)cm.blocks), dim3(kThreads), 0, st, g, cm, c, static_cast<const T*>(q),
                     static_cast<const T*>(work), static_cast<T*>(qbar));
  return hipGetLastError();
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
