// Discrete adjoint of the residual, of the RK stage and of eps^S.
//
// For the residual R(Q) the adjoint Q_bar += (dR/dQ)^T R_bar is written in
// gather form.  With D the antisymmetric 4th-order first difference,
// D^T = -D, D2^T = D2 and (D_a D_b)^T = D_a D_b on the periodic grid, every
// stencil term of the forward residual turns into a stencil of R_bar-weighted
// pointwise fields evaluated around the output point, plus pointwise terms.
// Three passes over a caller-provided workspace of 18 fields:
//   pass 0 (pointwise, viscous only) stores what pass A reads at stencil
//     neighbours: u_a and V_bar_a = R_bar_{m_a} + R_bar_E u_a;
//   pass A (viscous only) stores the adjoint of the viscous work sum
//     tau_ad G_ad, the symmetric G_bar_ad = 2 R_bar_E tau_ad (6 components),
//     and the inner derivatives of the mixed second-derivative terms,
//     sigma_a = sum_{b != a} D_b u_b and tau_b = sum_{a != b} D_a V_bar_a, so
//     that D_a D_b u_b and (D_a D_b)^T V_bar_a = D_b D_a V_bar_a become one
//     more first difference each in pass B (D_a and D_b commute on the
//     periodic grid);
//   pass B gathers every transposed-stencil and pointwise contribution,
//     re-deriving u_a, V_bar_a and sum_f R_bar_f Q_f at each neighbour from Q
//     and R_bar (which it loads there anyway) rather than reading them back.
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
  // 16 planes per block (measured 3-5 % faster than 64 or 128 at 512^3);
  // fewer where the grid would otherwise hold too few blocks to fill the chip
  m.kz = 16;
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
enum { W_U = 0, W_VB = 3, W_GB = 6, W_SIG = 12, W_TAU = 15, W_FIELDS = 18 };
static_assert(W_FIELDS == kResidualAdjointWorkFields, "workspace size");

// Pass 0: pointwise fields read at stencil neighbours by pass A.
template <class T>
__global__ void __launch_bounds__(kThreads) adj_prim(Grid g, const T* __restrict__ q, const T* __restrict__ rb,
                                                     T* __restrict__ w) {
  const long long N = g.N;
  for (long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x; id < N;
       id += (long long)gridDim.x * blockDim.x) {
  T q0[5], r0[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    q0[f] = q[f * N + id];
    r0[f] = rb[f * N + id];
  }
  const T ir = recip(q0[0]);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const T u = q0[a + 1] * ir;
    w[(W_U + a) * N + id] = u;
    w[(W_VB + a) * N + id] = r0[a + 1] + r0[4] * u;
  }
  }
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
// Along each direction the neighbours are visited in symmetric pairs, (-1, +1)
// and then (-2, +2).  At each neighbour u_a, V_bar_a and sum_f R_bar_f Q_f are
// derived from Q and R_bar with the expressions pass 0 uses, and every first
// and second difference is accumulated pair by pair,
//   8 (f_{+1} - f_{-1}) - (f_{+2} - f_{-2}),
//   16 ((f_{+1} - f_0) + (f_{-1} - f_0)) - ((f_{+2} - f_0) + (f_{-2} - f_0))
// (the factors 8 and 16 are exact), the neighbour differences always taken
// first.  Only the viscous fields G_bar, sigma and tau come from the
// workspace.
// The values of Q and R_bar at one neighbour and what is derived from them.
template <class T>
struct NbVals {
  T q[5], r[5], u[3], vb[3], srq;
};

template <class T>
__device__ __forceinline__ void load_nb(const T* __restrict__ q, const T* __restrict__ rb, long long N, long long n,
                                        NbVals<T>& v) {
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    v.q[f] = q[f * N + n];
    v.r[f] = rb[f * N + n];
  }
  const T ir = recip(v.q[0]);
  T srq = 0;
#pragma unroll
  for (int f = 0; f < 5; ++f) srq += v.r[f] * v.q[f];
  v.srq = srq;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const T u = v.q[a + 1] * ir;
    v.u[a] = u;
    v.vb[a] = v.r[a + 1] + v.r[4] * u;
  }
}

// Difference sums of one direction (before the 1/(12 h) or 1/(12 h^2) factor).
// `ubs` collects the terms that enter u_bar_d through a first difference:
// sum_f (-R_bar_f) D_d q_f + D_d (sum_f R_bar_f Q_f), each difference taken
// from the neighbour values first.
template <class T>
struct DirSums {
  T r[5], rud[5], ud, ubs, rE2, vb2[3], u2[3], gb[3], sig, tau;
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

// Pair K of direction d: neighbours at -K and +K.
template <int K, class T>
__device__ __forceinline__ void add_pair(DirSums<T>& S, const T* __restrict__ q, const T* __restrict__ rb,
                                         const T* __restrict__ w, long long N, long long nm, long long np, int d,
                                         bool viscous, const T (&r0)[5], const T (&vb0)[3], const T (&u0)[3]) {
  {
    NbVals<T> m, p;
    load_nb(q, rb, N, nm, m);
    load_nb(q, rb, N, np, p);
    const T udm = d == 0 ? m.u[0] : (d == 1 ? m.u[1] : m.u[2]);
    const T udp = d == 0 ? p.u[0] : (d == 1 ? p.u[1] : p.u[2]);
    T ubs = p.srq - m.srq;
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      d1_add<K>(S.r[f], p.r[f] - m.r[f]);
      const T pu = p.r[f] * udp;
      const T mu = m.r[f] * udm;
      d1_add<K>(S.rud[f], pu - mu);
      ubs -= r0[f] * (p.q[f] - m.q[f]);
    }
    d1_add<K>(S.ud, udp - udm);
    d1_add<K>(S.ubs, ubs);
    if (viscous) {
      d2_add<K>(S.rE2, p.r[4], m.r[4], r0[4]);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        d2_add<K>(S.vb2[a], p.vb[a], m.vb[a], vb0[a]);
        d2_add<K>(S.u2[a], p.u[a], m.u[a], u0[a]);
      }
    }
  }
  if (viscous) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const T* base = w + (W_GB + sym(a, d)) * N;
      d1_add<K>(S.gb[a], base[np] - base[nm]);
    }
    d1_add<K>(S.sig, w[(W_SIG + d) * N + np] - w[(W_SIG + d) * N + nm]);
    d1_add<K>(S.tau, w[(W_TAU + d) * N + np] - w[(W_TAU + d) * N + nm]);
  }
}

template <class T>
__global__ void __launch_bounds__(kThreads) adj_gather(Grid g, ColMarch cm, Coef<T> c, const T* __restrict__ q,
                                                       const T* __restrict__ rb, const T* __restrict__ w,
                                                       T* __restrict__ qbar) {
  const Column col = column(g, cm);
  if (!col.valid) return;
  const bool viscous = c.viscous != 0;
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
    T u0[3], vb0[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      u0[a] = q0[a + 1] * ir0;
      vb0[a] = r0[a + 1] + r0[4] * u0[a];
    }
    const T p0 = c.gm1 * (q0[4] - half * (q0[1] * u0[0] + q0[2] * u0[1] + q0[3] * u0[2]));
    const T T0 = c.gm2 * p0 * ir0;

    T qb[5] = {0, 0, 0, 0, 0};
    T ub[3] = {0, 0, 0};
    T pb = 0, Tb = 0;
    T lap[3] = {0, 0, 0}, X[3] = {0, 0, 0};  // forward viscous pieces at this point

    // The direction loop is not unrolled, so that one direction's sums and
    // one pair of neighbours are live at a time.
#pragma unroll 1
    for (int d = 0; d < 3; ++d) {
      const T u0d = d == 0 ? u0[0] : (d == 1 ? u0[1] : u0[2]);
      const T s1 = c.c1[d], s2 = c.c2[d];
      DirSums<T> S;
      add_pair<1>(S, q, rb, w, N, nb(g, id, ijk, d, -1), nb(g, id, ijk, d, 1), d, viscous, r0, vb0, u0);
      add_pair<2>(S, q, rb, w, N, nb(g, id, ijk, d, -2), nb(g, id, ijk, d, 2), d, viscous, r0, vb0, u0);
      T ubd = 0, Xd = 0;  // contributions to ub[d], X[d]
      const T dud = s1 * S.ud;  // forward D_d u_d at this point
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        const T Dr = s1 * S.r[f];
        // (1) flux term D_d(q_f u_d): F = 1/2 D_d(R_bar_f)
        const T F = half * Dr;
        qb[f] += F * u0d;
        ubd += F * q0[f];
        // (2) u_d D_d q_f
        qb[f] += half * (s1 * S.rud[f]);
        // (3) q_f D_d u_d, pointwise part
        qb[f] -= half * r0[f] * dud;
        // (4) momentum pressure gradient D_d p
        if (f == d + 1) pb += Dr;
        if (f == 4) {
          // (5) pressure work D_d(p u_d)
          pb += Dr * u0d;
          ubd += Dr * p0;
          // (8) heat flux
          if (viscous) Tb += c.kap * (s2 * S.rE2);
        }
      }
      // (2) -R_bar_f D_d q_f and (3) q_f D_d u_d, stencil part summed over f
      ubd += half * (s1 * S.ubs);
      if (viscous) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          // (6) viscous momentum, D2 parts, on V_bar_a = R_bar_{m_a} + R_bar_E u_a
          const T vb = s2 * S.vb2[a];
          ub[a] += c.ire * vb;
          if (a == d) ubd += c.ire * (T(1.0 / 3.0)) * vb;
          // forward pieces of V_{m_a} at this point
          const T l = s2 * S.u2[a];
          lap[a] += l;
          if (a == d) Xd += l;
          // (7) viscous work: u_a += D_d^T(G_bar_ad) = -D_d(G_bar_ad)
          ub[a] -= s1 * S.gb[a];
        }
        // (9) mixed second derivatives through the stored inner differences:
        //   forward X_d += D_d sigma_d ; adjoint u_d += (1/(3 Re)) D_d tau_d
        Xd += s1 * S.sig;
        ubd += c.ire * T(1.0 / 3.0) * (s1 * S.tau);
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        ub[a] += a == d ? ubd : T(0);
        X[a] += a == d ? Xd : T(0);
      }
    }

    if (viscous) {
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
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n5;
       i += (long long)gridDim.x * blockDim.x) {
    const T z = zeta[i] + B * qbar[i];
    rbar[i] = dt * z;
    zeta[i] = A * z;
  }
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

inline unsigned blocks_for(long long n) { return blocks_1d(n, kThreads); }

}  // namespace

long long adjoint_work_items(const Grid& g) { return col_march(g).blocks * kThreads; }

template <class T>
hipError_t launch_residual_adjoint(const Grid& g, const Coef<T>& c, const void* q, const void* rbar, void* qbar,
                                   void* work, hipStream_t st) {
  const T* qq = static_cast<const T*>(q);
  const T* rr = static_cast<const T*>(rbar);
  T* w = static_cast<T*>(work);
  const ColMarch cm = col_march(g);
  if (c.viscous) {
    hipLaunchKernelGGL((adj_prim<T>), dim3(blocks_for(g.N)), dim3(kThreads), 0, st, g, qq, rr, w);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
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
