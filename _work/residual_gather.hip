// Fused Navier-Stokes residual R = dQ/dt on a periodic grid (paper Sec. 2.3.1
// scheme and split form, Sec. 3.1 state vector and residual).
//
// Gather formulation: one thread per output point.  Every neighbour value a
// stencil needs is read from global memory (served by L1/L2: each value is
// re-read by the neighbouring threads) and the primitive variables are
// re-derived at each stencil point in the arithmetic type Tc.  Templated on
// the storage types of Q and R and the arithmetic type (Sec. 3.1 precision
// classes).
#include "tgv_device.h"
#include "tgv_kernels.h"

namespace tgv {

namespace {

template <class Tq, class Tc>
struct State {
  const Tq* __restrict__ q;
  long long N;
  __device__ __forceinline__ Tc at(int f, long long id) const { return load_as<Tc>(q[f * N + id]); }
};

template <class Tc>
struct Prim {
  Tc q[5];  // rho, m1, m2, m3, rho E
  Tc u[3];
  Tc p, T;
};

template <class Tq, class Tc>
__device__ __forceinline__ Prim<Tc> prim(const State<Tq, Tc>& s, const Coef<Tc>& c, long long id) {
  Prim<Tc> w;
#pragma unroll
  for (int f = 0; f < 5; ++f) w.q[f] = s.at(f, id);
  const Tc ir = Tc(1) / w.q[0];
#pragma unroll
  for (int a = 0; a < 3; ++a) w.u[a] = w.q[a + 1] * ir;
  const Tc ke = Tc(0.5) * (w.q[1] * w.u[0] + w.q[2] * w.u[1] + w.q[3] * w.u[2]);
  w.p = c.gm1 * (w.q[4] - ke);
  w.T = c.gm2 * w.p * ir;
  return w;
}

// Linear index of the point displaced by s cells along axis d (periodic).
__device__ __forceinline__ long long shift(const Grid& g, long long id, const int ijk[3], int d, int s) {
  if (d == 0) {
    int i = ijk[0] + s;
    i += (i < 0) ? g.nx : 0;
    i -= (i >= g.nx) ? g.nx : 0;
    return id + (i - ijk[0]);
  } else if (d == 1) {
    int j = ijk[1] + s;
    j += (j < 0) ? g.ny : 0;
    j -= (j >= g.ny) ? g.ny : 0;
    return id + (long long)(j - ijk[1]) * g.nx;
  } else {
    int k = ijk[2] + s;
    k += (k < 0) ? g.nz : 0;
    k -= (k >= g.nz) ? g.nz : 0;
    return id + (long long)(k - ijk[2]) * g.plane;
  }
}

// 4th-order central first and second differences in difference form.
template <class Tc>
__device__ __forceinline__ Tc d1(Tc fm2, Tc fm1, Tc fp1, Tc fp2, Tc scale) {
  return scale * (Tc(8) * (fp1 - fm1) - (fp2 - fm2));
}
template <class Tc>
__device__ __forceinline__ Tc d2(Tc fm2, Tc fm1, Tc f0, Tc fp1, Tc fp2, Tc scale) {
  return scale * (Tc(16) * ((fp1 - f0) + (fm1 - f0)) - ((fp2 - f0) + (fm2 - f0)));
}

template <class Tq, class Tr, class Tc>
__global__ void __launch_bounds__(256) residual_gather(Grid g, Coef<Tc> c, const Tq* __restrict__ q,
                                                       Tr* __restrict__ r) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= g.N) return;
  const int ijk[3] = {(int)(id % g.nx), (int)((id / g.nx) % g.ny), (int)(id / g.plane)};
  State<Tq, Tc> s{q, g.N};
  const Prim<Tc> w0 = prim(s, c, id);

  Tc C[5] = {0, 0, 0, 0, 0};  // convective terms (split form)
  Tc Pm[3] = {0, 0, 0};       // pressure gradient
  Tc PE = 0;                  // pressure work  sum_d D_d(p u_d)
  Tc G[3][3];                 // G[a][d] = D_d u_a
  Tc lap[3] = {0, 0, 0};      // sum_d D2_d u_a
  Tc X[3] = {0, 0, 0};        // D2_a u_a + sum_{d != a} D_a D_d u_d
  Tc lapT = 0;                // sum_d D2_d T

#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const Prim<Tc> A = prim(s, c, shift(g, id, ijk, d, -2));
    const Prim<Tc> B = prim(s, c, shift(g, id, ijk, d, -1));
    const Prim<Tc> Cc = prim(s, c, shift(g, id, ijk, d, +1));
    const Prim<Tc> D = prim(s, c, shift(g, id, ijk, d, +2));
    const Tc s1 = c.c1[d], s2 = c.c2[d];
    const Tc dud = d1(A.u[d], B.u[d], Cc.u[d], D.u[d], s1);
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      const Tc flux = d1(A.q[f] * A.u[d], B.q[f] * B.u[d], Cc.q[f] * Cc.u[d], D.q[f] * D.u[d], s1);
      const Tc dq = d1(A.q[f], B.q[f], Cc.q[f], D.q[f], s1);
      C[f] += Tc(0.5) * (flux + w0.u[d] * dq + w0.q[f] * dud);
    }
    Pm[d] = d1(A.p, B.p, Cc.p, D.p, s1);
    PE += d1(A.p * A.u[d], B.p * B.u[d], Cc.p * Cc.u[d], D.p * D.u[d], s1);
    if (c.viscous) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        G[a][d] = d1(A.u[a], B.u[a], Cc.u[a], D.u[a], s1);
        const Tc l = d2(A.u[a], B.u[a], w0.u[a], Cc.u[a], D.u[a], s2);
        lap[a] += l;
        if (a == d) X[a] += l;
      }
      lapT += d2(A.T, B.T, w0.T, Cc.T, D.T, s2);
    }
  }

  Tc R[5];
  R[0] = -C[0];
#pragma unroll
  for (int a = 0; a < 3; ++a) R[a + 1] = -C[a + 1] - Pm[a];
  R[4] = -C[4] - PE;

  if (c.viscous) {
    // Mixed derivatives on each coordinate plane (a, b), a < b: at the 16
    // points (s_a, s_b) in {-2,-1,1,2}^2 form u_a and u_b once, then
    // X_a += D_a D_b u_b and X_b += D_b D_a u_a (the two operators commute).
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
      for (int b = a + 1; b < 3; ++b) {
        const int offs[4] = {-2, -1, 1, 2};
        Tc inner_b[4], inner_a[4];  // D_b u_b and D_a ... see below, per s_a
        Tc ub_rows[4][4], ua_rows[4][4];
#pragma unroll
        for (int ia = 0; ia < 4; ++ia) {
          const long long ida = shift(g, id, ijk, a, offs[ia]);
          int ijk_a[3] = {ijk[0], ijk[1], ijk[2]};
          ijk_a[a] = ijk_a[a] + offs[ia];
          const int na = (a == 0) ? g.nx : (a == 1) ? g.ny : g.nz;
          ijk_a[a] += (ijk_a[a] < 0) ? na : 0;
          ijk_a[a] -= (ijk_a[a] >= na) ? na : 0;
#pragma unroll
          for (int ib = 0; ib < 4; ++ib) {
            const long long idab = shift(g, ida, ijk_a, b, offs[ib]);
            const Tc rho = s.at(0, idab);
            const Tc ir = Tc(1) / rho;
            ua_rows[ia][ib] = s.at(a + 1, idab) * ir;
            ub_rows[ia][ib] = s.at(b + 1, idab) * ir;
          }
        }
        // D_b at each a-offset, then D_a of that (for u_b); and the same
        // weights with the roles of the two offsets swapped for u_a.
#pragma unroll
        for (int ia = 0; ia < 4; ++ia)
          inner_b[ia] = d1(ub_rows[ia][0], ub_rows[ia][1], ub_rows[ia][2], ub_rows[ia][3], c.c1[b]);
#pragma unroll
        for (int ib = 0; ib < 4; ++ib)
          inner_a[ib] = d1(ua_rows[0][ib], ua_rows[1][ib], ua_rows[2][ib], ua_rows[3][ib], c.c1[a]);
        X[a] += d1(inner_b[0], inner_b[1], inner_b[2], inner_b[3], c.c1[a]);
        X[b] += d1(inner_a[0], inner_a[1], inner_a[2], inner_a[3], c.c1[b]);
      }
    }
    const Tc div = G[0][0] + G[1][1] + G[2][2];
    Tc VE = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const Tc Vm = c.ire * (lap[a] + X[a] * Tc(1.0 / 3.0));
      R[a + 1] += Vm;
      VE += w0.u[a] * Vm;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const Tc tau = c.ire * (G[a][d] + G[d][a] - (a == d ? Tc(2.0 / 3.0) * div : Tc(0)));
        VE += tau * G[a][d];
      }
    VE += c.kap * lapT;
    R[4] += VE;
  }
#pragma unroll
  for (int f = 0; f < 5; ++f) r[f * g.N + id] = store_as<Tr>(R[f]);
}

}  // namespace

template <class Tq, class Tr, class Tc>
hipError_t launch_residual(const Grid& g, const Coef<Tc>& c, const void* q, void* r, hipStream_t st) {
  const int threads = 256;
  const long long blocks = (g.N + threads - 1) / threads;
  hipLaunchKernelGGL((residual_gather<Tq, Tr, Tc>), dim3((unsigned)blocks), dim3(threads), 0, st, g, c,
                     static_cast<const Tq*>(q), static_cast<Tr*>(r));
  return hipGetLastError();
}

#define TGV_INST_RES(Tq, Tr, Tc) \
  template hipError_t launch_residual<Tq, Tr, Tc>(const Grid&, const Coef<Tc>&, const void*, void*, hipStream_t);
TGV_INST_RES(double, double, double)
TGV_INST_RES(double, float, float)
TGV_INST_RES(double, float, double)
TGV_INST_RES(float, float, double)
TGV_INST_RES(float, float, float)
TGV_INST_RES(float, f16, float)
TGV_INST_RES(float, bf16, float)
TGV_INST_RES(f16, f16, float)

}  // namespace tgv
