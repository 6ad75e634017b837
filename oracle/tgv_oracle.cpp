// TEST INFRASTRUCTURE ONLY -- the FP64 CPU oracle.
//
// A plain, slow, deliberately unoptimised implementation of what the explicit
// finite-difference time step of the compressible Navier-Stokes equations for
// the Taylor-Green vortex computes (paper: Sec. 2.3.1, Sec. 3.1, Sec. 4.1).
// Only the tests, __graft_entry__.smoke() and the CPU-baseline leg of the
// benchmark may load it.  It shares no code, header or constant with the GPU
// library; the product path never calls it.
//
// Every routine is templated on the scalar S so that the same source runs in
// double and in std::complex<double> (complex-step differentiation pins the
// hand-written adjoint).  Loops are plain (k, j, i) sweeps with modular
// periodic indexing; whole intermediate fields are materialised; nothing is
// fused or reordered beyond what the formulas say.  Built with
// -O2 -ffp-contract=off so no multiply-add is contracted.
//
// Readings of the paper used here (the paper leaves these open):
//   * grid x_i = i * L/n, no duplicated periodic end point;
//   * first derivative  D1 f_i = (f_{i-2} - 8 f_{i-1} + 8 f_{i+1} - f_{i+2}) / (12 h),
//     second derivative D2 f_i = (-f_{i-2} + 16 f_{i-1} - 30 f_i + 16 f_{i+1} - f_{i+2}) / (12 h^2)
//     (4th-order central, Sec. 2.3.1), each evaluated in difference form
//     (8 (f_{i+1} - f_{i-1}) - (f_{i+2} - f_{i-2})) / (12 h) and
//     (16 ((f_{i+1} - f_i) + (f_{i-1} - f_i)) - ((f_{i+2} - f_i) + (f_{i-2} - f_i))) / (12 h^2),
//     the same operators, written so that a constant field gives exactly zero;
//   * Blaisdell split of the convective term d(rho u_j phi)/dx_j with the pairing
//     (rho phi) x (u_j):  1/2 [ D(rho phi u_j) + u_j D(rho phi) + rho phi D(u_j) ],
//     applied to phi = 1, u_i, E (Sec. 2.3.1, convective form equation);
//     the other split forms the paper compares in the inviscid limit (Sec. 4.2),
//     selected by `split`: divergence D(rho u_j phi); Feiereisen (printed in
//     Sec. 2.3.1), pairing (rho u_j) x (phi); Jameson, pairing (rho) x (u_j phi);
//     Kennedy-Gruber-Pirozzoli, the cubic split averaging the divergence form
//     and all six product-rule expansions of the triple product (weights 1/4);
//     phi = E is the specific total energy (rho E)/rho; Kok's form (Kok 2009),
//     Feiereisen's pairing for mass and momentum, and the kinetic energy and
//     entropy preserving form KEEP (Kuya, Totani and Kawai 2018), the cubic
//     split for mass and momentum; both carry the energy as internal plus
//     kinetic energy and split the pressure work (see residual());
//   * pressure terms in divergence form, not split (Kok and KEEP: the pressure
//     gradient in divergence form, the pressure work split);
//   * constant viscosity mu = 1, Stokes stress, Fourier heat flux with
//     kappa = 1/((gamma-1) M^2 Pr Re), T = gamma M^2 p / rho (equation of state
//     consistent with the isothermal initial density of Sec. 4.1);
//   * viscous momentum term (1/Re)(sum_d D2_d u_a + X_a/3), X_a = D2_a u_a +
//     sum_{d!=a} D1_a D1_d u_d; viscous energy term expanded by the product rule;
//   * Williamson's 2N-storage RK3 for the two-register update of Sec. 3.1.

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

using cplx = std::complex<double>;

struct Params {
  int n[3];
  double L[3];
  double gamma, mach, re, pr;
  int viscous;
  int split;  // 0 Blaisdell, 1 divergence, 2 Feiereisen, 3 Jameson, 4 KGP, 5 Kok, 6 KEEP
};

Params unpack(const double* pv) {
  Params P;
  for (int d = 0; d < 3; ++d) P.n[d] = (int)pv[d];
  for (int d = 0; d < 3; ++d) P.L[d] = pv[3 + d];
  P.gamma = pv[6];
  P.mach = pv[7];
  P.re = pv[8];
  P.pr = pv[9];
  P.viscous = (int)pv[10];
  P.split = (int)pv[11];
  return P;
}

inline long npts(const Params& P) { return (long)P.n[0] * P.n[1] * P.n[2]; }

inline int wrap(int i, int n) { return ((i % n) + n) % n; }

// Linear index of point (i, j, k) = (x, y, z), x fastest, periodic.
inline long at(const Params& P, int i, int j, int k) {
  i = wrap(i, P.n[0]);
  j = wrap(j, P.n[1]);
  k = wrap(k, P.n[2]);
  return ((long)k * P.n[1] + j) * P.n[0] + i;
}

// Index of the point shifted by s cells along axis d.
inline long shifted(const Params& P, int i, int j, int k, int d, int s) {
  if (d == 0) return at(P, i + s, j, k);
  if (d == 1) return at(P, i, j + s, k);
  return at(P, i, j, k + s);
}

inline double spacing(const Params& P, int d) { return P.L[d] / P.n[d]; }

template <class S>
using Field = std::vector<S>;

// First derivative along axis d, 4th-order central (Sec. 2.3.1).
template <class S>
Field<S> D1(const Params& P, const Field<S>& f, int d) {
  Field<S> out(f.size());
  const double h = spacing(P, d);
#pragma omp parallel for
  for (int k = 0; k < P.n[2]; ++k)
    for (int j = 0; j < P.n[1]; ++j)
      for (int i = 0; i < P.n[0]; ++i) {
        S fm2 = f[shifted(P, i, j, k, d, -2)];
        S fm1 = f[shifted(P, i, j, k, d, -1)];
        S fp1 = f[shifted(P, i, j, k, d, +1)];
        S fp2 = f[shifted(P, i, j, k, d, +2)];
        out[at(P, i, j, k)] = (8.0 * (fp1 - fm1) - (fp2 - fm2)) / (12.0 * h);
      }
  return out;
}

// Second derivative along axis d, 4th-order central.
template <class S>
Field<S> D2(const Params& P, const Field<S>& f, int d) {
  Field<S> out(f.size());
  const double h = spacing(P, d);
#pragma omp parallel for
  for (int k = 0; k < P.n[2]; ++k)
    for (int j = 0; j < P.n[1]; ++j)
      for (int i = 0; i < P.n[0]; ++i) {
        S fm2 = f[shifted(P, i, j, k, d, -2)];
        S fm1 = f[shifted(P, i, j, k, d, -1)];
        S f0 = f[at(P, i, j, k)];
        S fp1 = f[shifted(P, i, j, k, d, +1)];
        S fp2 = f[shifted(P, i, j, k, d, +2)];
        out[at(P, i, j, k)] =
            (16.0 * ((fp1 - f0) + (fm1 - f0)) - ((fp2 - f0) + (fm2 - f0))) / (12.0 * h * h);
      }
  return out;
}

// Transposes.  With (D f)_i = sum_s c_s f_{i+s}, the matrix entry is
// A[i][i+s] = c_s, so (A^T g)_j = sum_i A[i][j] g_i = sum_s c_s g_{j-s}.
// For D1 (c_{+-1} = +-8, c_{+-2} = -+1, over 12 h) this is
// (8 (g_{j-1} - g_{j+1}) - (g_{j-2} - g_{j+2})) / (12 h); D2 is symmetric
// (c_s = c_{-s}), so its transpose has the D2 weights again.
template <class S>
Field<S> D1T(const Params& P, const Field<S>& g, int d) {
  Field<S> out(g.size());
  const double h = spacing(P, d);
#pragma omp parallel for
  for (int k = 0; k < P.n[2]; ++k)
    for (int j = 0; j < P.n[1]; ++j)
      for (int i = 0; i < P.n[0]; ++i) {
        S gm2 = g[shifted(P, i, j, k, d, -2)];
        S gm1 = g[shifted(P, i, j, k, d, -1)];
        S gp1 = g[shifted(P, i, j, k, d, +1)];
        S gp2 = g[shifted(P, i, j, k, d, +2)];
        out[at(P, i, j, k)] = (8.0 * (gm1 - gp1) - (gm2 - gp2)) / (12.0 * h);
      }
  return out;
}

template <class S>
Field<S> D2T(const Params& P, const Field<S>& g, int d) {
  Field<S> out(g.size());
  const double h = spacing(P, d);
#pragma omp parallel for
  for (int k = 0; k < P.n[2]; ++k)
    for (int j = 0; j < P.n[1]; ++j)
      for (int i = 0; i < P.n[0]; ++i) {
        // sum_s c_s g_{j-s} with c_s = c_{-s}: the D2 weights on the mirrored neighbours
        S gm2 = g[shifted(P, i, j, k, d, +2)];
        S gm1 = g[shifted(P, i, j, k, d, +1)];
        S g0 = g[at(P, i, j, k)];
        S gp1 = g[shifted(P, i, j, k, d, -1)];
        S gp2 = g[shifted(P, i, j, k, d, -2)];
        out[at(P, i, j, k)] =
            (16.0 * ((gp1 - g0) + (gm1 - g0)) - ((gp2 - g0) + (gm2 - g0))) / (12.0 * h * h);
      }
  return out;
}

// Pointwise helpers on whole fields.
template <class S>
Field<S> mul(const Field<S>& a, const Field<S>& b) {
  Field<S> out(a.size());
  for (size_t i = 0; i < a.size(); ++i) out[i] = a[i] * b[i];
  return out;
}

template <class S>
void axpy(Field<S>& y, double a, const Field<S>& x) {  // y += a x
  for (size_t i = 0; i < y.size(); ++i) y[i] += a * x[i];
}

template <class S>
void add(Field<S>& y, const Field<S>& x) {  // y += x
  for (size_t i = 0; i < y.size(); ++i) y[i] += x[i];
}

template <class S>
Field<S> copy_field(const S* base, long N) {
  return Field<S>(base, base + N);
}

// Primitive variables from the conserved vector Q = (rho, rho u, rho v, rho w, rho E)
// (Sec. 3.1): u_a = m_a / rho, p = (gamma-1)(rho E - 1/2 sum m_a u_a),
// T = gamma M^2 p / rho.
template <class S>
struct Prim {
  Field<S> rho, m[3], E, u[3], p, T;
};

template <class S>
Prim<S> primitives(const Params& P, const S* q) {
  const long N = npts(P);
  Prim<S> w;
  w.rho = copy_field(q, N);
  for (int a = 0; a < 3; ++a) w.m[a] = copy_field(q + (a + 1) * N, N);
  w.E = copy_field(q + 4 * N, N);
  for (int a = 0; a < 3; ++a) w.u[a].resize(N);
  w.p.resize(N);
  w.T.resize(N);
  const double gm2 = P.gamma * P.mach * P.mach;
  for (long i = 0; i < N; ++i) {
    for (int a = 0; a < 3; ++a) w.u[a][i] = w.m[a][i] / w.rho[i];
    S ke = 0.5 * (w.m[0][i] * w.u[0][i] + w.m[1][i] * w.u[1][i] + w.m[2][i] * w.u[2][i]);
    w.p[i] = (P.gamma - 1.0) * (w.E[i] - ke);
    w.T[i] = gm2 * w.p[i] / w.rho[i];
  }
  return w;
}

inline double kappa_of(const Params& P) {
  return 1.0 / ((P.gamma - 1.0) * P.mach * P.mach * P.pr * P.re);
}

// R = dQ/dt (Sec. 3.1): R_q = -C_q - P_q + V_q for q in (rho, m1, m2, m3, E).
template <class S>
void residual(const Params& P, const S* q, S* r) {
  const long N = npts(P);
  Prim<S> w = primitives(P, q);
  const Field<S>* cons[5] = {&w.rho, &w.m[0], &w.m[1], &w.m[2], &w.E};

  // Convection C_q for q = rho phi, phi in (1, u_1, u_2, u_3, E/rho).
  Field<S> C[5];
  Field<S> Du[3];
  for (int d = 0; d < 3; ++d) Du[d] = D1(P, w.u[d], d);  // D_d u_d
  if (P.split == 0) {
    // Blaisdell: C_q = 1/2 sum_d [D_d(q u_d) + u_d D_d q + q D_d u_d].
    for (int f = 0; f < 5; ++f) {
      C[f].assign(N, S(0.0));
      for (int d = 0; d < 3; ++d) {
        Field<S> t1 = D1(P, mul(*cons[f], w.u[d]), d);
        Field<S> t2 = mul(w.u[d], D1(P, *cons[f], d));
        Field<S> t3 = mul(*cons[f], Du[d]);
        for (long i = 0; i < N; ++i) C[f][i] += 0.5 * (t1[i] + t2[i] + t3[i]);
      }
    }
  } else {
    // The seven terms the other forms combine, for direction d:
    //   t_div  = D(rho u phi)      t_uDq  = u D(rho phi)    t_qDu   = rho phi D(u)
    //   t_phDm = phi D(rho u)      t_mDph = rho u D(phi)
    //   t_rDuf = rho D(u phi)      t_ufDr = u phi D(rho)
    Field<S> phi[5];
    phi[0].assign(N, S(1.0));
    for (int a = 0; a < 3; ++a) phi[a + 1] = w.u[a];
    phi[4].resize(N);
    for (long i = 0; i < N; ++i) phi[4][i] = w.E[i] / w.rho[i];
    Field<S> Drho[3];
    for (int d = 0; d < 3; ++d) Drho[d] = D1(P, w.rho, d);
    // (Kok and KEEP treat the energy apart, below: the loop stops at m3 for them.)
    const int nf = P.split >= 5 ? 4 : 5;
    for (int f = 0; f < nf; ++f) {
      C[f].assign(N, S(0.0));
      for (int d = 0; d < 3; ++d) {
        Field<S> t_div = D1(P, mul(*cons[f], w.u[d]), d);
        Field<S> t_uDq = mul(w.u[d], D1(P, *cons[f], d));
        Field<S> t_qDu = mul(*cons[f], Du[d]);
        Field<S> t_phDm = mul(phi[f], D1(P, w.m[d], d));
        Field<S> t_mDph = mul(w.m[d], D1(P, phi[f], d));
        Field<S> t_rDuf = mul(w.rho, D1(P, mul(w.u[d], phi[f]), d));
        Field<S> t_ufDr = mul(mul(w.u[d], phi[f]), Drho[d]);
        for (long i = 0; i < N; ++i) {
          S c;
          if (P.split == 1)
            c = t_div[i];
          else if (P.split == 2 || P.split == 5)
            c = 0.5 * (t_div[i] + t_phDm[i] + t_mDph[i]);
          else if (P.split == 3)
            c = 0.5 * (t_div[i] + t_rDuf[i] + t_ufDr[i]);
          else
            c = 0.25 * (t_div[i] + t_rDuf[i] + t_uDq[i] + t_phDm[i] + t_mDph[i] + t_qDu[i] + t_ufDr[i]);
          C[f][i] += c;
        }
      }
    }
  }
  if (P.split >= 5) {
    // Kok (split 5) and KEEP (split 6) transport the total energy as internal
    // energy e = p / ((gamma - 1) rho) plus kinetic energy |u|^2 / 2.  The
    // internal part takes the pairing of the momentum: Kok's (rho u_d) x (e),
    // KEEP's cubic rho x u_d x e.  The kinetic part is the split form whose
    // two-point flux is the mass flux times u_a(left) u_a(right) / 2 (Kok:
    // mass flux (rho u_d) averaged; KEEP: rho and u_d averaged apart):
    //   Kok:  1/2 sum_a [ m_d u_a D(u_a) + u_a D(m_d u_a) ]
    //   KEEP: 1/4 sum_a [ m_d u_a D(u_a) + u_a D(m_d u_a) + m_a D(u_d u_a) + u_d u_a D(m_a) ]
    // The pressure work is split as p D(u_d) + u_d D(p) (below).
    Field<S> e(N), rhoe(N);
    for (long i = 0; i < N; ++i) {
      rhoe[i] = w.p[i] / (P.gamma - 1.0);
      e[i] = rhoe[i] / w.rho[i];
    }
    C[4].assign(N, S(0.0));
    for (int d = 0; d < 3; ++d) {
      Field<S> t_div = D1(P, mul(w.m[d], e), d);   // D(rho u_d e)
      Field<S> t_eDm = mul(e, D1(P, w.m[d], d));    // e D(m_d)
      Field<S> t_mDe = mul(w.m[d], D1(P, e, d));    // m_d D(e)
      Field<S> internal(N);
      if (P.split == 5) {
        for (long i = 0; i < N; ++i) internal[i] = 0.5 * (t_div[i] + t_eDm[i] + t_mDe[i]);
      } else {
        Field<S> t_rDue = mul(w.rho, D1(P, mul(w.u[d], e), d));          // rho D(u_d e)
        Field<S> t_uDre = mul(w.u[d], D1(P, rhoe, d));                    // u_d D(rho e)
        Field<S> t_reDu = mul(rhoe, Du[d]);                               // rho e D(u_d)
        Field<S> t_ueDr = mul(mul(w.u[d], e), D1(P, w.rho, d));          // u_d e D(rho)
        for (long i = 0; i < N; ++i)
          internal[i] = 0.25 * (t_div[i] + t_rDue[i] + t_uDre[i] + t_eDm[i] + t_mDe[i] + t_reDu[i] + t_ueDr[i]);
      }
      add(C[4], internal);
      for (int a = 0; a < 3; ++a) {
        Field<S> mu = mul(w.m[d], w.u[a]);                      // m_d u_a
        Field<S> k1 = mul(mu, D1(P, w.u[a], d));                // m_d u_a D(u_a)
        Field<S> k2 = mul(w.u[a], D1(P, mu, d));                // u_a D(m_d u_a)
        if (P.split == 5) {
          for (long i = 0; i < N; ++i) C[4][i] += 0.5 * (k1[i] + k2[i]);
        } else {
          Field<S> k3 = mul(w.m[a], D1(P, mul(w.u[d], w.u[a]), d));   // m_a D(u_d u_a)
          Field<S> k4 = mul(mul(w.u[d], w.u[a]), D1(P, w.m[a], d));   // u_d u_a D(m_a)
          for (long i = 0; i < N; ++i) C[4][i] += 0.25 * (k1[i] + k2[i] + k3[i] + k4[i]);
        }
      }
    }
  }

  // Pressure: P_rho = 0, P_{m_a} = D_a p, P_E = sum_d D_d(p u_d).
  Field<S> Pr[5];
  Pr[0].assign(N, S(0.0));
  for (int a = 0; a < 3; ++a) Pr[a + 1] = D1(P, w.p, a);
  Pr[4].assign(N, S(0.0));
  for (int d = 0; d < 3; ++d) {
    if (P.split >= 5) {
      // Kok and KEEP: pressure work split as p D(u_d) + u_d D(p)
      add(Pr[4], mul(w.p, Du[d]));
      add(Pr[4], mul(w.u[d], D1(P, w.p, d)));
    } else {
      add(Pr[4], D1(P, mul(w.p, w.u[d]), d));
    }
  }

  // Viscous and heat-flux terms.
  Field<S> V[5];
  for (int f = 0; f < 5; ++f) V[f].assign(N, S(0.0));
  if (P.viscous) {
    const double ire = 1.0 / P.re;
    Field<S> G[3][3];  // G[a][d] = D_d u_a
    for (int a = 0; a < 3; ++a)
      for (int d = 0; d < 3; ++d) G[a][d] = D1(P, w.u[a], d);
    Field<S> div(N);
    for (long i = 0; i < N; ++i) div[i] = G[0][0][i] + G[1][1][i] + G[2][2][i];
    for (int a = 0; a < 3; ++a) {
      Field<S> lap(N, S(0.0));
      for (int d = 0; d < 3; ++d) add(lap, D2(P, w.u[a], d));
      Field<S> X = D2(P, w.u[a], a);
      for (int d = 0; d < 3; ++d)
        if (d != a) add(X, D1(P, D1(P, w.u[d], d), a));
      for (long i = 0; i < N; ++i) V[a + 1][i] = ire * (lap[i] + X[i] / 3.0);
    }
    // Energy: sum_a u_a V_{m_a} + sum_{a,d} tau_ad G_ad + kappa sum_d D2_d T.
    for (int a = 0; a < 3; ++a) add(V[4], mul(w.u[a], V[a + 1]));
    for (int a = 0; a < 3; ++a)
      for (int d = 0; d < 3; ++d)
        for (long i = 0; i < N; ++i) {
          S tau = ire * (G[a][d][i] + G[d][a][i] - (a == d ? (2.0 / 3.0) * div[i] : S(0.0)));
          V[4][i] += tau * G[a][d][i];
        }
    const double kap = kappa_of(P);
    for (int d = 0; d < 3; ++d) axpy(V[4], kap, D2(P, w.T, d));
  }

  for (int f = 0; f < 5; ++f)
    for (long i = 0; i < N; ++i) r[f * N + i] = -C[f][i] - Pr[f][i] + V[f][i];
}

// Reverse-mode transpose of residual(): qbar += (dR/dQ)^T rbar.  Written by
// walking the forward computation backwards, one statement at a time.
template <class S>
void residual_adjoint(const Params& P, const S* q, const S* rbar, S* qbar) {
  const long N = npts(P);
  Prim<S> w = primitives(P, q);
  const Field<S>* cons[5] = {&w.rho, &w.m[0], &w.m[1], &w.m[2], &w.E};

  Field<S> Rb[5];
  for (int f = 0; f < 5; ++f) Rb[f] = copy_field(rbar + f * N, N);

  // Adjoints of the primitives and conserved variables, accumulated.
  Field<S> consb[5], ub[3], pb(N, S(0.0)), Tb(N, S(0.0));
  for (int f = 0; f < 5; ++f) consb[f].assign(N, S(0.0));
  for (int a = 0; a < 3; ++a) ub[a].assign(N, S(0.0));

  // R_q = -C_q - P_q + V_q.
  Field<S> Cb[5], Pb[5], Vb[5];
  for (int f = 0; f < 5; ++f) {
    Cb[f].resize(N);
    Pb[f].resize(N);
    Vb[f].resize(N);
    for (long i = 0; i < N; ++i) {
      Cb[f][i] = -Rb[f][i];
      Pb[f][i] = -Rb[f][i];
      Vb[f][i] = Rb[f][i];
    }
  }

  // Viscous terms.
  if (P.viscous) {
    const double ire = 1.0 / P.re;
    Field<S> G[3][3];
    for (int a = 0; a < 3; ++a)
      for (int d = 0; d < 3; ++d) G[a][d] = D1(P, w.u[a], d);
    Field<S> div(N);
    for (long i = 0; i < N; ++i) div[i] = G[0][0][i] + G[1][1][i] + G[2][2][i];
    // Recompute V_{m_a} (needed as a coefficient in the energy term).
    Field<S> Vm[3];
    for (int a = 0; a < 3; ++a) {
      Field<S> lap(N, S(0.0));
      for (int d = 0; d < 3; ++d) add(lap, D2(P, w.u[a], d));
      Field<S> X = D2(P, w.u[a], a);
      for (int d = 0; d < 3; ++d)
        if (d != a) add(X, D1(P, D1(P, w.u[d], d), a));
      Vm[a].resize(N);
      for (long i = 0; i < N; ++i) Vm[a][i] = ire * (lap[i] + X[i] / 3.0);
    }
    // V_E = sum_a u_a Vm_a + sum tau_ad G_ad + kappa sum_d D2_d T.
    const Field<S>& VEb = Vb[4];
    const double kap = kappa_of(P);
    for (int d = 0; d < 3; ++d) {
      Field<S> t(N);
      for (long i = 0; i < N; ++i) t[i] = kap * VEb[i];
      add(Tb, D2T(P, t, d));
    }
    Field<S> Gb[3][3];
    for (int a = 0; a < 3; ++a)
      for (int d = 0; d < 3; ++d) Gb[a][d].assign(N, S(0.0));
    Field<S> divb(N, S(0.0));
    for (int a = 0; a < 3; ++a)
      for (int d = 0; d < 3; ++d)
        for (long i = 0; i < N; ++i) {
          S tau = ire * (G[a][d][i] + G[d][a][i] - (a == d ? (2.0 / 3.0) * div[i] : S(0.0)));
          // term tau * G_ad
          S taub = VEb[i] * G[a][d][i];
          Gb[a][d][i] += VEb[i] * tau;
          // tau = ire (G_ad + G_da - 2/3 delta_ad div)
          Gb[a][d][i] += ire * taub;
          Gb[d][a][i] += ire * taub;
          if (a == d) divb[i] += -ire * (2.0 / 3.0) * taub;
        }
    for (long i = 0; i < N; ++i)
      for (int a = 0; a < 3; ++a) Gb[a][a][i] += divb[i];
    // sum_a u_a Vm_a
    Field<S> Vmb[3];
    for (int a = 0; a < 3; ++a) {
      Vmb[a].resize(N);
      for (long i = 0; i < N; ++i) {
        ub[a][i] += VEb[i] * Vm[a][i];
        Vmb[a][i] = Vb[a + 1][i] + VEb[i] * w.u[a][i];
      }
    }
    // Vm_a = ire (lap_a + X_a / 3)
    for (int a = 0; a < 3; ++a) {
      Field<S> lapb(N), Xb(N);
      for (long i = 0; i < N; ++i) {
        lapb[i] = ire * Vmb[a][i];
        Xb[i] = ire * Vmb[a][i] / 3.0;
      }
      for (int d = 0; d < 3; ++d) add(ub[a], D2T(P, lapb, d));
      add(ub[a], D2T(P, Xb, a));
      for (int d = 0; d < 3; ++d)
        if (d != a) add(ub[d], D1T(P, D1T(P, Xb, a), d));
    }
    // G_ad = D_d u_a
    for (int a = 0; a < 3; ++a)
      for (int d = 0; d < 3; ++d) add(ub[a], D1T(P, Gb[a][d], d));
  }

  // Pressure: P_{m_a} = D_a p ; P_E = sum_d D_d(p u_d).
  for (int a = 0; a < 3; ++a) add(pb, D1T(P, Pb[a + 1], a));
  for (int d = 0; d < 3; ++d) {
    Field<S> Fb = D1T(P, Pb[4], d);
    for (long i = 0; i < N; ++i) {
      pb[i] += Fb[i] * w.u[d][i];
      ub[d][i] += Fb[i] * w.p[i];
    }
  }

  // Convection: C_q = 1/2 sum_d [D_d(q u_d) + u_d D_d q + q D_d u_d].
  Field<S> Du[3];
  for (int d = 0; d < 3; ++d) Du[d] = D1(P, w.u[d], d);
  for (int f = 0; f < 5; ++f) {
    for (int d = 0; d < 3; ++d) {
      Field<S> cb(N);
      for (long i = 0; i < N; ++i) cb[i] = 0.5 * Cb[f][i];
      // D_d(q u_d)
      Field<S> Fb = D1T(P, cb, d);
      for (long i = 0; i < N; ++i) {
        consb[f][i] += Fb[i] * w.u[d][i];
        ub[d][i] += Fb[i] * (*cons[f])[i];
      }
      // u_d D_d q
      Field<S> Dq = D1(P, *cons[f], d);
      Field<S> t(N);
      for (long i = 0; i < N; ++i) {
        ub[d][i] += cb[i] * Dq[i];
        t[i] = cb[i] * w.u[d][i];
      }
      add(consb[f], D1T(P, t, d));
      // q D_d u_d
      for (long i = 0; i < N; ++i) {
        consb[f][i] += cb[i] * Du[d][i];
        t[i] = cb[i] * (*cons[f])[i];
      }
      add(ub[d], D1T(P, t, d));
    }
  }

  // Primitives, in reverse: T = gm2 p / rho ; p = (g-1)(E - 1/2 sum m_a u_a) ; u_a = m_a / rho.
  const double gm2 = P.gamma * P.mach * P.mach;
  for (long i = 0; i < N; ++i) {
    pb[i] += gm2 * Tb[i] / w.rho[i];
    consb[0][i] += -gm2 * w.p[i] * Tb[i] / (w.rho[i] * w.rho[i]);
    consb[4][i] += (P.gamma - 1.0) * pb[i];
    for (int a = 0; a < 3; ++a) {
      consb[a + 1][i] += -0.5 * (P.gamma - 1.0) * pb[i] * w.u[a][i];
      ub[a][i] += -0.5 * (P.gamma - 1.0) * pb[i] * w.m[a][i];
    }
    for (int a = 0; a < 3; ++a) {
      consb[a + 1][i] += ub[a][i] / w.rho[i];
      consb[0][i] += -ub[a][i] * w.m[a][i] / (w.rho[i] * w.rho[i]);
    }
  }
  for (int f = 0; f < 5; ++f)
    for (long i = 0; i < N; ++i) qbar[f * N + i] += consb[f][i];
}

// Williamson 2N-storage RK3 coefficients for the update of Sec. 3.1:
// Qt <- A_i Qt + dt R ; Q <- Q + B_i Qt.
const double RK_A[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
const double RK_B[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};

template <class S>
void rk_stage(int stage, double dt, long n5, S* q, S* qt, const S* r) {
  for (long i = 0; i < n5; ++i) {
    S t = (stage == 0) ? S(dt * r[i]) : S(RK_A[stage] * qt[i] + dt * r[i]);
    qt[i] = t;
    q[i] = q[i] + RK_B[stage] * t;
  }
}

// Neumaier compensated summation.
struct Neumaier {
  double s = 0.0, c = 0.0;
  void add(double x) {
    double t = s + x;
    if (std::fabs(s) >= std::fabs(x))
      c += (s - t) + x;
    else
      c += (x - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};

struct NeumaierC {
  Neumaier re, im;
  void add(double x) { re.add(x); }
  void add(cplx x) {
    re.add(x.real());
    im.add(x.imag());
  }
  cplx value() const { return cplx(re.value(), im.value()); }
};

template <class S>
struct Acc;
template <>
struct Acc<double> {
  using type = Neumaier;
};
template <>
struct Acc<cplx> {
  using type = NeumaierC;
};

// Flow integrals (Sec. 4.1, equations for K and eps^S) as volume averages:
//   out[0] K      = <1/2 u_i u_i>
//   out[1] K_rho  = <1/2 rho u_i u_i>
//   out[2] eps^S  = (1/Re) <|omega|^2>, omega = curl u with 4th-order D1
//   out[3..7]     = <rho>, <m1>, <m2>, <m3>, <rho E>
template <class S>
void integrals(const Params& P, const S* q, S* out) {
  const long N = npts(P);
  Prim<S> w = primitives(P, q);
  Field<S> G[3][3];
  for (int a = 0; a < 3; ++a)
    for (int d = 0; d < 3; ++d) G[a][d] = D1(P, w.u[a], d);
  typename Acc<S>::type sk, skr, se, sq[5];
  for (long i = 0; i < N; ++i) {
    S uu = w.u[0][i] * w.u[0][i] + w.u[1][i] * w.u[1][i] + w.u[2][i] * w.u[2][i];
    sk.add(0.5 * uu);
    skr.add(0.5 * w.rho[i] * uu);
    S o1 = G[2][1][i] - G[1][2][i];
    S o2 = G[0][2][i] - G[2][0][i];
    S o3 = G[1][0][i] - G[0][1][i];
    se.add(o1 * o1 + o2 * o2 + o3 * o3);
    for (int f = 0; f < 5; ++f) sq[f].add(q[f * N + i]);
  }
  out[0] = sk.value() / (double)N;
  out[1] = skr.value() / (double)N;
  out[2] = se.value() / ((double)N * P.re);
  for (int f = 0; f < 5; ++f) out[3 + f] = sq[f].value() / (double)N;
}

// qbar += eps_bar * d(eps^S)/dQ.
template <class S>
void integrals_adjoint(const Params& P, const S* q, S eps_bar, S* qbar) {
  const long N = npts(P);
  Prim<S> w = primitives(P, q);
  Field<S> G[3][3];
  for (int a = 0; a < 3; ++a)
    for (int d = 0; d < 3; ++d) G[a][d] = D1(P, w.u[a], d);
  Field<S> Gb[3][3];
  for (int a = 0; a < 3; ++a)
    for (int d = 0; d < 3; ++d) Gb[a][d].assign(N, S(0.0));
  const double scale = 1.0 / ((double)N * P.re);
  for (long i = 0; i < N; ++i) {
    S o1 = G[2][1][i] - G[1][2][i];
    S o2 = G[0][2][i] - G[2][0][i];
    S o3 = G[1][0][i] - G[0][1][i];
    S o1b = eps_bar * scale * 2.0 * o1;
    S o2b = eps_bar * scale * 2.0 * o2;
    S o3b = eps_bar * scale * 2.0 * o3;
    Gb[2][1][i] += o1b;
    Gb[1][2][i] -= o1b;
    Gb[0][2][i] += o2b;
    Gb[2][0][i] -= o2b;
    Gb[1][0][i] += o3b;
    Gb[0][1][i] -= o3b;
  }
  Field<S> ub[3];
  for (int a = 0; a < 3; ++a) {
    ub[a].assign(N, S(0.0));
    for (int d = 0; d < 3; ++d) add(ub[a], D1T(P, Gb[a][d], d));
  }
  for (long i = 0; i < N; ++i)
    for (int a = 0; a < 3; ++a) {
      qbar[(a + 1) * N + i] += ub[a][i] / w.rho[i];
      qbar[i] += -ub[a][i] * w.m[a][i] / (w.rho[i] * w.rho[i]);
    }
}

// Taylor-Green initial condition (Sec. 4.1): velocity and pressure as printed,
// isothermal density rho = gamma M^2 p, then Q = (rho, rho u, rho v, rho w,
// p/(gamma-1) + 1/2 rho |u|^2).
void init(const Params& P, double* q) {
  const long N = npts(P);
  const double gm2 = P.gamma * P.mach * P.mach;
#pragma omp parallel for
  for (int k = 0; k < P.n[2]; ++k)
    for (int j = 0; j < P.n[1]; ++j)
      for (int i = 0; i < P.n[0]; ++i) {
        const double x = i * spacing(P, 0), y = j * spacing(P, 1), z = k * spacing(P, 2);
        const double u = std::sin(x) * std::cos(y) * std::cos(z);
        const double v = -std::cos(x) * std::sin(y) * std::cos(z);
        const double ww = 0.0;
        const double p = 1.0 / gm2 + (1.0 / 16.0) * (std::cos(2 * x) + std::cos(2 * y)) * (2.0 + std::cos(2 * z));
        const double rho = gm2 * p;
        const long id = at(P, i, j, k);
        q[id] = rho;
        q[N + id] = rho * u;
        q[2 * N + id] = rho * v;
        q[3 * N + id] = rho * ww;
        q[4 * N + id] = p / (P.gamma - 1.0) + 0.5 * rho * (u * u + v * v + ww * ww);
      }
}

// Pointwise evaluation of the same residual at one grid point, reading the
// conserved state directly from its neighbourhood.  Used to check sampled
// outputs at grid sizes where the whole-field routine is too slow; it is
// checked against residual() on small grids.
struct PointEval {
  const Params& P;
  const double* q;
  long N;
  double gm2;
  PointEval(const Params& P_, const double* q_) : P(P_), q(q_), N(npts(P_)) {
    gm2 = P.gamma * P.mach * P.mach;
  }
  double cons(int f, int i, int j, int k) const { return q[f * N + at(P, i, j, k)]; }
  double vel(int a, int i, int j, int k) const { return cons(a + 1, i, j, k) / cons(0, i, j, k); }
  double pres(int i, int j, int k) const {
    double ke = 0.0;
    for (int a = 0; a < 3; ++a) ke += cons(a + 1, i, j, k) * vel(a, i, j, k);
    return (P.gamma - 1.0) * (cons(4, i, j, k) - 0.5 * ke);
  }
  double temp(int i, int j, int k) const { return gm2 * pres(i, j, k) / cons(0, i, j, k); }

  // 4th-order stencils applied to a pointwise function F(i, j, k) along axis d.
  template <class F>
  double d1(F f, int d, int i, int j, int k) const {
    auto g = [&](int s) {
      return d == 0 ? f(i + s, j, k) : d == 1 ? f(i, j + s, k) : f(i, j, k + s);
    };
    return (8.0 * (g(1) - g(-1)) - (g(2) - g(-2))) / (12.0 * spacing(P, d));
  }
  template <class F>
  double d2(F f, int d, int i, int j, int k) const {
    auto g = [&](int s) {
      return d == 0 ? f(i + s, j, k) : d == 1 ? f(i, j + s, k) : f(i, j, k + s);
    };
    const double h = spacing(P, d);
    const double g0 = g(0);
    return (16.0 * ((g(1) - g0) + (g(-1) - g0)) - ((g(2) - g0) + (g(-2) - g0))) / (12.0 * h * h);
  }

  void residual_at(int i, int j, int k, double* r) const {
    auto U = [&](int a) { return [this, a](int x, int y, int z) { return vel(a, x, y, z); }; };
    auto Qf = [&](int f) { return [this, f](int x, int y, int z) { return cons(f, x, y, z); }; };
    auto Pf = [this](int x, int y, int z) { return pres(x, y, z); };
    auto Tf = [this](int x, int y, int z) { return temp(x, y, z); };
    double u[3];
    for (int a = 0; a < 3; ++a) u[a] = vel(a, i, j, k);
    double out[5] = {0, 0, 0, 0, 0};
    // phi of conserved component f (rho phi = q_f): 1, u_a, E/rho
    auto phi = [this](int f, int x, int y, int z) {
      return f == 0 ? 1.0 : f < 4 ? vel(f - 1, x, y, z) : cons(4, x, y, z) / cons(0, x, y, z);
    };
    const int nf = P.split >= 5 ? 4 : 5;  // Kok and KEEP: energy below
    for (int f = 0; f < nf; ++f) {
      double C = 0.0;
      for (int d = 0; d < 3; ++d) {
        auto qu = [&, f, d](int x, int y, int z) { return cons(f, x, y, z) * vel(d, x, y, z); };
        if (P.split == 0) {
          C += 0.5 * (d1(qu, d, i, j, k) + u[d] * d1(Qf(f), d, i, j, k) +
                      cons(f, i, j, k) * d1(U(d), d, i, j, k));
          continue;
        }
        // the seven terms of the whole-field residual, at this point
        auto Ph = [&, f](int x, int y, int z) { return phi(f, x, y, z); };
        auto uph = [&, f, d](int x, int y, int z) { return vel(d, x, y, z) * phi(f, x, y, z); };
        const double ph0 = phi(f, i, j, k);
        const double t_div = d1(qu, d, i, j, k);
        const double t_uDq = u[d] * d1(Qf(f), d, i, j, k);
        const double t_qDu = cons(f, i, j, k) * d1(U(d), d, i, j, k);
        const double t_phDm = ph0 * d1(Qf(d + 1), d, i, j, k);
        const double t_mDph = cons(d + 1, i, j, k) * d1(Ph, d, i, j, k);
        const double t_rDuf = cons(0, i, j, k) * d1(uph, d, i, j, k);
        const double t_ufDr = u[d] * ph0 * d1(Qf(0), d, i, j, k);
        if (P.split == 1)
          C += t_div;
        else if (P.split == 2 || P.split == 5)
          C += 0.5 * (t_div + t_phDm + t_mDph);
        else if (P.split == 3)
          C += 0.5 * (t_div + t_rDuf + t_ufDr);
        else
          C += 0.25 * (t_div + t_rDuf + t_uDq + t_phDm + t_mDph + t_qDu + t_ufDr);
      }
      out[f] -= C;
    }
    if (P.split >= 5) {
      // Kok / KEEP energy: internal energy e = p/((gamma-1) rho) by the
      // momentum's pairing, kinetic energy by the split of the two-point flux
      // (mass flux) u_a(left) u_a(right)/2, pressure work p D u_d + u_d D p.
      auto eint = [this](int x, int y, int z) { return pres(x, y, z) / ((P.gamma - 1.0) * cons(0, x, y, z)); };
      const double e0 = eint(i, j, k), rho0 = cons(0, i, j, k);
      double C = 0.0;
      for (int d = 0; d < 3; ++d) {
        auto me = [&, d](int x, int y, int z) { return cons(d + 1, x, y, z) * eint(x, y, z); };
        const double md = cons(d + 1, i, j, k);
        const double Dm = d1(Qf(d + 1), d, i, j, k), De = d1(eint, d, i, j, k);
        if (P.split == 5) {
          C += 0.5 * (d1(me, d, i, j, k) + e0 * Dm + md * De);
        } else {
          auto ue = [&, d](int x, int y, int z) { return vel(d, x, y, z) * eint(x, y, z); };
          auto re = [&](int x, int y, int z) { return pres(x, y, z) / (P.gamma - 1.0); };
          C += 0.25 * (d1(me, d, i, j, k) + rho0 * d1(ue, d, i, j, k) + u[d] * d1(re, d, i, j, k) + e0 * Dm +
                       md * De + rho0 * e0 * d1(U(d), d, i, j, k) + u[d] * e0 * d1(Qf(0), d, i, j, k));
        }
        for (int a = 0; a < 3; ++a) {
          auto mu = [&, d, a](int x, int y, int z) { return cons(d + 1, x, y, z) * vel(a, x, y, z); };
          const double kin = md * u[a] * d1(U(a), d, i, j, k) + u[a] * d1(mu, d, i, j, k);
          if (P.split == 5) {
            C += 0.5 * kin;
          } else {
            auto uu = [&, d, a](int x, int y, int z) { return vel(d, x, y, z) * vel(a, x, y, z); };
            C += 0.25 * (kin + cons(a + 1, i, j, k) * d1(uu, d, i, j, k) + u[d] * u[a] * d1(Qf(a + 1), d, i, j, k));
          }
        }
      }
      out[4] -= C;
    }
    for (int a = 0; a < 3; ++a) out[a + 1] -= d1(Pf, a, i, j, k);
    for (int d = 0; d < 3; ++d) {
      if (P.split >= 5) {
        out[4] -= pres(i, j, k) * d1(U(d), d, i, j, k) + u[d] * d1(Pf, d, i, j, k);
        continue;
      }
      auto pu = [&, d](int x, int y, int z) { return pres(x, y, z) * vel(d, x, y, z); };
      out[4] -= d1(pu, d, i, j, k);
    }
    if (P.viscous) {
      const double ire = 1.0 / P.re;
      double G[3][3];
      for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 3; ++d) G[a][d] = d1(U(a), d, i, j, k);
      const double div = G[0][0] + G[1][1] + G[2][2];
      double Vm[3];
      for (int a = 0; a < 3; ++a) {
        double lap = 0.0;
        for (int d = 0; d < 3; ++d) lap += d2(U(a), d, i, j, k);
        double X = d2(U(a), a, i, j, k);
        for (int d = 0; d < 3; ++d)
          if (d != a) {
            auto dud = [&, d](int x, int y, int z) { return d1(U(d), d, x, y, z); };
            X += d1(dud, a, i, j, k);
          }
        Vm[a] = ire * (lap + X / 3.0);
        out[a + 1] += Vm[a];
      }
      double VE = 0.0;
      for (int a = 0; a < 3; ++a) VE += u[a] * Vm[a];
      for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 3; ++d) {
          double tau = ire * (G[a][d] + G[d][a] - (a == d ? (2.0 / 3.0) * div : 0.0));
          VE += tau * G[a][d];
        }
      const double kap = kappa_of(P);
      for (int d = 0; d < 3; ++d) VE += kap * d2(Tf, d, i, j, k);
      out[4] += VE;
    }
    for (int f = 0; f < 5; ++f) r[f] = out[f];
  }
};

// One full RK3 step: three (residual, stage) pairs.
template <class S>
void step(const Params& P, double dt, S* q, S* qt, S* r) {
  const long n5 = 5 * npts(P);
  for (int s = 0; s < 3; ++s) {
    residual(P, q, r);
    rk_stage(s, dt, n5, q, qt, r);
  }
}

}  // namespace

extern "C" {

void oracle_init(const double* pv, double* q) { init(unpack(pv), q); }

void oracle_residual(const double* pv, const double* q, double* r) {
  residual(unpack(pv), q, r);
}

void oracle_residual_c(const double* pv, const cplx* q, cplx* r) {
  residual(unpack(pv), q, r);
}

// The adjoint is the transpose of the Blaisdell-split residual only: any
// other split form is refused (return -1, qbar untouched).
int oracle_residual_adjoint(const double* pv, const double* q, const double* rbar, double* qbar) {
  const Params P = unpack(pv);
  if (P.split != 0) return -1;
  residual_adjoint(P, q, rbar, qbar);
  return 0;
}

void oracle_rk_stage(int stage, double dt, long n5, double* q, double* qt, const double* r) {
  rk_stage(stage, dt, n5, q, qt, r);
}

void oracle_rk_stage_c(int stage, double dt, long n5, cplx* q, cplx* qt, const cplx* r) {
  rk_stage(stage, dt, n5, q, qt, r);
}

void oracle_integrals(const double* pv, const double* q, double* out8) {
  integrals(unpack(pv), q, out8);
}

void oracle_integrals_c(const double* pv, const cplx* q, cplx* out8) {
  integrals(unpack(pv), q, out8);
}

void oracle_integrals_adjoint(const double* pv, const double* q, double eps_bar, double* qbar) {
  integrals_adjoint(unpack(pv), q, eps_bar, qbar);
}

// Residual at `count` listed points (linear indices into one field);
// out is [count][5].
void oracle_residual_at(const double* pv, const double* q, long count, const long* idx, double* out) {
  Params P = unpack(pv);
  PointEval ev(P, q);
#pragma omp parallel for
  for (long s = 0; s < count; ++s) {
    const long id = idx[s];
    const int i = (int)(id % P.n[0]);
    const int j = (int)((id / P.n[0]) % P.n[1]);
    const int k = (int)(id / ((long)P.n[0] * P.n[1]));
    ev.residual_at(i, j, k, out + 5 * s);
  }
}

// Initial state at `count` listed points; out is [count][5].
void oracle_init_at(const double* pv, long count, const long* idx, double* out) {
  Params P = unpack(pv);
  const double gm2 = P.gamma * P.mach * P.mach;
  for (long s = 0; s < count; ++s) {
    const long id = idx[s];
    const int i = (int)(id % P.n[0]);
    const int j = (int)((id / P.n[0]) % P.n[1]);
    const int k = (int)(id / ((long)P.n[0] * P.n[1]));
    const double x = i * spacing(P, 0), y = j * spacing(P, 1), z = k * spacing(P, 2);
    const double u = std::sin(x) * std::cos(y) * std::cos(z);
    const double v = -std::cos(x) * std::sin(y) * std::cos(z);
    const double p = 1.0 / gm2 + (1.0 / 16.0) * (std::cos(2 * x) + std::cos(2 * y)) * (2.0 + std::cos(2 * z));
    const double rho = gm2 * p;
    out[5 * s + 0] = rho;
    out[5 * s + 1] = rho * u;
    out[5 * s + 2] = rho * v;
    out[5 * s + 3] = 0.0;
    out[5 * s + 4] = p / (P.gamma - 1.0) + 0.5 * rho * (u * u + v * v);
  }
}

void oracle_d1(const double* pv, const double* f, int axis, double* out) {
  Params P = unpack(pv);
  const long N = npts(P);
  Field<double> g = D1(P, Field<double>(f, f + N), axis);
  std::memcpy(out, g.data(), N * sizeof(double));
}

void oracle_d2(const double* pv, const double* f, int axis, double* out) {
  Params P = unpack(pv);
  const long N = npts(P);
  Field<double> g = D2(P, Field<double>(f, f + N), axis);
  std::memcpy(out, g.data(), N * sizeof(double));
}

// Advance `nsteps` full RK3 steps from q (in place).  If hist != nullptr, the
// eight integrals are written every `every` steps starting at step 0
// (hist row m holds the integrals after m*every steps).
void oracle_run(const double* pv, double dt, int nsteps, int every, double* q, double* hist) {
  Params P = unpack(pv);
  const long N = npts(P);
  std::vector<double> qt(5 * N, 0.0), r(5 * N, 0.0);
  int row = 0;
  for (int n = 0; n <= nsteps; ++n) {
    if (hist && every > 0 && n % every == 0) integrals(P, q, hist + 8 * (row++));
    if (n == nsteps) break;
    step(P, dt, q, qt.data(), r.data());
  }
}

void oracle_run_c(const double* pv, double dt, int nsteps, cplx* q) {
  Params P = unpack(pv);
  const long N = npts(P);
  std::vector<cplx> qt(5 * N, 0.0), r(5 * N, 0.0);
  for (int n = 0; n < nsteps; ++n) step(P, dt, q, qt.data(), r.data());
}

// Time-integrated dissipation J = dt sum_{n=0}^{nsteps} w_n eps^S(Q^n)
// (trapezoid weights) for a complex initial state; used for complex-step
// checks of the gradient.
void oracle_dissipation_c(const double* pv, double dt, int nsteps, cplx* q, cplx* J) {
  Params P = unpack(pv);
  const long N = npts(P);
  std::vector<cplx> qt(5 * N, 0.0), r(5 * N, 0.0);
  cplx out[8];
  cplx acc = 0.0;
  for (int n = 0; n <= nsteps; ++n) {
    integrals(P, q, out);
    double wgt = (n == 0 || n == nsteps) ? 0.5 : 1.0;
    acc += dt * wgt * out[2];
    if (n == nsteps) break;
    step(P, dt, q, qt.data(), r.data());
  }
  *J = acc;
}

// Same J in double, plus its gradient with respect to the initial state Q^0
// by store-all reverse mode over the RK3 stages (the reverse of
// Qt^i = A_i Qt^{i-1} + dt R(Q^{i-1}),  Q^i = Q^{i-1} + B_i Qt^i).
int oracle_dissipation_grad(const double* pv, double dt, int nsteps, const double* q0,
                            double* J, double* qbar0) {
  Params P = unpack(pv);
  if (P.split != 0) return -1;  // reverse mode of the Blaisdell form only
  const long N = npts(P), n5 = 5 * N;
  // Stage inputs for every stage of every step.
  std::vector<std::vector<double>> Y((size_t)nsteps * 3 + 1, std::vector<double>());
  std::vector<double> q(q0, q0 + n5), qt(n5, 0.0), r(n5, 0.0);
  double out[8];
  double acc = 0.0;
  for (int n = 0; n <= nsteps; ++n) {
    integrals(P, q.data(), out);
    double wgt = (n == 0 || n == nsteps) ? 0.5 : 1.0;
    acc += dt * wgt * out[2];
    if (n == nsteps) break;
    for (int s = 0; s < 3; ++s) {
      Y[(size_t)n * 3 + s] = q;
      residual(P, q.data(), r.data());
      rk_stage(s, dt, n5, q.data(), qt.data(), r.data());
    }
  }
  Y[(size_t)nsteps * 3] = q;
  *J = acc;
  // Reverse sweep.
  std::vector<double> qb(n5, 0.0), zeta(n5, 0.0), rb(n5, 0.0);
  for (int n = nsteps; n >= 0; --n) {
    const std::vector<double>& Qn = Y[(size_t)n * 3];
    double wgt = (n == 0 || n == nsteps) ? 0.5 : 1.0;
    integrals_adjoint(P, Qn.data(), dt * wgt, qb.data());
    if (n == 0) break;
    // Undo step n-1: stages 2, 1, 0 with stage inputs Y[(n-1)*3 + s].
    std::fill(zeta.begin(), zeta.end(), 0.0);
    for (int s = 2; s >= 0; --s) {
      // Q^s = Q^{s-1} + B_s Qt^s  ->  zeta += B_s qbar (qbar passes through)
      for (long i = 0; i < n5; ++i) zeta[i] += RK_B[s] * qb[i];
      // Qt^s = A_s Qt^{s-1} + dt R(Y)  ->  rbar = dt zeta ; qbar += J_R^T rbar ; zeta = A_s zeta
      for (long i = 0; i < n5; ++i) rb[i] = dt * zeta[i];
      residual_adjoint(P, Y[(size_t)(n - 1) * 3 + s].data(), rb.data(), qb.data());
      for (long i = 0; i < n5; ++i) zeta[i] = RK_A[s] * zeta[i];
    }
  }
  std::memcpy(qbar0, qb.data(), n5 * sizeof(double));
  return 0;
}

}  // extern "C"
