// Fused Navier-Stokes residual R = dQ/dt on a periodic grid (paper Sec. 2.3.1
// scheme and Blaisdell split form, Sec. 3.1 state vector and residual),
// tiled for CDNA4.
//
// Work decomposition.  A block of 64 x TY threads owns a 64 x TY tile of
// (x, y) columns and marches along z over a chunk of planes.  Per plane p it
//   1. loads Q on the tile plus a 2-point halo (coalesced along x; two
//      consecutive x-points per lane and field when nx is even), converts
//      to the arithmetic type Tc and derives the primitive variables once per
//      point into one LDS plane of 10 fields (rho, m1, m2, m3, rho E, u, v, w,
//      p, T);
//   2. evaluates every x- and y-derivative term of R at its own column from
//      LDS (split convective fluxes, pressure, viscous and heat-flux terms,
//      the x-y mixed derivatives, and the part of the viscous work tau : grad u
//      made of in-plane gradients only) and parks that partial R in a
//      thread-private LDS ring; it keeps three gradient combinations in
//      registers: D_x w, D_y w and D_x u + D_y v;
//   3. emits R (or, fused, the RK stage) for plane p - 2: its z-derivative
//      terms come from a 5-plane register window of (rho, m, rho E, 1/rho),
//      from which u, v, w, p and T are re-derived where needed; the z-mixed
//      derivatives of the viscous term are z-differences of the three stored
//      combinations, which are also all that the remaining (in-plane x z) part
//      of tau : grad u needs.
// The z loop is unrolled by the window length (5) so that the window rotates
// by renaming, not by register moves.  The next plane's loads are issued
// before the current plane's arithmetic.  Tiles are ordered x fastest in
// contiguous runs per XCD, so the blocks resident on one XCD cover whole rows
// of tiles and their halo re-reads hit that XCD's L2.  Outputs are streamed
// with the nontemporal hint.  The other split forms of the convective term
// (Sec. 2.3.1, compared in Sec. 4.2) replace the grouped fluxes by a generic
// seven-term combination (split_convection).  Most instances run the
// warp-specialised variant of the same step (residual_ws, below); the kernel
// choice per precision form is made in launch_tiled.
//
// Every 4th-order stencil is taken as S(f) = 8 (f_{+1} - f_{-1}) - (f_{+2} - f_{-2})
// (times 1/(12 h)) and S2(f) = 16 (f_{+1} + f_{-1} - 2 f_0) - (f_{+2} + f_{-2} - 2 f_0)
// (times 1/(12 h^2)).  Flux products are grouped so that each direction d
// needs one stencil per conserved component:
//   rho:        1/2 m_d
//   m_a, a!=d:  1/2 m_a u_d
//   m_d:        1/2 m_d u_d + p          (split flux plus pressure gradient)
//   rho E:      (1/2 rho E + p) u_d      (split flux plus pressure work)
#include <type_traits>

#include "tgv_device.h"
#include "tgv_kernels.h"

namespace tgv {

namespace {

constexpr int TX = 64, TY = 8, NT = TX * TY;
// A 512-thread block is two waves on each of the CU's four SIMDs, so every
// instance has at most 256 VGPRs per lane; of the instances that run this
// kernel, only the fused one with FP64 arithmetic on FP32 storage spills (a
// few registers).
template <class Tc>
constexpr int kWavesPerEU = 2;
// Waves per SIMD the warp-specialised kernel is compiled for.  The fused
// stage with FP16 storage and packed FP16 arithmetic fits two 512-thread
// blocks per CU (59 KB of LDS each) at 128 registers, a few of them spilled:
// 2.13 against 2.22 ms at 512^3; its residual-only instance spills more and
// was slower that way (1.86 against 1.52 ms), so it keeps two waves.
template <class Tq, class Tc, bool FUSED>
constexpr int kWsWaves = kWavesPerEU<Tc>;
template <>
constexpr int kWsWaves<f16, h2, true> = 4;
constexpr int HX = TX + 4, HY = TY + 4, NPL = HX * HY;  // LDS plane incl. halo
// Plane loads in runs of V consecutive x-points per lane (V = 2 when nx is
// even: a run then never crosses the periodic wrap and is V-element aligned).
template <int V>
struct Sr {
  static_assert(HX % V == 0, "a load run must not cross a halo row");
  static constexpr int VPR = HX / V, NVS = NPL / V, LOADS = (NVS + NT - 1) / NT;
};
template <class T, int V>
struct alignas(sizeof(T) * V) Run {
  T e[V];
};
constexpr int NF = 10;
enum { F_RHO = 0, F_M = 1, F_E = 4, F_U = 5, F_P = 8, F_T = 9 };

// Fields kept per plane in the z-window: the conserved variables and 1/rho,
// and for FP32 arithmetic (registers to spare at two waves per SIMD) also u,
// v, w, p and T; the FP64 instances re-derive those five where the
// z-stencils need them, exactly as primitives() derives them.
template <class Tc>
constexpr bool kFullWindow = sizeof(Tc) < 8;
template <class Tc>
constexpr int NW = kFullWindow<Tc> ? 11 : 6;
enum { W_IR = 5 };  // then u, v, w, p, T at 6..10 in the full window

template <class Tc>
struct Ctx {
  // z-window of this column at the last 5 planes
  Tc W[5][NW<Tc>];
  // per plane slot: 0: D_x w, 1: D_y w, 2: D_x u + D_y v
  Tc A[5][3];
};

// Fused stage, forms whose window does not hold Q_in exactly (storage type
// wider than the arithmetic type, as FP64 Q with FP32 arithmetic): Q_in of
// the own column in its storage type, read when its plane arrives (the block
// has just loaded that plane, so the read hits in cache) and kept for the two
// steps until that plane is emitted.  Slot = window slot of the plane.
template <class Tq>
struct QRing {
  Tq v[5][5];
};

// Thread-private ring of in-plane partial residuals in LDS: [3 slots][5][NT].
constexpr int RI_SLOTS = 3;

template <class Tc>
__device__ __forceinline__ Tc S1(Tc m2, Tc m1, Tc p1, Tc p2) {
  return Tc(8) * (p1 - m1) - (p2 - m2);
}
template <class Tc>
__device__ __forceinline__ Tc S2(Tc m2, Tc m1, Tc c, Tc p1, Tc p2) {
  return Tc(16) * ((p1 - c) + (m1 - c)) - ((p2 - c) + (m2 - c));
}

template <class Tc>
__device__ __forceinline__ void primitives(const Tc q[5], Tc* out, const Coef<Tc>& c) {
  const Tc ir = recip(q[0]);
#pragma unroll
  for (int f = 0; f < 5; ++f) out[f] = q[f];
  const Tc u = q[1] * ir, v = q[2] * ir, w = q[3] * ir;
  out[F_U] = u;
  out[F_U + 1] = v;
  out[F_U + 2] = w;
  const Tc p = c.gm1 * (q[4] - Tc(0.5) * (q[1] * u + q[2] * v + q[3] * w));
  out[F_P] = p;
  out[F_T] = c.gm2 * p * ir;
}

// x-neighbour s (0..3 = -2, -1, +1, +2 points) of LDS slot i in a row.  With
// packed FP16 pairs a slot holds two x-points, so the +-2 neighbours are the
// adjacent slots and the +-1 neighbours straddle two slots.
template <class Tc>
__device__ __forceinline__ Tc xnb(const Tc* row, int i, int s) {
  if constexpr (kLanes<Tc> == 1) {
    return row[i + ((s < 2) ? (s - 2) : (s - 1))];
  } else {
    if (s == 0) return row[i - 1];
    if (s == 3) return row[i + 1];
    return s == 1 ? __builtin_shufflevector(row[i - 1], row[i], 1, 2)
                  : __builtin_shufflevector(row[i], row[i + 1], 1, 2);
  }
}

// The four x-neighbours of slot i from per-slot values at i - 1, i, i + 1
// (packed pairs), or at i - 2 .. i + 2 through `at` (one point per slot).
template <class Tc, class F>
__device__ __forceinline__ void xnb4(F at, int i, Tc (&out)[4]) {
  if constexpr (kLanes<Tc> == 1) {
    out[0] = at(i - 2);
    out[1] = at(i - 1);
    out[2] = at(i + 1);
    out[3] = at(i + 2);
  } else {
    const Tc a = at(i - 1), b = at(i), d = at(i + 1);
    out[0] = a;
    out[1] = __builtin_shufflevector(a, b, 1, 2);
    out[2] = __builtin_shufflevector(b, d, 1, 2);
    out[3] = d;
  }
}

// Neighbour accessors: field f at offset index s (0..3 = -2, -1, +1, +2)
// along one direction, from the LDS plane (x, y) or the z-window.
template <class Tc, int STRIDE, int PLANE = NPL>
struct LdsNb {
  const Tc* lds;
  int own;
  __device__ __forceinline__ Tc operator()(int f, int s) const {
    if constexpr (STRIDE == 1) return xnb(lds + f * PLANE, own, s);
    const int o = (s < 2) ? (s - 2) : (s - 1);
    return lds[f * PLANE + own + o * STRIDE];
  }
  // 1/rho at the neighbour (only the non-Blaisdell split forms need it)
  __device__ __forceinline__ Tc ir(int s) const { return recip((*this)(F_RHO, s)); }
};

// The 10 fields of one z-window slot: stored, or re-derived from
// (rho, m, rho E, 1/rho) exactly as primitives() derives them.
template <class Tc, bool FULL = kFullWindow<Tc>>
__device__ __forceinline__ Tc derived(const Tc* w, int f, const Coef<Tc>& c) {
  if (f < 5) return w[f];
  if constexpr (FULL) return w[f + 1];
  if (f < F_P) return w[f - 4] * w[W_IR];
  const Tc u = w[1] * w[W_IR], v = w[2] * w[W_IR], x = w[3] * w[W_IR];
  const Tc p = c.gm1 * (w[4] - Tc(0.5) * (w[1] * u + w[2] * v + w[3] * x));
  return f == F_P ? p : c.gm2 * p * w[W_IR];
}

template <class Tc, int A, int B, int C, int D>
struct WinNb {
  const Tc (&W)[5][NW<Tc>];
  const Coef<Tc>& c;
  __device__ __forceinline__ Tc operator()(int f, int s) const {
    return derived(s == 0 ? W[A] : s == 1 ? W[B] : s == 2 ? W[C] : W[D], f, c);
  }
  __device__ __forceinline__ Tc ir(int s) const { return (s == 0 ? W[A] : s == 1 ? W[B] : s == 2 ? W[C] : W[D])[W_IR]; }
};

// The split forms of the convective term D_d(rho u_d phi), phi = (1, u_a, E/rho)
// for q = rho phi = (rho, m_a, rho E) (Sec. 2.3.1; compared in the inviscid
// limit in Sec. 4.2).  Blaisdell is the grouped, flux-merged code path in
// direction_terms; these are the other forms, built from the seven terms
//   t_div  = D(q u_d)     t_uDq = u_d D(q)     t_qDu  = q D(u_d)
//   t_phDm = phi D(m_d)   t_mDph = m_d D(phi)  t_rDuf = rho D(u_d phi)
//   t_ufDr = u_d phi D(rho)
// combined as: divergence t_div; Feiereisen (t_div + t_phDm + t_mDph)/2;
// Jameson (t_div + t_rDuf + t_ufDr)/2; Kennedy-Gruber-Pirozzoli the sum of all
// seven / 4.  The pressure terms stay in divergence form.
//
// Kok's form (Kok 2009) and KEEP (Kuya, Totani and Kawai 2018) take the
// Feiereisen resp. KGP terms for mass and momentum, and carry the energy as
// internal energy e = p / ((gamma - 1) rho), transported with the same
// pairing, plus kinetic energy in the split whose two-point flux is the mass
// flux times u_a(left) u_a(right) / 2:
//   Kok:  1/2 sum_a [ m_d u_a D(u_a) + u_a D(m_d u_a) ]
//   KEEP: 1/4 sum_a [ m_d u_a D(u_a) + u_a D(m_d u_a) + m_a D(u_d u_a) + u_d u_a D(m_a) ]
// with the pressure work split as p D(u_d) + u_d D(p).
enum {
  SPLIT_BLAISDELL = 0,
  SPLIT_DIVERGENCE = 1,
  SPLIT_FEIEREISEN = 2,
  SPLIT_JAMESON = 3,
  SPLIT_KGP = 4,
  SPLIT_KOK = 5,
  SPLIT_KEEP = 6
};

// Kok / KEEP energy convection and pressure work of direction d (see above).
template <class Tc, int d, int SPLIT, class Nb>
__device__ __forceinline__ Tc kinetic_internal_energy(const Nb& nb, const Tc* c0, Tc ir0, const Coef<Tc>& c,
                                                      const Tc (&ud)[4], const Tc (&rh)[4], const Tc (&md)[4],
                                                      const Tc (&pn)[4], Tc Dud, Tc Drho, Tc Dmd) {
  const Tc u0 = c0[F_U + d], r0 = c0[F_RHO], m0 = c0[F_M + d], p0 = c0[F_P];
  Tc en[4];  // specific internal energy at the neighbours
#pragma unroll
  for (int s = 0; s < 4; ++s) en[s] = pn[s] * nb.ir(s) * c.igm1;
  const Tc e0 = p0 * ir0 * c.igm1;
  const Tc t_div = S1(md[0] * en[0], md[1] * en[1], md[2] * en[2], md[3] * en[3]);
  const Tc t_eDm = e0 * Dmd, t_mDe = m0 * S1(en[0], en[1], en[2], en[3]);
  Tc cv;
  if constexpr (SPLIT == SPLIT_KOK) {
    cv = Tc(0.5) * (t_div + t_eDm + t_mDe);
  } else {
    const Tc t_rDue = r0 * S1(ud[0] * en[0], ud[1] * en[1], ud[2] * en[2], ud[3] * en[3]);
    const Tc t_uDre = u0 * c.igm1 * S1(pn[0], pn[1], pn[2], pn[3]);
    const Tc t_reDu = p0 * c.igm1 * Dud;
    const Tc t_ueDr = u0 * e0 * Drho;
    cv = Tc(0.25) * (t_div + t_rDue + t_uDre + t_eDm + t_mDe + t_reDu + t_ueDr);
  }
  Tc kin = Tc(0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Tc un[4], mu[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      un[s] = (a == d) ? ud[s] : nb(F_U + a, s);
      mu[s] = md[s] * un[s];
    }
    const Tc ua0 = c0[F_U + a];
    const Tc k12 = m0 * ua0 * S1(un[0], un[1], un[2], un[3]) + ua0 * S1(mu[0], mu[1], mu[2], mu[3]);
    if constexpr (SPLIT == SPLIT_KOK) {
      kin += k12;
    } else {
      Tc ma[4], uu[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        ma[s] = (a == d) ? md[s] : nb(F_M + a, s);
        uu[s] = ud[s] * un[s];
      }
      kin += k12 + c0[F_M + a] * S1(uu[0], uu[1], uu[2], uu[3]) + u0 * ua0 * S1(ma[0], ma[1], ma[2], ma[3]);
    }
  }
  cv += (SPLIT == SPLIT_KOK ? Tc(0.5) : Tc(0.25)) * kin;
  // pressure work p D(u_d) + u_d D(p)
  return cv + p0 * Dud + u0 * S1(pn[0], pn[1], pn[2], pn[3]);
}

template <class Tc, int d, int SPLIT, class Nb>
__device__ __forceinline__ void split_convection(const Nb& nb, const Tc* c0, Tc ir0, const Coef<Tc>& c,
                                                 Tc (&R)[5]) {
  const Tc sc1 = c.c1[d];
  Tc ud[4], rh[4], md[4], pn[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    ud[s] = nb(F_U + d, s);
    rh[s] = nb(F_RHO, s);
    md[s] = nb(F_M + d, s);
    pn[s] = nb(F_P, s);
  }
  const Tc u0 = c0[F_U + d], r0 = c0[F_RHO], m0 = c0[F_M + d];
  const Tc Dud = S1(ud[0], ud[1], ud[2], ud[3]);
  const Tc Drho = S1(rh[0], rh[1], rh[2], rh[3]);
  const Tc Dmd = S1(md[0], md[1], md[2], md[3]);
  constexpr bool kEnergyApart = SPLIT == SPLIT_KOK || SPLIT == SPLIT_KEEP;
#pragma unroll
  for (int f = 0; f < (kEnergyApart ? 4 : 5); ++f) {
    Tc qn[4], ph[4], q0, ph0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if (f == 0) {
        qn[s] = rh[s];
        ph[s] = Tc(1);
      } else if (f < 4) {
        qn[s] = nb(F_M + f - 1, s);
        ph[s] = nb(F_U + f - 1, s);
      } else {
        qn[s] = nb(F_E, s);
        ph[s] = qn[s] * nb.ir(s);
      }
    }
    if (f == 0) {
      q0 = r0;
      ph0 = Tc(1);
    } else if (f < 4) {
      q0 = c0[F_M + f - 1];
      ph0 = c0[F_U + f - 1];
    } else {
      q0 = c0[F_E];
      ph0 = c0[F_E] * ir0;
    }
    const Tc t_div = S1(qn[0] * ud[0], qn[1] * ud[1], qn[2] * ud[2], qn[3] * ud[3]);
    Tc cv;
    if constexpr (SPLIT == SPLIT_DIVERGENCE) {
      cv = t_div;
    } else if constexpr (SPLIT == SPLIT_FEIEREISEN || SPLIT == SPLIT_KOK) {
      const Tc t_phDm = ph0 * Dmd, t_mDph = m0 * S1(ph[0], ph[1], ph[2], ph[3]);
      cv = Tc(0.5) * (t_div + t_phDm + t_mDph);
    } else if constexpr (SPLIT == SPLIT_JAMESON) {
      const Tc t_rDuf = r0 * S1(ud[0] * ph[0], ud[1] * ph[1], ud[2] * ph[2], ud[3] * ph[3]);
      const Tc t_ufDr = u0 * ph0 * Drho;
      cv = Tc(0.5) * (t_div + t_rDuf + t_ufDr);
    } else {
      const Tc t_uDq = u0 * S1(qn[0], qn[1], qn[2], qn[3]);
      const Tc t_qDu = q0 * Dud;
      const Tc t_phDm = ph0 * Dmd, t_mDph = m0 * S1(ph[0], ph[1], ph[2], ph[3]);
      const Tc t_rDuf = r0 * S1(ud[0] * ph[0], ud[1] * ph[1], ud[2] * ph[2], ud[3] * ph[3]);
      const Tc t_ufDr = u0 * ph0 * Drho;
      cv = Tc(0.25) * (t_div + t_rDuf + t_uDq + t_phDm + t_mDph + t_qDu + t_ufDr);
    }
    R[f] -= sc1 * cv;
  }
  R[1 + d] -= sc1 * S1(pn[0], pn[1], pn[2], pn[3]);
  if constexpr (kEnergyApart)
    R[4] -= sc1 * kinetic_internal_energy<Tc, d, SPLIT>(nb, c0, ir0, c, ud, rh, md, pn, Dud, Drho, Dmd);
  else
    R[4] -= sc1 * S1(pn[0] * ud[0], pn[1] * ud[1], pn[2] * ud[2], pn[3] * ud[3]);
}

// Convective + pressure + linear viscous terms of direction d at one point:
// adds into R and writes the three gradients D_d u_a.  Neighbour values are
// consumed one field at a time to keep few of them live.
template <class Tc, int d, int SPLIT, class Nb>
__device__ __forceinline__ void direction_terms(const Nb& nb, const Tc* c0, Tc ir0, const Coef<Tc>& c, Tc (&R)[5],
                                                Tc (&G)[3]) {
  const Tc sc1 = c.c1[d];
  const Tc h = Tc(0.5);
  Tc ud[4], pn[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    ud[s] = nb(F_U + d, s);
    pn[s] = nb(F_P, s);
  }
  const Tc Sud = S1(ud[0], ud[1], ud[2], ud[3]);
  if constexpr (SPLIT != SPLIT_BLAISDELL) {
    split_convection<Tc, d, SPLIT>(nb, c0, ir0, c, R);
  } else {
  const Tc hu = h * c0[F_U + d];  // 1/2 u_d at the centre
  const Tc hS = h * Sud;
  // density: flux 1/2 m_d (m_d is read with the momentum below)
  {
    const Tc Sr = S1(nb(F_RHO, 0), nb(F_RHO, 1), nb(F_RHO, 2), nb(F_RHO, 3));
    R[0] -= sc1 * (hu * Sr + c0[F_RHO] * hS);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Tc m[4], F[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      m[s] = nb(F_M + a, s);
      F[s] = (a == d) ? m[s] * (h * ud[s]) + pn[s] : m[s] * (h * ud[s]);
    }
    const Tc Sm = S1(m[0], m[1], m[2], m[3]);
    if (a == d) R[0] -= sc1 * h * Sm;
    R[1 + a] -= sc1 * (S1(F[0], F[1], F[2], F[3]) + hu * Sm + c0[F_M + a] * hS);
  }
  {
    Tc e[4], F[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      e[s] = nb(F_E, s);
      F[s] = (h * e[s] + pn[s]) * ud[s];
    }
    R[4] -= sc1 * (S1(F[0], F[1], F[2], F[3]) + hu * S1(e[0], e[1], e[2], e[3]) + c0[F_E] * hS);
  }
  }
  if (c.viscous) {
    // V_{m_a} gets (1/Re) D2_d u_a, plus (1/Re)(1/3) D2_a u_a for a == d;
    // rho E gets u_a times the same, plus kappa D2_d T.
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      Tc un[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) un[s] = (a == d) ? ud[s] : nb(F_U + a, s);
      G[a] = sc1 * ((a == d) ? Sud : S1(un[0], un[1], un[2], un[3]));
      const Tc v = ((a == d) ? c.vis2l[d] : c.vis2[d]) * S2(un[0], un[1], c0[F_U + a], un[2], un[3]);
      R[1 + a] += v;
      R[4] += c0[F_U + a] * v;
    }
    R[4] += c.kap2[d] * S2(nb(F_T, 0), nb(F_T, 1), c0[F_T], nb(F_T, 2), nb(F_T, 3));
  }
}

template <class Tq, class Tr, class Tc>
struct Kernel {
  Grid g;
  Coef<Tc> c;
  const Tq* __restrict__ q;
  Tr* __restrict__ r;  // residual output (residual-only launch)
};

// Extra arguments of the fused residual + RK stage launch.
template <class Tq, class Tqt, class Ta>
struct RkArgs {
  Tq* __restrict__ q_out;
  Tqt* __restrict__ qt;
  Ta A, B, dt;
  int first;  // stage 0: the register is not read
};

// One z-step with the newest plane in window slot PH.
template <class Tq, class Tr, class Tc, class Tqt, class Ta, bool FUSED, int SPLIT, int V, int PH>
__device__ __forceinline__ void zstep(const Kernel<Tq, Tr, Tc>& K, const RkArgs<Tq, Tqt, Ta>& rk, Ctx<Tc>& cx,
                                      QRing<Tq>& qr,
                                      Tc* lds, Tc* lds_ri, int ri_slot_p, int ri_slot_k,
                                      Tq (&nxt)[Sr<V>::LOADS][V][5], const long long (&off)[Sr<V>::LOADS], int p,
                                      int kout_lo, int kout_hi, bool col_valid, long long col_off, int p_last) {
  constexpr int VPR = Sr<V>::VPR, NVS = Sr<V>::NVS, VLOADS = Sr<V>::LOADS;
  // the window holds Q converted exactly to Tc when Tc is at least as wide as Tq
  constexpr bool kQinFromWindow = sizeof(Tc) >= sizeof(Tq) && std::is_same<Ta, Tc>::value;
  const int tid = threadIdx.x;
  const Grid& g = K.g;
  const Coef<Tc>& c = K.c;
  // register values of the plane emitted in this step, requested early
  const int k = p - 2;
  const bool emit = k >= kout_lo && k < kout_hi;
  Tqt qt_k[5] = {Tqt(), Tqt(), Tqt(), Tqt(), Tqt()};
  if (FUSED && emit && col_valid && !rk.first) {
    const long long id = (long long)k * g.plane + col_off;
#pragma unroll
    for (int f = 0; f < 5; ++f) qt_k[f] = rk.qt[f * g.N + id];
  }
  // 1. primitives of the prefetched plane into LDS
#pragma unroll
  for (int l = 0; l < VLOADS; ++l) {
    const int sv = tid + l * NT;
    if (sv < NVS) {
      const int s0 = (sv / VPR) * HX + (sv % VPR) * V;
#pragma unroll
      for (int e = 0; e < V; ++e) {
        Tc qv[5], f[NF];
#pragma unroll
        for (int m = 0; m < 5; ++m) qv[m] = load_as<Tc>(nxt[l][e][m]);
        primitives(qv, f, c);
#pragma unroll
        for (int k = 0; k < NF; ++k) lds[k * NPL + s0 + e] = f[k];
      }
    }
  }
  __syncthreads();
  if (FUSED && !kQinFromWindow && p >= kout_lo && p < kout_hi && col_valid) {
    const long long id = (long long)p * g.plane + col_off;
#pragma unroll
    for (int f = 0; f < 5; ++f) qr.v[PH][f] = K.q[f * g.N + id];
  }
  // prefetch plane p + 1
  if (p < p_last) {
    int z = p + 1;
    z += (z < 0) ? g.nz : 0;
    z -= (z >= g.nz) ? g.nz : 0;
    const long long zo = (long long)z * g.plane;
#pragma unroll
    for (int l = 0; l < VLOADS; ++l) {
      const int sv = tid + l * NT;
      if (sv < NVS) {
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          const Run<Tq, V> v = *reinterpret_cast<const Run<Tq, V>*>(K.q + f * g.N + zo + off[l]);
#pragma unroll
          for (int e = 0; e < V; ++e) nxt[l][e][f] = v.e[e];
        }
      }
    }
  }
  // 2. in-plane terms of plane p at this column
  const int tx = tid % TX, ty = tid / TX;
  const int own = (ty + 2) * HX + (tx + 2);
  Tc c0[NF];
#pragma unroll
  for (int k = 0; k < NF; ++k) c0[k] = lds[k * NPL + own];
#pragma unroll
  for (int k = 0; k < 5; ++k) cx.W[PH][k] = c0[k];
  cx.W[PH][W_IR] = recip(c0[F_RHO]);
  if constexpr (kFullWindow<Tc>) {
#pragma unroll
    for (int k = F_U; k < NF; ++k) cx.W[PH][k + 1] = c0[k];
  }
  Tc R[5] = {0, 0, 0, 0, 0};
  {
    Tc Gx[3] = {0, 0, 0}, Gy[3] = {0, 0, 0};  // D_x u_a, D_y u_a
    direction_terms<Tc, 0, SPLIT>(LdsNb<Tc, 1>{lds, own}, c0, cx.W[PH][W_IR], c, R, Gx);
    direction_terms<Tc, 1, SPLIT>(LdsNb<Tc, HX>{lds, own}, c0, cx.W[PH][W_IR], c, R, Gy);
    cx.A[PH][0] = Gx[2];
    cx.A[PH][1] = Gy[2];
    cx.A[PH][2] = Gx[0] + Gy[1];
    if (c.viscous) {
      // in-plane part of tau : grad u (times Re):
      //   sum_{a, d in x,y} G_ad^2 + G_xx^2 + G_yy^2 + 2 G_xy G_yx - 2/3 (G_xx + G_yy)^2
      const Tc a3 = cx.A[PH][2];
      const Tc sq = Gx[0] * Gx[0] + Gx[1] * Gx[1] + Gx[2] * Gx[2] + Gy[0] * Gy[0] + Gy[1] * Gy[1] + Gy[2] * Gy[2];
      const Tc cr = Gx[0] * Gx[0] + Gy[1] * Gy[1] + Tc(2) * Gy[0] * Gx[1];
      R[4] += c.ire * (sq + cr - Tc(2.0 / 3.0) * a3 * a3);
    }
  }
  if (c.viscous) {
    // x-y mixed derivatives: X_x += D_x D_y v, X_y += D_y D_x u (corners of the 5 x 5 patch)
    const int offs[4] = {-2, -1, 1, 2};
    Tc iv[4], iu[4];
#pragma unroll
    for (int sy = 0; sy < 4; ++sy) {
      const int row = own + offs[sy] * HX;
      iv[sy] = S1(lds[(F_U + 1) * NPL + row - 2], lds[(F_U + 1) * NPL + row - 1], lds[(F_U + 1) * NPL + row + 1],
                  lds[(F_U + 1) * NPL + row + 2]);
    }
#pragma unroll
    for (int sx = 0; sx < 4; ++sx) {
      const int col = own + offs[sx];
      iu[sx] = S1(lds[F_U * NPL + col - 2 * HX], lds[F_U * NPL + col - HX], lds[F_U * NPL + col + HX],
                  lds[F_U * NPL + col + 2 * HX]);
    }
    const Tc cxy = c.c1[0] * c.c1[1] * c.ire * Tc(1.0 / 3.0);
    const Tc mx = cxy * S1(iv[0], iv[1], iv[2], iv[3]);
    const Tc my = cxy * S1(iu[0], iu[1], iu[2], iu[3]);
    R[1] += mx;
    R[2] += my;
    R[4] += c0[F_U] * mx + c0[F_U + 1] * my;
  }
  {
    Tc* ri = lds_ri + (ri_slot_p * 5) * NT + tid;
#pragma unroll
    for (int f = 0; f < 5; ++f) ri[f * NT] = R[f];
  }

  // 3. emit plane k = p - 2 (window slots: k-2 .. k+2)
  if (emit) {
    constexpr int KM2 = (PH + 1) % 5, KM1 = (PH + 2) % 5, K0 = (PH + 3) % 5, KP1 = (PH + 4) % 5, KP2 = PH;
    Tc Rz[5];
    {
      const Tc* ri = lds_ri + (ri_slot_k * 5) * NT + tid;
#pragma unroll
      for (int f = 0; f < 5; ++f) Rz[f] = ri[f * NT];
    }
    Tc Gz[3] = {0, 0, 0};
    Tc ck[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) ck[f] = derived(cx.W[K0], f, c);
    direction_terms<Tc, 2, SPLIT>(WinNb<Tc, KM2, KM1, KP1, KP2>{cx.W, c}, ck, cx.W[K0][W_IR], c, Rz, Gz);
    if (c.viscous) {
      const Tc* u0 = ck + F_U;
      // z-mixed: X_x += D_z(w_x), X_y += D_z(w_y), X_z += D_z(u_x + v_y)
      const Tc cz = c.c1[2] * c.ire * Tc(1.0 / 3.0);
      const Tc mx = cz * S1(cx.A[KM2][0], cx.A[KM1][0], cx.A[KP1][0], cx.A[KP2][0]);
      const Tc my = cz * S1(cx.A[KM2][1], cx.A[KM1][1], cx.A[KP1][1], cx.A[KP2][1]);
      const Tc mz = cz * S1(cx.A[KM2][2], cx.A[KM1][2], cx.A[KP1][2], cx.A[KP2][2]);
      Rz[1] += mx;
      Rz[2] += my;
      Rz[3] += mz;
      Rz[4] += u0[0] * mx + u0[1] * my + u0[2] * mz;
      // remaining part of tau : grad u (times Re), with G_az = Gz[a]:
      //   sum_a G_az^2 + 2 (G_xz G_zx + G_yz G_zy) + G_zz^2 - 2/3 (2 (G_xx + G_yy) G_zz + G_zz^2)
      const Tc a1 = cx.A[K0][0], a2 = cx.A[K0][1], a3 = cx.A[K0][2];
      const Tc sq = Gz[0] * Gz[0] + Gz[1] * Gz[1] + Gz[2] * Gz[2];
      const Tc cr = Tc(2) * (Gz[0] * a1 + Gz[1] * a2) + Gz[2] * Gz[2];
      Rz[4] += c.ire * (sq + cr - Tc(2.0 / 3.0) * (Tc(2) * a3 + Gz[2]) * Gz[2]);
    }
    if (col_valid) {
      const long long id = (long long)k * g.plane + col_off;
      if (!FUSED) {
#pragma unroll
        for (int f = 0; f < 5; ++f) stream_store(&K.r[f * g.N + id], store_as<Tr>(Rz[f]));
      } else {
        // Q~ <- A Q~ + dt R ; Q_out <- Q_in + B Q~, with R rounded to its
        // storage type as a stored residual would be.  Q_in at this point is
        // the window's centre when that holds it exactly, else the register
        // ring's copy in its storage type.
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          const Ta rr = load_as<Ta>(store_as<Tr>(Rz[f]));
          const Tqt ts = store_as<Tqt>(rk_register<Ta>(rk.first, rk.A, rk.dt, load_as<Ta>(qt_k[f]), rr));
          stream_store(&rk.qt[f * g.N + id], ts);
          Ta qin;
          if constexpr (kQinFromWindow)
            qin = ck[f];
          else
            qin = load_as<Ta>(qr.v[K0][f]);
          stream_store(&rk.q_out[f * g.N + id], store_as<Tq>(rk_state<Ta>(rk.B, qin, load_as<Ta>(ts))));
        }
      }
    }
  }
  // the next plane overwrites the LDS plane
  __syncthreads();
}

// Block order.  Hardware block b runs on XCD b % 8 (round robin); the remap
// gives each XCD a contiguous range of logical tiles.  The logical order walks
// strips kStripPoints wide across x, x fastest within a strip (on grids up to
// that width: rows of tiles, x fastest).  The 32 blocks resident on one XCD
// at a time then cover rows of at most kStripPoints columns, e.g. 2 rows of 16
// tiles of 32 x 8 columns, whose x- and y-halo loads meet in that XCD's L2; on
// a 1024-wide grid a whole row of 32 tiles was resident instead, and the
// stage fetched its Q at the full halo ratio from HBM.
constexpr int kStripPoints = 512;

struct TileIdx {
  int tx, ty, cz;
};

__device__ __forceinline__ TileIdx tile_of_block(int tiles_x, int tiles_y, int tile_w, int remap) {
  const int nb = gridDim.x;
  int b = blockIdx.x;
  if (remap) b = (b % 8) * (nb / 8) + b / 8;
  const int per_chunk = tiles_x * tiles_y;
  TileIdx t;
  t.cz = b / per_chunk;
  const int r = b % per_chunk;
  const int sw = max(1, kStripPoints / tile_w);  // strip width in tiles
  const int full = tiles_x / sw;                 // full-width strips
  if (r < full * sw * tiles_y) {
    const int s = r / (sw * tiles_y), i = r % (sw * tiles_y);
    t.tx = s * sw + i % sw;
    t.ty = i / sw;
  } else {
    const int w = tiles_x - full * sw, i = r - full * sw * tiles_y;
    t.tx = full * sw + i % w;
    t.ty = i / w;
  }
  return t;
}

template <class Tq, class Tr, class Tc, class Tqt, class Ta, bool FUSED, int SPLIT, int V>
__global__ void __launch_bounds__(NT, kWavesPerEU<Tc>) residual_tiled(Kernel<Tq, Tr, Tc> K, RkArgs<Tq, Tqt, Ta> rk, int tiles_x,
                                                     int tiles_y, int kz, int remap) {
  constexpr int VPR = Sr<V>::VPR, NVS = Sr<V>::NVS, VLOADS = Sr<V>::LOADS;
  __shared__ Tc lds[NF * NPL];
  __shared__ Tc lds_ri[RI_SLOTS * 5 * NT];
  const Grid& g = K.g;
  // XCD-aware block order (tile_of_block); at 512^3: 32 resident tiles =
  // 512 x 32 columns, halo fetch 1.16x the tile's own bytes instead of 1.6x
  const TileIdx tt = tile_of_block(tiles_x, tiles_y, TX, remap);
  const int cz = tt.cz;
  const int x0 = tt.tx * TX, y0 = tt.ty * TY;
  const int z0 = cz * kz;
  const int z1 = min(z0 + kz, g.nz);

  const int tid = threadIdx.x;
  // wrapped (x, y) offsets of the plane points this thread loads (fixed over z)
  long long off[VLOADS];
#pragma unroll
  for (int l = 0; l < VLOADS; ++l) {
    const int sv = tid + l * NT;
    const int lx = (sv % VPR) * V, ly = sv / VPR;
    int x = (x0 - 2 + lx) % g.nx;
    x += (x < 0) ? g.nx : 0;
    int y = (y0 - 2 + ly) % g.ny;
    y += (y < 0) ? g.ny : 0;
    off[l] = (long long)y * g.nx + x;
  }
  const int cxg = x0 + tid % TX, cyg = y0 + tid / TX;
  const bool col_valid = cxg < g.nx && cyg < g.ny;
  const long long col_off = (long long)cyg * g.nx + cxg;

  // prefetch the first plane (kept in the storage type until it is
  // converted for LDS a step later: a conversion right after the load would
  // make the wave wait for its data there)
  Tq nxt[VLOADS][V][5];
  {
    int z = z0 - 2;
    z += (z < 0) ? g.nz : 0;
    z -= (z >= g.nz) ? g.nz : 0;
    const long long zo = (long long)z * g.plane;
#pragma unroll
    for (int l = 0; l < VLOADS; ++l) {
      const int sv = tid + l * NT;
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        if (sv < NVS) {
          const Run<Tq, V> v = *reinterpret_cast<const Run<Tq, V>*>(K.q + f * g.N + zo + off[l]);
#pragma unroll
          for (int e = 0; e < V; ++e) nxt[l][e][f] = v.e[e];
        } else {
#pragma unroll
          for (int e = 0; e < V; ++e) nxt[l][e][f] = Tq(1);
        }
      }
    }
  }
  Ctx<Tc> cx;
  QRing<Tq> qr;
  const int p_first = z0 - 2, p_last = z1 + 1;  // planes entering the window
  // plane p = p_first + t sits in RI slot t % 3; the plane emitted with it,
  // p - 2, in slot (t - 2) % 3 = (t + 1) % 3.
  for (int p = p_first, t = 0; p <= p_last; p += 5, t += 5) {
    zstep<Tq, Tr, Tc, Tqt, Ta, FUSED, SPLIT, V, 0>(K, rk, cx, qr, lds, lds_ri, (t + 0) % RI_SLOTS, (t + 0 + 1) % RI_SLOTS, nxt, off, p, z0, z1, col_valid, col_off, p_last);
    if (p + 1 > p_last) break;
    zstep<Tq, Tr, Tc, Tqt, Ta, FUSED, SPLIT, V, 1>(K, rk, cx, qr, lds, lds_ri, (t + 1) % RI_SLOTS, (t + 1 + 1) % RI_SLOTS, nxt, off, p + 1, z0, z1, col_valid, col_off, p_last);
    if (p + 2 > p_last) break;
    zstep<Tq, Tr, Tc, Tqt, Ta, FUSED, SPLIT, V, 2>(K, rk, cx, qr, lds, lds_ri, (t + 2) % RI_SLOTS, (t + 2 + 1) % RI_SLOTS, nxt, off, p + 2, z0, z1, col_valid, col_off, p_last);
    if (p + 3 > p_last) break;
    zstep<Tq, Tr, Tc, Tqt, Ta, FUSED, SPLIT, V, 3>(K, rk, cx, qr, lds, lds_ri, (t + 3) % RI_SLOTS, (t + 3 + 1) % RI_SLOTS, nxt, off, p + 3, z0, z1, col_valid, col_off, p_last);
    if (p + 4 > p_last) break;
    zstep<Tq, Tr, Tc, Tqt, Ta, FUSED, SPLIT, V, 4>(K, rk, cx, qr, lds, lds_ri, (t + 4) % RI_SLOTS, (t + 4 + 1) % RI_SLOTS, nxt, off, p + 4, z0, z1, col_valid, col_off, p_last);
  }
}


// ---------------------------------------------------------------------------
// Warp-specialised variant.  A block of 2 x NCOL threads owns a WTX x WTY
// tile (32 x 8 for FP64 arithmetic, 64 x 8 for FP32): threads [0, NCOL) take the
// in-plane role, threads [NCOL, 2 NCOL) the z role, one column each, so that
// each SIMD holds waves of both kinds and the LDS-heavy in-plane phase of one
// overlaps the arithmetic of the other.  At step t (plane p = p_first + t):
//   in-plane: x/y terms of plane p from LDS buffer t % 2 -> partial R into ring
//             slot t % 4 and the gradient combinations into slot t % 2;
//   z:        primitives of plane p + 1 into LDS buffer (t + 1) % 2, loads of
//             plane p + 2, own column of plane p into window slot t % 6, the
//             combinations of plane p - 1 from the ring, and the emission of
//             plane p - 3 (z terms, z-mixed terms, store or RK stage).
// One barrier per step (double-buffered plane).
// The z role loads the plane in runs of V consecutive x-points per lane (one
// V-element load per field): V = 2 halves the load instructions of the halo
// plane.  A run never crosses the periodic wrap in x and is V-element aligned
// when nx is even (tile origins and the halo width are even); odd nx takes
// V = 1.
// Geometry in LDS slots: a slot is one x-point, or P = 2 consecutive x-points
// for the packed FP16 arithmetic (the tile is then 2 WTX points wide and the
// 2-point halo is one slot).  Loads of the plane go in runs of V slots.
template <int WTX, int WTY, int V = 1, int P = 1>
struct Ws {
  static constexpr int HALO = 2 / P;
  static constexpr int TX = WTX, HX = WTX + 2 * HALO, TY = WTY, NCOL = WTX * WTY, NT = 2 * NCOL, HY = WTY + 4,
                       NPL = HX * HY;
  static_assert(HX % V == 0, "a load run must not cross a halo row");
  static_assert(P == 1 || V == 1, "packed pairs load one slot per run");
  static constexpr int VPR = HX / V, NVS = NPL / V;  // runs per halo row and per plane
  static constexpr int LOADS = (NVS + NCOL - 1) / NCOL;
};
#define TGV_WS_DIMS                                                                          \
  constexpr int WS_P = kLanes<Tc>, WS_HALO = Ws<WTX, WTY, 1, WS_P>::HALO;                    \
  constexpr int WS_TX = Ws<WTX, WTY, 1, WS_P>::TX, WS_HX = Ws<WTX, WTY, 1, WS_P>::HX;       \
  constexpr int WS_TY = Ws<WTX, WTY, 1, WS_P>::TY;                                          \
  constexpr int WS_NCOL = Ws<WTX, WTY, 1, WS_P>::NCOL, WS_NPL = Ws<WTX, WTY, 1, WS_P>::NPL;  \
  (void)WS_TY;                                                                               \
  (void)WS_HALO;
#define TGV_WS_RUNS                                                                          \
  constexpr int WS_VPR = Ws<WTX, WTY, V, WS_P>::VPR, WS_NVS = Ws<WTX, WTY, V, WS_P>::NVS;    \
  constexpr int WS_LOADS = Ws<WTX, WTY, V, WS_P>::LOADS;


// The warp-specialised kernel keeps the reduced window (conserved variables
// and 1/rho) in every precision: its z role has half the registers.
constexpr int NWS = 6;

template <class Tc, int A, int B, int C, int D>
struct WinNb6 {
  const Tc (&W)[6][NWS];
  const Coef<Tc>& c;
  __device__ __forceinline__ Tc operator()(int f, int s) const {
    return derived<Tc, false>(s == 0 ? W[A] : s == 1 ? W[B] : s == 2 ? W[C] : W[D], f, c);
  }
  __device__ __forceinline__ Tc ir(int s) const { return (s == 0 ? W[A] : s == 1 ? W[B] : s == 2 ? W[C] : W[D])[W_IR]; }
};

constexpr int WL = 6;  // z-window length: emission lags the newest plane by 3
constexpr int RR_SLOTS = 4, RA_SLOTS = 2;

template <class Tc>
struct ZCtx {
  Tc W[WL][NWS];
  Tc A[WL][3];
};

template <class Tq>
struct QRing6 {
  Tq v[WL][5];
};

template <class Tc, int SPLIT, int WTX, int WTY>
__device__ __forceinline__ void ip_step(const Coef<Tc>& c, const Tc* lds, Tc* ring_r, Tc* ring_a, int col) {
  TGV_WS_DIMS
  const int tx = col % WS_TX, ty = col / WS_TX;
  const int own = (ty + 2) * WS_HX + (tx + WS_HALO);
  Tc c0[NF];
#pragma unroll
  for (int k = 0; k < NF; ++k) c0[k] = lds[k * WS_NPL + own];
  const Tc ir0 = SPLIT != SPLIT_BLAISDELL ? recip(c0[F_RHO]) : Tc(0);
  Tc R[5] = {0, 0, 0, 0, 0};
  Tc A3[3];
  {
    Tc Gx[3] = {0, 0, 0}, Gy[3] = {0, 0, 0};  // D_x u_a, D_y u_a
    direction_terms<Tc, 0, SPLIT>(LdsNb<Tc, 1, WS_NPL>{lds, own}, c0, ir0, c, R, Gx);
    direction_terms<Tc, 1, SPLIT>(LdsNb<Tc, WS_HX, WS_NPL>{lds, own}, c0, ir0, c, R, Gy);
    A3[0] = Gx[2];
    A3[1] = Gy[2];
    A3[2] = Gx[0] + Gy[1];
    if (c.viscous) {
      const Tc a3 = A3[2];
      const Tc sq = Gx[0] * Gx[0] + Gx[1] * Gx[1] + Gx[2] * Gx[2] + Gy[0] * Gy[0] + Gy[1] * Gy[1] + Gy[2] * Gy[2];
      const Tc cr = Gx[0] * Gx[0] + Gy[1] * Gy[1] + Tc(2) * Gy[0] * Gx[1];
      R[4] += c.ire * (sq + cr - Tc(2.0 / 3.0) * a3 * a3);
    }
  }
  if (c.viscous) {
    // X_x += D_x D_y v: x-differences of v on the rows y +- 1, 2; X_y +=
    // D_y D_x u: y-differences of u at the x-neighbour columns
    const int offs[4] = {-2, -1, 1, 2};
    Tc iv[4], iu[4];
    const Tc* vp = lds + (F_U + 1) * WS_NPL;
    const Tc* up = lds + F_U * WS_NPL;
#pragma unroll
    for (int sy = 0; sy < 4; ++sy) {
      const int row = own + offs[sy] * WS_HX;
      iv[sy] = S1(xnb(vp, row, 0), xnb(vp, row, 1), xnb(vp, row, 2), xnb(vp, row, 3));
    }
    xnb4<Tc>([&](int cl) { return S1(up[cl - 2 * WS_HX], up[cl - WS_HX], up[cl + WS_HX], up[cl + 2 * WS_HX]); },
             own, iu);
    const Tc cxy = c.c1[0] * c.c1[1] * c.ire * Tc(1.0 / 3.0);
    const Tc mx = cxy * S1(iv[0], iv[1], iv[2], iv[3]);
    const Tc my = cxy * S1(iu[0], iu[1], iu[2], iu[3]);
    R[1] += mx;
    R[2] += my;
    R[4] += c0[F_U] * mx + c0[F_U + 1] * my;
  }
#pragma unroll
  for (int f = 0; f < 5; ++f) ring_r[f * WS_NCOL + col] = R[f];
#pragma unroll
  for (int a = 0; a < 3; ++a) ring_a[a * WS_NCOL + col] = A3[a];
}

// Register type of the prefetched plane: the arithmetic type, or for packed
// FP16 pairs the stored pair itself, converted only when the plane is written
// to LDS a step later (a conversion right after the load would make the
// prefetch wait for its data).
template <class Tq, class Tc>
struct NxtOf {
  using type = Tc;
};
template <class Tq>
struct NxtOf<Tq, h2> {
  using type = Run<Tq, 2>;
};
template <>
struct NxtOf<f16, h2> {  // the stored pair is already the lane value
  using type = h2;
};
template <>
struct NxtOf<f16, float> {  // FP16 storage, FP32 arithmetic: converted when written to LDS
  using type = f16;
};
template <>
struct NxtOf<float, double> {  // FP32 storage, FP64 arithmetic: likewise (and half the registers)
  using type = float;
};
template <class Tc, class Tq, int N>
__device__ __forceinline__ typename NxtOf<Tq, Tc>::type nxt_load(const Tq (&e)[N], int i) {
  if constexpr (kLanes<Tc> == 1 && std::is_same<typename NxtOf<Tq, Tc>::type, Tq>::value)
    return e[i];
  else if constexpr (kLanes<Tc> == 1)
    return load_as<Tc>(e[i]);
  else if constexpr (std::is_same<Tq, f16>::value)
    return h2{e[2 * i], e[2 * i + 1]};
  else
    return Run<Tq, 2>{{e[2 * i], e[2 * i + 1]}};
}
template <class Tc, class N>
__device__ __forceinline__ Tc nxt_value(const N& v) {
  if constexpr (kLanes<Tc> == 1 && !std::is_same<N, Tc>::value)
    return load_as<Tc>(v);
  else if constexpr (kLanes<Tc> == 1 || std::is_same<N, h2>::value)
    return v;
  else
    return lane_load<Tc>(v.e);
}
template <class Tc, class Tq>
__device__ __forceinline__ typename NxtOf<Tq, Tc>::type nxt_pad() {
  if constexpr (kLanes<Tc> == 1)
    return typename NxtOf<Tq, Tc>::type(1);
  else if constexpr (std::is_same<Tq, f16>::value)
    return h2{f16(1), f16(1)};
  else
    return Run<Tq, 2>{{Tq(1), Tq(1)}};
}

// Two consecutive values in one nontemporal vector access (packed lanes).
template <class T>
__device__ __forceinline__ void stream_store2(T* p, T a, T b) {
  typedef T V2 __attribute__((ext_vector_type(2)));
  __builtin_nontemporal_store(V2{a, b}, reinterpret_cast<V2*>(p));
}
template <class T>
__device__ __forceinline__ void stream_load2(const T* p, T& a, T& b) {
  typedef T V2 __attribute__((ext_vector_type(2)));
  const V2 v = __builtin_nontemporal_load(reinterpret_cast<const V2*>(p));
  a = v.x;
  b = v.y;
}

template <class Tq, class Tr, class Tc, class Tqt, class Ta, bool FUSED, int SPLIT, int WTX, int WTY, int V, int PH>
__device__ __forceinline__ void z_step(const Kernel<Tq, Tr, Tc>& K, const RkArgs<Tq, Tqt, Ta>& rk, ZCtx<Tc>& zc,
                                       QRing6<Tq>& qr, const Tc* cur, Tc* next, const Tc* ring_r,
                                       const Tc* ring_a_prev, bool have_prev,
                                       typename NxtOf<Tq, Tc>::type (&nxt)[Ws<WTX, WTY, V, kLanes<Tc>>::LOADS][V][5],
                                       const long long (&off)[Ws<WTX, WTY, V, kLanes<Tc>>::LOADS], int p, int z0,
                                       int z1, int p_last, bool col_valid, long long col_off, int zt) {
  TGV_WS_DIMS
  TGV_WS_RUNS
  constexpr int P = WS_P;
  // the window holds Q converted exactly when each point's arithmetic type is
  // at least as wide as its storage type
  constexpr bool kQinFromWindow =
      sizeof(typename LaneT<Tc>::E) >= sizeof(Tq) && (std::is_same<Ta, Tc>::value || P == 2);
  // Q_in of the emitted point otherwise: a register ring of the own column's
  // stored values (one point per lane), or, for packed pairs, re-read at
  // emission (three planes after the block loaded it)
  constexpr bool kQinRing = !kQinFromWindow && P == 1;
  const Grid& g = K.g;
  const Coef<Tc>& c = K.c;
  const int k = p - 3;
  const bool emit = k >= z0 && k < z1;
  Tqt qt_k[5][P];
#pragma unroll
  for (int f = 0; f < 5; ++f)
#pragma unroll
    for (int e = 0; e < P; ++e) qt_k[f][e] = Tqt();
  if (FUSED && emit && col_valid && !rk.first) {
    const long long id = (long long)k * g.plane + col_off;
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      if constexpr (P == 1)
        qt_k[f][0] = stream_load(&rk.qt[f * g.N + id]);
      else
        stream_load2(&rk.qt[f * g.N + id], qt_k[f][0], qt_k[f][1]);
    }
  }
  // packed pairs: Q_in of the emitted points, requested with the register
  Tq qin_k[5][P];
  if constexpr (FUSED && !kQinFromWindow && !kQinRing) {
    if (emit && col_valid) {
      const long long id = (long long)k * g.plane + col_off;
#pragma unroll
      for (int f = 0; f < 5; ++f) {
        const Run<Tq, P> v = *reinterpret_cast<const Run<Tq, P>*>(K.q + f * g.N + id);
#pragma unroll
        for (int e = 0; e < P; ++e) qin_k[f][e] = v.e[e];
      }
    }
  }
  // 1. primitives of plane p + 1 into the other buffer; loads of plane p + 2
  if (p + 1 <= p_last) {
#pragma unroll
    for (int l = 0; l < WS_LOADS; ++l) {
      const int sv = zt + l * WS_NCOL;
      if (sv < WS_NVS) {
        const int s0 = (sv / WS_VPR) * WS_HX + (sv % WS_VPR) * V;
#pragma unroll
        for (int e = 0; e < V; ++e) {
          Tc qv[5], f[NF];
#pragma unroll
          for (int m = 0; m < 5; ++m) qv[m] = nxt_value<Tc>(nxt[l][e][m]);
          primitives(qv, f, c);
#pragma unroll
          for (int m = 0; m < NF; ++m) next[m * WS_NPL + s0 + e] = f[m];
        }
      }
    }
    if (p + 2 <= p_last) {
      int z = p + 2;
      z += (z < 0) ? g.nz : 0;
      z -= (z >= g.nz) ? g.nz : 0;
      const long long zo = (long long)z * g.plane;
#pragma unroll
      for (int l = 0; l < WS_LOADS; ++l) {
        const int sv = zt + l * WS_NCOL;
        if (sv < WS_NVS) {
#pragma unroll
          for (int f = 0; f < 5; ++f) {
            const Run<Tq, V * P> v = *reinterpret_cast<const Run<Tq, V * P>*>(K.q + f * g.N + zo + off[l]);
#pragma unroll
            for (int e = 0; e < V; ++e) nxt[l][e][f] = nxt_load<Tc>(v.e, e);
          }
        }
      }
    }
  }
  // 2. own column of plane p into window slot PH
  if (p <= p_last) {
    const int tx = zt % WS_TX, ty = zt / WS_TX;
    const int own = (ty + 2) * WS_HX + (tx + WS_HALO);
    Tc c0[NF];
#pragma unroll
    for (int m = 0; m < NF; ++m) c0[m] = cur[m * WS_NPL + own];
#pragma unroll
    for (int m = 0; m < 5; ++m) zc.W[PH][m] = c0[m];
    zc.W[PH][W_IR] = recip(c0[F_RHO]);
    if constexpr (FUSED && kQinRing) {
      if (p >= z0 && p < z1 && col_valid) {
        const long long id = (long long)p * g.plane + col_off;
#pragma unroll
        for (int f = 0; f < 5; ++f) qr.v[PH][f] = K.q[f * g.N + id];
      }
    }
  }
  // 3. gradient combinations of plane p - 1
  if (have_prev) {
#pragma unroll
    for (int a = 0; a < 3; ++a) zc.A[(PH + WL - 1) % WL][a] = ring_a_prev[a * WS_NCOL + zt];
  }
  // 4. emit plane k = p - 3 (window slots of k - 2 .. k + 2)
  if (emit) {
    constexpr int KM2 = (PH + 1) % WL, KM1 = (PH + 2) % WL, K0 = (PH + 3) % WL, KP1 = (PH + 4) % WL,
                  KP2 = (PH + 5) % WL;
    Tc Rz[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) Rz[f] = ring_r[f * WS_NCOL + zt];
    Tc Gz[3] = {0, 0, 0};
    Tc ck[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) ck[f] = derived<Tc, false>(zc.W[K0], f, c);
    direction_terms<Tc, 2, SPLIT>(WinNb6<Tc, KM2, KM1, KP1, KP2>{zc.W, c}, ck, zc.W[K0][W_IR], c, Rz, Gz);
    if (c.viscous) {
      const Tc* u0 = ck + F_U;
      const Tc cz = c.c1[2] * c.ire * Tc(1.0 / 3.0);
      const Tc mx = cz * S1(zc.A[KM2][0], zc.A[KM1][0], zc.A[KP1][0], zc.A[KP2][0]);
      const Tc my = cz * S1(zc.A[KM2][1], zc.A[KM1][1], zc.A[KP1][1], zc.A[KP2][1]);
      const Tc mz = cz * S1(zc.A[KM2][2], zc.A[KM1][2], zc.A[KP1][2], zc.A[KP2][2]);
      Rz[1] += mx;
      Rz[2] += my;
      Rz[3] += mz;
      Rz[4] += u0[0] * mx + u0[1] * my + u0[2] * mz;
      const Tc a1 = zc.A[K0][0], a2 = zc.A[K0][1], a3 = zc.A[K0][2];
      const Tc sq = Gz[0] * Gz[0] + Gz[1] * Gz[1] + Gz[2] * Gz[2];
      const Tc cr = Tc(2) * (Gz[0] * a1 + Gz[1] * a2) + Gz[2] * Gz[2];
      Rz[4] += c.ire * (sq + cr - Tc(2.0 / 3.0) * (Tc(2) * a3 + Gz[2]) * Gz[2]);
    }
    if (col_valid) {
      const long long id = (long long)k * g.plane + col_off;
      if (!FUSED) {
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          if constexpr (P == 1)
            stream_store(&K.r[f * g.N + id], store_as<Tr>(Rz[f]));
          else
            stream_store2(&K.r[f * g.N + id], store_as<Tr>(lane_get(Rz[f], 0)), store_as<Tr>(lane_get(Rz[f], 1)));
        }
      } else {
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          Tqt ts[P];
          Tq qo[P];
#pragma unroll
          for (int e = 0; e < P; ++e) {
            const Ta rr = load_as<Ta>(store_as<Tr>(lane_get(Rz[f], e)));
            ts[e] = store_as<Tqt>(rk_register<Ta>(rk.first, rk.A, rk.dt, load_as<Ta>(qt_k[f][e]), rr));
            Ta qin;
            if constexpr (kQinFromWindow)
              qin = load_as<Ta>(lane_get(ck[f], e));
            else if constexpr (kQinRing)
              qin = load_as<Ta>(qr.v[K0][f]);
            else
              qin = load_as<Ta>(qin_k[f][e]);
            qo[e] = store_as<Tq>(rk_state<Ta>(rk.B, qin, load_as<Ta>(ts[e])));
          }
          if constexpr (P == 1) {
            stream_store(&rk.qt[f * g.N + id], ts[0]);
            stream_store(&rk.q_out[f * g.N + id], qo[0]);
          } else {
            stream_store2(&rk.qt[f * g.N + id], ts[0], ts[1]);
            stream_store2(&rk.q_out[f * g.N + id], qo[0], qo[1]);
          }
        }
      }
    }
  }
}

template <class Tq, class Tr, class Tc, class Tqt, class Ta, bool FUSED, int SPLIT, int WTX, int WTY, int V>
__global__ void __launch_bounds__((Ws<WTX, WTY>::NT), (kWsWaves<Tq, Tc, FUSED>)) residual_ws(Kernel<Tq, Tr, Tc> K, RkArgs<Tq, Tqt, Ta> rk,
                                                                      int tiles_x, int tiles_y, int kz, int remap) {
  TGV_WS_DIMS
  TGV_WS_RUNS
  __shared__ Tc lds[2][NF * WS_NPL];
  __shared__ Tc ring_r[RR_SLOTS][5 * WS_NCOL];
  __shared__ Tc ring_a[RA_SLOTS][3 * WS_NCOL];
  const Grid& g = K.g;
  const TileIdx tt = tile_of_block(tiles_x, tiles_y, WS_TX * WS_P, remap);
  const int cz = tt.cz;
  const int x0 = tt.tx * WS_TX * WS_P, y0 = tt.ty * WS_TY;  // in grid points
  const int z0 = cz * kz;
  const int z1 = min(z0 + kz, g.nz);
  const bool zrole = threadIdx.x >= WS_NCOL;
  const int col = zrole ? threadIdx.x - WS_NCOL : threadIdx.x;

  long long off[WS_LOADS];
#pragma unroll
  for (int l = 0; l < WS_LOADS; ++l) {
    const int sv = col + l * WS_NCOL;
    const int lx = (sv % WS_VPR) * V * WS_P, ly = sv / WS_VPR;
    int x = (x0 - 2 + lx) % g.nx;
    x += (x < 0) ? g.nx : 0;
    int y = (y0 - 2 + ly) % g.ny;
    y += (y < 0) ? g.ny : 0;
    off[l] = (long long)y * g.nx + x;
  }
  const int cxg = x0 + (col % WS_TX) * WS_P, cyg = y0 + col / WS_TX;
  const bool col_valid = cxg < g.nx && cyg < g.ny;  // nx is even for pairs: both points in the grid
  const long long col_off = (long long)cyg * g.nx + cxg;
  const int p_first = z0 - 2, p_last = z1 + 1;  // planes entering the window
  typename NxtOf<Tq, Tc>::type nxt[WS_LOADS][V][5];
  if (zrole) {
    // plane p_first into buffer 0, plane p_first + 1 into registers
    for (int h = 0; h < 2; ++h) {
      int z = p_first + h;
      z += (z < 0) ? g.nz : 0;
      z -= (z >= g.nz) ? g.nz : 0;
      const long long zo = (long long)z * g.plane;
#pragma unroll
      for (int l = 0; l < WS_LOADS; ++l) {
        const int sv = col + l * WS_NCOL;
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          Run<Tq, V * WS_P> v;
          if (sv < WS_NVS) v = *reinterpret_cast<const Run<Tq, V * WS_P>*>(K.q + f * g.N + zo + off[l]);
#pragma unroll
          for (int e = 0; e < V; ++e) nxt[l][e][f] = sv < WS_NVS ? nxt_load<Tc>(v.e, e) : nxt_pad<Tc, Tq>();
        }
      }
      if (h == 0) {
#pragma unroll
        for (int l = 0; l < WS_LOADS; ++l) {
          const int sv = col + l * WS_NCOL;
          if (sv < WS_NVS) {
            const int s0 = (sv / WS_VPR) * WS_HX + (sv % WS_VPR) * V;
#pragma unroll
            for (int e = 0; e < V; ++e) {
              Tc qv[5], f[NF];
#pragma unroll
              for (int m = 0; m < 5; ++m) qv[m] = nxt_value<Tc>(nxt[l][e][m]);
              primitives(qv, f, K.c);
#pragma unroll
              for (int m = 0; m < NF; ++m) lds[0][m * WS_NPL + s0 + e] = f[m];
            }
          }
        }
      }
    }
  }
  __syncthreads();
  ZCtx<Tc> zc;
  QRing6<Tq> qr;
  const int T = p_last + 1 - p_first + 1;  // one more step than planes: the last emission
#define TGV_WS_STEP(PH)                                                                                          \
  {                                                                                                              \
    const int tt = t + PH, pp = p_first + tt;                                                                    \
    if (!zrole) {                                                                                                \
      if (pp <= p_last) ip_step<Tc, SPLIT, WTX, WTY>(K.c, lds[tt % 2], ring_r[tt % RR_SLOTS], ring_a[tt % RA_SLOTS], col); \
    } else {                                                                                                     \
      z_step<Tq, Tr, Tc, Tqt, Ta, FUSED, SPLIT, WTX, WTY, V, PH>(K, rk, zc, qr, lds[tt % 2], lds[(tt + 1) % 2],              \
                                                    ring_r[(tt + 1) % RR_SLOTS], ring_a[(tt + 1) % RA_SLOTS],    \
                                                    tt >= 1, nxt, off, pp, z0, z1, p_last, col_valid, col_off, col); \
    }                                                                                                            \
    __syncthreads();                                                                                             \
  }
  for (int t = 0; t < T; t += WL) {
    TGV_WS_STEP(0)
    if (t + 1 >= T) break;
    TGV_WS_STEP(1)
    if (t + 2 >= T) break;
    TGV_WS_STEP(2)
    if (t + 3 >= T) break;
    TGV_WS_STEP(3)
    if (t + 4 >= T) break;
    TGV_WS_STEP(4)
    if (t + 5 >= T) break;
    TGV_WS_STEP(5)
  }
#undef TGV_WS_STEP
}

struct TileLaunch {
  int tiles_x, tiles_y, kz;
  long long blocks;
};

// Planes per block: long z-marches amortise the 4 halo planes a block loads
// at its ends, but the grid must still hold enough blocks to fill the chip
// several times over.
TileLaunch tile_launch(const Grid& g, int tx, int ty) {
  TileLaunch L;
  L.tiles_x = (g.nx + tx - 1) / tx;
  L.tiles_y = (g.ny + ty - 1) / ty;
  L.kz = 512;
  while (L.kz > 16 && (long long)L.tiles_x * L.tiles_y * ((g.nz + L.kz - 1) / L.kz) < 1024) L.kz /= 2;
  L.blocks = (long long)L.tiles_x * L.tiles_y * ((g.nz + L.kz - 1) / L.kz);
  return L;
}

}  // namespace

// Packed FP16 tile: 32 x 8 lanes of two x-points (64 x 8 grid points), two
// roles of 256 threads at two waves per SIMD (with 32 x 16 lanes and 128
// registers the kernel spills 18-22 of them).
constexpr int kH2Tx = 32, kH2Ty = 8;

long long residual_work_items(const Grid& g) {
  // the launch geometries: warp-specialised 32 x 8 (512 threads), 64 x 8
  // (1024 threads) and packed 64 x 16 points (1024 threads), single-role
  // 64 x 8 (512 threads)
  const long long a = tile_launch(g, 32, 8).blocks * Ws<32, 8>::NT;
  const long long b = tile_launch(g, 64, 8).blocks * Ws<64, 8>::NT;
  const long long c = tile_launch(g, TX, TY).blocks * NT;
  const long long d = tile_launch(g, 2 * kH2Tx, kH2Ty).blocks * Ws<kH2Tx, kH2Ty>::NT;
  const long long m = a > b ? (a > c ? a : c) : (b > c ? b : c);
  return m > d ? m : d;
}

// FP16 arithmetic coefficients as packed pairs.
Coef<h2> splat(const Coef<f16>& c) {
  Coef<h2> o;
  auto sp = [](f16 v) { return h2{v, v}; };
  for (int d = 0; d < 3; ++d) {
    o.c1[d] = sp(c.c1[d]);
    o.c2[d] = sp(c.c2[d]);
    o.vis2[d] = sp(c.vis2[d]);
    o.vis2l[d] = sp(c.vis2l[d]);
    o.kap2[d] = sp(c.kap2[d]);
  }
  o.gm1 = sp(c.gm1);
  o.igm1 = sp(c.igm1);
  o.gm2 = sp(c.gm2);
  o.ire = sp(c.ire);
  o.kap = sp(c.kap);
  o.viscous = c.viscous;
  return o;
}

template <class Tq, class Tr, class Tc, class Tqt, class Ta, bool FUSED, int SPLIT>
hipError_t launch_tiled(const Grid& g, const Coef<Tc>& c, const void* q, void* r, const RkArgs<Tq, Tqt, Ta>& rk,
                        hipStream_t st) {
  // Kernel choice (measured at 512^3 and 1024^3): the warp-specialised
  // kernel, on 32 x 8 tiles for FP64 arithmetic (256 columns per role, as
  // many as the registers allow; a 36 x 12 plane has fewer halo points to
  // load and convert than 68 x 8) and 64 x 8 tiles for FP32 arithmetic; the
  // single-role kernel for the fused stage with FP64 Q and FP32 arithmetic,
  // where it is faster (its Q_in ring does not fit the z role's registers).
  // FP32 Q with FP64 arithmetic runs the warp-specialised kernel on FP64
  // geometry, its prefetched plane held in FP32 until written to LDS.
  if constexpr (std::is_same<Tc, f16>::value) {
    // FP16 arithmetic: packed pairs of x-points in the warp-specialised
    // kernel when nx is even (pairs never cross the periodic wrap and are
    // aligned); one point per lane otherwise.
    if (g.nx % 2 == 0) {
      const TileLaunch L = tile_launch(g, 2 * kH2Tx, kH2Ty);
      const int remap = L.blocks % 8 == 0 ? 1 : 0;
      Kernel<Tq, Tr, h2> K{g, splat(c), static_cast<const Tq*>(q), static_cast<Tr*>(r)};
      hipLaunchKernelGGL((residual_ws<Tq, Tr, h2, Tqt, Ta, FUSED, SPLIT, kH2Tx, kH2Ty, 1>), dim3((unsigned)L.blocks),
                         dim3(Ws<kH2Tx, kH2Ty>::NT), 0, st, K, rk, L.tiles_x, L.tiles_y, L.kz, remap);
      return hipGetLastError();
    }
  }
  constexpr bool kQinExact = sizeof(Tc) >= sizeof(Tq) && std::is_same<Ta, Tc>::value;
  constexpr bool kWs = !(FUSED && !kQinExact && sizeof(Tc) < 8);
  constexpr int kWtx = sizeof(Tc) == 8 ? 32 : 64, kWty = 8;
  constexpr int kTx = kWs ? kWtx : TX, kTy = kWs ? kWty : TY;
  const TileLaunch L = tile_launch(g, kTx, kTy);
  const int tiles_x = L.tiles_x, tiles_y = L.tiles_y, kz = L.kz;
  const long long nb = L.blocks;
  const int remap = nb % 8 == 0 ? 1 : 0;
  Kernel<Tq, Tr, Tc> K{g, c, static_cast<const Tq*>(q), static_cast<Tr*>(r)};
  if constexpr (kWs) {
    // Paired halo loads (V = 2) for FP64 arithmetic only: the fused stage
    // gains 1-4 % (bitwise the same results); the FP32-arithmetic instances
    // run 2-12 % slower with them (a few spilled registers) and keep V = 1.
    // The single-role kernel below takes pairs in every form it runs (SPDP
    // fused 2 %, SP_DPC 3.5 % faster).
    constexpr bool kPairs = sizeof(Tc) == 8 || std::is_same<Tq, f16>::value;
    if (kPairs && g.nx % 2 == 0)
      hipLaunchKernelGGL((residual_ws<Tq, Tr, Tc, Tqt, Ta, FUSED, SPLIT, kWtx, kWty, kPairs ? 2 : 1>),
                         dim3((unsigned)nb), dim3(Ws<kWtx, kWty>::NT), 0, st, K, rk, tiles_x, tiles_y, kz, remap);
    else
      hipLaunchKernelGGL((residual_ws<Tq, Tr, Tc, Tqt, Ta, FUSED, SPLIT, kWtx, kWty, 1>), dim3((unsigned)nb),
                         dim3(Ws<kWtx, kWty>::NT), 0, st, K, rk, tiles_x, tiles_y, kz, remap);
  } else {
    if (g.nx % 2 == 0)
      hipLaunchKernelGGL((residual_tiled<Tq, Tr, Tc, Tqt, Ta, FUSED, SPLIT, 2>), dim3((unsigned)nb), dim3(NT), 0, st,
                         K, rk, tiles_x, tiles_y, kz, remap);
    else
      hipLaunchKernelGGL((residual_tiled<Tq, Tr, Tc, Tqt, Ta, FUSED, SPLIT, 1>), dim3((unsigned)nb), dim3(NT), 0, st,
                         K, rk, tiles_x, tiles_y, kz, remap);
  }
  return hipGetLastError();
}

// The non-Blaisdell split forms are instantiated for the FP64 and the
// half-single forms only (the pair the paper compares them in).
template <class Tq, class Tr, class Tc>
constexpr bool kAllSplits = (std::is_same<Tq, double>::value && std::is_same<Tr, double>::value &&
                             std::is_same<Tc, double>::value) ||
                            (std::is_same<Tq, float>::value && std::is_same<Tr, f16>::value &&
                             std::is_same<Tc, float>::value);

template <class Tq, class Tr, class Tc, class Tqt, class Ta, bool FUSED>
hipError_t launch_split(int split, const Grid& g, const Coef<Tc>& c, const void* q, void* r,
                        const RkArgs<Tq, Tqt, Ta>& rk, hipStream_t st) {
  if (split == SPLIT_BLAISDELL) return launch_tiled<Tq, Tr, Tc, Tqt, Ta, FUSED, SPLIT_BLAISDELL>(g, c, q, r, rk, st);
  if constexpr (kAllSplits<Tq, Tr, Tc>) {
    switch (split) {
      case SPLIT_DIVERGENCE: return launch_tiled<Tq, Tr, Tc, Tqt, Ta, FUSED, SPLIT_DIVERGENCE>(g, c, q, r, rk, st);
      case SPLIT_FEIEREISEN: return launch_tiled<Tq, Tr, Tc, Tqt, Ta, FUSED, SPLIT_FEIEREISEN>(g, c, q, r, rk, st);
      case SPLIT_JAMESON: return launch_tiled<Tq, Tr, Tc, Tqt, Ta, FUSED, SPLIT_JAMESON>(g, c, q, r, rk, st);
      case SPLIT_KGP: return launch_tiled<Tq, Tr, Tc, Tqt, Ta, FUSED, SPLIT_KGP>(g, c, q, r, rk, st);
      case SPLIT_KOK: return launch_tiled<Tq, Tr, Tc, Tqt, Ta, FUSED, SPLIT_KOK>(g, c, q, r, rk, st);
      case SPLIT_KEEP: return launch_tiled<Tq, Tr, Tc, Tqt, Ta, FUSED, SPLIT_KEEP>(g, c, q, r, rk, st);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

template <class Tq, class Tr, class Tc>
hipError_t launch_residual(const Grid& g, const Coef<Tc>& c, int split, const void* q, void* r, hipStream_t st) {
  // (the stage arguments are unused; their arithmetic type is FP32 for FP16 arithmetic)
  using Ta = typename std::conditional<std::is_same<Tc, f16>::value, float, Tc>::type;
  const RkArgs<Tq, Tq, Ta> none{nullptr, nullptr, Ta(0), Ta(0), Ta(0), 1};
  return launch_split<Tq, Tr, Tc, Tq, Ta, false>(split, g, c, q, r, none, st);
}

template <class Tq, class Tqt, class Tr, class Tc, class Ta>
hipError_t launch_residual_rk(const Grid& g, const Coef<Tc>& c, int split, int stage, double dt, const void* q_in,
                              void* q_out, void* qt, hipStream_t st) {
  static const double kA[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
  static const double kB[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
  const RkArgs<Tq, Tqt, Ta> rk{static_cast<Tq*>(q_out), static_cast<Tqt*>(qt), (Ta)kA[stage], (Ta)kB[stage],
                               (Ta)dt, stage == 0 ? 1 : 0};
  return launch_split<Tq, Tr, Tc, Tqt, Ta, true>(split, g, c, q_in, nullptr, rk, st);
}

#define TGV_INST_RES(Tq, Tr, Tc) \
  template hipError_t launch_residual<Tq, Tr, Tc>(const Grid&, const Coef<Tc>&, int, const void*, void*, hipStream_t);
TGV_INST_RES(double, double, double)
TGV_INST_RES(double, float, float)
TGV_INST_RES(double, float, double)
TGV_INST_RES(float, float, double)
TGV_INST_RES(float, float, float)
TGV_INST_RES(float, f16, float)
TGV_INST_RES(float, bf16, float)
TGV_INST_RES(f16, f16, float)
TGV_INST_RES(double, double, float)
TGV_INST_RES(float, float, f16)
TGV_INST_RES(float, f16, f16)
TGV_INST_RES(f16, f16, f16)

#define TGV_INST_RRK(Tq, Tqt, Tr, Tc, Ta)                                                                     \
  template hipError_t launch_residual_rk<Tq, Tqt, Tr, Tc, Ta>(const Grid&, const Coef<Tc>&, int, int, double,\
                                                              const void*, void*, void*, hipStream_t);
TGV_INST_RRK(double, double, double, double, double)
TGV_INST_RRK(double, double, float, float, double)
TGV_INST_RRK(double, double, float, double, double)
TGV_INST_RRK(float, float, float, double, double)
TGV_INST_RRK(float, float, float, float, float)
TGV_INST_RRK(float, float, f16, float, float)
TGV_INST_RRK(float, float, bf16, float, float)
TGV_INST_RRK(f16, f16, f16, float, float)
TGV_INST_RRK(double, double, double, float, double)
TGV_INST_RRK(float, float, float, f16, float)
TGV_INST_RRK(float, float, f16, f16, float)
TGV_INST_RRK(f16, f16, f16, f16, float)

}  // namespace tgv
