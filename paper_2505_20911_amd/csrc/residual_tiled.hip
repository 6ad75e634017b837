// Fused Navier-Stokes residual R = dQ/dt on a periodic grid (paper Sec. 2.3.1
// scheme and Blaisdell split form, Sec. 3.1 state vector and residual),
// tiled for CDNA4.
//
// Work decomposition.  A 256-thread block owns a 64 x 4 tile of (x, y)
// columns and marches along z over a chunk of planes.  Per plane p it
//   1. loads Q on the tile plus a 2-point halo (68 x 8 points, coalesced
//      along x), converts to the arithmetic type Tc and derives the
//      primitive variables once per point into one LDS plane of 10 fields
//      (rho, m1, m2, m3, rho E, u, v, w, p, T);
//   2. evaluates every x- and y-derivative term of R at its own column from
//      LDS (split convective fluxes, pressure, viscous and heat-flux terms,
//      the x-y mixed derivatives) and keeps the result, plus the six
//      in-plane velocity gradients, in registers;
//   3. emits R for plane p - 2: its z-derivative terms come from a 5-plane
//      register window of the 10 fields, the z-mixed derivatives are
//      z-differences of the stored in-plane gradients, and the viscous work
//      tau : grad u needs all nine gradients at once.
// The z loop is unrolled by the window length (5) so that the window rotates
// by renaming, not by register moves.  The next plane's loads are issued
// before the current plane's arithmetic.  Tiles are ordered so that
// y-neighbours (which share halo rows) run on the same XCD, whose L2 then
// serves the halo re-reads.
//
// Every 4th-order stencil is taken as S(f) = 8 (f_{+1} - f_{-1}) - (f_{+2} - f_{-2})
// (times 1/(12 h)) and S2(f) = 16 (f_{+1} + f_{-1} - 2 f_0) - (f_{+2} + f_{-2} - 2 f_0)
// (times 1/(12 h^2)).  Flux products are grouped so that each direction d
// needs one stencil per conserved component:
//   rho:        1/2 m_d
//   m_a, a!=d:  1/2 m_a u_d
//   m_d:        1/2 m_d u_d + p          (split flux plus pressure gradient)
//   rho E:      (1/2 rho E + p) u_d      (split flux plus pressure work)
#include "tgv_device.h"
#include "tgv_kernels.h"

namespace tgv {

namespace {

constexpr int TX = 64, TY = 4, NT = TX * TY;
constexpr int HX = TX + 4, HY = TY + 4, NPL = HX * HY;  // LDS plane incl. halo
constexpr int LOADS = (NPL + NT - 1) / NT;              // plane points per thread
constexpr int NF = 10;
enum { F_RHO = 0, F_M = 1, F_E = 4, F_U = 5, F_P = 8, F_T = 9 };
constexpr int KZ = 64;  // planes per block

template <class Tc>
struct Ctx {
  // z-window: the 10 fields of this column at the last 5 planes
  Tc W[5][NF];
  // in-plane velocity gradients G[a][d] (d = x, y) per plane slot:
  // 0: u_x 1: u_y 2: v_x 3: v_y 4: w_x 5: w_y
  Tc GI[5][6];
  // in-plane part of R per plane slot
  Tc RI[5][5];
};

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
  const Tc ir = Tc(1) / q[0];
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

// Neighbour accessors: field f at offset index s (0..3 = -2, -1, +1, +2)
// along one direction, from the LDS plane (x, y) or the z-window.
template <class Tc, int STRIDE>
struct LdsNb {
  const Tc* lds;
  int own;
  __device__ __forceinline__ Tc operator()(int f, int s) const {
    const int o = (s < 2) ? (s - 2) : (s - 1);
    return lds[f * NPL + own + o * STRIDE];
  }
};

template <class Tc, int A, int B, int C, int D>
struct WinNb {
  const Tc (&W)[5][NF];
  __device__ __forceinline__ Tc operator()(int f, int s) const {
    return s == 0 ? W[A][f] : s == 1 ? W[B][f] : s == 2 ? W[C][f] : W[D][f];
  }
};

// Convective + pressure + linear viscous terms of direction d at one point:
// adds into R and writes the three gradients D_d u_a.  Neighbour values are
// consumed one field at a time to keep few of them live.
template <class Tc, int d, class Nb>
__device__ __forceinline__ void direction_terms(const Nb& nb, const Tc* c0, const Coef<Tc>& c, Tc sc1, Tc sc2,
                                                Tc (&R)[5], Tc (&G)[3]) {
  const Tc h = Tc(0.5);
  Tc ud[4], pn[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    ud[s] = nb(F_U + d, s);
    pn[s] = nb(F_P, s);
  }
  const Tc Sud = S1(ud[0], ud[1], ud[2], ud[3]);
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
  if (c.viscous) {
    // V_{m_a} gets (1/Re) D2_d u_a, plus (1/Re)(1/3) D2_a u_a for a == d;
    // rho E gets u_a times the same, plus kappa D2_d T.
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      Tc un[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) un[s] = (a == d) ? ud[s] : nb(F_U + a, s);
      G[a] = sc1 * ((a == d) ? Sud : S1(un[0], un[1], un[2], un[3]));
      const Tc l = sc2 * S2(un[0], un[1], c0[F_U + a], un[2], un[3]);
      const Tc v = (a == d) ? c.ire * Tc(4.0 / 3.0) * l : c.ire * l;
      R[1 + a] += v;
      R[4] += c0[F_U + a] * v;
    }
    R[4] += c.kap * sc2 * S2(nb(F_T, 0), nb(F_T, 1), c0[F_T], nb(F_T, 2), nb(F_T, 3));
  }
}

template <class Tq, class Tr, class Tc>
struct Kernel {
  Grid g;
  Coef<Tc> c;
  const Tq* __restrict__ q;
  Tr* __restrict__ r;
};

// One z-step with the newest plane in window slot PH.
template <class Tq, class Tr, class Tc, int PH>
__device__ __forceinline__ void zstep(const Kernel<Tq, Tr, Tc>& K, Ctx<Tc>& cx, Tc* lds, Tc (&nxt)[LOADS][5],
                                      const long long (&off)[LOADS], int p, int kout_lo, int kout_hi,
                                      bool col_valid, long long col_off, int p_last) {
  const int tid = threadIdx.x;
  const Grid& g = K.g;
  const Coef<Tc>& c = K.c;
  // 1. primitives of the prefetched plane into LDS
#pragma unroll
  for (int l = 0; l < LOADS; ++l) {
    const int s = tid + l * NT;
    if (s < NPL) {
      Tc f[NF];
      primitives(nxt[l], f, c);
#pragma unroll
      for (int k = 0; k < NF; ++k) lds[k * NPL + s] = f[k];
    }
  }
  __syncthreads();
  // prefetch plane p + 1
  if (p < p_last) {
    int z = p + 1;
    z += (z < 0) ? g.nz : 0;
    z -= (z >= g.nz) ? g.nz : 0;
    const long long zo = (long long)z * g.plane;
#pragma unroll
    for (int l = 0; l < LOADS; ++l) {
      const int s = tid + l * NT;
      if (s < NPL) {
#pragma unroll
        for (int f = 0; f < 5; ++f) nxt[l][f] = load_as<Tc>(K.q[f * g.N + zo + off[l]]);
      }
    }
  }
  // 2. in-plane terms of plane p at this column
  const int tx = tid % TX, ty = tid / TX;
  const int own = (ty + 2) * HX + (tx + 2);
#pragma unroll
  for (int k = 0; k < NF; ++k) cx.W[PH][k] = lds[k * NPL + own];
  const Tc* c0 = cx.W[PH];
  Tc R[5] = {0, 0, 0, 0, 0};
  {
    Tc G[3] = {0, 0, 0};
    direction_terms<Tc, 0>(LdsNb<Tc, 1>{lds, own}, c0, c, c.c1[0], c.c2[0], R, G);
    cx.GI[PH][0] = G[0];
    cx.GI[PH][2] = G[1];
    cx.GI[PH][4] = G[2];
    direction_terms<Tc, 1>(LdsNb<Tc, HX>{lds, own}, c0, c, c.c1[1], c.c2[1], R, G);
    cx.GI[PH][1] = G[0];
    cx.GI[PH][3] = G[1];
    cx.GI[PH][5] = G[2];
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
#pragma unroll
  for (int f = 0; f < 5; ++f) cx.RI[PH][f] = R[f];
  __syncthreads();

  // 3. emit plane k = p - 2 (window slots: k-2 .. k+2)
  const int k = p - 2;
  if (k >= kout_lo && k < kout_hi) {
    constexpr int KM2 = (PH + 1) % 5, KM1 = (PH + 2) % 5, K0 = (PH + 3) % 5, KP1 = (PH + 4) % 5, KP2 = PH;
    Tc Rz[5] = {cx.RI[K0][0], cx.RI[K0][1], cx.RI[K0][2], cx.RI[K0][3], cx.RI[K0][4]};
    Tc Gz[3] = {0, 0, 0};
    direction_terms<Tc, 2>(WinNb<Tc, KM2, KM1, KP1, KP2>{cx.W}, cx.W[K0], c, c.c1[2], c.c2[2], Rz, Gz);
    if (c.viscous) {
      const Tc* u0 = cx.W[K0] + F_U;
      // z-mixed: X_x += D_z(w_x), X_y += D_z(w_y), X_z += D_z(u_x) + D_z(v_y)
      const Tc cz = c.c1[2] * c.ire * Tc(1.0 / 3.0);
      const Tc mx = cz * S1(cx.GI[KM2][4], cx.GI[KM1][4], cx.GI[KP1][4], cx.GI[KP2][4]);
      const Tc my = cz * S1(cx.GI[KM2][5], cx.GI[KM1][5], cx.GI[KP1][5], cx.GI[KP2][5]);
      const Tc mz = cz * (S1(cx.GI[KM2][0], cx.GI[KM1][0], cx.GI[KP1][0], cx.GI[KP2][0]) +
                          S1(cx.GI[KM2][3], cx.GI[KM1][3], cx.GI[KP1][3], cx.GI[KP2][3]));
      Rz[1] += mx;
      Rz[2] += my;
      Rz[3] += mz;
      Rz[4] += u0[0] * mx + u0[1] * my + u0[2] * mz;
      // viscous work tau : grad u = (1/Re)[sum G_ad^2 + sum G_ad G_da - 2/3 div^2]
      const Tc G00 = cx.GI[K0][0], G01 = cx.GI[K0][1], G02 = Gz[0];
      const Tc G10 = cx.GI[K0][2], G11 = cx.GI[K0][3], G12 = Gz[1];
      const Tc G20 = cx.GI[K0][4], G21 = cx.GI[K0][5], G22 = Gz[2];
      const Tc div = G00 + G11 + G22;
      const Tc sq = G00 * G00 + G01 * G01 + G02 * G02 + G10 * G10 + G11 * G11 + G12 * G12 + G20 * G20 +
                    G21 * G21 + G22 * G22;
      const Tc cr = G00 * G00 + G11 * G11 + G22 * G22 + Tc(2) * (G01 * G10 + G02 * G20 + G12 * G21);
      Rz[4] += c.ire * (sq + cr - Tc(2.0 / 3.0) * div * div);
    }
    if (col_valid) {
      const long long id = (long long)k * g.plane + col_off;
#pragma unroll
      for (int f = 0; f < 5; ++f) K.r[f * g.N + id] = store_as<Tr>(Rz[f]);
    }
  }
}

template <class Tq, class Tr, class Tc>
__global__ void __launch_bounds__(NT) residual_tiled(Kernel<Tq, Tr, Tc> K, int tiles_x, int tiles_y, int chunks_z,
                                                     int remap) {
  __shared__ Tc lds[NF * NPL];
  const Grid& g = K.g;
  // XCD-aware order: hardware block b runs on XCD b % 8; give each XCD a
  // contiguous range of logical tiles so that y-neighbours share an L2.
  const int nb = tiles_x * tiles_y * chunks_z;
  int b = blockIdx.x;
  if (remap) b = (b % 8) * (nb / 8) + b / 8;
  const int ty_t = b % tiles_y;
  const int tx_t = (b / tiles_y) % tiles_x;
  const int cz = b / (tiles_y * tiles_x);
  const int x0 = tx_t * TX, y0 = ty_t * TY;
  const int z0 = cz * KZ;
  const int z1 = min(z0 + KZ, g.nz);

  const int tid = threadIdx.x;
  // wrapped (x, y) offsets of the plane points this thread loads (fixed over z)
  long long off[LOADS];
#pragma unroll
  for (int l = 0; l < LOADS; ++l) {
    const int s = tid + l * NT;
    const int lx = s % HX, ly = s / HX;
    int x = (x0 - 2 + lx) % g.nx;
    x += (x < 0) ? g.nx : 0;
    int y = (y0 - 2 + ly) % g.ny;
    y += (y < 0) ? g.ny : 0;
    off[l] = (long long)y * g.nx + x;
  }
  const int cxg = x0 + tid % TX, cyg = y0 + tid / TX;
  const bool col_valid = cxg < g.nx && cyg < g.ny;
  const long long col_off = (long long)cyg * g.nx + cxg;

  // prefetch the first plane
  Tc nxt[LOADS][5];
  {
    int z = z0 - 2;
    z += (z < 0) ? g.nz : 0;
    z -= (z >= g.nz) ? g.nz : 0;
    const long long zo = (long long)z * g.plane;
#pragma unroll
    for (int l = 0; l < LOADS; ++l) {
      const int s = tid + l * NT;
      if (s < NPL) {
#pragma unroll
        for (int f = 0; f < 5; ++f) nxt[l][f] = load_as<Tc>(K.q[f * g.N + zo + off[l]]);
      } else {
#pragma unroll
        for (int f = 0; f < 5; ++f) nxt[l][f] = Tc(1);
      }
    }
  }
  Ctx<Tc> cx;
  const int p_first = z0 - 2, p_last = z1 + 1;  // planes entering the window
  for (int p = p_first; p <= p_last; p += 5) {
    zstep<Tq, Tr, Tc, 0>(K, cx, lds, nxt, off, p, z0, z1, col_valid, col_off, p_last);
    if (p + 1 > p_last) break;
    zstep<Tq, Tr, Tc, 1>(K, cx, lds, nxt, off, p + 1, z0, z1, col_valid, col_off, p_last);
    if (p + 2 > p_last) break;
    zstep<Tq, Tr, Tc, 2>(K, cx, lds, nxt, off, p + 2, z0, z1, col_valid, col_off, p_last);
    if (p + 3 > p_last) break;
    zstep<Tq, Tr, Tc, 3>(K, cx, lds, nxt, off, p + 3, z0, z1, col_valid, col_off, p_last);
    if (p + 4 > p_last) break;
    zstep<Tq, Tr, Tc, 4>(K, cx, lds, nxt, off, p + 4, z0, z1, col_valid, col_off, p_last);
  }
}

}  // namespace

template <class Tq, class Tr, class Tc>
hipError_t launch_residual(const Grid& g, const Coef<Tc>& c, const void* q, void* r, hipStream_t st) {
  const int tiles_x = (g.nx + TX - 1) / TX;
  const int tiles_y = (g.ny + TY - 1) / TY;
  const int chunks_z = (g.nz + KZ - 1) / KZ;
  const long long nb = (long long)tiles_x * tiles_y * chunks_z;
  const int remap = (nb % 8 == 0) ? 1 : 0;
  Kernel<Tq, Tr, Tc> K{g, c, static_cast<const Tq*>(q), static_cast<Tr*>(r)};
  hipLaunchKernelGGL((residual_tiled<Tq, Tr, Tc>), dim3((unsigned)nb), dim3(NT), 0, st, K, tiles_x, tiles_y,
                     chunks_z, remap);
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
