/*
 * tgv.h -- C-ABI of libtgv.so: the explicit finite-difference time step of the
 * 3-D compressible Navier-Stokes equations on a periodic Cartesian grid, with
 * the Taylor-Green vortex as workload, for AMD Instinct MI355X (gfx950).
 *
 * Paper: "Reduced and mixed precision turbulent flow simulations using explicit
 * finite difference schemes" (arXiv 2505.20911).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Arrays are caller-owned DEVICE memory (e.g. torch tensors), never
 *    allocated, freed or retained by the library.  A state-like array holds the
 *    five conserved fields Q = (rho, rho u, rho v, rho w, rho E) (Sec. 3.1) as
 *    [5][nz][ny][nx], x fastest, no ghost cells; field f starts at element
 *    f*N, N = nx*ny*nz (64-bit offsets).  Base pointers must be 16-byte aligned.
 *  - Element types are chosen per array class by ns_prec_t (Sec. 3.1 storage
 *    classes Q, Q~, R and work arrays W; Sec. 3.2 per-class precision):
 *    q = Q, qt = RK register Q~, r = residual R, compute = arithmetic type
 *    of the fused residual (it stands in for the paper's W arrays, which
 *    here live in registers/LDS).  Supported combinations (q, qt, r, compute):
 *      DP        (f64, f64, f64, f64)
 *      SPDP      (f64, f64, f32, f32)   paper's single-double
 *      SPDP_C64  (f64, f64, f32, f64)
 *      SP_DPC    (f32, f32, f32, f64)   FP32 storage, FP64 arithmetic
 *      SP        (f32, f32, f32, f32)
 *      HPSP      (f32, f32, f16, f32)   paper's half-single
 *      HPSP_BF16 (f32, f32, bf16, f32)
 *      HP        (f16, f16, f16, f32)
 *    Anything else returns NS_ERR_DTYPE.  Every narrowing conversion rounds
 *    to nearest even; FP16 overflow gives +-inf.
 *  - `stream` is a hipStream_t (NULL = default stream).  Every call only
 *    enqueues work on it and returns without synchronising.
 *  - Return value: NS_OK (0) on success, a negative NS_ERR_* code otherwise.
 *    Arguments are validated on the host before any HIP call; on error nothing
 *    is launched and ns_last_error() returns a description (thread-local,
 *    valid until the next call on the same thread).  NS_ERR_HIP reports a
 *    failed kernel launch.
 *  - Grid: n_d >= 5 points per axis, spacing h_d = L_d / n_d, x_i = i h_d
 *    (no duplicated periodic end point), N <= 2^34 points (more than any
 *    precision form fits in device memory).  The tiled kernels also need
 *    fewer than 2^32 work-items per dispatch; their launch rules (long z
 *    chunks on large grids) keep every grid within the point limit below it,
 *    and the host check returns NS_ERR_SHAPE should one not be.
 *  - Physics: non-dimensional, constant viscosity mu = 1, Stokes stress,
 *    Fourier heat flux with kappa = 1 / ((gamma-1) M^2 Pr Re),
 *    p = (gamma-1)(rho E - rho |u|^2 / 2), T = gamma M^2 p / rho
 *    (consistent with the isothermal initial density rho = gamma M^2 p, Sec. 4.1).
 */
#ifndef TGV_H
#define TGV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { NS_F64 = 0, NS_F32 = 1, NS_F16 = 2, NS_BF16 = 3 } ns_dtype_t;

/* Split form of the convective term d(rho u_j phi)/dx_j, phi = (1, u_i, E)
 * (Sec. 2.3.1; the forms the paper compares in the inviscid limit, Sec. 4.2).
 * D is the 4th-order central first difference.
 *   BLAISDELL  (rho phi) x (u_j):  [D(rho phi u_j) + u_j D(rho phi) + rho phi D(u_j)] / 2
 *   DIVERGENCE D(rho u_j phi)
 *   FEIEREISEN (rho u_j) x (phi):  [D(rho u_j phi) + phi D(rho u_j) + rho u_j D(phi)] / 2
 *   JAMESON    (rho) x (u_j phi):  [D(rho u_j phi) + rho D(u_j phi) + u_j phi D(rho)] / 2
 *   KGP        Kennedy-Gruber-Pirozzoli cubic form: the divergence term and
 *              the six product-rule expansions of the triple product, each / 4.
 *   KOK        Kok (2009): FEIEREISEN for mass and momentum; the energy as
 *              internal energy e = p/((gamma-1) rho) with the (rho u_j) x (e)
 *              pairing plus kinetic energy split as
 *              [m_j u_a D(u_a) + u_a D(m_j u_a)] / 2 (two-point flux: mass flux
 *              times u_a(left) u_a(right) / 2); pressure work p D(u_j) + u_j D(p).
 *   KEEP       kinetic energy and entropy preserving form (Kuya, Totani and
 *              Kawai 2018): KGP for mass, momentum and internal energy; kinetic
 *              energy [m_j u_a D(u_a) + u_a D(m_j u_a) + m_a D(u_j u_a)
 *              + u_j u_a D(m_a)] / 4; pressure work as KOK.
 * The pressure gradient stays in divergence form in every variant, and so does
 * the pressure work except in KOK and KEEP.  Forms other
 * than BLAISDELL are available in the DP and HPSP precision forms, and the
 * adjoint supports BLAISDELL only (NS_ERR_ARG otherwise). */
typedef enum {
  NS_SPLIT_BLAISDELL = 0,
  NS_SPLIT_DIVERGENCE = 1,
  NS_SPLIT_FEIEREISEN = 2,
  NS_SPLIT_JAMESON = 3,
  NS_SPLIT_KGP = 4,
  NS_SPLIT_KOK = 5,
  NS_SPLIT_KEEP = 6
} ns_split_t;

typedef struct {
  int32_t n[3];     /* nx, ny, nz */
  double L[3];      /* box lengths (2 pi for the Taylor-Green vortex) */
  double gamma;     /* ratio of specific heats (1.4, Sec. 4.1) */
  double mach;      /* reference Mach number M */
  double reynolds;  /* Reynolds number Re */
  double prandtl;   /* Prandtl number Pr */
  int32_t viscous;  /* 1: full equations; 0: diffusive terms omitted (inviscid variant, Sec. 4.2) */
  int32_t split;    /* ns_split_t; only the residual entry points read it */
} ns_params_t;

typedef struct {
  ns_dtype_t q, qt, r, compute;
} ns_prec_t;

enum {
  NS_OK = 0,
  NS_ERR_ARG = -1,   /* null pointer, bad stage, non-finite or out-of-range scalar */
  NS_ERR_DTYPE = -2, /* unsupported precision combination */
  NS_ERR_SHAPE = -3, /* grid too small or too large */
  NS_ERR_ALIGN = -4, /* base pointer not 16-byte aligned */
  NS_ERR_HIP = -5    /* HIP launch error */
};

/* Taylor-Green initial state (Sec. 4.1 initial-condition equations):
 *   u = sin x cos y cos z, v = -cos x sin y cos z, w = 0,
 *   p = 1/(gamma M^2) + (1/16)(cos 2x + cos 2y)(2 + cos 2z),
 *   rho = gamma M^2 p, rho E = p/(gamma-1) + rho |u|^2 / 2,
 * evaluated in FP64 and rounded to q_dtype.  Writes q [5][nz][ny][nx]. */
int tgv_init(const ns_params_t* params, ns_dtype_t q_dtype, void* q, void* stream);

/* The same Taylor-Green initial fields in primitive form: velocity u
 * [3][nz][ny][nx], density rho and pressure p [nz][ny][nx], evaluated in FP64
 * and rounded to dtype (NS_F64 or NS_F32).  u, rho, p: distinct 16-byte
 * aligned device arrays. */
int tgv_init_primitive(const ns_params_t* params, ns_dtype_t dtype, void* u, void* rho, void* p, void* stream);

/* Conserved state of a velocity field at given density and pressure (Sec. 3.1
 * state vector; the total energy rho E = p/(gamma-1) + rho |u|^2 / 2 of the
 * equation of state above):
 *   q = (rho, rho u, rho v, rho w, p/(gamma-1) + (rho/2)(u^2 + v^2 + w^2)),
 * arithmetic and storage in dtype (NS_F64 or NS_F32).  This is how the
 * differentiation form builds Q^0 from its control, the initial velocity
 * (density and pressure held fixed).  u [3][N], rho [N], p [N] are read, q
 * [5][N] written; q must not overlap the inputs. */
int ns_state_from_velocity(const ns_params_t* params, ns_dtype_t dtype, const void* u, const void* rho,
                           const void* p, void* q, void* stream);

/* Reverse of ns_state_from_velocity at fixed rho and p:
 *   u_bar_a = rho (q_bar_{m_a} + u_a q_bar_E),   a = 1..3,
 * the gradient with respect to the velocity of a function of q whose gradient
 * with respect to q is q_bar.  u_bar [3][N] is overwritten (not accumulated). */
int ns_state_from_velocity_adjoint(const ns_params_t* params, ns_dtype_t dtype, const void* u, const void* rho,
                                   const void* q_bar, void* u_bar, void* stream);

/* Time-integrated dissipation by the trapezoid rule over a history of flow
 * integrals (the objective of the differentiation form):
 *   J = dt sum_{n=0}^{rows-1} w_n hist[n * stride + col],  w_0 = w_{rows-1} = 1/2, else 1
 * (rows = 1: J = dt hist[col] / 2).  With stride 8 and col 2 over rows written
 * by flow_integrals this is dt sum_n w_n eps_S(Q^n).  hist and J are device
 * memory; one block sums in a fixed order, so J is deterministic. */
int dissipation_trapezoid(const double* hist, int64_t rows, int32_t stride, int32_t col, double dt, double* J,
                          void* stream);

/* Residual R = dQ/dt (Sec. 3.1: R holds all terms of the equations except the
 * time derivative), 4th-order central differences for the convective and
 * diffusive parts (Sec. 2.3.1):
 *   R_q = -C_q - P_q + V_q,
 *   C_q = 1/2 sum_d [ D_d(q u_d) + u_d D_d q + q D_d u_d ]   (Blaisdell split, Sec. 2.3.1)
 *   P_rho = 0, P_{m_a} = D_a p, P_E = sum_d D_d(p u_d),
 *   V_rho = 0, V_{m_a} = (1/Re)(sum_d D2_d u_a + X_a/3), X_a = D2_a u_a + sum_{d!=a} D_a D_d u_d,
 *   V_E = sum_a u_a V_{m_a} + sum_{a,d} tau_ad D_d u_a + kappa sum_d D2_d T,
 * D f_i = (8 (f_{i+1} - f_{i-1}) - (f_{i+2} - f_{i-2})) / (12 h),
 * D2 f_i = (16 (f_{i+1} - 2 f_i + f_{i-1}) - (f_{i+2} - 2 f_i + f_{i-2})) / (12 h^2),
 * periodic.  Reads q (type prec->q), writes r (type prec->r), arithmetic in
 * prec->compute.  q and r must not overlap. */
int ns_residual(const ns_params_t* params, const ns_prec_t* prec, const void* q, void* r,
                void* stream);

/* One stage of the two-register low-storage RK3 update (Sec. 3.1 update equations),
 * Williamson coefficients A = (0, -5/9, -153/128), B = (1/3, 15/16, 8/15):
 *   Q~ <- A_i Q~ + dt R ;  Q <- Q + B_i Q~        (stage i = 0, 1, 2)
 * Stage 0 does not read Q~ (A_0 = 0).  q (prec->q) and qt (prec->qt) are
 * updated in place, r (prec->r) is read.  Arithmetic in FP64 when q or compute
 * is f64, else FP32. */
int rk_stage(const ns_params_t* params, const ns_prec_t* prec, int stage, double dt, void* q,
             void* qt, const void* r, void* stream);

/* Residual and RK stage in one pass over the grid (the two calls above fused,
 * so R never goes through memory):
 *   Q~ <- A_i Q~ + dt R(q_in) ;  q_out <- q_in + B_i Q~
 * with R rounded to prec->r exactly as ns_residual would store it and rk_stage
 * read it back, so the result equals ns_residual followed by rk_stage.
 * q_in (prec->q) is read, q_out (prec->q) written, qt (prec->qt) updated in
 * place (not read at stage 0).  q_in, q_out and qt must be distinct arrays:
 * every point's stencil reads q_in around it while q_out is written. */
int ns_residual_rk_stage(const ns_params_t* params, const ns_prec_t* prec, int stage, double dt,
                         const void* q_in, void* q_out, void* qt, void* stream);

/* Bytes of device workspace flow_integrals() needs for this grid. */
size_t flow_integrals_workspace_bytes(const ns_params_t* params);

/* Flow integrals of Sec. 4.1 as volume averages, accumulated in FP64 for every
 * precision form, written to device memory out8[8]:
 *   K = <|u|^2/2>, K_rho = <rho |u|^2/2>, eps_S = (1/Re) <|curl u|^2> (curl with
 *   the 4th-order D), <rho>, <rho u>, <rho v>, <rho w>, <rho E>.
 * Deterministic: a fixed two-pass reduction order.  workspace: device memory of
 * flow_integrals_workspace_bytes(params) bytes, 16-byte aligned. */
int flow_integrals(const ns_params_t* params, const ns_prec_t* prec, const void* q,
                   void* workspace, double* out8, void* stream);

/* flow_integrals() for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results, but the first pass's partial sums go to a
 * static device array inside the library (4 MiB per device, held until the
 * process ends) instead of a caller workspace, and the call allocates nothing.
 * Grids whose flow_integrals_workspace_bytes() exceeds 4 MiB (more than 65536
 * first-pass blocks; every cube up to 1024^3 fits) return NS_ERR_SHAPE.  All
 * calls on one device share that array: calls that overlap in time on one
 * device (different streams, or host threads) race and give wrong sums; calls
 * ordered on one stream are safe.  The first call on a device looks up the
 * array's device address (once per device). */
int flow_integrals_noalloc(const ns_params_t* params, const ns_prec_t* prec, const void* q, double* out8,
                           void* stream);

/* Bytes of device workspace ns_residual_adjoint() needs: 15 fields of N values
 * of prec->q's type (the symmetric viscous-work adjoint and the inner
 * differences of the mixed derivatives, read at stencil neighbours by a later
 * pass, and the velocity adjoint of those terms; only the viscous residual
 * uses it). */
size_t ns_residual_adjoint_workspace_bytes(const ns_params_t* params, const ns_prec_t* prec);

/* Discrete adjoint of ns_residual at state q:  q_bar += (dR/dQ)(q)^T r_bar.
 * q, r_bar and q_bar use prec->q as element type, arithmetic in prec->compute;
 * supported for the DP and SP forms.  q_bar is accumulated into (read-modify-
 * write) and must not overlap q or r_bar.  workspace: device memory of
 * ns_residual_adjoint_workspace_bytes() bytes (contents on return unspecified). */
int ns_residual_adjoint(const ns_params_t* params, const ns_prec_t* prec, const void* q,
                        const void* r_bar, void* q_bar, void* workspace, void* stream);

/* Reverse of rk_stage(stage) for the adjoint variables of Q (q_bar) and of the
 * register Q~ (zeta):  zeta <- zeta + B_i q_bar ;  r_bar <- dt zeta ;
 * zeta <- A_i zeta.  The caller then adds (dR/dQ)^T r_bar at the stage's input
 * state into q_bar with ns_residual_adjoint.  All three arrays of type prec->q. */
int rk_stage_adjoint(const ns_params_t* params, const ns_prec_t* prec, int stage, double dt,
                     const void* q_bar, void* zeta, void* r_bar, void* stream);

/* Bytes of device workspace flow_integrals_adjoint() needs. */
size_t flow_integrals_adjoint_workspace_bytes(const ns_params_t* params, const ns_prec_t* prec);

/* q_bar += eps_bar * d(eps_S)/dQ at state q (eps_S as in flow_integrals). */
int flow_integrals_adjoint(const ns_params_t* params, const ns_prec_t* prec, const void* q,
                           double eps_bar, void* q_bar, void* workspace, void* stream);

/* Description of the last error on this thread ("" if none). */
const char* ns_last_error(void);

/* ABI version of this header (incremented on incompatible change). */
int tgv_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TGV_H */
