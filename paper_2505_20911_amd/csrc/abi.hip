// C-ABI of libtgv.so (declarations and contracts in include/tgv.h): host-side
// argument validation, precision-form dispatch to the kernel template
// instances, and launch on the caller's stream.  No allocation, no
// synchronisation, no global state beyond the thread-local error message.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>

#include "tgv.h"
#include "tgv_device.h"
#include "tgv_kernels.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int ok() {
  g_err.clear();
  return NS_OK;
}

// The supported precision forms (q, qt, r, compute).
enum Form { DP, SPDP, SPDP_C64, SP_DPC, SP, HPSP, HPSP_BF16, HP, SPDP_WK, HPSP_WK, HPSP_RESWK, HP_C16, BAD };

Form form_of(const ns_prec_t& p) {
  auto is = [&](ns_dtype_t a, ns_dtype_t b, ns_dtype_t c, ns_dtype_t d) {
    return p.q == a && p.qt == b && p.r == c && p.compute == d;
  };
  if (is(NS_F64, NS_F64, NS_F64, NS_F64)) return DP;
  if (is(NS_F64, NS_F64, NS_F32, NS_F32)) return SPDP;
  if (is(NS_F64, NS_F64, NS_F32, NS_F64)) return SPDP_C64;
  if (is(NS_F32, NS_F32, NS_F32, NS_F64)) return SP_DPC;
  if (is(NS_F32, NS_F32, NS_F32, NS_F32)) return SP;
  if (is(NS_F32, NS_F32, NS_F16, NS_F32)) return HPSP;
  if (is(NS_F32, NS_F32, NS_BF16, NS_F32)) return HPSP_BF16;
  if (is(NS_F16, NS_F16, NS_F16, NS_F32)) return HP;
  if (is(NS_F64, NS_F64, NS_F64, NS_F32)) return SPDP_WK;
  if (is(NS_F32, NS_F32, NS_F32, NS_F16)) return HPSP_WK;
  if (is(NS_F32, NS_F32, NS_F16, NS_F16)) return HPSP_RESWK;
  if (is(NS_F16, NS_F16, NS_F16, NS_F16)) return HP_C16;
  return BAD;
}

const char* dtype_name(ns_dtype_t t) {
  switch (t) {
    case NS_F64: return "f64";
    case NS_F32: return "f32";
    case NS_F16: return "f16";
    case NS_BF16: return "bf16";
  }
  return "?";
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

int check_params(const ns_params_t* p, tgv::Grid* g) {
  if (!p) return fail(NS_ERR_ARG, "params is NULL");
  for (int d = 0; d < 3; ++d) {
    if (p->n[d] < 5)
      return fail(NS_ERR_SHAPE, "n[" + std::to_string(d) + "] = " + std::to_string(p->n[d]) +
                                    " < 5 (the 4th-order stencil needs 5 distinct points per axis)");
    if (!finite_pos(p->L[d])) return fail(NS_ERR_ARG, "L[" + std::to_string(d) + "] must be finite and > 0");
  }
  const long long N = (long long)p->n[0] * p->n[1] * p->n[2];
  // Element-wise kernels loop grid-stride, so only the tiled kernels' block
  // counts limit the grid (checked per entry point by check_launch); 2^34
  // points exceed the device memory of any precision form.
  if (N > (1LL << 34)) return fail(NS_ERR_SHAPE, "grid has more than 2^34 points");
  if (!(std::isfinite(p->gamma) && p->gamma > 1.0)) return fail(NS_ERR_ARG, "gamma must be finite and > 1");
  if (!finite_pos(p->mach)) return fail(NS_ERR_ARG, "mach must be finite and > 0");
  if (p->viscous != 0 && p->viscous != 1) return fail(NS_ERR_ARG, "viscous must be 0 or 1");
  if (p->split < NS_SPLIT_BLAISDELL || p->split > NS_SPLIT_KEEP)
    return fail(NS_ERR_ARG, "split must be one of NS_SPLIT_BLAISDELL .. NS_SPLIT_KEEP");
  if (!finite_pos(p->reynolds)) return fail(NS_ERR_ARG, "reynolds must be finite and > 0");
  if (!finite_pos(p->prandtl)) return fail(NS_ERR_ARG, "prandtl must be finite and > 0");
  g->nx = p->n[0];
  g->ny = p->n[1];
  g->nz = p->n[2];
  g->N = N;
  g->plane = (long long)p->n[0] * p->n[1];
  return NS_OK;
}

int check_prec(const ns_prec_t* p, Form* f) {
  if (!p) return fail(NS_ERR_ARG, "prec is NULL");
  *f = form_of(*p);
  if (*f == BAD)
    return fail(NS_ERR_DTYPE, std::string("unsupported precision form (q, qt, r, compute) = (") +
                                  dtype_name(p->q) + ", " + dtype_name(p->qt) + ", " + dtype_name(p->r) + ", " +
                                  dtype_name(p->compute) + ")");
  return NS_OK;
}

int check_ptr(const void* ptr, const char* name) {
  if (!ptr) return fail(NS_ERR_ARG, std::string(name) + " is NULL");
  if (reinterpret_cast<uintptr_t>(ptr) % 16 != 0)
    return fail(NS_ERR_ALIGN, std::string(name) + " is not 16-byte aligned");
  return NS_OK;
}

// A dispatch holds fewer than 2^32 work-items; grids whose tiled launch would
// need more (very large, or extremely elongated) are refused before any HIP call.
int check_launch(long long work_items, const char* what) {
  if (work_items > (long long)0xffffffffu)
    return fail(NS_ERR_SHAPE, std::string(what) + ": the grid needs " + std::to_string(work_items) +
                                  " work-items in one dispatch (at most 2^32 - 1)");
  return NS_OK;
}

int hip_status(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(NS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return ok();
}

template <class Tc>
tgv::Coef<Tc> make_coef(const ns_params_t* p) {
  tgv::Coef<Tc> c;
  for (int d = 0; d < 3; ++d) {
    const double h = p->L[d] / p->n[d];
    c.c1[d] = (Tc)(1.0 / (12.0 * h));
    c.c2[d] = (Tc)(1.0 / (12.0 * h * h));
  }
  c.gm1 = (Tc)(p->gamma - 1.0);
  c.igm1 = (Tc)(1.0 / (p->gamma - 1.0));
  c.gm2 = (Tc)(p->gamma * p->mach * p->mach);
  c.ire = (Tc)(1.0 / p->reynolds);
  const double kap = 1.0 / ((p->gamma - 1.0) * p->mach * p->mach * p->prandtl * p->reynolds);
  c.kap = (Tc)kap;
  for (int d = 0; d < 3; ++d) {
    const double h = p->L[d] / p->n[d];
    const double c2 = 1.0 / (12.0 * h * h);
    c.vis2[d] = (Tc)(c2 / p->reynolds);
    c.vis2l[d] = (Tc)(c2 * (4.0 / 3.0) / p->reynolds);
    c.kap2[d] = (Tc)(c2 * kap);
  }
  c.viscous = p->viscous;
  return c;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Split forms other than Blaisdell are built for the DP and HPSP forms.
int check_split(const ns_params_t* p, Form f) {
  if (p->split != NS_SPLIT_BLAISDELL && f != DP && f != HPSP)
    return fail(NS_ERR_ARG, "split forms other than Blaisdell are available for the DP and HPSP precision forms");
  return NS_OK;
}

// The adjoint is written for the Blaisdell split form.
int check_adjoint_split(const ns_params_t* p) {
  if (p->split != NS_SPLIT_BLAISDELL) return fail(NS_ERR_ARG, "the adjoint supports the Blaisdell split form only");
  return NS_OK;
}

}  // namespace

extern "C" {

int tgv_abi_version(void) { return 2; }

const char* ns_last_error(void) { return g_err.c_str(); }

int tgv_init(const ns_params_t* params, ns_dtype_t q_dtype, void* q, void* stream) {
  tgv::Grid g;
  int rc = check_params(params, &g);
  if (rc) return rc;
  if ((rc = check_ptr(q, "q"))) return rc;
  hipError_t e;
  switch (q_dtype) {
    case NS_F64: e = tgv::launch_init<double>(g, params->L, params->gamma, params->mach, q, as_stream(stream)); break;
    case NS_F32: e = tgv::launch_init<float>(g, params->L, params->gamma, params->mach, q, as_stream(stream)); break;
    case NS_F16: e = tgv::launch_init<tgv::f16>(g, params->L, params->gamma, params->mach, q, as_stream(stream)); break;
    case NS_BF16: e = tgv::launch_init<tgv::bf16>(g, params->L, params->gamma, params->mach, q, as_stream(stream)); break;
    default: return fail(NS_ERR_DTYPE, "q_dtype must be one of NS_F64, NS_F32, NS_F16, NS_BF16");
  }
  return hip_status(e, "tgv_init");
}

int tgv_init_primitive(const ns_params_t* params, ns_dtype_t dtype, void* u, void* rho, void* p, void* stream) {
  tgv::Grid g;
  int rc = check_params(params, &g);
  if (rc) return rc;
  if ((rc = check_ptr(u, "u")) || (rc = check_ptr(rho, "rho")) || (rc = check_ptr(p, "p"))) return rc;
  if (u == rho || u == p || rho == p) return fail(NS_ERR_ARG, "u, rho and p must be distinct arrays");
  hipError_t e;
  switch (dtype) {
    case NS_F64: e = tgv::launch_init_primitive<double>(g, params->L, params->gamma, params->mach, u, rho, p, as_stream(stream)); break;
    case NS_F32: e = tgv::launch_init_primitive<float>(g, params->L, params->gamma, params->mach, u, rho, p, as_stream(stream)); break;
    default: return fail(NS_ERR_DTYPE, "dtype must be NS_F64 or NS_F32");
  }
  return hip_status(e, "tgv_init_primitive");
}

int ns_state_from_velocity(const ns_params_t* params, ns_dtype_t dtype, const void* u, const void* rho,
                           const void* p, void* q, void* stream) {
  tgv::Grid g;
  int rc = check_params(params, &g);
  if (rc) return rc;
  if ((rc = check_ptr(u, "u")) || (rc = check_ptr(rho, "rho")) || (rc = check_ptr(p, "p")) ||
      (rc = check_ptr(q, "q")))
    return rc;
  if (q == u || q == rho || q == p) return fail(NS_ERR_ARG, "q must not overlap the inputs");
  hipError_t e;
  switch (dtype) {
    case NS_F64: e = tgv::launch_state_from_velocity<double>(g, params->gamma, u, rho, p, q, as_stream(stream)); break;
    case NS_F32: e = tgv::launch_state_from_velocity<float>(g, params->gamma, u, rho, p, q, as_stream(stream)); break;
    default: return fail(NS_ERR_DTYPE, "dtype must be NS_F64 or NS_F32");
  }
  return hip_status(e, "ns_state_from_velocity");
}

int ns_state_from_velocity_adjoint(const ns_params_t* params, ns_dtype_t dtype, const void* u, const void* rho,
                                   const void* q_bar, void* u_bar, void* stream) {
  tgv::Grid g;
  int rc = check_params(params, &g);
  if (rc) return rc;
  if ((rc = check_ptr(u, "u")) || (rc = check_ptr(rho, "rho")) || (rc = check_ptr(q_bar, "q_bar")) ||
      (rc = check_ptr(u_bar, "u_bar")))
    return rc;
  if (u_bar == u || u_bar == rho || u_bar == q_bar) return fail(NS_ERR_ARG, "u_bar must not overlap the inputs");
  hipError_t e;
  switch (dtype) {
    case NS_F64: e = tgv::launch_state_from_velocity_adjoint<double>(g, u, rho, q_bar, u_bar, as_stream(stream)); break;
    case NS_F32: e = tgv::launch_state_from_velocity_adjoint<float>(g, u, rho, q_bar, u_bar, as_stream(stream)); break;
    default: return fail(NS_ERR_DTYPE, "dtype must be NS_F64 or NS_F32");
  }
  return hip_status(e, "ns_state_from_velocity_adjoint");
}

int dissipation_trapezoid(const double* hist, int64_t rows, int32_t stride, int32_t col, double dt, double* J,
                          void* stream) {
  if (!hist || !J) return fail(NS_ERR_ARG, "hist and J must not be NULL");
  if (reinterpret_cast<uintptr_t>(hist) % 8 != 0 || reinterpret_cast<uintptr_t>(J) % 8 != 0)
    return fail(NS_ERR_ALIGN, "hist and J must be 8-byte aligned");
  if (rows < 1) return fail(NS_ERR_ARG, "rows must be >= 1");
  if (stride < 1 || col < 0 || col >= stride) return fail(NS_ERR_ARG, "need 0 <= col < stride");
  if (!std::isfinite(dt)) return fail(NS_ERR_ARG, "dt must be finite");
  return hip_status(tgv::launch_trapezoid(hist, rows, stride, col, dt, J, as_stream(stream)), "dissipation_trapezoid");
}

int ns_residual(const ns_params_t* params, const ns_prec_t* prec, const void* q, void* r, void* stream) {
  tgv::Grid g;
  Form f;
  int rc = check_params(params, &g);
  if (rc) return rc;
  if ((rc = check_prec(prec, &f)) || (rc = check_split(params, f))) return rc;
  if ((rc = check_ptr(q, "q")) || (rc = check_ptr(r, "r"))) return rc;
  if (q == r) return fail(NS_ERR_ARG, "q and r must not overlap");
  if ((rc = check_launch(tgv::residual_work_items(g), "ns_residual"))) return rc;
  hipStream_t st = as_stream(stream);
  hipError_t e = hipSuccess;
  using tgv::bf16;
  using tgv::f16;
  switch (f) {
    case DP: e = tgv::launch_residual<double, double, double>(g, make_coef<double>(params), params->split, q, r, st); break;
    case SPDP: e = tgv::launch_residual<double, float, float>(g, make_coef<float>(params), params->split, q, r, st); break;
    case SPDP_C64: e = tgv::launch_residual<double, float, double>(g, make_coef<double>(params), params->split, q, r, st); break;
    case SP_DPC: e = tgv::launch_residual<float, float, double>(g, make_coef<double>(params), params->split, q, r, st); break;
    case SP: e = tgv::launch_residual<float, float, float>(g, make_coef<float>(params), params->split, q, r, st); break;
    case HPSP: e = tgv::launch_residual<float, f16, float>(g, make_coef<float>(params), params->split, q, r, st); break;
    case HPSP_BF16: e = tgv::launch_residual<float, bf16, float>(g, make_coef<float>(params), params->split, q, r, st); break;
    case HP: e = tgv::launch_residual<f16, f16, float>(g, make_coef<float>(params), params->split, q, r, st); break;
    case SPDP_WK: e = tgv::launch_residual<double, double, float>(g, make_coef<float>(params), params->split, q, r, st); break;
    case HPSP_WK: e = tgv::launch_residual<float, float, f16>(g, make_coef<f16>(params), params->split, q, r, st); break;
    case HPSP_RESWK: e = tgv::launch_residual<float, f16, f16>(g, make_coef<f16>(params), params->split, q, r, st); break;
    case HP_C16: e = tgv::launch_residual<f16, f16, f16>(g, make_coef<f16>(params), params->split, q, r, st); break;
    default: break;
  }
  return hip_status(e, "ns_residual");
}

int rk_stage(const ns_params_t* params, const ns_prec_t* prec, int stage, double dt, void* q, void* qt,
             const void* r, void* stream) {
  tgv::Grid g;
  Form f;
  int rc = check_params(params, &g);
  if (rc) return rc;
  if ((rc = check_prec(prec, &f))) return rc;
  if (stage < 0 || stage > 2) return fail(NS_ERR_ARG, "stage must be 0, 1 or 2");
  if (!std::isfinite(dt)) return fail(NS_ERR_ARG, "dt must be finite");
  if ((rc = check_ptr(q, "q")) || (rc = check_ptr(qt, "qt")) || (rc = check_ptr(r, "r"))) return rc;
  if (q == qt || q == r || qt == r) return fail(NS_ERR_ARG, "q, qt and r must be distinct arrays");
  hipStream_t st = as_stream(stream);
  hipError_t e = hipSuccess;
  using tgv::bf16;
  using tgv::f16;
  switch (f) {
    case DP:
    case SPDP_WK: e = tgv::launch_rk_stage<double, double, double, double>(g, stage, dt, q, qt, r, st); break;
    case SPDP:
    case SPDP_C64: e = tgv::launch_rk_stage<double, double, float, double>(g, stage, dt, q, qt, r, st); break;
    case SP_DPC: e = tgv::launch_rk_stage<float, float, float, double>(g, stage, dt, q, qt, r, st); break;
    case SP:
    case HPSP_WK: e = tgv::launch_rk_stage<float, float, float, float>(g, stage, dt, q, qt, r, st); break;
    case HPSP:
    case HPSP_RESWK: e = tgv::launch_rk_stage<float, float, f16, float>(g, stage, dt, q, qt, r, st); break;
    case HPSP_BF16: e = tgv::launch_rk_stage<float, float, bf16, float>(g, stage, dt, q, qt, r, st); break;
    case HP:
    case HP_C16: e = tgv::launch_rk_stage<f16, f16, f16, float>(g, stage, dt, q, qt, r, st); break;
    default: break;
  }
  return hip_status(e, "rk_stage");
}

int ns_residual_rk_stage(const ns_params_t* params, const ns_prec_t* prec, int stage, double dt, const void* q_in,
                         void* q_out, void* qt, void* stream) {
  tgv::Grid g;
  Form f;
  int rc = check_params(params, &g);
  if (rc) return rc;
  if ((rc = check_prec(prec, &f)) || (rc = check_split(params, f))) return rc;
  if (stage < 0 || stage > 2) return fail(NS_ERR_ARG, "stage must be 0, 1 or 2");
  if (!std::isfinite(dt)) return fail(NS_ERR_ARG, "dt must be finite");
  if ((rc = check_ptr(q_in, "q_in")) || (rc = check_ptr(q_out, "q_out")) || (rc = check_ptr(qt, "qt"))) return rc;
  if (q_in == q_out || q_in == qt || q_out == qt) return fail(NS_ERR_ARG, "q_in, q_out and qt must be distinct arrays");
  if ((rc = check_launch(tgv::residual_work_items(g), "ns_residual_rk_stage"))) return rc;
  hipStream_t st = as_stream(stream);
  hipError_t e = hipSuccess;
  using tgv::bf16;
  using tgv::f16;
  switch (f) {
    case DP:
      e = tgv::launch_residual_rk<double, double, double, double, double>(g, make_coef<double>(params), params->split, stage, dt,
                                                                          q_in, q_out, qt, st);
      break;
    case SPDP:
      e = tgv::launch_residual_rk<double, double, float, float, double>(g, make_coef<float>(params), params->split, stage, dt, q_in,
                                                                        q_out, qt, st);
      break;
    case SPDP_C64:
      e = tgv::launch_residual_rk<double, double, float, double, double>(g, make_coef<double>(params), params->split, stage, dt,
                                                                         q_in, q_out, qt, st);
      break;
    case SP_DPC:
      e = tgv::launch_residual_rk<float, float, float, double, double>(g, make_coef<double>(params), params->split, stage, dt, q_in,
                                                                       q_out, qt, st);
      break;
    case SP:
      e = tgv::launch_residual_rk<float, float, float, float, float>(g, make_coef<float>(params), params->split, stage, dt, q_in,
                                                                     q_out, qt, st);
      break;
    case HPSP:
      e = tgv::launch_residual_rk<float, float, f16, float, float>(g, make_coef<float>(params), params->split, stage, dt, q_in, q_out,
                                                                   qt, st);
      break;
    case HPSP_BF16:
      e = tgv::launch_residual_rk<float, float, bf16, float, float>(g, make_coef<float>(params), params->split, stage, dt, q_in,
                                                                    q_out, qt, st);
      break;
    case HP:
      e = tgv::launch_residual_rk<f16, f16, f16, float, float>(g, make_coef<float>(params), params->split, stage, dt, q_in, q_out, qt,
                                                               st);
      break;
    case SPDP_WK:
      e = tgv::launch_residual_rk<double, double, double, float, double>(g, make_coef<float>(params), params->split, stage, dt,
                                                                         q_in, q_out, qt, st);
      break;
    case HPSP_WK:
      e = tgv::launch_residual_rk<float, float, float, f16, float>(g, make_coef<f16>(params), params->split, stage, dt, q_in,
                                                                   q_out, qt, st);
      break;
    case HPSP_RESWK:
      e = tgv::launch_residual_rk<float, float, f16, f16, float>(g, make_coef<f16>(params), params->split, stage, dt, q_in,
                                                                 q_out, qt, st);
      break;
    case HP_C16:
      e = tgv::launch_residual_rk<f16, f16, f16, f16, float>(g, make_coef<f16>(params), params->split, stage, dt, q_in, q_out,
                                                             qt, st);
      break;
    default: break;
  }
  return hip_status(e, "ns_residual_rk_stage");
}

size_t flow_integrals_workspace_bytes(const ns_params_t* params) {
  tgv::Grid g;
  if (check_params(params, &g)) return 0;
  return (size_t)tgv::integrals_blocks(g) * 8 * sizeof(double);
}

int flow_integrals(const ns_params_t* params, const ns_prec_t* prec, const void* q, void* workspace, double* out8,
                   void* stream) {
  tgv::Grid g;
  Form f;
  int rc = check_params(params, &g);
  if (rc) return rc;
  if ((rc = check_prec(prec, &f))) return rc;
  if ((rc = check_ptr(q, "q")) || (rc = check_ptr(workspace, "workspace")) || (rc = check_ptr(out8, "out8")))
    return rc;
  if ((rc = check_launch(tgv::integrals_work_items(g), "flow_integrals"))) return rc;
  hipStream_t st = as_stream(stream);
  const tgv::Coef<double> c = make_coef<double>(params);
  hipError_t e;
  double* w = static_cast<double*>(workspace);
  switch (prec->q) {
    case NS_F64: e = tgv::launch_integrals<double>(g, c, q, w, out8, st); break;
    case NS_F32: e = tgv::launch_integrals<float>(g, c, q, w, out8, st); break;
    case NS_F16: e = tgv::launch_integrals<tgv::f16>(g, c, q, w, out8, st); break;
    default: return fail(NS_ERR_DTYPE, "unsupported q dtype for flow_integrals");
  }
  return hip_status(e, "flow_integrals");
}

int flow_integrals_noalloc(const ns_params_t* params, const ns_prec_t* prec, const void* q, double* out8,
                           void* stream) {
  tgv::Grid g;
  Form f;
  int rc = check_params(params, &g);
  if (rc) return rc;
  if ((rc = check_prec(prec, &f))) return rc;
  if ((rc = check_ptr(q, "q")) || (rc = check_ptr(out8, "out8"))) return rc;
  if ((rc = check_launch(tgv::integrals_work_items(g), "flow_integrals_noalloc"))) return rc;
  const long long rows = tgv::integrals_blocks(g);
  if (rows > tgv::kNoAllocRows)
    return fail(NS_ERR_SHAPE, "flow_integrals_noalloc: the grid needs " + std::to_string(rows) +
                                  " partial-sum rows, the static scratch holds " +
                                  std::to_string(tgv::kNoAllocRows) +
                                  " (flow_integrals_workspace_bytes() must be at most 4 MiB)");
  hipStream_t st = as_stream(stream);
  const tgv::Coef<double> c = make_coef<double>(params);
  hipError_t e;
  switch (prec->q) {
    case NS_F64: e = tgv::launch_integrals_noalloc<double>(g, c, q, out8, st); break;
    case NS_F32: e = tgv::launch_integrals_noalloc<float>(g, c, q, out8, st); break;
    case NS_F16: e = tgv::launch_integrals_noalloc<tgv::f16>(g, c, q, out8, st); break;
    default: return fail(NS_ERR_DTYPE, "unsupported q dtype for flow_integrals_noalloc");
  }
  return hip_status(e, "flow_integrals_noalloc");
}

}  // extern "C"

namespace {
int check_adjoint_prec(const ns_prec_t* prec, bool* f64) {
  Form f;
  int rc = check_prec(prec, &f);
  if (rc) return rc;
  if (f == DP) {
    *f64 = true;
    return NS_OK;
  }
  if (f == SP) {
    *f64 = false;
    return NS_OK;
  }
  return fail(NS_ERR_DTYPE, "the adjoint supports the DP (f64) and SP (f32) forms only");
}
}  // namespace

extern "C" {

size_t ns_residual_adjoint_workspace_bytes(const ns_params_t* params, const ns_prec_t* prec) {
  tgv::Grid g;
  bool f64;
  if (check_params(params, &g) || check_adjoint_prec(prec, &f64)) return 0;
  return (size_t)(tgv::kResidualAdjointWorkFields * g.N) * (f64 ? sizeof(double) : sizeof(float));
}

int ns_residual_adjoint(const ns_params_t* params, const ns_prec_t* prec, const void* q, const void* r_bar,
                        void* q_bar, void* workspace, void* stream) {
  tgv::Grid g;
  bool f64;
  int rc = check_params(params, &g);
  if (rc) return rc;
  if ((rc = check_adjoint_split(params))) return rc;
  if ((rc = check_adjoint_prec(prec, &f64))) return rc;
  if ((rc = check_ptr(q, "q")) || (rc = check_ptr(r_bar, "r_bar")) || (rc = check_ptr(q_bar, "q_bar")) ||
      (rc = check_ptr(workspace, "workspace")))
    return rc;
  if (q_bar == q || q_bar == r_bar) return fail(NS_ERR_ARG, "q_bar must not overlap q or r_bar");
  if ((rc = check_launch(tgv::adjoint_work_items(g), "ns_residual_adjoint"))) return rc;
  hipStream_t st = as_stream(stream);
  hipError_t e = f64 ? tgv::launch_residual_adjoint<double>(g, make_coef<double>(params), q, r_bar, q_bar,
                                                           workspace, st)
                     : tgv::launch_residual_adjoint<float>(g, make_coef<float>(params), q, r_bar, q_bar,
                                                          workspace, st);
  return hip_status(e, "ns_residual_adjoint");
}

int rk_stage_adjoint(const ns_params_t* params, const ns_prec_t* prec, int stage, double dt, const void* q_bar,
                     void* zeta, void* r_bar, void* stream) {
  tgv::Grid g;
  bool f64;
  int rc = check_params(params, &g);
  if (rc) return rc;
  if ((rc = check_adjoint_prec(prec, &f64))) return rc;
  if (stage < 0 || stage > 2) return fail(NS_ERR_ARG, "stage must be 0, 1 or 2");
  if (!std::isfinite(dt)) return fail(NS_ERR_ARG, "dt must be finite");
  if ((rc = check_ptr(q_bar, "q_bar")) || (rc = check_ptr(zeta, "zeta")) || (rc = check_ptr(r_bar, "r_bar")))
    return rc;
  hipStream_t st = as_stream(stream);
  hipError_t e = f64 ? tgv::launch_rk_stage_adjoint<double>(g, stage, dt, q_bar, zeta, r_bar, st)
                     : tgv::launch_rk_stage_adjoint<float>(g, stage, dt, q_bar, zeta, r_bar, st);
  return hip_status(e, "rk_stage_adjoint");
}

size_t flow_integrals_adjoint_workspace_bytes(const ns_params_t* params, const ns_prec_t* prec) {
  tgv::Grid g;
  bool f64;
  if (check_params(params, &g) || check_adjoint_prec(prec, &f64)) return 0;
  return (size_t)(3 * g.N) * (f64 ? sizeof(double) : sizeof(float));
}

int flow_integrals_adjoint(const ns_params_t* params, const ns_prec_t* prec, const void* q, double eps_bar,
                           void* q_bar, void* workspace, void* stream) {
  tgv::Grid g;
  bool f64;
  int rc = check_params(params, &g);
  if (rc) return rc;
  if ((rc = check_adjoint_prec(prec, &f64))) return rc;
  if (!std::isfinite(eps_bar)) return fail(NS_ERR_ARG, "eps_bar must be finite");
  if ((rc = check_ptr(q, "q")) || (rc = check_ptr(q_bar, "q_bar")) || (rc = check_ptr(workspace, "workspace")))
    return rc;
  if ((rc = check_launch(tgv::adjoint_work_items(g), "flow_integrals_adjoint"))) return rc;
  hipStream_t st = as_stream(stream);
  hipError_t e = f64 ? tgv::launch_integrals_adjoint<double>(g, make_coef<double>(params), q, eps_bar, q_bar,
                                                            workspace, st)
                     : tgv::launch_integrals_adjoint<float>(g, make_coef<float>(params), q, eps_bar, q_bar,
                                                           workspace, st);
  return hip_status(e, "flow_integrals_adjoint");
}

}  // extern "C"
