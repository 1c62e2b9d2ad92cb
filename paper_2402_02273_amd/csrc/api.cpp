// Host runtime of the C ABI declared in include/expint.h: argument
// validation, coefficient tables, the (s, m) plan, the Taylor-term schedule
// of one exponential Euler step and its HIP graph.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "context.hpp"
#include "internal.hpp"
#include "plan.hpp"
#include "autotune.hpp"
#include "modal.hpp"
#include "schedule.hpp"
#include "trace.hpp"

using namespace expint;

namespace expint {

namespace {
thread_local std::string g_last_error;
}

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

const char* last_error() { return g_last_error.c_str(); }
void clear_error() { g_last_error.clear(); }

size_t dtype_size(expint_dtype dt) { return dt == EXPINT_F64 ? 8 : 4; }

Arena::Arena() {
  const char* env = std::getenv("EXPINT_MAX_BYTES");
  if (env && *env) cap_ = static_cast<size_t>(std::strtoull(env, nullptr, 10));
}

Arena::~Arena() {
  for (auto& e : ptrs_) (void)hipFree(e.first);
}

void Arena::release(void* p) {
  if (!p) return;
  for (size_t i = 0; i < ptrs_.size(); ++i) {
    if (ptrs_[i].first == p) {
      (void)hipFree(p);
      bytes_ -= ptrs_[i].second;
      ptrs_.erase(ptrs_.begin() + static_cast<long>(i));
      return;
    }
  }
}

int Arena::alloc(void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 1;
  if (cap_ && bytes_ + bytes > cap_)
    return set_error(EXPINT_ENOMEM, "allocation of %zu bytes exceeds EXPINT_MAX_BYTES=%zu (in use %zu)", bytes,
                     cap_, bytes_);
  const hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return set_error(EXPINT_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  ptrs_.emplace_back(*p, bytes);
  bytes_ += bytes;
  return EXPINT_OK;
}

void destroy_graphs(std::vector<GraphEntry>& gs) {
  for (auto& e : gs) {
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (e.graph) (void)hipGraphDestroy(e.graph);
  }
  gs.clear();
}

}  // namespace expint

namespace expint {

bool finite_nonneg(double v) { return std::isfinite(v) && v >= 0.0; }

double harmonic_mean(double a, double b) {
  const double s = a + b;
  return s > 0.0 ? 2.0 * a * b / s : 0.0;
}

int ensure_device(expint_ctx* c) {
  int cur = -1;
  HIP_TRY(c, hipGetDevice(&cur));
  if (cur != c->device) HIP_TRY(c, hipSetDevice(c->device));
  return EXPINT_OK;
}

// Upload the class-pair tables for the current class_D (label form).
int upload_tables(expint_ctx* c) {
  double t64[kTab] = {0}, w64[kMaxClasses] = {0};
  const double inv_h2 = 1.0 / (c->h * c->h);
  for (int a = 0; a < c->nclass; ++a) {
    w64[a] = c->class_D[a] * inv_h2;
    for (int b = 0; b < c->nclass; ++b) t64[a * kMaxClasses + b] = harmonic_mean(c->class_D[a], c->class_D[b]) * inv_h2;
  }
  HIP_TRY(c, hipMemcpyAsync(c->tab64, t64, sizeof(t64), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->wall64, w64, sizeof(w64), hipMemcpyHostToDevice, c->stream));
  if (c->dtype == EXPINT_F64) {
    HIP_TRY(c, hipMemcpyAsync(c->tab, t64, sizeof(t64), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->wallc, w64, sizeof(w64), hipMemcpyHostToDevice, c->stream));
  } else {
    float t32[kTab], w32[kMaxClasses];
    for (int i = 0; i < kTab; ++i) t32[i] = static_cast<float>(t64[i]);
    for (int i = 0; i < kMaxClasses; ++i) w32[i] = static_cast<float>(w64[i]);
    HIP_TRY(c, hipMemcpyAsync(c->tab, t32, sizeof(t32), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->wallc, w32, sizeof(w32), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));  // the host arrays die at return
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return EXPINT_OK;
}

// Label scan: ||A||_1 and label validation (one synchronisation).
int scan_labels(expint_ctx* c, double* bad) {
  HIP_TRY(c, launch_scan_labels(c->bc, c->g, c->labels, c->nclass, c->tab64, c->wall64, c->partial, c->red,
                                c->stream));
  double out[2];
  HIP_TRY(c, hipMemcpyAsync(out, c->red, sizeof(out), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->norm1 = out[0];
  *bad = out[1];
  return EXPINT_OK;
}

double plan_norm(const expint_ctx* c) {
  return c->scheme == EXPINT_SCHEME_LINEARISED ? c->norm1 + c->rho : c->norm1;
}

int make_plan(expint_ctx* c) {
  if (c->fixed_plan) return EXPINT_OK;
  int s = 0, m = 0;
  const double nu = c->tau * plan_norm(c);
  const int m_min = c->scheme == EXPINT_SCHEME_EXPRK2 ? 2 : 1;
  if (!choose_plan(nu, c->tol, c->theta_max, &s, &m, m_min))
    return set_error(EXPINT_EINVAL, "no admissible plan for nu = %g (tol %g, theta_max %g)", nu, c->tol,
                     c->theta_max);
  c->s = s;
  c->m = m;
  return EXPINT_OK;
}

int run_ops(expint_ctx* c, const std::vector<TermOp>& ops, hipStream_t st) {
  const Coef cf = c->coef();
  for (const TermOp& op : ops) {
    if (op.pair) HIP_TRY(c, launch_pair(c->dtype, c->bc, c->g, c->ptiling, cf, op, st));
    else HIP_TRY(c, launch_term(c->dtype, c->bc, c->g, c->tiling, cf, op, st));
  }
  return EXPINT_OK;
}

int run_ops(expint_ctx* c, const std::vector<TermOp>& ops) { return run_ops(c, ops, c->stream); }

StepBuffers step_buffers(expint_ctx* c) {
  StepBuffers sb;
  sb.b = c->b;
  sb.y[0] = c->y[0];
  sb.y[1] = c->y[1];
  sb.acc[0] = c->acc[0];
  sb.acc[1] = c->acc[1];
  return sb;
}

std::vector<TermOp> step_schedule(expint_ctx* c, const void* b, void* x_out, void* u, const StepBuffers* sb) {
  const StepBuffers ws = sb ? *sb : step_buffers(c);
  if (c->ptiling.ty != 0 && c->labels_form && c->m >= 2)
    return phi1_schedule_pairs(ws, c->s, c->m, c->tau, b, x_out, u);
  return phi1_schedule(ws, c->s, c->m, c->tau, b, x_out, u);
}

// Launches of one step on stream st (no synchronisation), with the step
// buffers sb as workspace (NULL: the context's).  The right-hand side is
// A u + f(u) for both schemes (for LINEARISED it is J_n u_n + rho u_n^2, the
// same field); LINEARISED applies phi1 to J_n, taken at u before the last
// sweep adds the result into it.  The modal and EXPRK2 forms run on the
// context stream with the context's buffers only.
int enqueue_step_on(expint_ctx* c, void* u, hipStream_t st, const StepBuffers* sb) {
  if ((st != c->stream || sb) && (c->algo == EXPINT_ALGO_MODAL || c->scheme == EXPINT_SCHEME_EXPRK2))
    return set_error(EXPINT_EUNSUPPORTED, "this step runs on the context stream only");
  void* const bv = sb ? sb->b : c->b;
  // the modal form with z transforms forms b inside its first pass
  if (c->algo == EXPINT_ALGO_MODAL && modal_fuses_rhs(c)) return modal_phi1(c, nullptr, u, true, u);
  HIP_TRY(c, launch_rhs(c->dtype, c->bc, c->g, c->tiling, c->coef(), u, bv, c->rho, st));
  if (c->algo == EXPINT_ALGO_MODAL) return modal_phi1(c, c->b, u, true);
  if (c->scheme == EXPINT_SCHEME_EXPRK2) {
    // stage 1: X = tau phi1(tau A) b; d = f(u + X) - f(u); stage 2 adds
    // tau phi1(tau A) b + tau phi2(tau A) d into u (phi1 b recomputed: the
    // phi2 part needs the same sweeps, d enters two of them per sub-step)
    int rc = run_ops(c, phi1_schedule(step_buffers(c), c->s, c->m, c->tau, c->b, c->stage, nullptr));
    if (rc) return rc;
    HIP_TRY(c, launch_reaction_increment(c->dtype, c->g.n, c->rho, u, c->stage, c->dvec, c->stream));
    return run_ops(c, phi1_schedule(step_buffers(c), c->s, c->m, c->tau, c->b, nullptr, u, c->dvec));
  }
  std::vector<TermOp> ops = step_schedule(c, bv, nullptr, u, sb);
  if (c->scheme == EXPINT_SCHEME_LINEARISED) set_linearised(ops, u, c->rho);
  return run_ops(c, ops, st);
}

int enqueue_step(expint_ctx* c, void* u) { return enqueue_step_on(c, u, c->stream, nullptr); }

int check_finite_field(expint_ctx* c, const void* u) {
  HIP_TRY(c, launch_reduce(c->dtype, 3, u, nullptr, c->g.n, c->partial, c->red, c->stream));
  double cnt = 0.0;
  HIP_TRY(c, hipMemcpyAsync(&cnt, c->red, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (cnt != 0.0) return set_error(EXPINT_ENONFINITE, "state holds %.0f non-finite values", cnt);
  return EXPINT_OK;
}

}  // namespace expint

namespace {

int validate_opts(const expint_opts* o) {
  const int dt = enum_value(o->dtype);
  if (dt != EXPINT_F64 && dt != EXPINT_F32) return set_error(EXPINT_EINVAL, "unknown dtype %d", dt);
  if (!(o->tau > 0.0) || !std::isfinite(o->tau)) return set_error(EXPINT_EINVAL, "tau must be finite and > 0");
  if (!(o->tol >= 0.0) || !std::isfinite(o->tol)) return set_error(EXPINT_EINVAL, "tol must be finite and >= 0");
  if (!(o->theta_max >= 0.0) || !std::isfinite(o->theta_max))
    return set_error(EXPINT_EINVAL, "theta_max must be finite and >= 0");
  if ((o->s > 0) != (o->m > 0) || o->s < 0 || o->m < 0)
    return set_error(EXPINT_EINVAL, "give both s and m (> 0) or neither");
  if (o->m > kPlanMaxDegree) return set_error(EXPINT_EINVAL, "m must be <= %d", kPlanMaxDegree);
  const int algo = enum_value(o->algo), mp = enum_value(o->mp), sw = enum_value(o->sweeps);
  const int scheme = enum_value(o->scheme);
  if (algo < EXPINT_ALGO_AUTO || algo > EXPINT_ALGO_MODAL) return set_error(EXPINT_EINVAL, "unknown algo");
  if (mp < EXPINT_MP_NONE || mp > EXPINT_MP_FP16_SPLIT) return set_error(EXPINT_EINVAL, "unknown mp");
  if (sw < EXPINT_SWEEPS_AUTO || sw > EXPINT_SWEEPS_PAIRS) return set_error(EXPINT_EINVAL, "unknown sweeps");
  if (scheme < EXPINT_SCHEME_EXP_EULER || scheme > EXPINT_SCHEME_EXPRK2)
    return set_error(EXPINT_EINVAL, "unknown scheme");
  return EXPINT_OK;
}

}  // namespace

extern "C" {

int expint_opts_default(expint_opts* o) {
  if (!o) return set_error(EXPINT_EINVAL, "opts is NULL");
  std::memset(o, 0, sizeof(*o));
  o->dtype = EXPINT_F32;
  o->tau = 7.3;
  o->algo = EXPINT_ALGO_AUTO;
  o->mp = EXPINT_MP_NONE;
  return EXPINT_OK;
}

const char* expint_last_error(void) { return expint::last_error(); }

int expint_create(const expint_grid* grid, const expint_dfield* df, double rho, expint_bc bc,
                  const expint_opts* opts, expint_ctx** out) {
  PhaseRange range("expint_create");
  if (out) *out = nullptr;
  if (!grid || !df || !opts || !out) return set_error(EXPINT_EINVAL, "NULL argument");
  if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1)
    return set_error(EXPINT_EINVAL, "grid dims must be >= 1 (got %d %d %d)", grid->nx, grid->ny, grid->nz);
  if (!(grid->h > 0.0) || !std::isfinite(grid->h)) return set_error(EXPINT_EINVAL, "h must be finite and > 0");
  if (!finite_nonneg(rho)) return set_error(EXPINT_EINVAL, "rho must be finite and >= 0");
  if (enum_value(bc) != EXPINT_NOFLUX && enum_value(bc) != EXPINT_DIRICHLET0)
    return set_error(EXPINT_EINVAL, "unknown bc %d", enum_value(bc));
  int rc = validate_opts(opts);
  if (rc) return rc;
  if ((df->labels == nullptr) == (df->D == nullptr))
    return set_error(EXPINT_EINVAL, "give exactly one of labels and D");
  // 32-bit voxel indices, with room for the sweeps' one-past-the-chunk offsets
  if (product_within(static_cast<int64_t>(grid->nx) + 16, grid->ny, grid->nz, (int64_t(1) << 31) - 1) < 0)
    return set_error(EXPINT_EINVAL, "grid too large (%d x %d x %d)", grid->nx, grid->ny, grid->nz);
  const int64_t n = static_cast<int64_t>(grid->nx) * grid->ny * grid->nz;
  if (df->labels) {
    if (df->n_classes < 1 || df->n_classes > EXPINT_MAX_CLASSES)
      return set_error(EXPINT_EINVAL, "n_classes must be in 1..%d", EXPINT_MAX_CLASSES);
    if (!df->class_D) return set_error(EXPINT_EINVAL, "class_D is NULL");
    for (int a = 0; a < df->n_classes; ++a)
      if (!finite_nonneg(df->class_D[a])) return set_error(EXPINT_EINVAL, "class_D[%d] must be finite and >= 0", a);
  }
  const expint_algo algo = opts->algo == EXPINT_ALGO_AUTO ? EXPINT_ALGO_STENCIL_TAYLOR : opts->algo;
  if (opts->mp != EXPINT_MP_NONE && algo != EXPINT_ALGO_MODAL)
    return set_error(EXPINT_EUNSUPPORTED, "split matrix-core products belong to the modal algorithm");
  if (opts->mp != EXPINT_MP_NONE && opts->dtype == EXPINT_F64)
    return set_error(EXPINT_EUNSUPPORTED, "split matrix-core products are for FP32 contexts");
  if (opts->sweeps == EXPINT_SWEEPS_PAIRS && !df->labels)
    return set_error(EXPINT_EUNSUPPORTED, "pair sweeps need the label form of D");
  if (opts->scheme == EXPINT_SCHEME_LINEARISED && algo == EXPINT_ALGO_MODAL)
    return set_error(EXPINT_EUNSUPPORTED, "the linearised operator is not separable: no modal path");
  if (opts->scheme == EXPINT_SCHEME_EXPRK2 && algo == EXPINT_ALGO_MODAL)
    return set_error(EXPINT_EUNSUPPORTED, "the EXPRK2 scheme runs on the stencil-Taylor path");
  if (opts->scheme != EXPINT_SCHEME_EXP_EULER && opts->sweeps == EXPINT_SWEEPS_PAIRS)
    return set_error(EXPINT_EUNSUPPORTED, "the LINEARISED and EXPRK2 schemes use single-term sweeps");
  if (algo == EXPINT_ALGO_MODAL) {
    if (!df->labels) return set_error(EXPINT_EUNSUPPORTED, "the modal path needs the label form of D");
    if (grid->nx % 32 || grid->ny % 32 || grid->nz % 32)
      return set_error(EXPINT_EUNSUPPORTED, "the modal path needs every grid dimension to be a multiple of 32");
  }

  expint_ctx* c = new (std::nothrow) expint_ctx();
  if (!c) return set_error(EXPINT_ENOMEM, "host allocation failed");
  auto bail = [&](int code) {
    expint_destroy(c);
    return code;
  };
  c->g.nx = grid->nx;
  c->g.ny = grid->ny;
  c->g.nz = grid->nz;
  c->g.n = n;
  c->h = grid->h;
  c->dtype = opts->dtype;
  c->bc = bc;
  c->algo = algo;
  c->mp = opts->mp;
  c->scheme = opts->scheme;
  c->rho = rho;
  c->tau = opts->tau;
  default_tolerances(c->dtype, &c->tol, &c->theta_max);
  if (opts->tol > 0.0) c->tol = opts->tol;
  if (opts->theta_max > 0.0) c->theta_max = opts->theta_max;
  c->fixed_plan = opts->s > 0;
  if (c->fixed_plan) {
    c->s = opts->s;
    c->m = opts->m;
  }
  c->check_finite = opts->check_finite;
  c->labels_form = df->labels != nullptr;
  {
    const char* ge = std::getenv("EXPINT_GRAPH");
    c->use_graph = !(ge && ge[0] == '0');
  }

  if (field_block_count(c->g) > (int64_t(1) << 31) - 1) return bail(set_error(EXPINT_EINVAL, "grid too large"));
  {
    // The field buffers every context needs (b, two terms, two running sums;
    // the stage and increment of EXPRK2; the labels or the four dense face
    // fields) against EXPINT_MAX_BYTES, before the device is touched.
    const size_t fb = c->field_bytes();
    size_t need = (c->scheme == EXPINT_SCHEME_EXPRK2 ? 7 : 5) * fb;
    need += c->labels_form ? static_cast<size_t>(n) : 4 * fb;
    if (c->arena.cap() && need > c->arena.cap())
      return bail(set_error(EXPINT_ENOMEM, "the workspace needs at least %zu bytes, above EXPINT_MAX_BYTES=%zu", need,
                            c->arena.cap()));
  }
  if (hipGetDevice(&c->device) != hipSuccess) {
    (void)hipGetLastError();
    return bail(set_error(EXPINT_EHIP, "no HIP device"));
  }
  if (opts->stream) {
    c->stream = static_cast<hipStream_t>(opts->stream);
  } else {
    // A blocking stream of our own: ordered with the null stream, and
    // capturable into a graph (the null stream is not).
    if (hipStreamCreate(&c->stream) != hipSuccess) {
      (void)hipGetLastError();
      return bail(set_error(EXPINT_EHIP, "hipStreamCreate failed"));
    }
    c->own_stream = true;
  }

  const size_t fb = c->field_bytes();
  // partial sums: the scans write two per voxel-kernel workgroup, the
  // reductions one per reduction workgroup
  const int64_t nparts = std::max<int64_t>(field_block_count(c->g), kReduceBlocks);
  if ((rc = c->arena.alloc(reinterpret_cast<void**>(&c->partial), 2 * nparts * sizeof(double)))) return bail(rc);
  if ((rc = c->arena.alloc(reinterpret_cast<void**>(&c->red), 2 * sizeof(double)))) return bail(rc);

  double bad = 0.0;
  PhaseRange scan_range("expint_create: coefficients, norm scan, plan");
  if (c->labels_form) {
    c->nclass = df->n_classes;
    for (int a = 0; a < c->nclass; ++a) c->class_D[a] = df->class_D[a];
    if ((rc = c->arena.alloc(reinterpret_cast<void**>(&c->labels), static_cast<size_t>(n)))) return bail(rc);
    if ((rc = c->arena.alloc(reinterpret_cast<void**>(&c->tab64), kTab * sizeof(double)))) return bail(rc);
    if ((rc = c->arena.alloc(reinterpret_cast<void**>(&c->wall64), kMaxClasses * sizeof(double)))) return bail(rc);
    if ((rc = c->arena.alloc(&c->tab, kTab * sizeof(double)))) return bail(rc);
    if ((rc = c->arena.alloc(&c->wallc, kMaxClasses * sizeof(double)))) return bail(rc);
    if (hipMemcpyAsync(c->labels, df->labels, static_cast<size_t>(n), hipMemcpyDefault, c->stream) != hipSuccess) {
      (void)hipGetLastError();
      return bail(set_error(EXPINT_EINVAL, "labels pointer is not readable"));
    }
    if ((rc = upload_tables(c))) return bail(rc);
    if ((rc = scan_labels(c, &bad))) return bail(rc);
    if (bad != 0.0) return bail(set_error(EXPINT_EINVAL, "a label is >= n_classes (%d)", c->nclass));
  } else {
    if ((rc = c->arena.alloc(&c->fx, fb))) return bail(rc);
    if ((rc = c->arena.alloc(&c->fy, fb))) return bail(rc);
    if ((rc = c->arena.alloc(&c->fz, fb))) return bail(rc);
    if ((rc = c->arena.alloc(&c->wallv, fb))) return bail(rc);
    const hipError_t e = launch_scan_dense(c->dtype, c->bc, c->g, df->D, 1.0 / (c->h * c->h), c->fx, c->fy, c->fz,
                                           c->wallv, c->partial, c->red, c->stream);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return bail(set_error(EXPINT_EHIP, "dense scan failed: %s", hipGetErrorString(e)));
    }
    double out2[2];
    if (hipMemcpyAsync(out2, c->red, sizeof(out2), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
      (void)hipGetLastError();
      return bail(set_error(EXPINT_EHIP, "dense scan readback failed"));
    }
    c->norm1 = out2[0];
    if (out2[1] != 0.0) return bail(set_error(EXPINT_EINVAL, "D holds a negative or non-finite value"));
  }
  if ((rc = make_plan(c))) return bail(rc);

  if ((rc = c->arena.alloc(&c->b, fb))) return bail(rc);
  if (c->scheme == EXPINT_SCHEME_EXPRK2) {
    if ((rc = c->arena.alloc(&c->stage, fb))) return bail(rc);
    if ((rc = c->arena.alloc(&c->dvec, fb))) return bail(rc);
  }
  for (int i = 0; i < 2; ++i) {
    if ((rc = c->arena.alloc(&c->y[i], fb))) return bail(rc);
    if ((rc = c->arena.alloc(&c->acc[i], fb))) return bail(rc);
  }
  scan_range.end();
  PhaseRange tune_range("expint_create: sweep autotuning");
  {
    const bool lin = c->scheme == EXPINT_SCHEME_LINEARISED;
    const hipError_t e = autotune_sweep(c->dtype, c->bc, c->g, c->coef(), c->y[0], c->acc[0], c->y[1], c->stream,
                                        true, &c->tiling, lin ? c->acc[1] : nullptr, c->rho);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return bail(set_error(EXPINT_EHIP, "autotune failed: %s", hipGetErrorString(e)));
    }
  }
  if (const char* f = std::getenv("EXPINT_FACE_LP")) {
    // planes per lane of the adjoint's fused reverse sweeps (default 1)
    const int v = std::atoi(f);
    if (v == 1 || v == 2 || v == 4) c->tiling.flp = v;
  }
  if (c->algo != EXPINT_ALGO_MODAL && c->scheme == EXPINT_SCHEME_EXP_EULER) {
    const hipError_t e = autotune_pairs(c->dtype, c->bc, c->g, c->coef(), c->y[0], c->acc[0], c->y[1], c->stream,
                                        c->tiling, opts->sweeps, &c->ptiling);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return bail(set_error(EXPINT_EHIP, "pair-sweep autotune failed: %s", hipGetErrorString(e)));
    }
  }
  tune_range.end();
  if (c->algo == EXPINT_ALGO_MODAL) {
    PhaseRange modal_range("expint_create: modal set-up");
    if ((rc = modal_setup(c))) return bail(rc);
  }
  if (std::getenv("EXPINT_LOG"))
    std::fprintf(stderr,
                 "[expint] grid %dx%dx%d h=%g dtype=%s scheme=%s ||A||_1=%.17g nu=%.6g plan s=%d m=%d workspace %zu B\n",
                 c->g.nx, c->g.ny, c->g.nz, c->h, c->dtype == EXPINT_F64 ? "f64" : "f32",
                 c->scheme == EXPINT_SCHEME_LINEARISED ? "linearised"
                 : c->scheme == EXPINT_SCHEME_EXPRK2  ? "exprk2"
                                                      : "exp-euler",
                 c->norm1, c->tau * plan_norm(c),
                 c->s, c->m, c->arena.bytes());
  if (const char* f = std::getenv("EXPINT_FAIL_NTH_HIP")) c->fail_countdown = std::strtoll(f, nullptr, 10);
  *out = c;
  expint::clear_error();
  return EXPINT_OK;
}

void expint_destroy(expint_ctx* c) {
  if (!c) return;
  int cur = -1;
  if (hipGetDevice(&cur) == hipSuccess && cur != c->device) (void)hipSetDevice(c->device);
  if (c->stream && !c->poisoned) (void)hipStreamSynchronize(c->stream);
  destroy_graphs(c->graphs);
  auto& a = c->adj;
  if (a.rec) {
    if (!c->poisoned) (void)hipStreamSynchronize(a.rec);
    (void)hipStreamDestroy(a.rec);
  }
  for (hipEvent_t e : {a.ev_fwd, a.ev_seg[0], a.ev_seg[1], a.ev_segfree[0], a.ev_segfree[1]})
    if (e) (void)hipEventDestroy(e);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  const int dev = c->device;
  delete c;  // the arena frees the device buffers
  if (cur >= 0 && cur != dev) (void)hipSetDevice(cur);
}

int expint_get_plan(const expint_ctx* c, int32_t* s, int32_t* m, double* norm1) {
  if (!c) return set_error(EXPINT_EINVAL, "context is NULL");
  if (s) *s = c->s;
  if (m) *m = c->m;
  if (norm1) *norm1 = c->norm1;
  return EXPINT_OK;
}

int expint_get_launch(const expint_ctx* c, expint_launch_info* info) {
  if (!c || !info) return set_error(EXPINT_EINVAL, "NULL argument");
  const bool pairs = c->ptiling.ty != 0;
  info->sweeps = pairs ? EXPINT_SWEEPS_PAIRS : EXPINT_SWEEPS_SINGLE;
  info->pair_ty = pairs ? c->ptiling.ty : 0;
  info->pair_lp = pairs ? c->ptiling.lp : 0;
  info->vec = c->tiling.vec ? 1 : 0;
  info->bx = c->tiling.vec ? 0 : c->tiling.bx;
  info->by = c->tiling.vec ? 0 : c->tiling.by;
  info->rw = c->tiling.vec ? c->tiling.rw : 0;
  info->lp = c->tiling.lp;
  info->nt = c->tiling.vec && c->scheme != EXPINT_SCHEME_LINEARISED ? c->tiling.nt : 0;
  info->modal_dct = 0;
  if (c->algo == EXPINT_ALGO_MODAL)
    for (int ax = 0; ax < 3; ++ax)
      if (c->modal.dct_tw[ax]) info->modal_dct |= 1 << ax;
  return EXPINT_OK;
}

int expint_set_params(expint_ctx* c, double rho, const double* class_D, int32_t replan) {
  CHECK_CTX(c);
  if (!finite_nonneg(rho)) return set_error(EXPINT_EINVAL, "rho must be finite and >= 0");
  int rc = ensure_device(c);
  if (rc) return rc;
  if (class_D) {
    if (!c->labels_form) return set_error(EXPINT_EINVAL, "class_D given for a dense-D context");
    for (int a = 0; a < c->nclass; ++a)
      if (!finite_nonneg(class_D[a])) return set_error(EXPINT_EINVAL, "class_D[%d] must be finite and >= 0", a);
    // the modal form keeps a uniform D: checked before anything changes
    if (c->algo == EXPINT_ALGO_MODAL && (rc = modal_diffusivity(c, class_D, false))) return rc;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int a = 0; a < c->nclass; ++a) c->class_D[a] = class_D[a];
    if (c->algo == EXPINT_ALGO_MODAL) (void)modal_diffusivity(c, class_D, true);
    if ((rc = upload_tables(c))) return rc;
  }
  c->rho = rho;
  if (replan) {
    // ||A||_1 changes with class_D (label form); the LINEARISED bound also with rho
    if (c->labels_form) {
      double bad = 0.0;
      if ((rc = scan_labels(c, &bad))) return rc;
    }
    if ((rc = make_plan(c))) return rc;
  }
  // rho and the schedule are baked into recorded graphs; a launch of one may
  // still be running on the stream
  if (!c->graphs.empty()) HIP_TRY(c, hipStreamSynchronize(c->stream));
  destroy_graphs(c->graphs);
  return EXPINT_OK;
}

int expint_apply(expint_ctx* c, const void* x, void* y) {
  CHECK_CTX(c);
  if (!x || !y) return set_error(EXPINT_EINVAL, "NULL field");
  if (x == y) return set_error(EXPINT_EINVAL, "x and y must not overlap");
  int rc = ensure_device(c);
  if (rc) return rc;
  HIP_TRY(c, launch_apply(c->dtype, c->bc, c->g, c->tiling, c->coef(), x, y, c->stream));
  return EXPINT_OK;
}

int expint_rhs(expint_ctx* c, const void* u, void* b) {
  CHECK_CTX(c);
  if (!u || !b) return set_error(EXPINT_EINVAL, "NULL field");
  if (u == b) return set_error(EXPINT_EINVAL, "u and b must not overlap");
  int rc = ensure_device(c);
  if (rc) return rc;
  HIP_TRY(c, launch_rhs(c->dtype, c->bc, c->g, c->tiling, c->coef(), u, b, c->rho, c->stream));
  return EXPINT_OK;
}

int expint_phi1(expint_ctx* c, const void* b, void* x) {
  CHECK_CTX(c);
  if (!b || !x) return set_error(EXPINT_EINVAL, "NULL field");
  if (b == x) return set_error(EXPINT_EINVAL, "b and x must not overlap");
  int rc = ensure_device(c);
  if (rc) return rc;
  if (c->algo == EXPINT_ALGO_MODAL) return modal_phi1(c, b, x, false);
  return run_ops(c, step_schedule(c, b, x, nullptr, nullptr));
}

int expint_phi12(expint_ctx* c, const void* b, const void* d, void* x) {
  CHECK_CTX(c);
  if (!b || !d || !x) return set_error(EXPINT_EINVAL, "NULL field");
  if (c->algo == EXPINT_ALGO_MODAL || c->scheme == EXPINT_SCHEME_LINEARISED)
    return set_error(EXPINT_EUNSUPPORTED, "phi1 + phi2 needs a stencil-Taylor EXP_EULER or EXPRK2 context");
  if (b == x || d == x) return set_error(EXPINT_EINVAL, "x must overlap neither b nor d");
  int rc = ensure_device(c);
  if (rc) return rc;
  return run_ops(c, phi1_schedule(step_buffers(c), c->s, c->m, c->tau, b, x, nullptr, d));
}

int expint_phi1_lin(expint_ctx* c, const void* u, const void* b, void* x) {
  CHECK_CTX(c);
  if (!u || !b || !x) return set_error(EXPINT_EINVAL, "NULL field");
  if (c->scheme != EXPINT_SCHEME_LINEARISED)
    return set_error(EXPINT_EUNSUPPORTED, "phi1 of the linearised operator needs a LINEARISED context");
  if (b == x || u == x) return set_error(EXPINT_EINVAL, "x must overlap neither u nor b");
  int rc = ensure_device(c);
  if (rc) return rc;
  std::vector<TermOp> ops = step_schedule(c, b, x, nullptr, nullptr);
  set_linearised(ops, u, c->rho);
  return run_ops(c, ops);
}

int expint_step(expint_ctx* c, void* u) {
  CHECK_CTX(c);
  if (!u) return set_error(EXPINT_EINVAL, "u is NULL");
  int rc = ensure_device(c);
  if (rc) return rc;
  if ((rc = enqueue_step(c, u))) return rc;
  if (c->check_finite) return check_finite_field(c, u);
  return EXPINT_OK;
}

int expint_advance(expint_ctx* c, void* u, int32_t nsteps) {
  PhaseRange range("expint_advance");
  CHECK_CTX(c);
  if (!u) return set_error(EXPINT_EINVAL, "u is NULL");
  if (nsteps < 0) return set_error(EXPINT_EINVAL, "nsteps must be >= 0");
  int rc = ensure_device(c);
  if (rc) return rc;
  if (nsteps == 0) return EXPINT_OK;
  if ((rc = run_steps(c, u, nsteps))) return rc;
  if (c->check_finite) return check_finite_field(c, u);
  return EXPINT_OK;
}

int expint_advance_volumes(expint_ctx* c, void* u, int32_t nsteps, double* volumes) {
  CHECK_CTX(c);
  if (!u || (nsteps > 0 && !volumes)) return set_error(EXPINT_EINVAL, "NULL argument");
  if (nsteps < 0) return set_error(EXPINT_EINVAL, "nsteps must be >= 0");
  int rc = ensure_device(c);
  if (rc) return rc;
  if (nsteps == 0) return EXPINT_OK;
  auto& d = c->diag;
  if (d.vol_cap < nsteps) {
    c->arena.release(d.vol);
    d.vol = nullptr;
    d.vol_cap = 0;
    if ((rc = c->arena.alloc(reinterpret_cast<void**>(&d.vol), static_cast<size_t>(nsteps) * sizeof(double))))
      return rc;
    d.vol_cap = nsteps;
  }
  // each step, then sum u (fixed-order FP64 reduction) into slot k
  for (int32_t k = 0; k < nsteps; ++k) {
    if ((rc = run_steps(c, u, 1))) return rc;
    HIP_TRY(c, launch_reduce(c->dtype, 0, u, nullptr, c->g.n, c->partial, d.vol + k, c->stream));
  }
  HIP_TRY(c, hipMemcpyAsync(volumes, d.vol, static_cast<size_t>(nsteps) * sizeof(double), hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int32_t k = 0; k < nsteps; ++k) volumes[k] /= static_cast<double>(c->g.n);
  if (c->check_finite) return check_finite_field(c, u);
  return EXPINT_OK;
}

}  // extern "C"

namespace expint {

int run_steps(expint_ctx* c, void* u, int32_t nsteps) {
  int rc = EXPINT_OK;
  if (!c->use_graph) {
    for (int32_t i = 0; i < nsteps; ++i)
      if ((rc = enqueue_step(c, u))) return rc;
    return EXPINT_OK;
  }
  GraphEntry* ge = nullptr;
  for (auto& e : c->graphs)
    if (e.key0 == u) ge = &e;
  if (!ge) {
    if (c->graphs.size() >= 4) {
      // a launch of the evicted graph may still be running on the stream
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      std::vector<GraphEntry> old(c->graphs.begin(), c->graphs.begin() + 1);
      destroy_graphs(old);
      c->graphs.erase(c->graphs.begin());
    }
    GraphEntry e;
    e.key0 = u;
    e.nsteps = 1;
    PhaseRange range("record step graph");
    HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    rc = enqueue_step(c, u);
    hipGraph_t gr = nullptr;
    const hipError_t ec = hipStreamEndCapture(c->stream, &gr);
    if (rc) {
      if (gr) (void)hipGraphDestroy(gr);
      return rc;
    }
    if (ec != hipSuccess) {
      c->poisoned = true;
      return set_error(EXPINT_EHIP, "hipStreamEndCapture failed: %s", hipGetErrorString(ec));
    }
    e.graph = gr;
    const hipError_t ei = hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      (void)hipGraphDestroy(e.graph);
      c->poisoned = true;
      return set_error(EXPINT_EHIP, "hipGraphInstantiate failed: %s", hipGetErrorString(ei));
    }
    c->graphs.push_back(e);
    ge = &c->graphs.back();
  }
  for (int32_t i = 0; i < nsteps; ++i) HIP_TRY(c, hipGraphLaunch(ge->exec, c->stream));
  return EXPINT_OK;
}

}  // namespace expint

extern "C" {

int expint_reduce(expint_ctx* c, int32_t op, const void* x, const void* y, double* out) {
  CHECK_CTX(c);
  if (op < 0 || op > 3) return set_error(EXPINT_EINVAL, "reduce op must be 0, 1, 2 or 3");
  if (!x || !out || (op == 1 && !y)) return set_error(EXPINT_EINVAL, "NULL argument");
  int rc = ensure_device(c);
  if (rc) return rc;
  // op 3, the mean, is the sum (op 0) over the voxel count
  HIP_TRY(c, launch_reduce(c->dtype, op == 3 ? 0 : op, x, y, c->g.n, c->partial, c->red, c->stream));
  HIP_TRY(c, hipMemcpyAsync(out, c->red, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (op == 3) *out /= static_cast<double>(c->g.n);
  return EXPINT_OK;
}

int expint_profile(expint_ctx* c, int32_t kernel, int32_t reps, double* ms) {
  CHECK_CTX(c);
  if (reps < 1 || !ms) return set_error(EXPINT_EINVAL, "reps must be >= 1 and ms non-NULL");
  if (kernel < 0 || kernel > 6) return set_error(EXPINT_EINVAL, "kernel id must be in 0..6");
  if (kernel == 6 && !c->adj.fpart)
    return set_error(EXPINT_EUNSUPPORTED, "kernel id 6 times the gradient's reverse sweep: run a gradient first");
  if ((kernel == 3 || kernel == 4) && c->algo != EXPINT_ALGO_MODAL)
    return set_error(EXPINT_EINVAL, "kernel ids 3 and 4 time the modal path's mode products");
  if (kernel == 5 && c->ptiling.ty == 0)
    return set_error(EXPINT_EUNSUPPORTED, "this context does not use pair sweeps");
  int rc = ensure_device(c);
  if (rc) return rc;
  // The sweeps of the step schedule, on the context workspace:
  // 0 = pair-flush term (src y0, running sum updated in place, y1 written),
  // 1 = skip term (src y0, y1 written), 2 = right-hand side (u = acc1, b),
  // 5 = pair sweep inside a sub-step (src y0, two terms added to the running
  // sum in place, the second term written to y1).  LINEARISED contexts time
  // 0 and 1 as sweeps of the linearised operator (u_n = acc1).
  TermOp op;
  op.src = c->y[0];
  op.c = c->tau / c->s / 2.0;
  op.y_out = c->y[1];
  if (kernel == 0 || kernel == 5) {
    op.acc_in = c->acc[0];
    op.ca = 1.0;
    op.cs = kernel == 0 ? 1.0 : 0.0;
    op.acc_out = c->acc[0];
  }
  if (kernel == 5) {
    op.pair = 1;
    op.c2 = c->tau / c->s / 3.0;
  } else {
    classify_term(op);
  }
  if ((kernel == 0 || kernel == 1) && c->scheme == EXPINT_SCHEME_LINEARISED) {
    op.ju = c->acc[1];  // the state u_n (filled below)
    op.jrho = c->rho;
  }
  const Coef cf = c->coef();
  ModalArgs ma;
  const bool mode = kernel == 3 || kernel == 4;
  if (mode) {
    ma.q = c->modal.q[kernel == 3 ? 0 : 2][0];
    ma.in = c->acc[1];
    ma.out = c->y[1];
    if (kernel == 3) {  // x axis: left product over (1, nx, ny*nz)
      ma.pre = 1;
      ma.n = c->g.nx;
      ma.post = static_cast<long>(c->g.ny) * c->g.nz;
    } else {  // z axis: right product over (nx*ny, nz)
      ma.pre = c->g.nx * c->g.ny;
      ma.n = c->g.nz;
      ma.post = 1;
    }
  }
  // an axis whose products run as fast transforms: the pass the step runs
  // (x: forward transform, multiplier and inverse transform; z: the forward
  // transform)
  const int max = kernel == 3 ? 0 : 2;
  const bool dct = mode && c->modal.dct_tw[max] != nullptr;
  DctArgs da;
  if (dct) {
    da.in = ma.in;
    da.out = ma.out;
    da.pre = ma.pre;
    da.n = ma.n;
    da.post = ma.post;
    da.tw = c->modal.dct_tw[max];
    da.mk = c->modal.dct_mk[max];
    da.lam_x = c->modal.lam[0];
    da.lam_y = c->modal.lam[1];
    da.lam_z = c->modal.lam[2];
    da.tauD = c->tau * c->modal.Dc;
    da.tau = c->tau;
    da.nz = c->g.nz;
  }
  // 6: the gradient's fused reverse sweep, a Taylor term (source y0, second
  // source acc0, term written to y1) with the class face products against the
  // tape field acc1 into the gradient's slots (zeroed again afterwards)
  TermOp rop;
  const bool lin = c->scheme == EXPINT_SCHEME_LINEARISED;
  if (kernel == 6) {
    rop.src = c->y[0];
    rop.bsrc = c->acc[0];
    rop.cb = 1.0;
    rop.c = c->tau / c->s / 2.0;
    rop.y_out = c->y[1];
    classify_term(rop);
    if (lin) {
      rop.ju = c->b;  // u_n
      rop.jrho = c->rho;
    }
    if (rop.flavor != kGeneric ||
        !sweep_face_ok(c->dtype, c->g, c->tiling, c->coef(), {rop.src, rop.bsrc, rop.y_out, c->acc[1], c->b}))
      return set_error(EXPINT_EUNSUPPORTED, "this context's reverse sweeps do not take the fused form");
  }
  auto launch = [&]() -> hipError_t {
    if (kernel == 6)
      return launch_term_face(c->dtype, c->bc, c->g, c->tiling, c->coef(), rop, c->nclass, c->acc[1], c->adj.dtab,
                              c->adj.dwall, 1.0, c->adj.fpart, lin ? c->adj.dbar : nullptr, c->stream);
    if (dct)
      return launch_mode_dct(c->modal.prec, kernel == 3 ? 0 : 1, kernel == 3 ? kDctFwdMulInv : kDctFwd, kEpiStore,
                             da, c->stream);
    if (mode) return launch_mode_product(c->modal.prec, kernel == 3 ? 0 : 1, kEpiStore, ma, c->stream);
    if (kernel == 2) return launch_rhs(c->dtype, c->bc, c->g, c->tiling, cf, c->acc[1], c->b, c->rho, c->stream);
    if (kernel == 5) return launch_pair(c->dtype, c->bc, c->g, c->ptiling, cf, op, c->stream);
    return launch_term(c->dtype, c->bc, c->g, c->tiling, cf, op, c->stream);
  };
  hipEvent_t e0, e1;
  HIP_TRY(c, hipEventCreate(&e0));
  HIP_TRY(c, hipEventCreate(&e1));
  // defined inputs for the timed sweeps
  HIP_TRY(c, launch_fill(c->dtype, c->g.n, 0.25, c->y[0], c->stream));
  HIP_TRY(c, launch_fill(c->dtype, c->g.n, 0.0, c->acc[0], c->stream));
  HIP_TRY(c, launch_fill(c->dtype, c->g.n, 0.5, c->acc[1], c->stream));
  HIP_TRY(c, launch());
  HIP_TRY(c, hipEventRecord(e0, c->stream));
  for (int r = 0; r < reps; ++r) HIP_TRY(c, launch());
  HIP_TRY(c, hipEventRecord(e1, c->stream));
  HIP_TRY(c, hipEventSynchronize(e1));
  float t = 0.f;
  HIP_TRY(c, hipEventElapsedTime(&t, e0, e1));
  *ms = static_cast<double>(t) / reps;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (kernel == 6) {
    HIP_TRY(c, launch_fill(EXPINT_F64, faceprod_slots(c->g, c->tiling) * kMaxClasses, 0.0, c->adj.fpart, c->stream));
    if (lin) HIP_TRY(c, launch_fill(c->dtype, c->g.n, 0.0, c->adj.dbar, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  return EXPINT_OK;
}

int expint_get_stream(const expint_ctx* c, void** stream) {
  if (!c || !stream) return set_error(EXPINT_EINVAL, "NULL argument");
  *stream = c->stream;
  return EXPINT_OK;
}

}  // extern "C"
