// Discrete adjoint of the exponential Euler advance (host orchestration).
//
// The forward map with the plan frozen is, per step n,
//   b_n = A u_n + f(u_n),  x_0 = 0,
//   sub-step sigma: y_1 = h (A x + b_n), y_j = (h/j) A y_{j-1}, x <- x + sum_j y_j,
//   u_{n+1} = u_n + x_s,   h = tau / s.
// For a cotangent lambda_{n+1} = dL/du_{n+1} the reverse sweep runs the Taylor
// recurrence backwards (A is symmetric):
//   ybar_m = xbar,  ybar_j = xbar + (h/(j+1)) A ybar_{j+1},
//   bbar += h ybar_1,  xbar <- xbar + h A ybar_1,
// starting from xbar = lambda_{n+1}; g = bbar equals P(A) lambda_{n+1} and
//   lambda_n = lambda_{n+1} + A g + rho (1 - 2 u_n) g,
//   dL/drho += <g, u_n (1 - u_n)>,
//   dL/dD_c += <g, A_c u_n> + sum_sigma [h <ybar_1, A_c x_{sigma-1}> + sum_{j>=2} (h/j) <ybar_j, A_c y_{j-1}>],
// with A_c = dA/dD_c.  u is checkpointed every ckpt_every steps and recomputed
// inside a segment; each step's Taylor terms are recomputed once and kept.
//
// The LINEARISED scheme (section 2.1's splitting) runs every recurrence with
// J_n = A + diag(d_n), d_n = rho (1 - 2 u_n), in place of A (J_n is
// symmetric as well); the diagonal's adjoint
//   dbar = sum_sigma [h ybar_1 * x_{sigma-1} + sum_{j>=2} (h/j) ybar_j * y_{j-1}]
// (pointwise, the pairs of the class terms) adds lambda_n += -2 rho dbar and
// dL/drho += <dbar, 1 - 2 u_n>.

#include <algorithm>
#include <cmath>
#include <vector>

#include "context.hpp"
#include "internal.hpp"
#include "schedule.hpp"
#include "trace.hpp"

using namespace expint;

namespace {

int grow(expint_ctx* c, std::vector<void*>& v, size_t count) {
  const size_t fb = c->field_bytes();
  while (v.size() < count) {
    void* p = nullptr;
    const int rc = c->arena.alloc(&p, fb);
    if (rc) return rc;
    v.push_back(p);
  }
  return EXPINT_OK;
}

int ensure_adj(expint_ctx* c, int nck, int seg) {
  auto& a = c->adj;
  const size_t fb = c->field_bytes();
  int rc;
  if (!a.lam) {
    // all or nothing, lam last: it marks the set as complete
    struct Want {
      void** p;
      size_t bytes;
    } want[] = {
        {&a.gb, fb},
        {&a.work, fb},
        {&a.xb[0], fb},
        {&a.xb[1], fb},
        {&a.yb[0], fb},
        {&a.yb[1], fb},
        {&a.dbar, fb},
        {reinterpret_cast<void**>(&a.fpart),
         static_cast<size_t>(faceprod_slots(c->g, c->tiling)) * kMaxClasses * sizeof(double)},
        {reinterpret_cast<void**>(&a.dev), 16 * sizeof(double)},
        {reinterpret_cast<void**>(&a.dtab), kMaxClasses * kTab * sizeof(double)},
        {reinterpret_cast<void**>(&a.dwall), kMaxClasses * kMaxClasses * sizeof(double)},
        {&a.lam, fb},
    };
    for (const Want& wnt : want) {
      if ((rc = c->arena.alloc(wnt.p, wnt.bytes))) {
        for (const Want& q : want) {
          c->arena.release(*q.p);
          *q.p = nullptr;
        }
        return rc;
      }
    }
  }
  // the most steps per segment any call asked for (slot t's buffers do not
  // depend on it, so a larger value only adds slots)
  if (seg > a.seg) a.seg = seg;
  const size_t slots = 2 * static_cast<size_t>(a.seg);
  if ((rc = grow(c, a.ckpt, static_cast<size_t>(nck)))) return rc;
  if ((rc = grow(c, a.segs, static_cast<size_t>(a.seg)))) return rc;
  if ((rc = grow(c, a.segs2, static_cast<size_t>(a.seg)))) return rc;
  if ((rc = grow(c, a.xs, slots * (static_cast<size_t>(c->s) + 1)))) return rc;
  if ((rc = grow(c, a.tape, slots * static_cast<size_t>(c->s) * c->m))) return rc;
  if ((rc = grow(c, a.bts, slots))) return rc;
  if (!a.rec) {
    // the segment stream and its events (default priority, like every stream here)
    hipStream_t st = nullptr;
    HIP_TRY(c, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    a.rec = st;
    HIP_TRY(c, hipEventCreateWithFlags(&a.ev_fwd, hipEventDisableTiming));
    for (int q = 0; q < 2; ++q) {
      HIP_TRY(c, hipEventCreateWithFlags(&a.ev_seg[q], hipEventDisableTiming));
      HIP_TRY(c, hipEventCreateWithFlags(&a.ev_segfree[q], hipEventDisableTiming));
    }
  }
  return EXPINT_OK;
}

// Tape slot t: the sub-step state x_sig, the Taylor terms of sub-step sig.
void* xs_at(expint_ctx* c, int t, int sig) { return c->adj.xs[static_cast<size_t>(t) * (c->s + 1) + sig]; }
void** tape_of(expint_ctx* c, int t, int sig) {
  return &c->adj.tape[(static_cast<size_t>(t) * c->s + (sig - 1)) * c->m];
}

// Face weights -dK(D_a, D_b)/dD_c / h^2 and wall weights -[a == c] / h^2.
int upload_weights(expint_ctx* c) {
  double dt[kMaxClasses * kTab] = {0}, dw[kMaxClasses * kMaxClasses] = {0};
  const double inv_h2 = 1.0 / (c->h * c->h);
  for (int cc = 0; cc < c->nclass; ++cc) {
    dw[cc * kMaxClasses + cc] = -inv_h2;
    for (int a = 0; a < c->nclass; ++a) {
      for (int b = 0; b < c->nclass; ++b) {
        const double da = c->class_D[a], db = c->class_D[b], s = da + db;
        double d = 0.0;
        if (a == cc && b == cc) {
          d = 1.0;  // K(D, D) = D
        } else if (s > 0.0) {
          if (a == cc) d += 2.0 * db * db / (s * s);
          if (b == cc) d += 2.0 * da * da / (s * s);
        }
        dt[cc * kTab + a * kMaxClasses + b] = -d * inv_h2;
      }
    }
  }
  HIP_TRY(c, hipMemcpyAsync(c->adj.dtab, dt, sizeof(dt), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->adj.dwall, dw, sizeof(dw), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return EXPINT_OK;
}

// Adds w <ybar, (dA/dD_c) y> for every class into the face-product slots.
// For a Taylor term (taylor) of the LINEARISED scheme also dbar += w ybar * y:
// the term applied the diagonal to y as well.
int faceprod(expint_ctx* c, const void* ybar, const void* y, double w, bool taylor) {
  HIP_TRY(c, launch_faceprod(c->dtype, c->bc, c->g, c->tiling, c->labels, c->nclass, c->adj.dtab, c->adj.dwall, ybar,
                             y, w, c->adj.fpart, c->stream));
  if (taylor && c->scheme == EXPINT_SCHEME_LINEARISED)
    HIP_TRY(c, launch_diag_accumulate(c->dtype, c->g.n, w, ybar, y, c->adj.dbar, c->stream));
  return EXPINT_OK;
}

// One Taylor sweep of the step's matrix: A, or J_n at the state un.
int term(expint_ctx* c, TermOp op, const void* un, hipStream_t st) {
  if (c->scheme == EXPINT_SCHEME_LINEARISED) {
    op.ju = un;
    op.jrho = c->rho;
  }
  classify_term(op);
  HIP_TRY(c, launch_term(c->dtype, c->bc, c->g, c->tiling, c->coef(), op, st));
  return EXPINT_OK;
}

// The reverse Taylor sweep op (stencil source op.src) preceded by the face
// products w <op.src, (dA/dD_c) y> (LINEARISED: and dbar += w op.src * y):
// one fused pass where it applies (vectorised shape, aligned fields), else
// the separate launches in that order.
int term_face(expint_ctx* c, TermOp op, const void* un, const void* y, double w) {
  classify_term(op);
  const bool lin = c->scheme == EXPINT_SCHEME_LINEARISED;
  if (op.flavor == kGeneric &&
      sweep_face_ok(c->dtype, c->g, c->tiling, c->coef(), {op.src, op.bsrc, op.y_out, y, un, c->adj.dbar})) {
    if (lin) {
      op.ju = un;
      op.jrho = c->rho;
    }
    HIP_TRY(c, launch_term_face(c->dtype, c->bc, c->g, c->tiling, c->coef(), op, c->nclass, y, c->adj.dtab,
                                c->adj.dwall, w, c->adj.fpart, lin ? c->adj.dbar : nullptr, c->stream));
    return EXPINT_OK;
  }
  int rc;
  if ((rc = faceprod(c, op.src, y, w, true))) return rc;
  return term(c, op, un, c->stream);
}

// Reverse sweep of one step; lambda (c->adj.lam) is updated in place.
// The forward tape of step n at the state un into tape slot p, on stream st:
// b_n, the sub-step states and every Taylor term.
int tape_step(expint_ctx* c, const void* un, int p, hipStream_t st) {
  auto& a = c->adj;
  const int s = c->s, m = c->m;
  const double h = c->tau / s;
  int rc;
  HIP_TRY(c, launch_rhs(c->dtype, c->bc, c->g, c->tiling, c->coef(), un, a.bts[p], c->rho, st));
  for (int sig = 1; sig <= s; ++sig) {
    void** T = tape_of(c, p, sig);
    TermOp t1;
    t1.src = xs_at(c, p, sig - 1);
    t1.bsrc = a.bts[p];
    t1.c = h;
    t1.cb = h;
    t1.cs = 1.0;
    t1.acc_out = xs_at(c, p, sig);
    t1.y_out = m >= 2 ? T[0] : nullptr;
    if ((rc = term(c, t1, un, st))) return rc;
    for (int j = 2; j <= m; ++j) {
      TermOp t;
      t.src = T[j - 2];
      t.c = h / j;
      t.acc_in = xs_at(c, p, sig);
      t.ca = 1.0;
      t.acc_out = xs_at(c, p, sig);
      t.y_out = j < m ? T[j - 1] : nullptr;
      if ((rc = term(c, t, un, st))) return rc;
    }
  }
  return EXPINT_OK;
}

// The reverse sweeps of step n from tape slot p, on the context stream;
// lambda (c->adj.lam) is updated in place.
int reverse_step(expint_ctx* c, const void* un, int p) {
  auto& a = c->adj;
  const int s = c->s, m = c->m;
  const double h = c->tau / s;
  const int64_t n = c->g.n;
  int rc;
  // reverse through the sub-steps
  int xi = 0;
  HIP_TRY(c, launch_copy(c->dtype, n, a.lam, a.xb[0], c->stream));
  HIP_TRY(c, launch_fill(c->dtype, n, 0.0, a.gb, c->stream));
  const bool lin = c->scheme == EXPINT_SCHEME_LINEARISED;
  if (lin) HIP_TRY(c, launch_fill(c->dtype, n, 0.0, a.dbar, c->stream));
  for (int sig = s; sig >= 1; --sig) {
    void** T = tape_of(c, p, sig);
    const void* xprev = xs_at(c, p, sig - 1);
    const void* ynext = a.xb[xi];  // ybar_m = xbar
    // the face products of ybar_j pair it with y_{j-1} (x_{sigma-1} for j = 1)
    // at weight h/j; each is taken with the next sweep, whose source is ybar_j
    const void* fy = m >= 2 ? T[m - 2] : xprev;
    double fw = m >= 2 ? h / m : h;
    int yi = 0;
    for (int j = m - 1; j >= 1; --j) {
      TermOp t;  // ybar_j = xbar + (h/(j+1)) A ybar_{j+1}
      t.src = ynext;
      t.bsrc = a.xb[xi];
      t.cb = 1.0;
      t.c = h / (j + 1);
      t.y_out = a.yb[yi];
      if ((rc = term_face(c, t, un, fy, fw))) return rc;
      ynext = a.yb[yi];
      yi ^= 1;
      fy = j >= 2 ? T[j - 2] : xprev;
      fw = j >= 2 ? h / j : h;
    }
    // bbar += h ybar_1;  xbar <- xbar + h A ybar_1
    HIP_TRY(c, launch_axpby(c->dtype, n, 1.0, a.gb, h, ynext, a.gb, c->stream));
    TermOp t;
    t.src = ynext;
    t.bsrc = a.xb[xi];
    t.cb = 1.0;
    t.c = h;
    t.y_out = a.xb[1 - xi];
    if ((rc = term_face(c, t, un, fy, fw))) return rc;
    xi ^= 1;
  }
  // g = bbar: rho and D contributions of b_n = A u_n + f(u_n), then lambda_n
  HIP_TRY(c, launch_reduce(c->dtype, 4, a.gb, un, n, c->partial, a.dev + 8, c->stream, true));
  // the D terms of b_n = A u_n + f(u_n) (no diagonal), then lambda_n
  if (sweep_face_ok(c->dtype, c->g, c->tiling, c->coef(), {a.gb, un, a.lam})) {
    HIP_TRY(c, launch_adj_rhs_face(c->dtype, c->bc, c->g, c->tiling, c->coef(), a.gb, un, a.lam, a.lam, c->rho,
                                   c->nclass, a.dtab, a.dwall, 1.0, a.fpart, c->stream));
  } else {
    if ((rc = faceprod(c, a.gb, un, 1.0, false))) return rc;
    HIP_TRY(c, launch_adj_rhs(c->dtype, c->bc, c->g, c->tiling, c->coef(), a.gb, un, a.lam, a.lam, c->rho,
                              c->stream));
  }
  if (lin) {  // the diagonal rho (1 - 2 u_n): d/drho and d/du_n
    HIP_TRY(c, launch_reduce(c->dtype, 6, a.dbar, un, n, c->partial, a.dev + 8, c->stream, true));
    HIP_TRY(c, launch_axpy(c->dtype, n, -2.0 * c->rho, a.dbar, a.lam, c->stream));
  }
  return EXPINT_OK;
}

// The launches of one gradient, from zeroing the accumulators to the
// class sums, on the context stream and the two helper streams (joined back
// into the context stream before the end); the result is left in lam.
int enqueue_gradient(expint_ctx* c, const void* u0, int32_t nsteps, const void* cot, bool cot_is_target,
                     int32_t ckpt_every) {
  int rc;
  const int nck = nsteps > 0 ? (nsteps + ckpt_every - 1) / ckpt_every : 0;
  auto& a = c->adj;
  const int64_t n = c->g.n;
  const int64_t slots = faceprod_slots(c->g, c->tiling);
  HIP_TRY(c, launch_fill(EXPINT_F64, 16, 0.0, a.dev, c->stream));
  HIP_TRY(c, launch_fill(EXPINT_F64, slots * kMaxClasses, 0.0, a.fpart, c->stream));
  for (int t = 0; t < 2 * a.seg; ++t) HIP_TRY(c, launch_fill(c->dtype, n, 0.0, xs_at(c, t, 0), c->stream));
  // both segment sets start free
  for (int q = 0; q < 2; ++q) HIP_TRY(c, hipEventRecord(a.ev_segfree[q], c->stream));

  // Segment sgi uses set sgi & 1: its states and one tape slot per step.
  auto seg_states = [&](int sgi) -> std::vector<void*>& { return (sgi & 1) ? a.segs2 : a.segs; };
  auto slot = [&](int sgi, int k) { return (sgi & 1) * a.seg + (k - sgi * ckpt_every); };
  // The tapes of segment sgi from its first state, already in its states[0],
  // on stream st: per step the tape (b, sub-step states, Taylor terms) and
  // the next state u_{k+1} = u_k + x_s.  last_out: where the state after the
  // segment goes (NULL: nowhere).
  auto build = [&](int sgi, hipStream_t st, void* last_out) -> int {
    const int start = sgi * ckpt_every;
    const int stop = std::min(start + ckpt_every, nsteps);
    std::vector<void*>& sv = seg_states(sgi);
    for (int k = start; k < stop; ++k) {
      const int t = slot(sgi, k);
      const int r = tape_step(c, sv[k - start], t, st);
      if (r) return r;
      void* next = k + 1 < stop ? sv[k - start + 1] : last_out;
      if (next) HIP_TRY(c, launch_axpby(c->dtype, n, 1.0, sv[k - start], 1.0, xs_at(c, t, c->s), next, st));
    }
    return EXPINT_OK;
  };

  // forward with checkpoints; the last segment's tapes are built as it passes
  PhaseRange fwd_range("gradient: forward with checkpoints");
  HIP_TRY(c, launch_copy(c->dtype, n, u0, a.work, c->stream));
  const int last_start = (nck - 1) * ckpt_every;
  for (int k = 0; k < last_start; ++k) {
    if (k % ckpt_every == 0) HIP_TRY(c, launch_copy(c->dtype, n, a.work, a.ckpt[k / ckpt_every], c->stream));
    // the tapes of the segments before the last may be built from here on
    if (k == last_start - ckpt_every) HIP_TRY(c, hipEventRecord(a.ev_fwd, c->stream));
    if ((rc = enqueue_step(c, a.work))) return rc;
  }
  if (nck > 0) {
    HIP_TRY(c, launch_copy(c->dtype, n, a.work, seg_states(nck - 1)[0], c->stream));
    if ((rc = build(nck - 1, c->stream, a.work))) return rc;
    HIP_TRY(c, hipEventRecord(a.ev_seg[(nck - 1) & 1], c->stream));
  }
  if (cot_is_target) {
    HIP_TRY(c, launch_reduce(c->dtype, 5, a.work, cot, n, c->partial, a.dev + 9, c->stream));
    HIP_TRY(c, launch_axpby(c->dtype, n, 1.0, a.work, -1.0, cot, a.lam, c->stream));
  } else {
    HIP_TRY(c, launch_copy(c->dtype, n, cot, a.lam, c->stream));
  }

  fwd_range.end();
  PhaseRange rev_range("gradient: reverse segments (tapes built one segment ahead on a second stream)");
  // Two streams from here on: the tapes of segment sgi - 1 are built on
  // `rec` from its checkpoint while segment sgi reverses on the context
  // stream.
  if (nck >= 2) HIP_TRY(c, hipStreamWaitEvent(a.rec, a.ev_fwd, 0));
  for (int sgi = nck - 1; sgi >= 0; --sgi) {
    const int start = sgi * ckpt_every;
    const int stop = std::min(start + ckpt_every, nsteps);
    const int q = sgi & 1;
    if (sgi >= 1) {
      const int qp = (sgi - 1) & 1;
      HIP_TRY(c, hipStreamWaitEvent(a.rec, a.ev_segfree[qp], 0));
      HIP_TRY(c, launch_copy(c->dtype, n, a.ckpt[sgi - 1], seg_states(sgi - 1)[0], a.rec));
      if ((rc = build(sgi - 1, a.rec, nullptr))) return rc;
      HIP_TRY(c, hipEventRecord(a.ev_seg[qp], a.rec));
    }
    HIP_TRY(c, hipStreamWaitEvent(c->stream, a.ev_seg[q], 0));
    std::vector<void*>& sv = seg_states(sgi);
    for (int k = stop - 1; k >= start; --k)
      if ((rc = reverse_step(c, sv[k - start], slot(sgi, k)))) return rc;
    // every read of this set (states and tapes) is behind this event
    HIP_TRY(c, hipEventRecord(a.ev_segfree[q], c->stream));
  }
  rev_range.end();
  HIP_TRY(c, launch_faceprod_final(a.fpart, slots, a.dev, c->stream));
  return EXPINT_OK;
}

int vjp_core(expint_ctx* c, const void* u0, int32_t nsteps, const void* cot, bool cot_is_target, int32_t ckpt_every,
             double* loss, void* grad_u0, double* grad_rho, double* grad_D) {
  PhaseRange range("gradient");
  CHECK_CTX(c);
  if (!u0 || !cot || !grad_u0) return set_error(EXPINT_EINVAL, "NULL field");
  if (nsteps < 0) return set_error(EXPINT_EINVAL, "nsteps must be >= 0");
  if (ckpt_every < 1) return set_error(EXPINT_EINVAL, "ckpt_every must be >= 1");
  if (!c->labels_form) return set_error(EXPINT_EINVAL, "gradients need the label form of D");
  if (c->scheme == EXPINT_SCHEME_EXPRK2)
    return set_error(EXPINT_EUNSUPPORTED, "gradients are for the EXP_EULER and LINEARISED schemes");
  if (c->algo == EXPINT_ALGO_MODAL)  // the reverse pass is that of the Taylor map, not of the mode products
    return set_error(EXPINT_EUNSUPPORTED, "gradients are for the stencil-Taylor algorithm");
  int rc = ensure_device(c);
  if (rc) return rc;
  const int nck = nsteps > 0 ? (nsteps + ckpt_every - 1) / ckpt_every : 0;
  const int seg = std::min(ckpt_every, std::max(nsteps, 1));
  if ((rc = ensure_adj(c, nck, seg))) return rc;
  if ((rc = upload_weights(c))) return rc;
  auto& a = c->adj;
  if ((rc = enqueue_gradient(c, u0, nsteps, cot, cot_is_target, ckpt_every))) return rc;
  HIP_TRY(c, launch_copy(c->dtype, c->g.n, a.lam, grad_u0, c->stream));
  PhaseRange sync_range("gradient: wait for the device");
  double host[16];
  HIP_TRY(c, hipMemcpyAsync(host, a.dev, sizeof(host), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (loss) *loss = 0.5 * host[9];
  if (grad_rho) *grad_rho = host[8];
  if (grad_D)
    for (int k = 0; k < c->nclass; ++k) grad_D[k] = host[k];
  return EXPINT_OK;
}

}  // namespace

extern "C" {

int expint_grad(expint_ctx* c, const void* u0, int32_t nsteps, const void* u_target, int32_t ckpt_every,
                double* loss, void* grad_u0, double* grad_rho, double* grad_class_D) {
  return vjp_core(c, u0, nsteps, u_target, true, ckpt_every, loss, grad_u0, grad_rho, grad_class_D);
}

int expint_vjp(expint_ctx* c, const void* u0, int32_t nsteps, const void* gout, int32_t ckpt_every, void* grad_u0,
               double* grad_rho, double* grad_class_D) {
  return vjp_core(c, u0, nsteps, gout, false, ckpt_every, nullptr, grad_u0, grad_rho, grad_class_D);
}

}  // extern "C"
