// Batched scenarios: many independent grids advanced together (host side).
//
// Every instance keeps its own plan (s_i, m_i), coefficient tables, tile
// shape (autotuned per grid size) and workspace.  One step of the batch is
// a sequence of launches: launch 0 computes every instance's right-hand side,
// launch t >= 1 runs Taylor sweep t of every instance that has one (their
// schedules have different lengths), split into one kernel launch per term
// flavour and plane count.  The sequence is recorded once as a HIP
// graph for a given set of state pointers and replayed per step.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <new>
#include <vector>

#include "autotune.hpp"
#include "batch.hpp"
#include "context.hpp"
#include "plan.hpp"
#include "schedule.hpp"
#include "trace.hpp"

using namespace expint;

namespace {

constexpr int kMaxGrid = 4096;  // workgroups of one batched launch (grid stride beyond)
// flags bit of the tuning entries a batch files its final tilings under, on
// top of the key flags of the grid's own sweep search
constexpr int kBatchTuneFlag = 16;

struct Inst {
  Geom g{};
  double h = 1.0;
  int nclass = 0;
  double class_D[kMaxClasses] = {0};
  double rho = 0.0;
  int s = 1, m = 1;
  double norm1 = 0.0;
  uint8_t* labels = nullptr;
  double* tab64 = nullptr;
  double* wall64 = nullptr;
  void* tab = nullptr;
  void* wallc = nullptr;
  Tiling tiling;
  int ctx_flags = 0;     // tuning key flags of this instance's batch-context entry
  bool ctx_set = false;  // tiling read from such an entry: the plane pass leaves it
  StepBuffers ws;
  std::vector<double> tab_host;  // class table (64) + wall table (8), FP64
  Coef coef() const {
    Coef c{};
    c.labels_form = true;
    c.labels = labels;
    c.tab = tab;
    c.wallc = wallc;
    return c;
  }
};

struct Launch {
  int offset, nitems, total, grid;
  bool rhs;
  int flavor, lp;
  int group;
};

}  // namespace

struct expint_batch {
  expint_dtype dtype = EXPINT_F32;
  expint_bc bc = EXPINT_NOFLUX;
  expint_scheme scheme = EXPINT_SCHEME_EXP_EULER;
  double tau = 0.0;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  Arena arena;
  std::vector<Inst> inst;
  double* partial = nullptr;
  double* red = nullptr;
  // schedule recorded for one set of state pointers
  std::vector<const void*> key;
  BatchItem* d_items = nullptr;
  void* d_tables = nullptr;
  size_t items_cap = 0;
  std::vector<Launch> launches;
  // groups are dealt round-robin to `lanes` streams inside the recorded
  // graph (lane 0 is `stream`, the others `side` streams), so the launch
  // chains of independent groups overlap; joined before the graph ends
  int lanes = 3;
  hipStream_t side[3] = {nullptr, nullptr, nullptr};
  hipEvent_t fork = nullptr, join[3] = {nullptr, nullptr, nullptr};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool poisoned = false;
};

namespace {

int fail_hip(expint_batch* b, hipError_t e, const char* what) {
  (void)hipGetLastError();
  b->poisoned = true;
  return set_error(EXPINT_EHIP, "%s failed: %s", what, hipGetErrorString(e));
}

#define BHIP(call)                                     \
  do {                                                 \
    const hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) return fail_hip(b, e_, #call); \
  } while (0)

int setup_instance(expint_batch* b, Inst& in, const uint8_t* labels_src) {
  const size_t w = dtype_size(b->dtype);
  const size_t fb = static_cast<size_t>(in.g.n) * w;
  int rc;
  if ((rc = b->arena.alloc(reinterpret_cast<void**>(&in.labels), static_cast<size_t>(in.g.n)))) return rc;
  if ((rc = b->arena.alloc(reinterpret_cast<void**>(&in.tab64), kTab * sizeof(double)))) return rc;
  if ((rc = b->arena.alloc(reinterpret_cast<void**>(&in.wall64), kMaxClasses * sizeof(double)))) return rc;
  if ((rc = b->arena.alloc(&in.tab, kTab * sizeof(double)))) return rc;
  if ((rc = b->arena.alloc(&in.wallc, kMaxClasses * sizeof(double)))) return rc;
  if ((rc = b->arena.alloc(&in.ws.b, fb))) return rc;
  for (int i = 0; i < 2; ++i) {
    if ((rc = b->arena.alloc(&in.ws.y[i], fb))) return rc;
    if ((rc = b->arena.alloc(&in.ws.acc[i], fb))) return rc;
  }
  BHIP(hipMemcpyAsync(in.labels, labels_src, static_cast<size_t>(in.g.n), hipMemcpyDefault, b->stream));
  double t64[kTab] = {0}, w64[kMaxClasses] = {0};
  float t32[kTab] = {0}, w32[kMaxClasses] = {0};
  const double inv_h2 = 1.0 / (in.h * in.h);
  for (int a = 0; a < in.nclass; ++a) {
    w64[a] = in.class_D[a] * inv_h2;
    for (int c = 0; c < in.nclass; ++c) t64[a * kMaxClasses + c] = harmonic_mean(in.class_D[a], in.class_D[c]) * inv_h2;
  }
  in.tab_host.assign(t64, t64 + kTab);
  in.tab_host.insert(in.tab_host.end(), w64, w64 + kMaxClasses);
  for (int i = 0; i < kTab; ++i) t32[i] = static_cast<float>(t64[i]);
  for (int i = 0; i < kMaxClasses; ++i) w32[i] = static_cast<float>(w64[i]);
  BHIP(hipMemcpyAsync(in.tab64, t64, sizeof(t64), hipMemcpyHostToDevice, b->stream));
  BHIP(hipMemcpyAsync(in.wall64, w64, sizeof(w64), hipMemcpyHostToDevice, b->stream));
  if (b->dtype == EXPINT_F64) {
    BHIP(hipMemcpyAsync(in.tab, t64, sizeof(t64), hipMemcpyHostToDevice, b->stream));
    BHIP(hipMemcpyAsync(in.wallc, w64, sizeof(w64), hipMemcpyHostToDevice, b->stream));
  } else {
    BHIP(hipMemcpyAsync(in.tab, t32, sizeof(t32), hipMemcpyHostToDevice, b->stream));
    BHIP(hipMemcpyAsync(in.wallc, w32, sizeof(w32), hipMemcpyHostToDevice, b->stream));
  }
  BHIP(launch_scan_labels(b->bc, in.g, in.labels, in.nclass, in.tab64, in.wall64, b->partial, b->red, b->stream));
  double out[2];
  BHIP(hipMemcpyAsync(out, b->red, sizeof(out), hipMemcpyDeviceToHost, b->stream));
  BHIP(hipStreamSynchronize(b->stream));  // also retires the host-array copies above
  if (out[1] != 0.0) return set_error(EXPINT_EINVAL, "a label is >= n_classes (%d)", in.nclass);
  in.norm1 = out[0];
  const bool lin = b->scheme == EXPINT_SCHEME_LINEARISED;
  in.ctx_flags = autotune_key_flags(in.g, in.coef(), true, lin, /*vec_only=*/true) | kBatchTuneFlag;
  in.ctx_set = autotune_find(b->dtype, b->bc, in.g, in.ctx_flags, &in.tiling);
  if (!in.ctx_set)
    BHIP(autotune_sweep(b->dtype, b->bc, in.g, in.coef(), in.ws.y[0], in.ws.acc[0], in.ws.y[1], b->stream, true,
                        &in.tiling, lin ? in.ws.acc[1] : nullptr, in.rho, /*vec_only=*/true));
  return EXPINT_OK;
}

void destroy_graph(expint_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->key.clear();
}

int build_schedule(expint_batch* b, void* const* u) {
  destroy_graph(b);
  const int count = static_cast<int>(b->inst.size());
  std::vector<std::vector<TermOp>> per(count);
  // launch shape per instance: its autotuned tiling, or the scalar default
  // when the caller's u is not aligned for 4-value vectors
  std::vector<Tiling> tl(count);
  const uintptr_t vmask = 4 * dtype_size(b->dtype) - 1;
  for (int i = 0; i < count; ++i) {
    Inst& in = b->inst[i];
    per[i] = phi1_schedule(in.ws, in.s, in.m, b->tau, in.ws.b, nullptr, u[i]);
    if (b->scheme == EXPINT_SCHEME_LINEARISED) set_linearised(per[i], u[i], in.rho);
    tl[i] = in.tiling;
    if (tl[i].vec && (reinterpret_cast<uintptr_t>(u[i]) & vmask) != 0) tl[i] = default_tiling(in.g);
  }
  // instances ordered by tile count, largest first, then packed greedily into
  // groups whose working set (u, b, two term buffers, two running sums,
  // labels) fits the byte budget: a group runs its whole step before the
  // next, so its fields stay in the Infinity Cache across the step's sweeps.
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    return sweep_blocks(b->inst[a].g, tl[a]) > sweep_blocks(b->inst[c].g, tl[c]);
  });
  const size_t w = dtype_size(b->dtype);
  size_t budget = static_cast<size_t>(128) << 20;
  if (const char* env = std::getenv("EXPINT_BATCH_GROUP_BYTES")) budget = std::strtoull(env, nullptr, 10);
  std::vector<std::vector<int>> groups;
  size_t used = 0;
  for (int i : order) {
    const size_t ws = static_cast<size_t>(b->inst[i].g.n) * (6 * w + 1);
    if (groups.empty() || (used + ws > budget && !groups.back().empty())) {
      groups.emplace_back();
      used = 0;
    }
    groups.back().push_back(i);
    used += ws;
  }
  std::vector<BatchItem> items;
  std::vector<double> tabs;  // per item: class table + wall table
  b->launches.clear();
  for (size_t gi = 0; gi < groups.size(); ++gi) {
  const std::vector<int>& grp = groups[gi];
  size_t gmax = 0;
  for (int i : grp) gmax = std::max(gmax, per[i].size());
  for (size_t t = 0; t <= gmax; ++t) {
    // the ops of position t, grouped by (flavour, lp), at most kBatchMaxOps
    // per launch
    for (int fl = kGeneric; fl <= kFirst; ++fl) {
      for (int lp : {1, 2, 4}) {
        Launch L{static_cast<int>(items.size()), 0, 0, 0, t == 0, fl, lp, static_cast<int>(gi)};
        auto close = [&]() {
          L.grid = std::min(L.total, kMaxGrid);
          if (L.nitems > 0) b->launches.push_back(L);
          L = Launch{static_cast<int>(items.size()), 0, 0, 0, t == 0, fl, lp, static_cast<int>(gi)};
        };
        for (int i : grp) {
          const Inst& in = b->inst[i];
          const Tiling& ti = tl[i];
          if (ti.lp != lp) continue;
          if (t == 0) {
            if (fl != kGeneric) continue;
          } else {
            if (per[i].size() < t || per[i][t - 1].flavor != fl) continue;
          }
          if (L.nitems == kBatchMaxOps) close();
          BatchItem it{};
          it.block_start = L.total;
          it.nx = in.g.nx;
          it.ny = in.g.ny;
          it.nz = in.g.nz;
          if (ti.vec) {
            it.vec = 1;
            it.bx = ti.rw;
            it.by = kBlock / ti.rw;
            it.gx = FastDiv(static_cast<uint32_t>(((in.g.nz >> 2) + ti.rw - 1) / ti.rw));
          } else {
            it.bx = ti.bx;
            it.by = ti.by;
            it.gx = FastDiv(static_cast<uint32_t>((in.g.nz + it.bx - 1) / it.bx));
          }
          it.bx_log2 = it.bx == 64 ? 6 : (it.bx == 32 ? 5 : 4);
          it.gy = FastDiv(static_cast<uint32_t>((in.g.ny + it.by - 1) / it.by));
          it.labels = in.labels;
          it.rho = in.rho;
          if (t == 0) {
            it.op.src = u[i];
            it.op.y_out = in.ws.b;
          } else {
            it.op = per[i][t - 1];
          }
          items.push_back(it);
          tabs.insert(tabs.end(), in.tab_host.begin(), in.tab_host.end());
          L.total += static_cast<int>(sweep_blocks(in.g, ti));
          ++L.nitems;
        }
        close();
      }
    }
  }
  }
  if (items.size() > b->items_cap) {
    b->arena.release(b->d_items);
    b->arena.release(b->d_tables);
    b->d_items = nullptr;
    b->d_tables = nullptr;
    int rc = b->arena.alloc(reinterpret_cast<void**>(&b->d_items), items.size() * sizeof(BatchItem));
    if (!rc) rc = b->arena.alloc(&b->d_tables, items.size() * (kTab + kMaxClasses) * w);
    if (rc) return rc;
    b->items_cap = items.size();
  }
  std::vector<float> tabs32;
  const void* tsrc = tabs.data();
  if (b->dtype == EXPINT_F32) {
    tabs32.assign(tabs.begin(), tabs.end());
    tsrc = tabs32.data();
  }
  BHIP(hipMemcpyAsync(b->d_items, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice, b->stream));
  BHIP(hipMemcpyAsync(b->d_tables, tsrc, tabs.size() * w, hipMemcpyHostToDevice, b->stream));
  BHIP(hipStreamSynchronize(b->stream));
  PhaseRange range("record batch graph");
  BHIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  hipError_t err = hipSuccess;
  const int lanes = std::min<int>(b->lanes, static_cast<int>(groups.size()));
  auto lane_stream = [&](int g) { return g % lanes == 0 ? b->stream : b->side[g % lanes - 1]; };
  if (lanes > 1) {  // fork: the side streams join the capture after the fork event
    err = hipEventRecord(b->fork, b->stream);
    for (int l = 1; l < lanes && err == hipSuccess; ++l) err = hipStreamWaitEvent(b->side[l - 1], b->fork, 0);
  }
  for (const Launch& L : b->launches) {
    if (err != hipSuccess) break;
    const void* tb = static_cast<const char*>(b->d_tables) + static_cast<size_t>(L.offset) * (kTab + kMaxClasses) * w;
    err = launch_batch(b->dtype, b->bc, L.rhs, b->scheme == EXPINT_SCHEME_LINEARISED, L.flavor, L.lp,
                       b->d_items + L.offset, tb, L.nitems, L.total, L.grid, lane_stream(L.group));
  }
  if (lanes > 1) {  // join every side stream back into the capturing stream
    for (int l = 1; l < lanes && err == hipSuccess; ++l) {
      err = hipEventRecord(b->join[l - 1], b->side[l - 1]);
      if (err == hipSuccess) err = hipStreamWaitEvent(b->stream, b->join[l - 1], 0);
    }
  }
  hipGraph_t gr = nullptr;
  const hipError_t ec = hipStreamEndCapture(b->stream, &gr);
  if (err != hipSuccess) {
    if (gr) (void)hipGraphDestroy(gr);
    return fail_hip(b, err, "batched launch");
  }
  if (ec != hipSuccess) return fail_hip(b, ec, "hipStreamEndCapture");
  b->graph = gr;
  BHIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  b->key.assign(u, u + count);
  return EXPINT_OK;
}

// Planes per lane of the instances, chosen on whole recorded steps.  Each
// grid's own search times one sweep launched alone, where one plane per lane
// (the most waves) tends to win; a batched step runs many instances per
// launch and several groups at once, so the waves are there anyway, and more
// planes per lane, which re-read fewer neighbour planes, can be faster.  Every
// candidate plane count (1, 2, 4, for every instance the pass may change) is
// recorded as the step it would run and timed over a few replays; the
// fastest is kept.  The timed steps read and write workspace fields only:
// each instance's state is stood in for by one of its two term or two sum
// fields that the step's last sweep does not read (it adds into the state
// element by element, so the stand-in must not be its stencil source or its
// running sum).  Their values are meaningless; the caller's fields are not
// touched.
int tune_batch_planes(expint_batch* b) {
  const int count = static_cast<int>(b->inst.size());
  std::vector<void*> su(count, nullptr);
  for (int i = 0; i < count; ++i) {
    Inst& in = b->inst[i];
    // the last sweep reads at most two fields: one of the four is free
    const std::vector<TermOp> ops = phi1_schedule(in.ws, in.s, in.m, b->tau, in.ws.b, nullptr, in.ws.b);
    for (void* f : {in.ws.y[0], in.ws.y[1], in.ws.acc[0], in.ws.acc[1]}) {
      if (f != ops.back().src && f != ops.back().acc_in) {
        su[i] = f;
        break;
      }
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t ev = hipEventCreate(&e0);
  if (ev == hipSuccess) ev = hipEventCreate(&e1);
  if (ev != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail_hip(b, ev, "hipEventCreate");
  }
  int rc = EXPINT_OK;
  int best_lp = 0;
  float best = -1.f;
  for (int lp : {1, 2, 4}) {
    for (Inst& in : b->inst)
      if (!in.ctx_set) in.tiling.lp = lp;
    if ((rc = build_schedule(b, su.data()))) break;
    // one replay to warm up and size the timed run (at least ~4 ms, 2..20 replays)
    hipError_t e = hipEventRecord(e0, b->stream);
    if (e == hipSuccess) e = hipGraphLaunch(b->exec, b->stream);
    if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    const int reps = std::max(2, std::min(20, static_cast<int>(4.0f / std::max(ms, 1e-3f)) + 1));
    if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = hipGraphLaunch(b->exec, b->stream);
    if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      rc = fail_hip(b, e, "timing a batched step");
      break;
    }
    ms /= reps;
    if (std::getenv("EXPINT_LOG")) std::fprintf(stderr, "[expint] batch planes per lane %d: %.3f ms per step\n", lp, ms);
    if (best < 0.f || ms < best) {
      best = ms;
      best_lp = lp;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  destroy_graph(b);
  if (rc) return rc;
  for (Inst& in : b->inst)
    if (!in.ctx_set) in.tiling.lp = best_lp;
  return EXPINT_OK;
}

}  // namespace

extern "C" {

int expint_batch_create(int32_t count, const expint_grid* grids, const expint_dfield* dfields, const double* rho,
                        expint_bc bc, const expint_opts* opts, expint_batch** out) {
  PhaseRange range("expint_batch_create");
  if (out) *out = nullptr;
  if (count < 1 || !grids || !dfields || !rho || !opts || !out) return set_error(EXPINT_EINVAL, "NULL argument or count < 1");
  if (enum_value(bc) != EXPINT_NOFLUX && enum_value(bc) != EXPINT_DIRICHLET0)
    return set_error(EXPINT_EINVAL, "unknown bc %d", enum_value(bc));
  if (enum_value(opts->dtype) != EXPINT_F64 && enum_value(opts->dtype) != EXPINT_F32)
    return set_error(EXPINT_EINVAL, "unknown dtype");
  if (!(opts->tau > 0.0) || !std::isfinite(opts->tau)) return set_error(EXPINT_EINVAL, "tau must be finite and > 0");
  if ((opts->s > 0) != (opts->m > 0) || opts->s < 0 || opts->m < 0 || opts->m > kPlanMaxDegree)
    return set_error(EXPINT_EINVAL, "give both s and m (m <= %d) or neither", kPlanMaxDegree);
  if (!(opts->tol >= 0.0) || !(opts->theta_max >= 0.0)) return set_error(EXPINT_EINVAL, "bad tolerances");
  {
    const int algo = enum_value(opts->algo), mp = enum_value(opts->mp), scheme = enum_value(opts->scheme);
    if (algo < EXPINT_ALGO_AUTO || algo > EXPINT_ALGO_MODAL || mp < EXPINT_MP_NONE || mp > EXPINT_MP_FP16_SPLIT ||
        scheme < EXPINT_SCHEME_EXP_EULER || scheme > EXPINT_SCHEME_EXPRK2)
      return set_error(EXPINT_EINVAL, "unknown algo, mp or scheme");
    if (algo == EXPINT_ALGO_MODAL || mp != EXPINT_MP_NONE)
      return set_error(EXPINT_EUNSUPPORTED, "batches run the stencil-Taylor path only");
    if (scheme != EXPINT_SCHEME_EXP_EULER && scheme != EXPINT_SCHEME_LINEARISED)
      return set_error(EXPINT_EUNSUPPORTED, "batches take the EXP_EULER or LINEARISED scheme");
  }
  for (int i = 0; i < count; ++i) {
    const expint_grid& g = grids[i];
    const expint_dfield& d = dfields[i];
    if (g.nx < 1 || g.ny < 1 || g.nz < 1 || !(g.h > 0.0) || !std::isfinite(g.h))
      return set_error(EXPINT_EINVAL, "instance %d: bad grid", i);
    if (product_within(static_cast<int64_t>(g.nx) + 16, g.ny, g.nz, (int64_t(1) << 31) - 1) < 0)
      return set_error(EXPINT_EINVAL, "instance %d: grid too large", i);
    if (!d.labels || d.D) return set_error(EXPINT_EINVAL, "instance %d: batches need the label form", i);
    if (d.n_classes < 1 || d.n_classes > EXPINT_MAX_CLASSES || !d.class_D)
      return set_error(EXPINT_EINVAL, "instance %d: n_classes must be in 1..%d", i, EXPINT_MAX_CLASSES);
    for (int a = 0; a < d.n_classes; ++a)
      if (!finite_nonneg(d.class_D[a])) return set_error(EXPINT_EINVAL, "instance %d: bad class_D[%d]", i, a);
    if (!finite_nonneg(rho[i])) return set_error(EXPINT_EINVAL, "instance %d: bad rho", i);
  }
  expint_batch* b = new (std::nothrow) expint_batch();
  if (!b) return set_error(EXPINT_ENOMEM, "host allocation failed");
  auto bail = [&](int code) {
    expint_batch_destroy(b);
    return code;
  };
  b->dtype = opts->dtype;
  b->bc = bc;
  b->scheme = opts->scheme;
  b->tau = opts->tau;
  double tol, theta_max;
  default_tolerances(b->dtype, &tol, &theta_max);
  if (opts->tol > 0.0) tol = opts->tol;
  if (opts->theta_max > 0.0) theta_max = opts->theta_max;
  if (hipGetDevice(&b->device) != hipSuccess) {
    (void)hipGetLastError();
    return bail(set_error(EXPINT_EHIP, "no HIP device"));
  }
  if (opts->stream) {
    b->stream = static_cast<hipStream_t>(opts->stream);
  } else {
    if (hipStreamCreate(&b->stream) != hipSuccess) {
      (void)hipGetLastError();
      return bail(set_error(EXPINT_EHIP, "hipStreamCreate failed"));
    }
    b->own_stream = true;
  }
  // lanes of the recorded step (default 3; EXPINT_BATCH_LANES, 1..4): side
  // streams (default priority) and the fork / join events of the capture
  if (const char* env = std::getenv("EXPINT_BATCH_LANES")) b->lanes = std::max(1, std::min(4, std::atoi(env)));
  for (int l = 1; l < b->lanes; ++l) {
    if (hipStreamCreateWithFlags(&b->side[l - 1], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->join[l - 1], hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      return bail(set_error(EXPINT_EHIP, "side stream creation failed"));
    }
  }
  if (b->lanes > 1 && hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    return bail(set_error(EXPINT_EHIP, "event creation failed"));
  }
  int64_t max_parts = kReduceBlocks;
  b->inst.resize(count);
  for (int i = 0; i < count; ++i) {
    Inst& in = b->inst[i];
    in.g.nx = grids[i].nx;
    in.g.ny = grids[i].ny;
    in.g.nz = grids[i].nz;
    in.g.n = static_cast<int64_t>(in.g.nx) * in.g.ny * in.g.nz;
    in.h = grids[i].h;
    in.nclass = dfields[i].n_classes;
    for (int a = 0; a < in.nclass; ++a) in.class_D[a] = dfields[i].class_D[a];
    in.rho = rho[i];
    max_parts = std::max(max_parts, field_block_count(in.g));
  }
  int rc;
  if ((rc = b->arena.alloc(reinterpret_cast<void**>(&b->partial), 2 * max_parts * sizeof(double)))) return bail(rc);
  if ((rc = b->arena.alloc(reinterpret_cast<void**>(&b->red), 2 * sizeof(double)))) return bail(rc);
  for (int i = 0; i < count; ++i) {
    Inst& in = b->inst[i];
    if ((rc = setup_instance(b, in, dfields[i].labels))) return bail(rc);
    if (opts->s > 0) {
      in.s = opts->s;
      in.m = opts->m;
    } else if (!choose_plan(b->tau * (in.norm1 + (b->scheme == EXPINT_SCHEME_LINEARISED ? in.rho : 0.0)), tol,
                            theta_max, &in.s, &in.m)) {
      return bail(set_error(EXPINT_EINVAL, "instance %d: no admissible plan", i));
    }
  }
  {
    // instances without a batch-context tuning entry: planes per lane chosen
    // on whole steps, then filed for later batches and processes
    bool any = false;
    for (const Inst& in : b->inst) any = any || !in.ctx_set;
    const char* env = std::getenv("EXPINT_AUTOTUNE");
    if (any && !(env && env[0] == '0')) {
      PhaseRange tr("batch plane tuning");
      if ((rc = tune_batch_planes(b))) return bail(rc);
      for (Inst& in : b->inst) {
        if (in.ctx_set) continue;
        Tiling t;
        if (!autotune_find(b->dtype, b->bc, in.g, in.ctx_flags, &t))
          autotune_keep(b->dtype, b->bc, in.g, in.ctx_flags, in.tiling);
      }
    }
  }
  if (std::getenv("EXPINT_LOG")) {
    int64_t vox = 0;
    long terms = 0;
    for (auto& in : b->inst) {
      vox += in.g.n;
      terms += static_cast<long>(in.s) * in.m;
    }
    std::fprintf(stderr, "[expint] batch of %d instances, %lld voxels, %ld Taylor terms per step in total, %zu B\n",
                 count, static_cast<long long>(vox), terms, b->arena.bytes());
  }
  *out = b;
  return EXPINT_OK;
}

int expint_batch_advance(expint_batch* b, void* const* u, int32_t nsteps) {
  PhaseRange range("expint_batch_advance");
  if (!b) return set_error(EXPINT_EINVAL, "batch is NULL");
  if (b->poisoned) return set_error(EXPINT_ESTATE, "batch poisoned by an earlier HIP error");
  if (!u) return set_error(EXPINT_EINVAL, "u is NULL");
  if (nsteps < 0) return set_error(EXPINT_EINVAL, "nsteps must be >= 0");
  const int count = static_cast<int>(b->inst.size());
  for (int i = 0; i < count; ++i)
    if (!u[i]) return set_error(EXPINT_EINVAL, "u[%d] is NULL", i);
  int cur = -1;
  BHIP(hipGetDevice(&cur));
  if (cur != b->device) BHIP(hipSetDevice(b->device));
  if (nsteps == 0) return EXPINT_OK;
  bool same = b->exec && static_cast<int>(b->key.size()) == count;
  for (int i = 0; same && i < count; ++i) same = b->key[i] == u[i];
  if (!same) {
    // a launch of the graph being replaced may still be running on the stream
    if (b->exec) BHIP(hipStreamSynchronize(b->stream));
    const int rc = build_schedule(b, u);
    if (rc) return rc;
  }
  for (int32_t k = 0; k < nsteps; ++k) BHIP(hipGraphLaunch(b->exec, b->stream));
  return EXPINT_OK;
}

int expint_batch_get_plan(const expint_batch* b, int32_t index, int32_t* s, int32_t* m, double* norm1) {
  if (!b || index < 0 || index >= static_cast<int32_t>(b->inst.size()))
    return set_error(EXPINT_EINVAL, "NULL batch or index out of range");
  const Inst& in = b->inst[index];
  if (s) *s = in.s;
  if (m) *m = in.m;
  if (norm1) *norm1 = in.norm1;
  return EXPINT_OK;
}

void expint_batch_destroy(expint_batch* b) {
  if (!b) return;
  if (b->stream && !b->poisoned) (void)hipStreamSynchronize(b->stream);
  destroy_graph(b);
  for (int l = 0; l < 3; ++l) {
    if (b->side[l]) (void)hipStreamDestroy(b->side[l]);
    if (b->join[l]) (void)hipEventDestroy(b->join[l]);
  }
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

}  // extern "C"
