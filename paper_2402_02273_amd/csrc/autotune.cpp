#include "autotune.hpp"

#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

namespace expint {

namespace {

using Key = std::tuple<int, int, int, int, int, int>;
std::mutex g_mu;
std::map<Key, Tiling> g_cache;

std::map<Key, PairTiling> g_pair_cache;

// Average time of `reps` launches after one warm-up launch, in ms.
template <typename F>
hipError_t time_launches(F&& launch, int reps, hipStream_t st, float* ms) {
  hipEvent_t e0, e1;
  hipError_t e;
  if ((e = hipEventCreate(&e0)) != hipSuccess) return e;
  if ((e = hipEventCreate(&e1)) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return e;
  }
  if ((e = launch()) == hipSuccess && (e = hipEventRecord(e0, st)) == hipSuccess) {
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
    if (e == hipSuccess && (e = hipEventRecord(e1, st)) == hipSuccess && (e = hipEventSynchronize(e1)) == hipSuccess) {
      float t = 0.f;
      if ((e = hipEventElapsedTime(&t, e0, e1)) == hipSuccess) *ms = t / reps;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return e;
}

}  // namespace

hipError_t autotune_pairs(expint_dtype dt, expint_bc bc, const Geom& g, const Coef& cf, void* f0, void* f1, void* f2,
                          hipStream_t st, const Tiling& single, expint_sweeps mode, PairTiling* out) {
  *out = PairTiling{};
  out->ty = 0;
  if (!cf.labels_form || mode == EXPINT_SWEEPS_SINGLE || !pair_grid_ok(g, dt)) return hipSuccess;
  const char* env = std::getenv("EXPINT_AUTOTUNE");
  if (env && env[0] == '0') {
    out->ty = 8;
    out->lp = 8;
    return hipSuccess;
  }
  const bool forced = mode == EXPINT_SWEEPS_PAIRS;
  const Key key{g.nx, g.ny, g.nz, static_cast<int>(dt), static_cast<int>(bc), forced ? 1 : 0};
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_pair_cache.find(key);
    if (it != g_pair_cache.end()) {
      *out = it->second;
      return hipSuccess;
    }
  }
  hipError_t e;
  if ((e = launch_fill(dt, g.n, 0.25, f0, st)) != hipSuccess) return e;
  if ((e = launch_fill(dt, g.n, 0.0, f1, st)) != hipSuccess) return e;
  const int reps = g.n > (1 << 22) ? 3 : 8;
  // the two single-term sweeps a pair sweep replaces
  TermOp skip;
  skip.src = f0;
  skip.y_out = f2;
  skip.c = 0.5;
  classify_term(skip);
  TermOp flush;
  flush.src = f0;
  flush.acc_in = f1;
  flush.ca = 1.0;
  flush.cs = 1.0;
  flush.acc_out = f1;
  flush.y_out = f2;
  flush.c = 0.5;
  classify_term(flush);
  float t_skip = 0.f, t_flush = 0.f;
  if ((e = time_launches([&] { return launch_term(dt, bc, g, single, cf, skip, st); }, reps, st, &t_skip)) !=
      hipSuccess)
    return e;
  if ((e = time_launches([&] { return launch_term(dt, bc, g, single, cf, flush, st); }, reps, st, &t_flush)) !=
      hipSuccess)
    return e;
  // a pair sweep in the middle of a sub-step
  TermOp pr;
  pr.src = f0;
  pr.acc_in = f1;
  pr.ca = 1.0;
  pr.acc_out = f1;
  pr.y_out = f2;
  pr.c = 0.5;
  pr.c2 = 0.25;
  pr.pair = 1;
  float best = -1.f;
  PairTiling best_t;
  for (int ty : {4, 8}) {
    for (int lp : {4, 8, 16}) {
      PairTiling t;
      t.ty = ty;
      t.lp = lp;
      float ms = 0.f;
      if ((e = time_launches([&] { return launch_pair(dt, bc, g, t, cf, pr, st); }, reps, st, &ms)) != hipSuccess)
        return e;
      if (std::getenv("EXPINT_LOG"))
        std::fprintf(stderr, "[expint]   pair ty=%d lp=%d: %.2f us\n", ty, lp, ms * 1000.f);
      if (best < 0.f || ms < best) {
        best = ms;
        best_t = t;
      }
    }
  }
  if (forced || best < t_skip + t_flush) *out = best_t;
  if (std::getenv("EXPINT_LOG"))
    std::fprintf(stderr, "[expint] pair sweeps %dx%dx%d %s: best ty=%d lp=%d %.2f us vs skip+flush %.2f+%.2f us -> %s\n",
                 g.nx, g.ny, g.nz, dt == EXPINT_F64 ? "f64" : "f32", best_t.ty, best_t.lp, best * 1000.f,
                 t_skip * 1000.f, t_flush * 1000.f, out->ty ? "pairs" : "single terms");
  std::lock_guard<std::mutex> lk(g_mu);
  g_pair_cache[key] = *out;
  return hipSuccess;
}

hipError_t autotune_sweep(expint_dtype dt, expint_bc bc, const Geom& g, const Coef& cf, void* f0, void* f1, void* f2,
                          hipStream_t st, bool allow_vec, Tiling* out) {
  *out = default_tiling(g);
  // EXPINT_TILE=scalar / vec restricts the candidates to one sweep shape
  const char* shape = std::getenv("EXPINT_TILE");
  const int only = shape ? (shape[0] == 'v' ? 2 : (shape[0] == 's' ? 1 : 0)) : 0;
  const bool vec_ok = allow_vec && vec_sweep_ok(g, cf.labels_form) && only != 1;
  const bool scalar_ok = !(only == 2 && vec_ok);
  const char* env = std::getenv("EXPINT_AUTOTUNE");
  if (env && env[0] == '0') {
    if (!scalar_ok) {
      out->vec = 1;
      out->rw = 16;
      while (out->rw < 64 && 4 * out->rw < g.nz) out->rw *= 2;
      out->lp = 2;
    }
    return hipSuccess;
  }
  const Key key{g.nx, g.ny, g.nz, static_cast<int>(dt), static_cast<int>(bc),
                (cf.labels_form ? 1 : 0) | (vec_ok ? 2 : 0) | (scalar_ok ? 4 : 0)};
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      *out = it->second;
      return hipSuccess;
    }
  }
  // defined inputs for the timed sweeps
  hipError_t e;
  if ((e = launch_fill(dt, g.n, 0.25, f0, st)) != hipSuccess) return e;
  if ((e = launch_fill(dt, g.n, 0.0, f1, st)) != hipSuccess) return e;
  // the flush sweep with a y output: the heaviest flavour of the schedule
  TermOp op;
  op.src = f0;
  op.acc_in = f1;
  op.ca = 1.0;
  op.cs = 1.0;
  op.acc_out = f1;
  op.y_out = f2;
  op.c = 0.5;
  classify_term(op);
  std::vector<Tiling> cands;
  if (scalar_ok) {
    for (int bx : {64, 32, 16}) {
      if (bx > 16 && g.nz <= bx / 2) continue;  // mostly idle lanes
      for (int lp : {1, 2, 4}) {
        Tiling t;
        t.bx = bx;
        t.by = kBlock / bx;
        t.lp = lp;
        cands.push_back(t);
      }
    }
  }
  if (vec_ok) {
    for (int rw : {16, 32, 64}) {
      if (rw > 16 && 4 * rw >= 2 * g.nz) continue;  // mostly idle lanes
      for (int lp : {1, 2, 4}) {
        Tiling t;
        t.vec = 1;
        t.rw = rw;
        t.lp = lp;
        cands.push_back(t);
      }
    }
  }
  const int reps = g.n > (1 << 22) ? 3 : 8;
  float best = -1.f;
  Tiling best_t = *out;
  for (const Tiling& t : cands) {
    float ms = 0.f;
    if ((e = time_launches([&] { return launch_term(dt, bc, g, t, cf, op, st); }, reps, st, &ms)) != hipSuccess)
      return e;
    if (best < 0.f || ms < best) {
      best = ms;
      best_t = t;
    }
  }
  *out = best_t;
  if (std::getenv("EXPINT_LOG")) {
    if (best_t.vec)
      std::fprintf(stderr, "[expint] autotune %dx%dx%d %s: vector sweep rw=%d lp=%d (%.2f us/sweep)\n", g.nx, g.ny,
                   g.nz, dt == EXPINT_F64 ? "f64" : "f32", best_t.rw, best_t.lp, best * 1000.f);
    else
      std::fprintf(stderr, "[expint] autotune %dx%dx%d %s: bx=%d by=%d lp=%d (%.2f us/sweep)\n", g.nx, g.ny, g.nz,
                   dt == EXPINT_F64 ? "f64" : "f32", best_t.bx, best_t.by, best_t.lp, best * 1000.f);
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache[key] = best_t;
  return hipSuccess;
}

}  // namespace expint
