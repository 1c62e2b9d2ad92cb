// The context object behind expint_ctx* and its helpers (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <string>
#include <vector>

#include "internal.hpp"

namespace expint {

int set_error(int code, const char* fmt, ...);

// Device memory owned by one context or batch, with an optional byte cap
// (environment variable EXPINT_MAX_BYTES) for out-of-memory tests.
class Arena {
 public:
  Arena();
  ~Arena();
  // 0 on success, EXPINT_ENOMEM otherwise (error message set).
  int alloc(void** p, size_t bytes);
  // frees one allocation made by this arena (no-op for NULL)
  void release(void* p);
  size_t bytes() const { return bytes_; }
  // the EXPINT_MAX_BYTES cap read at construction (0 = none)
  size_t cap() const { return cap_; }

 private:
  std::vector<std::pair<void*, size_t>> ptrs_;
  size_t bytes_ = 0;
  size_t cap_ = 0;
};

struct GraphEntry {
  const void* key0 = nullptr;
  int nsteps = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

void destroy_graphs(std::vector<GraphEntry>& gs);

size_t dtype_size(expint_dtype dt);

}  // namespace expint

// A checked HIP call.  A context created with EXPINT_FAIL_NTH_HIP=N counts
// its checked calls and reports the N-th one as failed (after making it), so
// that the poisoned-context path can be driven from the host.
#define HIP_TRY(ctxp, call)                                                                          \
  do {                                                                                               \
    hipError_t e_ = (call);                                                                          \
    if (e_ == hipSuccess && (ctxp)->fail_countdown > 0 && --(ctxp)->fail_countdown == 0)             \
      e_ = hipErrorUnknown;                                                                          \
    if (e_ != hipSuccess) {                                                                          \
      (ctxp)->poisoned = true;                                                                       \
      return set_error(EXPINT_EHIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                       __LINE__);                                                                    \
    }                                                                                                \
  } while (0)

#define CHECK_CTX(ctxp)                                                              \
  do {                                                                               \
    if (!(ctxp)) return set_error(EXPINT_EINVAL, "context is NULL");                 \
    if ((ctxp)->poisoned) return set_error(EXPINT_ESTATE, "context poisoned by an earlier HIP error"); \
  } while (0)


struct expint_ctx {
  expint::Geom g{};
  double h = 1.0;
  expint_dtype dtype = EXPINT_F32;
  expint_bc bc = EXPINT_NOFLUX;
  expint_algo algo = EXPINT_ALGO_STENCIL_TAYLOR;
  expint_mp mp = EXPINT_MP_NONE;
  expint_scheme scheme = EXPINT_SCHEME_EXP_EULER;
  double rho = 0.0, tau = 0.0, tol = 0.0, theta_max = 0.0;
  bool fixed_plan = false;
  int s = 1, m = 1;
  double norm1 = 0.0;
  int check_finite = 0;

  bool labels_form = true;
  int nclass = 0;
  double class_D[EXPINT_MAX_CLASSES] = {0};

  int device = 0;
  hipStream_t stream = nullptr;  // the stream every call works on
  bool own_stream = false;

  expint::Arena arena;
  uint8_t* labels = nullptr;
  double* tab64 = nullptr;   // K(D_a, D_b) / h^2, FP64, 8 x 8
  double* wall64 = nullptr;  // D_a / h^2, FP64
  void* tab = nullptr;       // same in the context dtype
  void* wallc = nullptr;
  void* fx = nullptr;  // dense form face coefficients
  void* fy = nullptr;
  void* fz = nullptr;
  void* wallv = nullptr;

  void* b = nullptr;  // step workspace
  void* stage = nullptr;  // EXPRK2: tau phi1(tau A) b of the first stage
  void* dvec = nullptr;   // EXPRK2: f(U) - f(u)
  void* y[2] = {nullptr, nullptr};
  void* acc[2] = {nullptr, nullptr};
  double* partial = nullptr;  // reduction partials (see expint_create)
  double* red = nullptr;      // 2 reduction results

  expint::Tiling tiling;  // launch shape of the stencil sweeps (autotuned)
  expint::PairTiling ptiling;  // pair sweeps (two terms per sweep) if ptiling.ty != 0

  // modal path (uniform D): per-axis operators and eigenvalues, two scratch fields
  struct Modal {
    int prec = 0;                       // ModalPrec
    double Dc = 0.0;                    // the uniform diffusivity
    unsigned present = 0;               // bit a: some voxel has class a
    void* q[3][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};  // [axis][fwd, inv]
    double* lam[3] = {nullptr, nullptr, nullptr};
    void* t[2] = {nullptr, nullptr};
    // fast-transform tables of the axes whose products run as DCTs (zero
    // flux, FP64 or FP32, a power-of-two length dct_axis_ok), else NULL
    double* dct_tw[3] = {nullptr, nullptr, nullptr};
    double* dct_mk[3] = {nullptr, nullptr, nullptr};
  } modal;

  // adjoint workspace: allocated on the first gradient call, regrown on demand
  struct Adj {
    std::vector<void*> ckpt;  // u every ckpt_every steps
    // Two segment sets, used by alternate checkpoint segments: the states
    // u_k of every step of the segment (segs, segs2) and its tape, one slot
    // per step.  Slot t holds b_k (bts[t]), the sub-step states x_0 .. x_s
    // (xs[t (s + 1) ..]) and the Taylor terms y_1 .. y_m of every sub-step
    // (tape[t s m ..]); segment sgi's step k uses slot (sgi & 1) seg + k - start.
    std::vector<void*> segs;
    std::vector<void*> segs2;
    std::vector<void*> xs;
    std::vector<void*> tape;
    std::vector<void*> bts;
    int seg = 0;  // steps per segment set
    // the tapes of segment k - 1 are built on `rec` while segment k reverses
    // on the context stream (the first of them while the forward pass still
    // runs); the last segment's are built by the forward pass itself
    hipStream_t rec = nullptr;
    hipEvent_t ev_fwd = nullptr;                    // checkpoint of the second-to-last segment written
    hipEvent_t ev_seg[2] = {nullptr, nullptr};      // segment set q built
    hipEvent_t ev_segfree[2] = {nullptr, nullptr};  // set q no longer read
    void* lam = nullptr;      // adjoint state
    void* gb = nullptr;       // adjoint of b (= P(A) lambda)
    void* work = nullptr;     // forward state
    void* xb[2] = {nullptr, nullptr};
    void* yb[2] = {nullptr, nullptr};
    void* dbar = nullptr;     // LINEARISED: adjoint of the diagonal rho (1 - 2 u_n)
    double* fpart = nullptr;  // face-product slots, faceprod_slots(g, tiling) * 8
    double* dev = nullptr;    // [0..7] class sums, [8] d/drho, [9] loss
    double* dtab = nullptr;   // 8 x 64 face weights
    double* dwall = nullptr;  // 8 x 8 wall weights
  } adj;

  // tumour diagnostics workspace: allocated on first use
  struct Diag {
    int* ext = nullptr;  // x lo/hi, y lo/hi, z lo/hi line extents, back to back
    int* cand = nullptr;  // candidate points (linear indices), up to 2 per x-line
    int* count = nullptr;  // candidate count; best d2 and pair key follow
    unsigned long long* best = nullptr;
    unsigned long long* key = nullptr;
    double* vol = nullptr;  // per-step sums of u
    int64_t vol_cap = 0;
  } diag;

  std::vector<expint::GraphEntry> graphs;
  bool use_graph = true;  // EXPINT_GRAPH=0: advance launches each step directly
  bool poisoned = false;
  int64_t fail_countdown = 0;  // EXPINT_FAIL_NTH_HIP (see HIP_TRY)

  expint::Coef coef() const {
    expint::Coef c{};
    c.labels_form = labels_form;
    c.labels = labels;
    c.tab = tab;
    c.wallc = wallc;
    c.fx = fx;
    c.fy = fy;
    c.fz = fz;
    c.wallv = wallv;
    return c;
  }
  size_t field_bytes() const { return static_cast<size_t>(g.n) * expint::dtype_size(dtype); }
};

namespace expint {

struct StepBuffers;

// Shared host runtime (api.cpp).
bool finite_nonneg(double v);
double harmonic_mean(double a, double b);
int ensure_device(expint_ctx* c);
int upload_tables(expint_ctx* c);
int enqueue_step(expint_ctx* c, void* u);
int enqueue_step_on(expint_ctx* c, void* u, hipStream_t st, const StepBuffers* sb);
// nsteps steps on the stream: replays (recording on first use) the step graph
// for u, or launches each step when graphs are off.  No synchronisation.
int run_steps(expint_ctx* c, void* u, int32_t nsteps);
int run_ops(expint_ctx* c, const std::vector<TermOp>& ops);
// The Taylor sweeps of tau phi1(tau A) b for this context's plan: pair sweeps
// when the context uses them, else one sweep per term (see phi1_schedule).
std::vector<TermOp> step_schedule(expint_ctx* c, const void* b, void* x_out, void* u, const StepBuffers* sb);
// ||A||_1 for EXP_EULER, ||A||_1 + rho (a bound on ||J_n||_1) for LINEARISED.
double plan_norm(const expint_ctx* c);
int check_finite_field(expint_ctx* c, const void* u);
// modal path (modal_host.cpp)
int modal_setup(expint_ctx* c);
// u_rhs non-NULL: b is the right-hand side A u_rhs + rho u_rhs (1 - u_rhs),
// computed inside the first pass where z runs as fast transforms (returns
// false if it does not: the caller forms b itself)
bool modal_fuses_rhs(const expint_ctx* c);
// The uniform diffusivity of class_D over the classes present in the grid
// (EXPINT_EUNSUPPORTED if they differ); with set, stored as the modal D.
int modal_diffusivity(expint_ctx* c, const double* class_D, bool set);
int modal_phi1(expint_ctx* c, const void* b, void* out, bool add_into_out, const void* u_rhs = nullptr);

}  // namespace expint
