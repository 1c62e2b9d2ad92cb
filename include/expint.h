/*
 * expint.h - C ABI of the MI355X exponential-integrator library.
 *
 * The library advances the finite-difference Fisher-Kolmogorov glioma model
 *
 *     du/dt = div(D(x) grad u) + rho u (1 - u),   zero normal flux   (PDE, section 2)
 *
 * by the exponential Euler method in its incremental form (section 2.2)
 *
 *     u_{n+1} = u_n + tau phi1(tau A) (A u_n + rho u_n (1 - u_n)),
 *
 * where A is the 7-point finite-difference diffusion operator (section 2.1,
 * taken in conservative flux form with harmonic face means, so that it is
 * symmetric, negative semidefinite and conserves mass) and the action of
 * tau phi1(tau A) is computed as exp(tau B) applied to a unit vector of the
 * augmented matrix B = [[A, b], [0, 0]], exp evaluated as s scaled factors of
 * a degree-m truncated Taylor series (section 2.2).
 *
 * Conventions for every call:
 *  - Grids are nx * ny * nz voxels of spacing h, stored contiguously in C
 *    order with z fastest: flat index (i * ny + j) * nz + k.
 *  - "device" pointers are HIP device allocations on the current device (for
 *    example the data pointer of a torch tensor); "host" pointers are
 *    ordinary host memory.  Field pointers carry the context's dtype
 *    (double for EXPINT_F64, float for EXPINT_F32).
 *  - Every call returns 0 (EXPINT_OK) or a negative error code; nothing
 *    throws across the ABI.  expint_last_error() gives a message for the last
 *    failure on the calling thread.
 *  - Field computations are asynchronous on the context's stream unless the
 *    call returns host scalars (then it synchronises that stream).
 *  - A context is not thread-safe; use one context per stream.  After an
 *    EXPINT_EHIP failure the context is poisoned and every later call on it
 *    returns EXPINT_ESTATE (expint_destroy still works).
 *  - Environment: EXPINT_MAX_BYTES=N caps the device memory of a context;
 *    expint_create gives EXPINT_ENOMEM, before touching the device, when the
 *    field buffers alone exceed it.  EXPINT_FAIL_NTH_HIP=N (for tests of the
 *    error paths) makes a context created with it report its N-th checked
 *    HIP call after creation as failed.
 */
#ifndef EXPINT_H
#define EXPINT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EXPINT_OK 0
#define EXPINT_EINVAL (-1)       /* invalid argument */
#define EXPINT_EUNSUPPORTED (-2) /* valid request this build does not handle */
#define EXPINT_ENOMEM (-3)       /* device allocation failed or over EXPINT_MAX_BYTES */
#define EXPINT_EHIP (-4)         /* a HIP runtime call failed; context poisoned */
#define EXPINT_ENONFINITE (-5)   /* check_finite found a NaN/Inf in the state */
#define EXPINT_ESTATE (-6)       /* context poisoned by an earlier EXPINT_EHIP */
#define EXPINT_EIO (-7)          /* a file could not be written */

#define EXPINT_MAX_CLASSES 8

typedef enum { EXPINT_F64 = 0, EXPINT_F32 = 1 } expint_dtype;

/* Box boundary: EXPINT_NOFLUX is the paper's grad u . n = 0 (PDE, section 2),
 * read as zero flux through the wall faces.  EXPINT_DIRICHLET0 puts a ghost
 * value u = 0 at distance h outside each wall face (used for closed-form
 * sine-mode tests). */
typedef enum { EXPINT_NOFLUX = 0, EXPINT_DIRICHLET0 = 1 } expint_bc;

/* EXPINT_ALGO_STENCIL_TAYLOR: matrix-free stencil inside the scaled Taylor
 * series (any D).  EXPINT_ALGO_MODAL: uniform D only, A diagonalised by
 * per-axis cosine (no-flux) or sine (Dirichlet) modes; phi1 applied exactly
 * in that basis by per-axis mode products: fast cosine transforms along
 * no-flux axes of 32, 64, 128 or 256 points (FP64 and FP32 arithmetic, the
 * step's right-hand side formed inside the first pass when z is one), dense
 * products otherwise.  AUTO picks STENCIL_TAYLOR. */
typedef enum {
  EXPINT_ALGO_AUTO = 0,
  EXPINT_ALGO_STENCIL_TAYLOR = 1,
  EXPINT_ALGO_MODAL = 2
} expint_algo;

/* Arithmetic of the modal path's mode products (EXPINT_F32 contexts only):
 * NONE = FP32 (fast transforms where they apply, else FP32 matrix-core
 * products); BF16_SPLIT / FP16_SPLIT = dense matrix-core products of hi + lo
 * split operands with fp32 accumulation, on every axis. */
typedef enum {
  EXPINT_MP_NONE = 0,
  EXPINT_MP_BF16_SPLIT = 1,
  EXPINT_MP_FP16_SPLIT = 2
} expint_mp;

/* How the stencil-Taylor path groups the Taylor terms of a sub-step into
 * sweeps over the grid.  SINGLE: one sweep per term.  PAIRS: two consecutive
 * terms per sweep, the first kept on chip (label form only, else
 * EXPINT_EUNSUPPORTED; grids whose x-planes hold 4 GiB or more of field data
 * fall back to SINGLE).  AUTO: times both at creation and keeps the faster
 * (PAIRS only where PAIRS applies).  Same polynomial either way; results
 * agree to rounding.  expint_get_launch reports the choice. */
typedef enum {
  EXPINT_SWEEPS_AUTO = 0,
  EXPINT_SWEEPS_SINGLE = 1,
  EXPINT_SWEEPS_PAIRS = 2
} expint_sweeps;

/* The step a context takes.
 * EXP_EULER: u <- u + tau phi1(tau A)(A u + f(u)), f(u) = rho u (1 - u): the
 *   reaction frozen at u_n over the step (section 2.2).
 * EXPRK2: the second-order exponential Runge-Kutta step, the higher-order
 *   extension section 1 mentions, with phi2 from section 2.2's augmented
 *   matrix with both columns of its omega block in use:
 *   U = u + tau phi1(tau A)(A u + f(u)), then
 *   u <- u + tau phi1(tau A)(A u + f(u)) + tau phi2(tau A)(f(U) - f(u)).
 *   Two phi evaluations per step.  The plan rule takes m >= 2 (the phi2
 *   vector enters the series through its degree-2 term).  Stencil-Taylor
 *   with single-term sweeps only; batches and gradients give
 *   EXPINT_EUNSUPPORTED.
 * LINEARISED: the paper's splitting of the reaction (section 2.1, the
 *   rewritten F and the new F after it).  The part linear in the new state
 *   moves into the matrix, J_n = A + rho diag(1 - 2 u_n), leaving the source
 *   rho u_n^2, and the section 2.2 step is taken with J_n:
 *   u <- u + tau phi1(tau J_n)(J_n u_n + rho u_n^2), which equals
 *   u + tau phi1(tau J_n)(A u_n + f(u_n)).  J_n is the Jacobian at u_n, so
 *   this is exponential Rosenbrock-Euler, second order in tau.  The plan is
 *   chosen for tau (||A||_1 + rho), which bounds tau ||J_n||_1 for every
 *   state with 0 <= u <= 1 (the tolerance is not guaranteed outside that
 *   range).  Stencil-Taylor algorithm with single-term sweeps only. */
typedef enum {
  EXPINT_SCHEME_EXP_EULER = 0,
  EXPINT_SCHEME_LINEARISED = 1,
  EXPINT_SCHEME_EXPRK2 = 2
} expint_scheme;

typedef struct {
  int32_t nx, ny, nz; /* voxels per axis, each >= 1 */
  double h;           /* grid spacing (> 0), same unit as sqrt(D * time) */
} expint_grid;

/* Diffusivity D(x) per voxel (section 2: one value per tissue class).
 * Exactly one of `labels` and `D` is non-NULL.
 *  - label form: labels (device, nx*ny*nz uint8, each < n_classes) and
 *    class_D (host, n_classes doubles >= 0), 1 <= n_classes <= 8.
 *  - dense form: D (device, nx*ny*nz values of the context dtype, >= 0).
 * The library copies what it needs during expint_create; the caller may free
 * these buffers afterwards. */
typedef struct {
  const uint8_t* labels;
  int32_t n_classes;
  const double* class_D;
  const void* D;
} expint_dfield;

typedef struct {
  expint_dtype dtype;   /* arithmetic of the fields */
  double tau;           /* time step (> 0) */
  double tol;           /* plan tolerance; 0 = 1e-13 (F64) / 1e-6 (F32) */
  double theta_max;     /* plan cap on tau*||A||_1/s; 0 = ln 1024 (F64) / ln 64 (F32) */
  expint_algo algo;
  expint_mp mp;
  int32_t s, m;         /* both > 0: use this plan; both 0: choose it */
  int32_t check_finite; /* nonzero: expint_step / expint_advance scan u for NaN/Inf */
  expint_sweeps sweeps; /* term grouping of the stencil-Taylor sweeps */
  expint_scheme scheme; /* the step: EXP_EULER (default), LINEARISED or EXPRK2 */
  void* stream;         /* hipStream_t the context works on; NULL = null stream */
} expint_opts;

typedef struct expint_ctx expint_ctx;

/* Fill *opts with defaults: F32, tau = 7.3, automatic plan, AUTO algorithm,
 * AUTO sweeps, EXP_EULER scheme, no check, null stream.  Returns
 * EXPINT_EINVAL for NULL. */
int expint_opts_default(expint_opts* opts);

/* Create a context for one grid, diffusivity field, rho and boundary.
 * Validates the arguments, copies the coefficients, computes ||A||_1 on the
 * device (one stream synchronisation), chooses (s, m) by the plan rule
 * (section 2.2 asks for a "proper selection"; the rule: minimise s*m subject
 * to s*theta^(m+1)/(m+1)! <= tol and theta = tau*||A||_1/s <= theta_max,
 * m <= 60, ties to the smaller s) and allocates the workspace.
 * Errors: EINVAL (NULL pointer, dims < 1, h <= 0, tau <= 0, rho < 0 or not
 * finite, n_classes outside 1..8, class_D < 0 or not finite, a label >=
 * n_classes, D < 0 or not finite, s/m partly set), EUNSUPPORTED (MODAL with a
 * non-uniform D, mp without MODAL F32, LINEARISED or EXPRK2 with MODAL or
 * PAIRS), ENOMEM, EHIP.  A LINEARISED context plans for tau*(||A||_1 + rho) in
 * place of tau*||A||_1; an EXPRK2 context plans with m >= 2.  *out is NULL on
 * error. */
int expint_create(const expint_grid* grid, const expint_dfield* dfield, double rho,
                  expint_bc bc, const expint_opts* opts, expint_ctx** out);

/* Release the context and its workspace.  NULL-safe. */
void expint_destroy(expint_ctx* ctx);

/* The plan in use: Taylor scaling s, degree m and ||A||_1 (host scalars;
 * ||A||_1 of the diffusion operator alone, also for LINEARISED contexts). */
int expint_get_plan(const expint_ctx* ctx, int32_t* s, int32_t* m, double* norm_A1);

/* Launch configuration the context resolved at creation (autotuned). */
typedef struct {
  expint_sweeps sweeps; /* EXPINT_SWEEPS_SINGLE or EXPINT_SWEEPS_PAIRS (modal: SINGLE) */
  int32_t pair_ty;      /* pair sweeps: output rows along y per workgroup (0 if SINGLE) */
  int32_t pair_lp;      /* pair sweeps: x-planes per workgroup (0 if SINGLE) */
  int32_t vec;          /* single-term sweeps: 1 = z-vectorised (4 voxels per lane) */
  int32_t bx, by;       /* scalar sweep: threads along z and y (0 if vec) */
  int32_t rw;           /* vectorised sweep: lanes per z-segment (0 if scalar) */
  int32_t lp;           /* single-term sweeps: x-planes per thread */
  int32_t nt;           /* vectorised sweep: 1 = the Taylor terms of A store their outputs
                         * non-temporally (autotuned; LINEARISED contexts: always 0) */
  int32_t modal_dct;    /* modal contexts: bit a set if the mode products along axis a
                         * (0 = x, 1 = y, 2 = z) run as fast cosine transforms (zero flux,
                         * FP64 or FP32, that axis 32, 64, 128 or 256 long;
                         * EXPINT_MODAL_DCT=0 in the environment at creation: none); 0 otherwise */
} expint_launch_info;

/* The context's launch configuration.  EXPINT_EINVAL for NULL arguments. */
int expint_get_launch(const expint_ctx* ctx, expint_launch_info* info);

/* Replace rho and (label form) the class diffusivities.  replan != 0
 * recomputes ||A||_1 and (s, m) unless the plan was fixed in the options;
 * replan == 0 keeps the current (s, m) (finite-difference checks need the
 * computed map to stay smooth).  class_D may be NULL to keep it.  Modal
 * contexts need class_D uniform over the classes present in the grid, else
 * EXPINT_EUNSUPPORTED and nothing changes. */
int expint_set_params(expint_ctx* ctx, double rho, const double* class_D, int32_t replan);

/* y = A x (device fields).  x and y must not overlap. */
int expint_apply(expint_ctx* ctx, const void* x, void* y);

/* b = A u + rho u (1 - u): the right-hand side the step applies phi1 to. */
int expint_rhs(expint_ctx* ctx, const void* u, void* b);

/* x = tau phi1(tau A) b by the scaled Taylor series (section 2.2); with the
 * MODAL algorithm, exactly in the mode basis.  b and x must not overlap. */
int expint_phi1(expint_ctx* ctx, const void* b, void* x);

/* x = tau phi1(tau A) b + tau phi2(tau A) d (section 2.2's augmented matrix
 * with omega = [d / tau, b] next to the nilpotent 2 x 2 block), by the scaled
 * Taylor series with the context's plan (phi2 needs m >= 2 to appear; EXPRK2
 * contexts plan with it).  Stencil-Taylor contexts of the EXP_EULER or
 * EXPRK2 scheme (else EXPINT_EUNSUPPORTED).  b, d: device fields, read only;
 * x: device field, written, overlapping neither. */
int expint_phi12(expint_ctx* ctx, const void* b, const void* d, void* x);

/* x = tau phi1(tau J) b with J = A + rho diag(1 - 2 u), the linearised
 * operator of section 2.1 at the state u, by the scaled Taylor series of
 * section 2.2 with the context's plan.  LINEARISED contexts only (else
 * EXPINT_EUNSUPPORTED).  u, b: device fields, read only (they may be the same
 * field); x: device field, written, overlapping neither u nor b. */
int expint_phi1_lin(expint_ctx* ctx, const void* u, const void* b, void* x);

/* One step in place, of the context's scheme: EXP_EULER
 * u <- u + tau phi1(tau A)(A u + f(u)); LINEARISED
 * u <- u + tau phi1(tau J_n)(A u + f(u)); EXPRK2 as described at
 * expint_scheme.  u: device field owned by the caller.  ENONFINITE with
 * check_finite set. */
int expint_step(expint_ctx* ctx, void* u);

/* nsteps >= 0 steps in place.  The first call for a given u records the step
 * as a HIP graph on the context stream; later calls replay it. */
int expint_advance(expint_ctx* ctx, void* u, int32_t nsteps);

/* Deterministic FP64 reductions over a device field of the context dtype:
 * op 0 = sum x, 1 = sum x*y, 2 = max |x|, 3 = sum x / (nx ny nz), the tumour
 * volume diagnostic of the paper's convergence study (section 3.5).  y is
 * used by op 1 only.  Writes the host scalar *out (synchronises the
 * stream). */
int expint_reduce(expint_ctx* ctx, int32_t op, const void* x, const void* y, double* out);

/* Gradient of loss = 0.5 ||u_T - u_target||^2, u_T = nsteps steps from u0,
 * by the discrete adjoint of the computed map with the plan frozen.
 * u0, u_target: device fields (read only); grad_u0: device field (written);
 * loss, grad_rho: host scalars; grad_class_D: host array of n_classes
 * (label form only; dense form gives EINVAL).  u is checkpointed every
 * ckpt_every steps (>= 1) and recomputed in between.  Stencil-Taylor
 * contexts only (MODAL gives EXPINT_EUNSUPPORTED).  The context creates two
 * more streams for it (default priority): one recomputes each step's Taylor
 * tape one step ahead of the reverse sweeps on the context stream, the
 * other the states of the next checkpoint segment one segment ahead.  The
 * call synchronises all three before it returns.  EXP_EULER and
 * LINEARISED contexts (the latter differentiates J_n's diagonal too); EXPRK2
 * gives EXPINT_EUNSUPPORTED. */
int expint_grad(expint_ctx* ctx, const void* u0, int32_t nsteps, const void* u_target,
                int32_t ckpt_every, double* loss, void* grad_u0, double* grad_rho,
                double* grad_class_D);

/* Vector-Jacobian product of the same map for a given cotangent gout = dL/du_T
 * (device field).  Outputs as in expint_grad. */
int expint_vjp(expint_ctx* ctx, const void* u0, int32_t nsteps, const void* gout,
               int32_t ckpt_every, void* grad_u0, double* grad_rho, double* grad_class_D);

/* ---- Batched scenarios: many independent instances advanced together. ---- */
typedef struct expint_batch expint_batch;

/* count instances, each with its own grid, label field, class table and rho
 * (arrays of length count; dfield entries must use the label form).  Shared
 * bc and opts (dtype, tau, tol, theta_max).  Every instance gets its own
 * plan (LINEARISED: for tau (||A||_1 + rho_i)).  Creation also picks each
 * instance's sweep shape: the grid's own search chooses among the
 * z-vectorised shapes where the grid allows them.  Then, unless every
 * instance already has a batch entry in the tuning cache or file, whole
 * steps of the batch are timed with 1, 2 and 4 x-planes per lane.  They run
 * on workspace stand-ins for the states (a few to twenty replays of each, a
 * few tens of ms for 64 heads), and the fastest count is kept and filed.
 * EXPINT_AUTOTUNE=0 skips all timing.  Errors as expint_create; EXPRK2 gives
 * EXPINT_EUNSUPPORTED. */
int expint_batch_create(int32_t count, const expint_grid* grids, const expint_dfield* dfields,
                        const double* rho, expint_bc bc, const expint_opts* opts,
                        expint_batch** out);

/* Advance every instance by nsteps: u[i] is instance i's device field.  The
 * first call for a given set of pointers records one HIP graph holding the
 * whole schedule; later calls replay it.  Inside the graph, groups of
 * instances sized for the Infinity Cache run on three streams concurrently
 * (EXPINT_BATCH_LANES=1..4 in the environment at expint_batch_create sets
 * the count); results do not depend on it. */
int expint_batch_advance(expint_batch* batch, void* const* u, int32_t nsteps);

/* Plan of instance `index` (0 <= index < count): s, m and ||A||_1 as for
 * expint_get_plan (host scalars; each may be NULL).  EXPINT_EINVAL for a
 * NULL batch or an index out of range. */
int expint_batch_get_plan(const expint_batch* batch, int32_t index, int32_t* s, int32_t* m,
                          double* norm_A1);

/* Release the batch, its workspace and its recorded graph.  NULL-safe. */
void expint_batch_destroy(expint_batch* batch);

/* ---- Introspection and measurement. ---- */

/* The HIP stream (hipStream_t) the context works on: opts.stream, or a
 * blocking stream the context created when opts.stream was NULL. */
int expint_get_stream(const expint_ctx* ctx, void** stream);

/* Times `reps` back-to-back launches of one kernel of this context's step
 * with HIP events on the context stream and writes the mean milliseconds per
 * launch: kernel 0 = Taylor term that adds a pair of terms to the running sum
 * (reads the source, the sum; writes the term, the sum), 1 = Taylor term that
 * only writes its term, 2 = right-hand side A u + rho u (1 - u); modal
 * contexts also 3 = the pass along x as the step runs it (the dense mode
 * product in the left GEMM shape, or, where x runs as fast transforms, the
 * forward transform, the phi1 multiplier and the inverse transform in one
 * pass), 4 = the forward pass along z (dense product in the right GEMM shape,
 * or the forward transform); contexts that take their Taylor terms two at a
 * time (pair sweeps, label form) also 5 = pair sweep inside a sub-step (reads
 * the source, the sum; writes the second term, the sum), else
 * EXPINT_EUNSUPPORTED; 6 = the gradient's fused reverse sweep (a Taylor term
 * reading the source and a second field and writing the term, with the class
 * face products against a tape field), after a first gradient call on the
 * context and where it takes the fused form (z-vectorised shape, label form),
 * else EXPINT_EUNSUPPORTED.  Uses only the context workspace; synchronises. */
int expint_profile(expint_ctx* ctx, int32_t kernel, int32_t reps, double* ms);

/* ---- Peak probes (measurement of the device; not part of the method). ---- */

/* Times `reps` copies of `bytes` bytes (a positive multiple of 16, at most
 * 256 * (2^31 - 1) 16-byte vectors) from src to dst (device buffers, 16-byte
 * aligned, not overlapping), one 16-byte vector per lane, on `stream`
 * (hipStream_t, NULL = null stream); writes the mean milliseconds per copy to
 * *ms (bytes moved per copy = 2 * bytes).  nontemporal != 0 uses
 * non-temporal loads and stores (the fastest form for HBM streams); 0 uses
 * ordinary ones (for buffers that stay in the Infinity Cache).  Buffers well
 * above 256 MB measure HBM; smaller ones the Infinity Cache.  Synchronises.
 * EXPINT_EINVAL for bad arguments. */
int expint_probe_copy(const void* src, void* dst, int64_t bytes, int32_t reps, int32_t nontemporal, void* stream,
                      double* ms);

/* Runs `blocks` workgroups of 4 wavefronts; each wavefront issues `iters` x 8
 * independent v_mfma_f32_32x32x16 instructions (f16 != 0: fp16 inputs, else
 * bf16) on register operands.  Writes the executed TFLOP/s (2*32*32*16 flops
 * per instruction) to *tflops.  sink: device buffer of blocks * 256 floats
 * that receives the accumulator sums (overwritten).  Synchronises. */
int expint_probe_mfma(int32_t f16, int32_t iters, int32_t blocks, void* sink, void* stream, double* tflops);

/* ---- Label ingestion, diagnostics and output (sections 3.1, 3.2, 3.5). ---- */

/* Labels on the stencil grid nx x ny x nz from an 8-bit scan volume
 * ni x nj x nk (device, uint8, z fastest like the fields).  Section 3.5 takes
 * the scan values at the stencil points; read as: stencil point i of n along
 * an axis of N samples takes sample floor((2i + 1) N / (2n)).  Section 3.1
 * assigns materials by intensity thresholds; the label is the number of
 * thresholds strictly below the intensity (the paper's thresholds 1, 115,
 * 240 give 0 air, 1 white, 2 gray, 3 skull).  thresholds: host array of
 * n_thresholds (1..7) strictly increasing values.  labels: device, nx*ny*nz
 * bytes, written.  Asynchronous on `stream` (hipStream_t, NULL = null
 * stream).  EXPINT_EINVAL for bad arguments or overlapping buffers,
 * EXPINT_EUNSUPPORTED for nx or ny above 65535. */
int expint_labels_from_intensity(const uint8_t* image, int32_t ni, int32_t nj, int32_t nk,
                                 const int32_t* thresholds, int32_t n_thresholds, int32_t nx,
                                 int32_t ny, int32_t nz, uint8_t* labels, void* stream);

/* nsteps steps of the context's scheme, in place, recording the tumour
 * volume of section 3.5 after each: volumes[k] = (sum of u after step k + 1)
 * / (number of voxels), by the fixed-order FP64 reduction.  volumes: host
 * array of nsteps doubles.  Synchronises once at the end.  Errors as
 * expint_advance. */
int expint_advance_volumes(expint_ctx* ctx, void* u, int32_t nsteps, double* volumes);

/* The tumour size of section 3.2, the largest distance between two grid
 * points holding tumour, here the points with u > threshold: *d2 = the
 * largest squared distance in grid steps (h * sqrt(*d2) in length units);
 * -1 without such points, 0 for one.  pair (may be NULL): the linear indices
 * (i * ny + j) * nz + k of the pair reaching it that is smallest in
 * (first, second) order with first < second (the point twice for one point).
 * u: device field of the context's dtype and grid.  The comparison u >
 * threshold is made in FP64.  Synchronises.  EXPINT_EUNSUPPORTED for grids
 * whose y-z cross-section exceeds 2^27 points. */
int expint_tumour_size(expint_ctx* ctx, const void* u, double threshold, int64_t* d2, int64_t* pair);

/* Bytes of the static device workspace of expint_tumour_size_static. */
#define EXPINT_STATIC_SCRATCH_BYTES (4 << 20)

/* expint_tumour_size without a context and without any allocation, for
 * callers that cannot allocate device memory (code running while a HIP graph
 * is captured, tight serving loops, hosts that forbid hipMalloc).  Same
 * result as expint_tumour_size for the same field.  u: device field of nx *
 * ny * nz values of `dtype` (expint_dtype), z fastest; d2 and pair (may be
 * NULL) as there.  Runs on `stream` (hipStream_t, NULL = null stream) and
 * synchronises it.  The pass's workspace (line extents, candidates and
 * counters, 8 (ny nz + nx nz + nx ny) + 8 ny nz bytes plus 320) lives in a
 * static device array of EXPINT_STATIC_SCRATCH_BYTES on each device the
 * library runs on, held until the process ends; grids needing more give
 * EXPINT_EINVAL (up to 362^3 for cubes).  All calls on one device share that
 * array: calls that overlap in time on one device race and must not be
 * made.  EXPINT_EUNSUPPORTED as expint_tumour_size; EXPINT_EHIP on a HIP
 * error. */
int expint_tumour_size_static(const void* u, int32_t dtype, int32_t nx, int32_t ny, int32_t nz, double threshold,
                              int64_t* d2, int64_t* pair, void* stream);

/* Writes a legacy VTK file (STRUCTURED_POINTS, binary, big-endian) for
 * ParaView, the viewer of section 3.3: the field (host, nx*ny*nz values of
 * dtype, the library's layout) as scalars `name` (1..64 letters, digits or
 * '_'), and the labels (host, may be NULL) as scalars "labels".  The
 * library's axis i is VTK's x axis; spacing h, origin 0.  Host only, no
 * device call.  EXPINT_EINVAL for bad arguments, EXPINT_EIO for file errors. */
int expint_write_vtk(const char* path, int32_t nx, int32_t ny, int32_t nz, double h, const void* field,
                     expint_dtype dtype, const char* name, const uint8_t* labels);

/* Message for the last failed call on this thread ("" if none). */
const char* expint_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EXPINT_H */
