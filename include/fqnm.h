/*
 * fqnm.h -- C ABI of the MI355X (gfx950) implementation of the Fast Quantised
 * Numerical Method (FQNM), arXiv 2604.06947.
 *
 * The method evolves integer states q_i instead of floating-point fields
 * (Sec. 2, eq:quantisation).  Every interface i+1/2 carries an integer count
 * flux F_{i+1/2} = T(q_i, q_{i+1}) built from rounded transfer maps
 * (eq:flux_table, eq:numerical_count_flux_definition), and every cell applies
 *     q_i <- q_i - (F_{i+1/2} - F_{i-1/2})         (eq:update_rule_conservative_form)
 * so the total count is conserved exactly by integer telescoping
 * (Sec. 2.3, eq:exact_conservation).  Fields are observables u_i = delta*q_i
 * (eq:reconstruction_operator).
 *
 * Conventions shared by every entry point
 *   - Every function returns fqnm_status: 0 on success, a negative code on
 *     failure.  fqnm_last_error() returns a thread-local message describing the
 *     last failure of the calling thread.  No C++ exception crosses this ABI.
 *   - Host pointers are read (or written) during the call only; the caller
 *     keeps ownership.  Device memory allocated by the library belongs to the
 *     object that allocated it and is freed by its destroy call.  A device
 *     pointer passed to fqnm_create_on_device is borrowed and must outlive the
 *     context.
 *   - hip_stream is a hipStream_t (NULL = the default stream).  Work is
 *     enqueued asynchronously on it; calls that return host data synchronise it.
 *   - An object is not thread-safe; distinct objects on distinct streams are
 *     independent.  After a HIP runtime error an object is poisoned and every
 *     later call on it returns FQNM_ERR_DEVICE.
 *   - Cells are indexed 0..n-1 with centres x_i = i*dx (Sec. 2).  A scalar
 *     state is n integers; an Euler state is three arrays of n integers
 *     (rho, m, E) stored one after the other (structure of arrays).
 *   - "round" is IEEE round-half-to-even; every floating-point operation of a
 *     transfer map is one IEEE operation in a fixed order with no contraction,
 *     so the integer trajectory is a deterministic function of the inputs.
 */
#ifndef FQNM_H
#define FQNM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FQNM_ABI_VERSION 1u

typedef enum {
  FQNM_OK = 0,
  FQNM_ERR_ARG = -1,         /* invalid argument (null pointer, bad enum, non-positive constant) */
  FQNM_ERR_CFL = -2,         /* CFL number nu = dt/dx * max|f'| exceeds 1 (Sec. 2.2, eq:cfl_number) */
  FQNM_ERR_RANGE = -3,       /* integer or FP64-exactness range would be exceeded                */
  FQNM_ERR_OOM = -4,         /* device allocation failed, or a server budget cannot hold a request */
  FQNM_ERR_DEVICE = -5,      /* HIP runtime error (sticky for the object)                         */
  FQNM_ERR_STATE = -6,       /* call not valid in the object's current state                      */
  FQNM_ERR_BUSY = -7,        /* resource temporarily unavailable (server queue full)              */
  FQNM_ERR_UNSUPPORTED = -8  /* valid request that the library does not implement                 */
} fqnm_status;

/* Flux kinds.  Split kinds round f+ and f- separately (eq:flux_table); two-point
 * kinds round the interface flux once
 * (Sec. 2.2, eq:transfer_operator_equivalence_definition). */
typedef enum {
  FQNM_FLUX_UPWIND = 0,          /* f = a u; f+ = max(a,0)u, f- = min(a,0)u; phi = rint((a*lambda)*q) */
  FQNM_FLUX_BURGERS_EO = 1,      /* f = u^2/2, Engquist-Osher split f+ = max(u,0)^2/2, f- = min(u,0)^2/2;
                                    phi = rint(((delta*lambda)*0.5) * s^2)                        */
  FQNM_FLUX_BURGERS_GODUNOV = 2, /* f = u^2/2, two-point Godunov flux, one rounding              */
  FQNM_FLUX_LF_LINEAR = 3,       /* f = a u, Lax-Friedrichs split (f +- alpha u)/2 (Sec. 2,
                                    eq:flux_splitting)                                           */
  FQNM_FLUX_LF_BURGERS = 4,      /* f = u^2/2, Lax-Friedrichs split                              */
  FQNM_FLUX_EULER_ROE = 5,       /* Euler equations, 3 components, Roe flux in FP64 then
                                    T_c = rint((F_c*lambda)/delta) per component (Sec. 3.3)      */
  FQNM_FLUX_EULER_ROE_EF = 6,    /* as above with an entropy fix of the acoustic waves            */
  FQNM_FLUX_BURGERS_MURMAN_ROE = 7, /* f = u^2/2, two-point Murman-Roe flux, one rounding        */
  FQNM_FLUX_EULER_ROE_DENSITY = 8, /* Euler, density-only quantisation (the prototype of Sec. 3.3):
                                    component 0 holds int64 density counts moved by
                                    T = rint((F_rho*lambda)/delta); components 1 and 2 hold FP64
                                    m and E (8-byte slots), updated U - lambda*(F_R - F_L); all
                                    fluxes from one FP64 Roe flux of (delta*q_rho, m, E)        */
  FQNM_FLUX_EULER_ROE_EF_DENSITY = 9 /* as above with the entropy fix of FQNM_FLUX_EULER_ROE_EF  */
} fqnm_flux;

typedef enum { FQNM_BC_PERIODIC = 0, FQNM_BC_OUTFLOW = 1 } fqnm_bc;
typedef enum { FQNM_I32 = 0, FQNM_I64 = 1 } fqnm_itype;

/* How a split transfer map is evaluated on the device.  Tabulation is an
 * execution strategy, not the method (Sec. 2, after eq:flux_table): both
 * modes produce the same integers.  LUT mode tabulates phi+ and phi- over the
 * initial state range [min q0, max q0], which bounds every later state by the
 * discrete maximum principle (Lemma cfl_monotone (i)); it is accepted for the
 * kinds for which that principle holds (UPWIND, BURGERS_EO).  Building the
 * table also checks that principle on the rounded maps themselves (phi+ never
 * falls, phi- never rises and q - phi+ + phi- never falls from one state to the
 * next); kernels 1 and 10 rely on it to step their LDS slices in the update's
 * per-cell form g(q_i) + phi+(q_{i-1}) - phi-(q_{i+1}), g(q) = q - phi+(q) +
 * phi-(q), from one unclamped read per cell, and take the flux-difference
 * form with clamped reads for a table that fails the check (or for every
 * table when the environment variable FQNM_TABLE_CLAMPED is set at create):
 * the integers are the same.  The temporally blocked
 * kernels (plan kernels 1, 3, 4, 5, 7, 8 and 10) read the table
 * from a per-tile slice in LDS when the tile's int32 states span fewer than
 * 512 levels (2048 for tiles of several wavefronts); their wider int32 tiles
 * and all their int64 tiles evaluate the maps the table was built from
 * instead, which gives the same entries.  The other kernels read the table
 * itself. */
typedef enum { FQNM_EVAL_AUTO = 0, FQNM_EVAL_DIRECT = 1, FQNM_EVAL_LUT = 2 } fqnm_eval;

/* Problem statement (Sec. 2): flux kind and its constants, resolution delta,
 * cell width dx, lambda = dt/dx, boundary kind, storage width, cell count. */
typedef struct {
  uint32_t abi_version; /* must equal FQNM_ABI_VERSION                                  */
  int32_t flux;         /* fqnm_flux                                                    */
  int32_t bc;           /* fqnm_bc                                                      */
  int32_t itype;        /* fqnm_itype; Euler kinds require FQNM_I64                     */
  int32_t eval;         /* fqnm_eval (scalar split kinds only; others ignore it)        */
  int32_t reserved;     /* must be 0                                                    */
  double a;             /* advection speed (UPWIND, LF_LINEAR)                          */
  double alpha;         /* LF dissipation speed, alpha >= max|f'| on the state range    */
  double gamma;         /* ratio of specific heats (Euler kinds), > 1                   */
  double delta;         /* quantisation resolution, > 0                                */
  double dx;            /* cell width, > 0 (informational: the update uses lambda)      */
  double lambda;        /* dt/dx, > 0                                                   */
  int64_t n;            /* cells, >= 1; components = 3 for Euler kinds, else 1          */
} fqnm_problem;

/* Exact diagnostics of a state (Sec. 2.2 Lemma cfl_monotone, Sec. 2.3).  Sums
 * and total variations are 128-bit two's-complement values split into a
 * signed high and an unsigned low word.  Unused components are zero. */
typedef struct {
  int32_t components;
  int32_t reserved;
  int64_t steps_done;   /* steps applied since create                                    */
  int64_t sum_hi[3];    /* sum_i q_i per component                                       */
  uint64_t sum_lo[3];
  int64_t qmin[3];
  int64_t qmax[3];
  int64_t tv_hi[3];     /* sum_i |q_{i+1} - q_i| (periodic: including the wrap term);
                           0 for d-D contexts                                            */
  uint64_t tv_lo[3];
  int64_t ledger[3];    /* outflow: sum over steps of F_{-1/2} - F_{n-1/2}, the net count
                           that entered through the boundaries (d-D: over every outflow
                           face); periodic: 0.  Invariant: sum(q) - sum(q0) == ledger    */
} fqnm_invariants;

/* Launch plan of the single-grid stepper.  kernel 0 = one step per pass
 * ("stream"); 1 = temporal blocking: every wavefront keeps a tile of 64*vec
 * consecutive cells in registers (vec consecutive cells per lane) and
 * advances it `depth` steps per pass over memory (vec 4, 8 or 16 for int32
 * states; 2, 4 or 8 for int64, and also 16 for int64 UPWIND maps evaluated
 * directly, whose windows away from outflow ends step as exact doubles); 2 = temporal blocking with
 * lane-interleaved cells (consecutive cells in consecutive lanes, so table
 * reads coalesce), split kinds only; 3, 4, 5 = temporal blocking in
 * workgroup tiles of 2, 4 or 8 wavefronts; 6 = the d-D marching kernel: a
 * wavefront owns 64*vec cells of axis 0 and marches `depth` cells along the
 * last axis, one step per pass; 7, 8 = workgroup tiles of 4 or 8 wavefronts
 * whose windows (64*vec cells, vec 2 or 4) overlap by 16 cells and are
 * refreshed from their neighbours every 8 steps, `depth` <= 64*vec - 16 steps
 * per pass (int32 tables on periodic grids only); 9 = d-D marching with
 * temporal blocking (2-D grids; vec 2 or 4 for int32, 2 for int64, dividing
 * the length of axis 0): `depth & 0xFF` steps per pass (1, 2, 4 or 8; a
 * remainder runs as smaller passes) and `depth >> 8` cells marched along
 * axis 1 per wavefront (0 = chosen from the grid size); 10 = kernel 1's
 * tiles (vec 4 or 8, `depth` steps per pass) with every pass in one
 * cooperative launch: each wavefront keeps its tile in registers between
 * passes and swaps its edge cells with its two neighbours through memory,
 * every wait bounded (a launch that times out makes the next syncing call
 * return FQNM_ERR_DEVICE); int32 states on periodic grids, UPWIND or
 * BURGERS_EO maps (table or direct), and only when every workgroup of the
 * launch can be resident at once (fqnm_set_plan checks).  d-D contexts run
 * kernels 6 and 9 only.  Zero fields mean "keep" (on a change between
 * kernels 6 and 9: that kernel's default, vec 4 (int64: 2) and 16 rows, or
 * vec 2 and 4 steps per pass).  A new 1-D context starts with the plan the
 * autotuner cached for its shape, else kernel 1 with vec 4 (int32) or 8
 * (int64), 52 steps per pass for int32 tables and 24 otherwise (int64 UPWIND:
 * vec 16, 48 steps); a grid small enough that a deeper pass keeps about one
 * wavefront per SIMD (at most 1.75 tiles per SIMD) takes instead the deepest
 * such pass of 4-cell lanes, up to 120 steps (int64 UPWIND also 16-cell lanes
 * at 200 steps), since there a pass costs about its launch whatever its
 * halo. */
typedef struct {
  int32_t kernel;
  int32_t vec;          /* cells per lane                                                */
  int32_t depth;        /* steps per pass (kernel 1)                                     */
  int32_t eval;         /* resolved fqnm_eval (read-only in fqnm_get_plan)               */
} fqnm_plan;

typedef struct fqnm_ctx fqnm_ctx;

const char* fqnm_last_error(void);
const char* fqnm_version(void);

/* Create a solver from an integer initial state q0_host (n or 3n integers of
 * the problem's itype; for the density-only Euler kinds 3n 8-byte slots: n
 * int64 density counts, then n FP64 momenta and n FP64 energies).  Validates
 * the problem: positive finite delta, dx, lambda (FQNM_ERR_ARG); the CFL
 * number over [min q0, max q0] for scalar
 * kinds (FQNM_ERR_CFL, Sec. 2.2 eq:cfl_number); |q| < 2^51 for int64 states
 * (the transfers convert through a 1.5*2^52 bias) so that q converts
 * to FP64 exactly, q^2 < 2^53 for Burgers kinds, and for I32 that
 * |q| + 2 max|F| < 2^31 on that range (FQNM_ERR_RANGE).  Copies q0 to the
 * device on hip_stream and builds the LUT when the eval mode asks for it. */
fqnm_status fqnm_create(const fqnm_problem* prob, const void* q0_host, void* hip_stream,
                        fqnm_ctx** out);

/* As fqnm_create, from a real initial field u0_host (n or 3n doubles): the
 * device quantises q0_i = rint(u0_i / delta) (Sec. 2, eq:quantisation); the
 * density-only Euler kinds quantise the density and keep m and E as given. */
fqnm_status fqnm_create_from_field(const fqnm_problem* prob, const double* u0_host,
                                   void* hip_stream, fqnm_ctx** out);

/* As fqnm_create, with the initial state already on the device in d_q
 * (components*n integers of the problem's itype, borrowed).  After every
 * fqnm_step the current state is again in d_q. */
fqnm_status fqnm_create_on_device(const fqnm_problem* prob, void* d_q, void* hip_stream,
                                  fqnm_ctx** out);

/* Advance n_steps >= 0 time steps of eq:update_rule_conservative_form.
 * Asynchronous: enqueued on the context's stream. */
fqnm_status fqnm_step(fqnm_ctx* ctx, int64_t n_steps);

/* Copy the current integer state to the host (components*n integers). Syncs. */
fqnm_status fqnm_get_state(fqnm_ctx* ctx, void* q_host);

/* Device address of the current state (valid until the next fqnm_step). */
fqnm_status fqnm_state_device(fqnm_ctx* ctx, void** d_q);

/* Reconstruct u_i = delta*q_i (eq:reconstruction_operator) into u_host
 * (components*n doubles; density-only Euler kinds: delta*q_rho, then m and E
 * as they are).  Syncs. */
fqnm_status fqnm_reconstruct(fqnm_ctx* ctx, double* u_host);

/* As fqnm_reconstruct into device memory d_u; asynchronous. */
fqnm_status fqnm_reconstruct_device(fqnm_ctx* ctx, double* d_u);

/* Exact sums, extrema, total variation and boundary ledger of the integer
 * components (density-only Euler kinds: the density alone).  Syncs. */
fqnm_status fqnm_invariants_get(fqnm_ctx* ctx, fqnm_invariants* out);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, such as tight serving loops or harnesses that forbid it): the
 * same results as fqnm_invariants_get, with no device allocation.  The
 * per-block partial records live in a static device array of the library
 * (4099 records of 48 bytes, 192 KiB per device, held until the process ends)
 * instead of a buffer the context allocates on first use; one block reduces
 * ceil(n/4096) cells (at least 16384), so every context size fits.  Calls of
 * one process are serialised by the library (the array is shared by all calls
 * on a device).  Switches to the context's device for the call.  Syncs.
 * FQNM_ERR_UNSUPPORTED for FP64 twin contexts, FQNM_ERR_RANGE should a state
 * need more than 4096 partial records. */
fqnm_status fqnm_invariants_get_noalloc(fqnm_ctx* ctx, fqnm_invariants* out);

/* The context's launch plan.  Euler contexts have a fixed one and report
 * kernel 0 with depth = the steps advanced per launch (8). */
fqnm_status fqnm_get_plan(fqnm_ctx* ctx, fqnm_plan* out);
/* Force a plan (zero fields keep the current choice).  FQNM_ERR_ARG if the
 * combination is not available for this problem. */
fqnm_status fqnm_set_plan(fqnm_ctx* ctx, const fqnm_plan* plan);
/* Time the candidate plans on a scratch copy of the state (the state itself is
 * not advanced), keep the fastest, and remember it for problems of the same
 * shape in this process and in the file named by FQNM_AUTOTUNE_CACHE, if set. */
fqnm_status fqnm_autotune(fqnm_ctx* ctx, int64_t steps_per_trial);

fqnm_status fqnm_destroy(fqnm_ctx* ctx); /* NULL-safe */

/* The FP64 split finite-volume twin of a problem (Sec. 2.1,
 * eq:classical_operator_definition): state u in FP64 (n doubles, u0_host is
 * copied), the same flux kind, boundary kind and lambda, update
 * u_i <- u_i - lambda*(F(u_i,u_{i+1}) - F(u_{i-1},u_i)) with
 * F(uL,uR) = f+(uL) + f-(uR) (or the two-point flux), every operation one
 * IEEE double op in a fixed order.  It exists to time the classical scheme
 * beside the integer one on the same workload.  fqnm_step, fqnm_get_state
 * (n doubles), fqnm_reconstruct (the state itself), plans and fqnm_destroy
 * apply; fqnm_invariants_get returns FQNM_ERR_UNSUPPORTED.  Validation:
 * FQNM_ERR_ARG as for fqnm_create (itype and eval are ignored, Euler kinds
 * are refused), FQNM_ERR_CFL if lambda*max|f'| > 1 on [min u0, max u0]. */
fqnm_status fqnm_create_classical(const fqnm_problem* prob, const double* u0_host,
                                  void* hip_stream, fqnm_ctx** out);

/* A d-dimensional Cartesian grid, d = 2 or 3, advanced by directional
 * composition (Thm dimension_extension, eq:nd_transfer_rule,
 * eq:nd_flux_definition): each step every cell subtracts, for every direction
 * m, the difference of the one-dimensional transfers across its two faces
 * orthogonal to m, all evaluated from the state before the step.  axes[m]
 * describes direction m: n = cells along the axis, bc, a, alpha, lambda
 * (= dt/dx_m) and dx; flux, itype and delta must be the same on every axis.
 * Axis 0 is contiguous: cell (i_0, .., i_{d-1}) is element
 * i_0 + n_0*(i_1 + n_1*i_2) of q0_host (prod n_m values of itype, copied).
 * Outflow ends copy the cell into its ghost, per direction.  The single-grid
 * calls (step, get/state, reconstruct, invariants, plans, autotune, level
 * statistics, destroy) apply with n = prod n_m.  2-D grids start on the
 * temporally blocked marching kernel (plan kernel 9: 2 cells per lane, 4
 * steps per launch), or on kernel 6 when n_0 is odd; 3-D grids start on the
 * one-step marching kernel (kernel 6).  Errors: FQNM_ERR_ARG for a
 * bad dim, an invalid axis, axes that disagree, more than 2^36 cells, or
 * an axis of 2^31 cells or more;
 * FQNM_ERR_UNSUPPORTED for Euler kinds and for eval = FQNM_EVAL_LUT (the
 * composed rounding keeps no exact maximum principle, on which the table
 * range rests); FQNM_ERR_CFL if the CFL numbers of the directions add up to
 * more than 1; FQNM_ERR_RANGE if states or transfers could overflow (int32
 * keeps a margin of 2^24 counts). */
fqnm_status fqnm_create_nd(const fqnm_problem* axes, int32_t dim, const void* q0_host,
                           void* hip_stream, fqnm_ctx** out);

/* Quantise a real field on the device (Sec. 2, eq:quantisation):
 * q_host[i] = rint(u_host[i] / delta) for i < n, stored as itype.
 * FQNM_ERR_RANGE if a value does not fit the storage type (or |q| >= 2^52
 * for FQNM_I64).  Syncs hip_stream. */
fqnm_status fqnm_quantise(const double* u_host, int64_t n, double delta, int32_t itype,
                          void* q_host, void* hip_stream);

/* Self-check of the FP64 operations the Euler transfer relies on: evaluates,
 * with the library's own device code generation, out_sqrt[i] = sqrt(d_a[i])
 * and out_div[i] = d_a[i] / d_b[i] for i < n (all device pointers), so that a
 * caller can compare them with a correctly rounded host reference.  Syncs. */
fqnm_status fqnm_fp64_selfcheck(const double* d_a, const double* d_b, double* d_out_sqrt,
                                double* d_out_div, int64_t n, void* hip_stream);

/* ------------------------------------------------------------------------
 * Level statistics of a scalar integer state (Supplementary Information).
 * c_k = #{i : q_i = k} and p_k = c_k / n (eq:pk_definition); these calls are
 * diagnostics, computed on the device by a radix sort of the state and a
 * run-length encoding, with temporary device memory allocated per call.  They
 * synchronise the context's stream.  FQNM_ERR_UNSUPPORTED for Euler and FP64
 * twin contexts and for n > 2^31 - 1.
 * ---------------------------------------------------------------------- */

/* Occupied levels of the current state in increasing order, with their
 * counts: levels[j], counts[j] for j < min(cap, *n_levels).  *n_levels
 * receives the number of occupied levels even when it exceeds cap (cap = 0
 * with NULL arrays asks for the count only).  FQNM_ERR_ARG for NULL
 * n_levels, cap < 0, or cap > 0 with a NULL array. */
fqnm_status fqnm_level_histogram(fqnm_ctx* ctx, int64_t* levels, int64_t* counts, int64_t cap,
                                 int64_t* n_levels);

/* Discrete entropy S = -sum_k p_k log p_k of the current state
 * (eq:discrete_entropy), summed over the occupied levels in increasing level
 * order, and N_eff = exp(S) (eq:neff) if n_eff is non-NULL. */
fqnm_status fqnm_entropy(fqnm_ctx* ctx, double* S, double* n_eff);

/* Advance the context by ONE step and report the level-transition counts of
 * that step (Definition level_transition): N_{k'k} = #{i : q_i^n = k and
 * q_i^{n+1} = k'} as triples (from[j] = k, to[j] = k', count[j] = N_{k'k}),
 * the nonzero ones, in increasing (k, k') order, for j < min(cap, *n_pairs).
 * *n_pairs receives the number of nonzero triples.  If row_defect is
 * non-NULL it receives rho = max over k' of |sum_k N_{k'k} / c_k^n - 1|
 * (eq:empirical_M, Remark doubly_stochastic_condition), k' running over the
 * levels occupied after the step, each row summed in increasing k.  The step
 * is the context's ordinary step (counted in its step total). */
fqnm_status fqnm_step_transitions(fqnm_ctx* ctx, int64_t* from, int64_t* to, int64_t* count,
                                  int64_t cap, int64_t* n_pairs, double* row_defect);

/* ------------------------------------------------------------------------
 * Batching: many independent instances (each its own problem, state and step
 * count) advanced together.  int32 instances with direct evaluation and at
 * most 65536 cells (32768 for the Godunov and Murman-Roe kinds) run every one
 * of their steps inside persistent launches with their state held in
 * registers: three kernels, one per size class, side by side on the caller's
 * stream and two library streams forked from it and joined back.  Other
 * instances (tables, 64-bit states, Lax-Friedrichs maps, larger grids) run
 * as tiled work items: one launch per step block advances every such
 * instance's tiles together, on a library stream beside the persistent
 * kernels.  The whole run is captured once as a HIP graph and replayed (with
 * the environment variable FQNM_BATCH_NO_GRAPH set when the batch is
 * created, the same launches are issued directly instead, for profilers that
 * cannot follow graph replays).
 * ---------------------------------------------------------------------- */
typedef struct fqnm_batch fqnm_batch;

/* probs[k], q0s[k] (host, the instance's itype) and steps[k] >= 0 describe
 * instance k.  Scalar kinds only. */
fqnm_status fqnm_batch_create(const fqnm_problem* probs, const void* const* q0s,
                              const int64_t* steps, int32_t count, void* hip_stream,
                              fqnm_batch** out);
/* How a batch lays out its work.  Register-resident instances: those of at
 * most class0_max_cells cells (<= 16384) run on 512-thread workgroups using
 * at most class0_lanes lanes (128, 256 or 512: cells per lane is the
 * smallest power of two that fits, at most 32); with wide_split_class 1 (or
 * 0), split kinds of up to 32768 cells run on 512 threads with 64 cells per
 * lane, with 2 they join the larger instances on 1024-thread workgroups.
 * Tiled instances: tiled_vec cells per lane (4 or 8) and tiled_depth steps
 * per block, or each instance's own single-grid plan where 0.  Every field
 * zero means the library's default layout. */
typedef struct {
  int32_t class0_max_cells;
  int32_t class0_lanes;
  int32_t wide_split_class;
  int32_t tiled_vec;
  int32_t tiled_depth;
  int32_t reserved;     /* must be 0 */
} fqnm_batch_config;

/* The batch's current layout (the default until set or tuned). */
fqnm_status fqnm_batch_get_config(fqnm_batch* b, fqnm_batch_config* out);
/* Lay the batch out anew (rebuilds its instance tables and graph; the
 * instances' states are not changed).  FQNM_ERR_ARG for values outside the
 * ranges above.  Syncs. */
fqnm_status fqnm_batch_set_config(fqnm_batch* b, const fqnm_batch_config* cfg);
/* Time candidate layouts of this batch -- the class boundary, lanes per
 * resident instance, the wide split class, and the tiled instances' cells
 * per lane and depth -- each on the real instances (the better of two runs,
 * HIP events on the library's stream), keep the fastest, and remember it for
 * batches of the same shape (count, storage type and a histogram of the
 * instances' sizes) in this process.  Every instance is reset to its initial
 * state afterwards.  Syncs. */
fqnm_status fqnm_batch_autotune(fqnm_batch* b);

/* Restore every instance to its initial state (for repeated runs). Async. */
fqnm_status fqnm_batch_reset(fqnm_batch* b);
/* Advance every instance by its own step count in one batched run. Async. */
fqnm_status fqnm_batch_run(fqnm_batch* b);
/* The comparison loop: the same work as one single-grid run per instance,
 * issued one instance after another on the stream. Async. */
fqnm_status fqnm_batch_run_per_instance(fqnm_batch* b);
fqnm_status fqnm_batch_get_state(fqnm_batch* b, int32_t idx, void* q_host); /* syncs */
fqnm_status fqnm_batch_destroy(fqnm_batch* b);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of solve requests.  A worker thread admits
 * queued requests while their device footprint fits the budget, keeps their
 * integer state resident, and advances every admitted request by up to
 * tick_steps steps per tick in one batched launch sequence.  Requests that
 * arrive while a tick runs join at the next tick.  Each request's trajectory
 * is the same integers it would have alone.
 * ---------------------------------------------------------------------- */
typedef struct fqnm_server fqnm_server;

typedef struct {
  uint64_t id;
  int32_t status;       /* fqnm_status of the request                                    */
  int32_t components;
  int64_t n;
  int64_t steps;
  double t_submit;      /* seconds on the library's monotonic clock                      */
  double t_admit;
  double t_done;
} fqnm_completion;

typedef struct {
  int64_t submitted, admitted, completed, queued, active;
  int64_t ticks;
  int64_t bytes_in_use;
  int64_t peak_bytes;
  double cell_updates;  /* total cells*steps*components... counted per cell-update       */
} fqnm_server_stats;

fqnm_status fqnm_server_create(size_t device_budget_bytes, int32_t tick_steps, void* hip_stream,
                               fqnm_server** out);
/* Queue a request.  q0_host is copied during the call; the final state is
 * written to out_host (same size) before the request is reported complete;
 * out_host must stay valid until then.  FQNM_ERR_OOM if the request alone
 * exceeds the budget. */
fqnm_status fqnm_server_submit(fqnm_server* s, const fqnm_problem* prob, const void* q0_host,
                               int64_t n_steps, void* out_host, uint64_t* req_id);
/* Move up to max completions into out; *n_out receives the count.  Never blocks. */
fqnm_status fqnm_server_poll(fqnm_server* s, fqnm_completion* out, int32_t max, int32_t* n_out);
/* Block until every submitted request has completed or timeout_s elapsed
 * (FQNM_ERR_BUSY on timeout). */
fqnm_status fqnm_server_drain(fqnm_server* s, double timeout_s);
fqnm_status fqnm_server_stats_get(fqnm_server* s, fqnm_server_stats* out);
double fqnm_server_now(void); /* the clock of fqnm_completion, in seconds */
fqnm_status fqnm_server_destroy(fqnm_server* s); /* cancels queued work; NULL-safe */

#ifdef __cplusplus
}
#endif
#endif /* FQNM_H */
