/*
 * fqnm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow CPU reference for the Fast Quantised Numerical Method (FQNM,
 * arXiv 2604.06947).  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load this library; the
 * product path (the HIP library and its Python binding) never does.  It shares
 * no code, header or constant table with the HIP implementation: both are
 * written independently from the paper and from the readings recorded in the
 * design notes, and they meet only on seeded inputs.
 *
 * Build: gcc -std=c11 -O2 -ffp-contract=off -fno-fast-math -fPIC -shared
 * (contraction off: every floating-point operation below is one IEEE op, in
 * the order written).  The same source also builds with -fopenmp: the
 * stepping loops run over cells or interfaces that read only the state
 * before the step, so the threads split independent work and both builds give
 * the same integers (tested); the threaded build serves the full-size
 * digests and the all-cores CPU baseline.  States are held in int64 regardless of the problem's
 * storage width; for 32-bit problems every intermediate integer is checked to
 * lie in the int32 range so that a 32-bit implementation computes the same
 * numbers.
 *
 * Paper sections followed (cited by section / equation label):
 *   quantisation          Sec. 2, eq:quantisation          q = round(u/delta)
 *   transfer maps         Sec. 2, eq:flux_table            phi+- = round(f+-(dq) dt/dx / d)
 *   conservative update   Sec. 2, eq:update_rule,
 *                         eq:update_rule_conservative_form,
 *                         eq:numerical_count_flux_definition
 *   reconstruction        Sec. 2.1, eq:reconstruction_operator   u = delta q
 *   classical operator    Sec. 2.1, eq:classical_operator_definition
 *   two-point rules       Sec. 2.2, eq:transfer_operator_equivalence_definition
 *   conservation          Sec. 2.3, eq:exact_conservation
 *   d-D composition       Thm dimension_extension, eq:nd_transfer_rule,
 *                         eq:nd_flux_definition
 *   entropy diagnostics   Supplementary Information, eq:pk_definition,
 *                         eq:discrete_entropy, eq:empirical_M, and the
 *                         row-sum defect of Remark doubly_stochastic_condition
 *
 * "round" is read as IEEE round-half-to-even (C rint in the default
 * rounding mode), the rounding of the NumPy prototype the paper describes.
 */
#include <fenv.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Flux kinds.  The numbering is part of the public interface (it is how a
 * caller names a kind), so it is restated here rather than shared. */
enum {
  OFQ_UPWIND = 0,            /* f = a u, split f+ = max(a,0)u, f- = min(a,0)u   */
  OFQ_BURGERS_EO = 1,        /* Engquist-Osher split of u^2/2                    */
  OFQ_BURGERS_GODUNOV = 2,   /* two-point Godunov flux of u^2/2                  */
  OFQ_LF_LINEAR = 3,         /* Lax-Friedrichs split (f +- alpha u)/2, f = a u   */
  OFQ_LF_BURGERS = 4,        /* Lax-Friedrichs split, f = u^2/2                  */
  OFQ_EULER_ROE = 5,         /* two-point Roe flux, 3 conserved components       */
  OFQ_EULER_ROE_EF = 6,      /* Roe flux with Harten-Hyman entropy fix           */
  OFQ_BURGERS_MURMAN_ROE = 7 /* two-point Murman-Roe flux of u^2/2               */
};
enum { OFQ_BC_PERIODIC = 0, OFQ_BC_OUTFLOW = 1 };
enum { OFQ_OK = 0, OFQ_E_ARG = 1, OFQ_E_RANGE = 2, OFQ_E_NONFINITE = 3 };

typedef struct {
  int32_t kind;
  int32_t bc;
  int32_t width;   /* 32 or 64: integer width whose range every value must fit */
  int32_t pad_;
  double a;        /* advection speed (UPWIND, LF_LINEAR)                       */
  double alpha;    /* Lax-Friedrichs dissipation speed (LF kinds)               */
  double gamma;    /* ratio of specific heats (Euler kinds)                     */
  double delta;    /* quantisation resolution                                   */
  double lambda;   /* dt/dx                                                     */
} ofq_problem;

#define TWO53 9007199254740992.0
#define I32_MIN (-2147483648LL)
#define I32_MAX 2147483647LL
#define I64_SAFE 4611686018427387904LL /* 2^62: headroom for one subtraction */

static int fits(const ofq_problem* p, int64_t v) {
  if (p->width == 32) return v >= I32_MIN && v <= I32_MAX;
  return v > -I64_SAFE && v < I64_SAFE;
}

/* int64 -> double, exact only below 2^53 in magnitude. */
static int to_double_exact(int64_t v, double* out) {
  if (v >= (int64_t)1 << 53 || v <= -((int64_t)1 << 53)) return OFQ_E_RANGE;
  *out = (double)v;
  return OFQ_OK;
}

/* A rounded double that holds an integer value -> int64. */
static int round_to_int(double x, int64_t* out) {
  double r = rint(x);
  if (!isfinite(r)) return OFQ_E_NONFINITE;
  if (r >= 4.6e18 || r <= -4.6e18) return OFQ_E_RANGE;
  *out = (int64_t)r;
  return OFQ_OK;
}

/* ---------------------------------------------------------------------------
 * Scalar transfer maps.  Sec. 2, eq:flux_table defines
 *     phi+-(q) = round( f+-(delta q) * (dt/dx) / delta ).
 * Each kind below writes that quantity in one fixed IEEE operation order (the
 * order is part of the method's definition at finite precision; the design
 * notes list it).  For the linear and quadratic fluxes delta cancels exactly
 * in real arithmetic and the cancelled form is the one evaluated.
 * ------------------------------------------------------------------------- */

/* f+ for UPWIND: max(a,0) u  ->  phi+(q) = rint(c q), c = a*lambda, when a >= 0. */
static int phi_upwind(const ofq_problem* p, int plus, int64_t q, int64_t* out) {
  double c = p->a * p->lambda;
  int pos = p->a >= 0.0;
  if ((plus && !pos) || (!plus && pos)) { *out = 0; return OFQ_OK; }
  double x;
  int st = to_double_exact(q, &x);
  if (st) return st;
  return round_to_int(c * x, out);
}

/* Engquist-Osher for f(u) = u^2/2: f+(u) = max(u,0)^2/2, f-(u) = min(u,0)^2/2.
 * phi(q) = rint(h * s^2) with h = (delta*lambda)*0.5 and s = max(q,0) or min(q,0). */
static int phi_eo(const ofq_problem* p, int plus, int64_t q, int64_t* out) {
  double h = (p->delta * p->lambda) * 0.5;
  int64_t s = plus ? (q > 0 ? q : 0) : (q < 0 ? q : 0);
  if (s > 3037000499LL || s < -3037000499LL) return OFQ_E_RANGE;
  int64_t ss = s * s;
  double x;
  int st = to_double_exact(ss, &x);
  if (st) return st;
  return round_to_int(h * x, out);
}

/* Lax-Friedrichs split (Sec. 2, eq:flux_splitting, the example given there):
 * f+-(u) = (f(u) +- alpha u)/2, evaluated on x = delta*q and divided by delta. */
static int phi_lf(const ofq_problem* p, int plus, int64_t q, int64_t* out) {
  double qd;
  int st = to_double_exact(q, &qd);
  if (st) return st;
  double x = p->delta * qd;
  double fx = (p->kind == OFQ_LF_LINEAR) ? p->a * x : (x * x) * 0.5;
  double ax = p->alpha * x;
  double g = plus ? fx + ax : fx - ax;
  g = g * 0.5;
  g = g * p->lambda;
  g = g / p->delta;
  return round_to_int(g, out);
}

static int phi(const ofq_problem* p, int plus, int64_t q, int64_t* out) {
  switch (p->kind) {
    case OFQ_UPWIND: return phi_upwind(p, plus, q, out);
    case OFQ_BURGERS_EO: return phi_eo(p, plus, q, out);
    case OFQ_LF_LINEAR:
    case OFQ_LF_BURGERS: return phi_lf(p, plus, q, out);
    default: return OFQ_E_ARG;
  }
}

/* Two-point rules for Burgers (Sec. 2.2, eq:transfer_operator_equivalence_definition):
 * Phi(qL,qR) = round(F(delta qL, delta qR) dt/dx / delta) rounded once.  For both
 * the Godunov and the Murman-Roe flux F equals f(delta s) for one state s chosen
 * by integer comparisons, so Phi = rint(h * s^2). */
static int64_t godunov_state(int64_t qL, int64_t qR) {
  if (qL <= qR) {          /* rarefaction: minimum of f over [uL, uR] */
    if (qL > 0) return qL;
    if (qR < 0) return qR;
    return 0;
  }
  /* shock: maximum of f over [uR, uL] is at an end point */
  return (qL * qL >= qR * qR) ? qL : qR;
}

static int two_point_burgers(const ofq_problem* p, int64_t qL, int64_t qR, int64_t* out) {
  if (qL > 3037000499LL || qL < -3037000499LL || qR > 3037000499LL || qR < -3037000499LL)
    return OFQ_E_RANGE;
  int64_t s = (p->kind == OFQ_BURGERS_GODUNOV) ? godunov_state(qL, qR)
                                               : ((qL + qR >= 0) ? qL : qR);
  double h = (p->delta * p->lambda) * 0.5;
  double x;
  int st = to_double_exact(s * s, &x);
  if (st) return st;
  return round_to_int(h * x, out);
}

/* Interface count flux F(qL,qR) (eq:numerical_count_flux_definition). */
static int interface_flux(const ofq_problem* p, int64_t qL, int64_t qR, int64_t* F) {
  if (p->kind == OFQ_BURGERS_GODUNOV || p->kind == OFQ_BURGERS_MURMAN_ROE)
    return two_point_burgers(p, qL, qR, F);
  int64_t fp, fm;
  int st = phi(p, 1, qL, &fp);
  if (st) return st;
  st = phi(p, 0, qR, &fm);
  if (st) return st;
  if (!fits(p, fp) || !fits(p, fm)) return OFQ_E_RANGE;
  *F = fp + fm;
  return fits(p, *F) ? OFQ_OK : OFQ_E_RANGE;
}

/* Exported single-map evaluation, used by tests of the map's closed forms. */
int ofq_phi(const ofq_problem* p, int32_t plus, int64_t q, int64_t* out) {
  return phi(p, plus, q, out);
}

int ofq_interface_flux(const ofq_problem* p, int64_t qL, int64_t qR, int64_t* F) {
  return interface_flux(p, qL, qR, F);
}

/* Threads the stepping loops use: 1 in the plain build, the OpenMP team size
 * in the build with -fopenmp (same source; every parallel loop runs over
 * cells or interfaces that read only the state before the step, so both
 * builds give the same integers). */
int ofq_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static int scalar_kind(int32_t k) {
  return k == OFQ_UPWIND || k == OFQ_BURGERS_EO || k == OFQ_BURGERS_GODUNOV ||
         k == OFQ_LF_LINEAR || k == OFQ_LF_BURGERS || k == OFQ_BURGERS_MURMAN_ROE;
}

static int check_problem(const ofq_problem* p) {
  if (!(p->delta > 0.0) || !(p->lambda > 0.0) || !isfinite(p->delta) || !isfinite(p->lambda))
    return OFQ_E_ARG;
  if (p->bc != OFQ_BC_PERIODIC && p->bc != OFQ_BC_OUTFLOW) return OFQ_E_ARG;
  if (p->width != 32 && p->width != 64) return OFQ_E_ARG;
  if (fegetround() != FE_TONEAREST) return OFQ_E_ARG;
  return OFQ_OK;
}

/* ---------------------------------------------------------------------------
 * Quantisation and reconstruction (eq:quantisation, eq:reconstruction_operator).
 * ------------------------------------------------------------------------- */
int ofq_quantise(const double* u, int64_t n, double delta, int32_t width, int64_t* q) {
  ofq_problem p;
  memset(&p, 0, sizeof p);
  p.width = width;
  for (int64_t i = 0; i < n; ++i) {
    int64_t v;
    int st = round_to_int(u[i] / delta, &v);
    if (st) return st;
    if (!fits(&p, v)) return OFQ_E_RANGE;
    q[i] = v;
  }
  return OFQ_OK;
}

void ofq_reconstruct(const int64_t* q, int64_t n, double delta, double* u) {
  for (int64_t i = 0; i < n; ++i) u[i] = delta * (double)q[i];
}

/* ---------------------------------------------------------------------------
 * One Jacobi step of the conservative integer update (eq:update_rule in the
 * flux-difference form eq:update_rule_conservative_form).  Cells are 0..n-1;
 * F[j] is the count flux through interface j-1/2, j = 0..n.
 *   periodic: F[0] = F[n] = F(q[n-1], q[0])
 *   outflow : F[0] = F(q[0], q[0]),  F[n] = F(q[n-1], q[n-1])   (copied ghost)
 * The ledger accumulates F[0] - F[n], the net count that entered the domain.
 * ------------------------------------------------------------------------- */
static int scalar_step(const ofq_problem* p, int64_t n, int64_t* q, int64_t* F, int64_t* ledger) {
  int err = OFQ_OK;
  /* every interface reads the state before the step only, so the interfaces
   * (and, below, the cells) are independent of one another */
#pragma omp parallel for schedule(static) reduction(max : err)
  for (int64_t j = 1; j < n; ++j) {
    int st = interface_flux(p, q[j - 1], q[j], &F[j]);
    if (st > err) err = st;
  }
  if (err) return err;
  int st;
  if (p->bc == OFQ_BC_PERIODIC) {
    st = interface_flux(p, q[n - 1], q[0], &F[0]);
    if (st) return st;
    F[n] = F[0];
  } else {
    st = interface_flux(p, q[0], q[0], &F[0]);
    if (st) return st;
    st = interface_flux(p, q[n - 1], q[n - 1], &F[n]);
    if (st) return st;
  }
#pragma omp parallel for schedule(static) reduction(max : err)
  for (int64_t i = 0; i < n; ++i) {
    int64_t d = F[i + 1] - F[i];
    if (!fits(p, d)) { err = OFQ_E_RANGE; continue; }
    int64_t v = q[i] - d;
    if (!fits(p, v)) { err = OFQ_E_RANGE; continue; }
    q[i] = v;
  }
  if (err) return err;
  if (ledger) *ledger += F[0] - F[n];
  return OFQ_OK;
}

int ofq_step(const ofq_problem* p, int64_t n, int64_t* q, int64_t nsteps, int64_t* ledger) {
  int st = check_problem(p);
  if (st) return st;
  if (!scalar_kind(p->kind) || n < 1 || nsteps < 0) return OFQ_E_ARG;
  for (int64_t i = 0; i < n; ++i)
    if (!fits(p, q[i])) return OFQ_E_RANGE;
  int64_t* F = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!F) return OFQ_E_ARG;
  st = OFQ_OK;
  for (int64_t s = 0; s < nsteps && st == OFQ_OK; ++s) st = scalar_step(p, n, q, F, ledger);
  free(F);
  return st;
}

/* ---------------------------------------------------------------------------
 * d-dimensional directional composition (Thm dimension_extension,
 * eq:nd_transfer_rule, eq:nd_flux_definition):
 *   q_i <- q_i - sum_m ( Phi_m(q_i, q_{i+e_m}) - Phi_m(q_{i-e_m}, q_i) ),
 * every directional flux taken from the state before the step.  Axis 0 is
 * the contiguous one: cell (i_0, .., i_{d-1}) sits at
 * i_0 + n_0*(i_1 + n_1*(i_2 + ...)).  axes[m] is the one-dimensional rule of
 * direction m: kind, width and delta must agree across axes; a, alpha,
 * lambda and the boundary kind may differ.  Outflow ends copy the cell into
 * its ghost in that direction, as in one dimension; the ledger collects
 * sum over boundary faces of (F_low face - F_high face).  The directional
 * differences are subtracted in axis order, each intermediate checked
 * against the storage range.
 * ------------------------------------------------------------------------- */
int ofq_step_nd(const ofq_problem* axes, int32_t dim, const int64_t* shape, int64_t* q,
                int64_t nsteps, int64_t* ledger) {
  if (dim < 1 || dim > 3 || nsteps < 0) return OFQ_E_ARG;
  int64_t n = 1, stride[3];
  for (int32_t m = 0; m < dim; ++m) {
    int st = check_problem(&axes[m]);
    if (st) return st;
    if (!scalar_kind(axes[m].kind) || shape[m] < 1) return OFQ_E_ARG;
    if (axes[m].kind != axes[0].kind || axes[m].width != axes[0].width ||
        axes[m].delta != axes[0].delta)
      return OFQ_E_ARG;
    stride[m] = n;
    n *= shape[m];
  }
  for (int64_t i = 0; i < n; ++i)
    if (!fits(&axes[0], q[i])) return OFQ_E_RANGE;
  int64_t* old = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  if (!old) return OFQ_E_ARG;
  int st = OFQ_OK;
  for (int64_t s = 0; s < nsteps && st == OFQ_OK; ++s) {
    memcpy(old, q, sizeof(int64_t) * (size_t)n);
    int err = OFQ_OK;
    int64_t led = 0;
    /* every cell reads the state before the step only */
#pragma omp parallel for schedule(static) reduction(max : err) reduction(+ : led)
    for (int64_t i = 0; i < n; ++i) {
      int64_t v = old[i];
      int sti = OFQ_OK;
      for (int32_t m = 0; m < dim; ++m) {
        const ofq_problem* p = &axes[m];
        const int64_t im = (i / stride[m]) % shape[m];
        int64_t lo_nb, hi_nb; /* neighbours across the low and high faces */
        if (im > 0) lo_nb = i - stride[m];
        else lo_nb = p->bc == OFQ_BC_PERIODIC ? i + (shape[m] - 1) * stride[m] : i;
        if (im < shape[m] - 1) hi_nb = i + stride[m];
        else hi_nb = p->bc == OFQ_BC_PERIODIC ? i - (shape[m] - 1) * stride[m] : i;
        int64_t Fhi, Flo;
        sti = interface_flux(p, old[i], old[hi_nb], &Fhi);
        if (sti) break;
        sti = interface_flux(p, old[lo_nb], old[i], &Flo);
        if (sti) break;
        const int64_t d = Fhi - Flo;
        if (!fits(p, d)) { sti = OFQ_E_RANGE; break; }
        v -= d;
        if (!fits(p, v)) { sti = OFQ_E_RANGE; break; }
        if (p->bc == OFQ_BC_OUTFLOW) {
          if (im == 0) led += Flo;
          if (im == shape[m] - 1) led -= Fhi;
        }
      }
      if (sti) { if (sti > err) err = sti; continue; }
      q[i] = v;
    }
    st = err;
    if (!st && ledger) *ledger += led;
  }
  free(old);
  return st;
}

/* ---------------------------------------------------------------------------
 * Invariants (Sec. 2.2 Lemma cfl_monotone, Sec. 2.3 eq:exact_conservation):
 * exact sum (as a 128-bit value split into hi/lo words), min, max and total
 * variation including the periodic wrap term.
 * ------------------------------------------------------------------------- */
void ofq_invariants(const int64_t* q, int64_t n, int32_t periodic, int64_t* sum_hi,
                    uint64_t* sum_lo, int64_t* qmin, int64_t* qmax, int64_t* tv_hi,
                    uint64_t* tv_lo) {
  __int128 s = 0, tv = 0;
  int64_t lo = q[0], hi = q[0];
  for (int64_t i = 0; i < n; ++i) {
    s += q[i];
    if (q[i] < lo) lo = q[i];
    if (q[i] > hi) hi = q[i];
    if (i + 1 < n) {
      __int128 d = (__int128)q[i + 1] - q[i];
      tv += d < 0 ? -d : d;
    }
  }
  if (periodic && n > 1) {
    __int128 d = (__int128)q[0] - q[n - 1];
    tv += d < 0 ? -d : d;
  }
  *sum_hi = (int64_t)(s >> 64);
  *sum_lo = (uint64_t)s;
  *qmin = lo;
  *qmax = hi;
  *tv_hi = (int64_t)(tv >> 64);
  *tv_lo = (uint64_t)tv;
}

/* ---------------------------------------------------------------------------
 * Classical split finite-volume flux and step in FP64
 * (Sec. 2.1, eq:classical_operator_definition): F(uL,uR) = f+(uL) + f-(uR)
 * for split kinds, the two-point flux itself for the Godunov and Murman-Roe
 * kinds.  Used as the comparator of the per-step correspondence
 * (Prop. operator_quantisation_error) and as the floating-point twin.
 * ------------------------------------------------------------------------- */
static double fplus(const ofq_problem* p, double u) {
  switch (p->kind) {
    case OFQ_UPWIND: return p->a >= 0.0 ? p->a * u : 0.0;
    case OFQ_BURGERS_EO: { double s = u > 0.0 ? u : 0.0; return (s * s) * 0.5; }
    case OFQ_LF_LINEAR: return (p->a * u + p->alpha * u) * 0.5;
    case OFQ_LF_BURGERS: return ((u * u) * 0.5 + p->alpha * u) * 0.5;
    default: return NAN;
  }
}
static double fminus(const ofq_problem* p, double u) {
  switch (p->kind) {
    case OFQ_UPWIND: return p->a < 0.0 ? p->a * u : 0.0;
    case OFQ_BURGERS_EO: { double s = u < 0.0 ? u : 0.0; return (s * s) * 0.5; }
    case OFQ_LF_LINEAR: return (p->a * u - p->alpha * u) * 0.5;
    case OFQ_LF_BURGERS: return ((u * u) * 0.5 - p->alpha * u) * 0.5;
    default: return NAN;
  }
}

double ofq_classical_flux(const ofq_problem* p, double uL, double uR) {
  if (p->kind == OFQ_BURGERS_GODUNOV || p->kind == OFQ_BURGERS_MURMAN_ROE) {
    double s;
    if (p->kind == OFQ_BURGERS_MURMAN_ROE) {
      s = (uL + uR >= 0.0) ? uL : uR;
    } else if (uL <= uR) {
      s = uL > 0.0 ? uL : (uR < 0.0 ? uR : 0.0);
    } else {
      s = (uL * uL >= uR * uR) ? uL : uR;
    }
    return (s * s) * 0.5;
  }
  return fplus(p, uL) + fminus(p, uR);
}

int ofq_classical_step(const ofq_problem* p, int64_t n, double* u, int64_t nsteps) {
  if (!scalar_kind(p->kind) || n < 1) return OFQ_E_ARG;
  double* F = (double*)malloc(sizeof(double) * (size_t)(n + 1));
  if (!F) return OFQ_E_ARG;
  for (int64_t s = 0; s < nsteps; ++s) {
    for (int64_t j = 1; j < n; ++j) F[j] = ofq_classical_flux(p, u[j - 1], u[j]);
    if (p->bc == OFQ_BC_PERIODIC) {
      F[0] = ofq_classical_flux(p, u[n - 1], u[0]);
      F[n] = F[0];
    } else {
      F[0] = ofq_classical_flux(p, u[0], u[0]);
      F[n] = ofq_classical_flux(p, u[n - 1], u[n - 1]);
    }
    for (int64_t i = 0; i < n; ++i) u[i] = u[i] - p->lambda * (F[i + 1] - F[i]);
  }
  free(F);
  return OFQ_OK;
}

/* ---------------------------------------------------------------------------
 * Euler system (Sec. 3.3: Sod shock tube under a Roe-type flux).  The paper
 * quantises only density in its prototype and names the componentwise variant;
 * this reference quantises all three conserved components (rho, m, E), each
 * with the same delta, and evaluates the Roe flux in FP64 before rounding each
 * component once:  T_c = rint((F_c * lambda) / delta).
 *
 * Per cell (one IEEE operation per statement):
 *   r = delta*qr; m = delta*qm; E = delta*qE; u = m/r;
 *   p = g1*(E - (0.5*m)*u); H = (E + p)/r; s = sqrt(r)
 *   [entropy fix only] c = sqrt(((g1 + 1)*p)/r)
 *   f0 = m; f1 = m*u + p; f2 = u*(E + p)
 * Per interface the Roe averages, wave strengths and dissipation follow
 * the standard Roe linearisation of the Euler equations (Toro, ch. 11), in
 * the operation order of roe_interface below.
 * ------------------------------------------------------------------------- */
typedef struct {
  double r, m, E, u, p, H, s, c, f0, f1, f2;
} ofq_cell;

static void euler_cell(double delta, double g1, int fix, int64_t qr, int64_t qm, int64_t qE,
                       ofq_cell* o) {
  double r = delta * (double)qr;
  double m = delta * (double)qm;
  double E = delta * (double)qE;
  double u = m / r;
  double t = 0.5 * m;
  t = t * u;
  t = E - t;
  double p = g1 * t;
  double H = E + p;
  H = H / r;
  double s = sqrt(r);
  double c = 0.0;
  if (fix) {
    c = g1 + 1.0;
    c = c * p;
    c = c / r;
    c = sqrt(c);
  }
  double f1 = m * u;
  f1 = f1 + p;
  double f2 = E + p;
  f2 = u * f2;
  o->r = r; o->m = m; o->E = E; o->u = u; o->p = p; o->H = H; o->s = s; o->c = c;
  o->f0 = m; o->f1 = f1; o->f2 = f2;
}

/* Harten-Hyman style entropy fix for the acoustic waves: the eigenvalue
 * modulus is replaced by (l^2 + d^2)/(2d) when |l| < d, with
 * d = max(0, l - lL, lR - l) built from the one-sided characteristic speeds. */
static double entropy_fix(double l, double e, double lLk, double lRk) {
  double d1 = l - lLk;
  double d2 = lRk - l;
  double d = 0.0;
  d = d > d1 ? d : d1;
  d = d > d2 ? d : d2;
  if (e < d) {
    double t = l * l;
    double v = d * d;
    t = t + v;
    v = 2.0 * d;
    e = t / v;
  }
  return e;
}

typedef struct {
  double ub, Hb, cb, c2, a1, a2, a3, l1, l2, l3;
} ofq_roe_waves;

static void roe_interface(double g1, int fix, const ofq_cell* L, const ofq_cell* R, double F[3],
                          ofq_roe_waves* wv) {
  double w = L->s + R->s;
  double ub = L->s * L->u;
  double t = R->s * R->u;
  ub = ub + t;
  ub = ub / w;
  double Hb = L->s * L->H;
  t = R->s * R->H;
  Hb = Hb + t;
  Hb = Hb / w;
  double c2 = ub * ub;
  c2 = 0.5 * c2;
  c2 = Hb - c2;
  c2 = g1 * c2;
  double cb = sqrt(c2);
  double rb = L->s * R->s;
  double dr = R->r - L->r;
  double du = R->u - L->u;
  double dp = R->p - L->p;
  double k = rb * cb;
  k = k * du;
  double d2 = 2.0 * c2;
  double a1 = dp - k;
  a1 = a1 / d2;
  double a3 = dp + k;
  a3 = a3 / d2;
  double a2 = dp / c2;
  a2 = dr - a2;
  double l1 = ub - cb;
  double l2 = ub;
  double l3 = ub + cb;
  double e1 = fabs(l1), e2 = fabs(l2), e3 = fabs(l3);
  if (fix) {
    e1 = entropy_fix(l1, e1, L->u - L->c, R->u - R->c);
    e3 = entropy_fix(l3, e3, L->u + L->c, R->u + R->c);
  }
  double w1 = e1 * a1;
  double w2 = e2 * a2;
  double w3 = e3 * a3;
  double D0 = w1 + w2;
  D0 = D0 + w3;
  double D1 = w1 * l1;
  t = w2 * ub;
  D1 = D1 + t;
  t = w3 * l3;
  D1 = D1 + t;
  double h1 = ub * cb;
  double hm = Hb - h1;
  double hp = Hb + h1;
  double kk = ub * ub;
  kk = 0.5 * kk;
  double D2 = w1 * hm;
  t = w2 * kk;
  D2 = D2 + t;
  t = w3 * hp;
  D2 = D2 + t;
  double fL[3] = {L->f0, L->f1, L->f2};
  double fR[3] = {R->f0, R->f1, R->f2};
  double D[3] = {D0, D1, D2};
  for (int c = 0; c < 3; ++c) {
    double Fc = fL[c] + fR[c];
    Fc = 0.5 * Fc;
    t = 0.5 * D[c];
    F[c] = Fc - t;
  }
  if (wv) {
    wv->ub = ub; wv->Hb = Hb; wv->cb = cb; wv->c2 = c2;
    wv->a1 = a1; wv->a2 = a2; wv->a3 = a3; wv->l1 = l1; wv->l2 = l2; wv->l3 = l3;
  }
}

static int euler_kind(int32_t k) { return k == OFQ_EULER_ROE || k == OFQ_EULER_ROE_EF; }

/* Exported: the FP64 Roe flux of two integer states and its wave decomposition
 * (used to pin the linearisation in tests). */
int ofq_euler_flux(const ofq_problem* p, const int64_t qL[3], const int64_t qR[3], double F[3],
                   double waves[10]) {
  if (!euler_kind(p->kind)) return OFQ_E_ARG;
  double g1 = p->gamma - 1.0;
  int fix = p->kind == OFQ_EULER_ROE_EF;
  ofq_cell L, R;
  euler_cell(p->delta, g1, fix, qL[0], qL[1], qL[2], &L);
  euler_cell(p->delta, g1, fix, qR[0], qR[1], qR[2], &R);
  ofq_roe_waves wv;
  roe_interface(g1, fix, &L, &R, F, &wv);
  if (waves) {
    waves[0] = wv.ub; waves[1] = wv.Hb; waves[2] = wv.cb; waves[3] = wv.c2;
    waves[4] = wv.a1; waves[5] = wv.a2; waves[6] = wv.a3;
    waves[7] = wv.l1; waves[8] = wv.l2; waves[9] = wv.l3;
  }
  return OFQ_OK;
}

static int euler_transfer(const ofq_problem* p, const double F[3], int64_t T[3]) {
  for (int c = 0; c < 3; ++c) {
    double v = F[c] * p->lambda;
    v = v / p->delta;
    int st = round_to_int(v, &T[c]);
    if (st) return st;
    if (!fits(p, T[c])) return OFQ_E_RANGE;
  }
  return OFQ_OK;
}

/* Euler state: three arrays (rho, m, E) of n cells each, structure of arrays. */
int ofq_step_euler(const ofq_problem* p, int64_t n, int64_t* qr, int64_t* qm, int64_t* qE,
                   int64_t nsteps, int64_t ledger[3]) {
  int st = check_problem(p);
  if (st) return st;
  if (!euler_kind(p->kind) || n < 1 || nsteps < 0) return OFQ_E_ARG;
  double g1 = p->gamma - 1.0;
  int fix = p->kind == OFQ_EULER_ROE_EF;
  ofq_cell* cell = (ofq_cell*)malloc(sizeof(ofq_cell) * (size_t)n);
  int64_t* T = (int64_t*)malloc(sizeof(int64_t) * 3 * (size_t)(n + 1));
  if (!cell || !T) { free(cell); free(T); return OFQ_E_ARG; }
  int64_t* q[3] = {qr, qm, qE};
  st = OFQ_OK;
  for (int64_t s = 0; s < nsteps && st == OFQ_OK; ++s) {
    int err = OFQ_OK;
    /* per cell: primitives of the state before the step */
#pragma omp parallel for schedule(static) reduction(max : err)
    for (int64_t i = 0; i < n; ++i) {
      int sti = OFQ_OK;
      for (int c = 0; c < 3 && !sti; ++c) {
        double x;
        sti = to_double_exact(q[c][i], &x);
      }
      if (sti) { if (sti > err) err = sti; continue; }
      euler_cell(p->delta, g1, fix, qr[i], qm[i], qE[i], &cell[i]);
      if (!(cell[i].r > 0.0) || !(cell[i].p > 0.0)) err = OFQ_E_NONFINITE;
    }
    if ((st = err)) goto done;
    /* per interface: the Roe flux and its three rounded transfers */
#pragma omp parallel for schedule(static) reduction(max : err)
    for (int64_t j = 1; j < n; ++j) {
      double Fj[3];
      roe_interface(g1, fix, &cell[j - 1], &cell[j], Fj, NULL);
      int sti = euler_transfer(p, Fj, &T[3 * j]);
      if (sti > err) err = sti;
    }
    if ((st = err)) goto done;
    double F[3];
    if (p->bc == OFQ_BC_PERIODIC) {
      roe_interface(g1, fix, &cell[n - 1], &cell[0], F, NULL);
      if ((st = euler_transfer(p, F, &T[0]))) goto done;
      for (int c = 0; c < 3; ++c) T[3 * n + c] = T[c];
    } else {
      roe_interface(g1, fix, &cell[0], &cell[0], F, NULL);
      if ((st = euler_transfer(p, F, &T[0]))) goto done;
      roe_interface(g1, fix, &cell[n - 1], &cell[n - 1], F, NULL);
      if ((st = euler_transfer(p, F, &T[3 * n]))) goto done;
    }
    /* per cell: the telescoping update of each component */
#pragma omp parallel for schedule(static) reduction(max : err)
    for (int64_t i = 0; i < n; ++i) {
      for (int c = 0; c < 3; ++c) {
        int64_t d = T[3 * (i + 1) + c] - T[3 * i + c];
        if (!fits(p, d)) { err = OFQ_E_RANGE; break; }
        int64_t v = q[c][i] - d;
        if (!fits(p, v)) { err = OFQ_E_RANGE; break; }
        q[c][i] = v;
      }
    }
    if ((st = err)) goto done;
    if (ledger)
      for (int c = 0; c < 3; ++c) ledger[c] += T[c] - T[3 * n + c];
  }
done:
  free(cell);
  free(T);
  return st;
}

/* FP64 Roe finite-volume scheme on reconstructed conserved variables (the
 * floating-point reference trajectory of Sec. 3.3):  U <- U - lambda (F_R - F_L). */
int ofq_classical_step_euler(const ofq_problem* p, int64_t n, double* r, double* m, double* E,
                             int64_t nsteps) {
  if (!euler_kind(p->kind) || n < 1) return OFQ_E_ARG;
  double g1 = p->gamma - 1.0;
  int fix = p->kind == OFQ_EULER_ROE_EF;
  ofq_cell* cell = (ofq_cell*)malloc(sizeof(ofq_cell) * (size_t)n);
  double* F = (double*)malloc(sizeof(double) * 3 * (size_t)(n + 1));
  if (!cell || !F) { free(cell); free(F); return OFQ_E_ARG; }
  double* U[3] = {r, m, E};
  for (int64_t s = 0; s < nsteps; ++s) {
    for (int64_t i = 0; i < n; ++i) {
      /* same per-cell formulas with delta = 1 applied to real-valued states */
      ofq_cell* o = &cell[i];
      double rr = r[i], mm = m[i], EE = E[i];
      double u = mm / rr;
      double t = 0.5 * mm;
      t = t * u;
      t = EE - t;
      double pp = g1 * t;
      double H = EE + pp;
      H = H / rr;
      o->r = rr; o->m = mm; o->E = EE; o->u = u; o->p = pp; o->H = H; o->s = sqrt(rr);
      o->c = fix ? sqrt(((g1 + 1.0) * pp) / rr) : 0.0;
      o->f0 = mm; o->f1 = mm * u + pp; o->f2 = u * (EE + pp);
    }
    for (int64_t j = 1; j < n; ++j) roe_interface(g1, fix, &cell[j - 1], &cell[j], &F[3 * j], NULL);
    if (p->bc == OFQ_BC_PERIODIC) {
      roe_interface(g1, fix, &cell[n - 1], &cell[0], &F[0], NULL);
      for (int c = 0; c < 3; ++c) F[3 * n + c] = F[c];
    } else {
      roe_interface(g1, fix, &cell[0], &cell[0], &F[0], NULL);
      roe_interface(g1, fix, &cell[n - 1], &cell[n - 1], &F[3 * n], NULL);
    }
    for (int64_t i = 0; i < n; ++i)
      for (int c = 0; c < 3; ++c)
        U[c][i] = U[c][i] - p->lambda * (F[3 * (i + 1) + c] - F[3 * i + c]);
  }
  free(cell);
  free(F);
  return OFQ_OK;
}

/* Density-only quantisation of the Roe update (Sec. 3.3, the prototype the
 * paper runs): the density is an integer count, rho = delta*qr, and moves by
 * the rounded transfer T = rint((F_rho*lambda)/delta); momentum and energy
 * stay real-valued and take the classical update U <- U - lambda*(F_R - F_L).
 * All three fluxes come from the same FP64 Roe flux of the coupled state
 * (rho, m, E), with the operation order of the other Euler functions.  The
 * ledger (may be NULL) collects the density counts through outflow ends. */
int ofq_step_euler_density(const ofq_problem* p, int64_t n, int64_t* qr, double* m, double* E,
                           int64_t nsteps, int64_t* ledger) {
  int st = check_problem(p);
  if (st) return st;
  if (!euler_kind(p->kind) || n < 1 || nsteps < 0) return OFQ_E_ARG;
  const double g1 = p->gamma - 1.0;
  const int fix = p->kind == OFQ_EULER_ROE_EF;
  ofq_cell* cell = (ofq_cell*)malloc(sizeof(ofq_cell) * (size_t)n);
  double* F = (double*)malloc(sizeof(double) * 3 * (size_t)(n + 1));
  int64_t* T = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!cell || !F || !T) { free(cell); free(F); free(T); return OFQ_E_ARG; }
  for (int64_t s = 0; s < nsteps && st == OFQ_OK; ++s) {
    for (int64_t i = 0; i < n; ++i) {
      ofq_cell* o = &cell[i];
      const double rr = p->delta * (double)qr[i];
      const double mm = m[i], EE = E[i];
      double u = mm / rr;
      double t = 0.5 * mm;
      t = t * u;
      t = EE - t;
      double pp = g1 * t;
      double H = EE + pp;
      H = H / rr;
      o->r = rr; o->m = mm; o->E = EE; o->u = u; o->p = pp; o->H = H; o->s = sqrt(rr);
      o->c = 0.0;
      if (fix) {
        double c = g1 + 1.0;
        c = c * pp;
        c = c / rr;
        o->c = sqrt(c);
      }
      o->f0 = mm;
      double f1 = mm * u;
      o->f1 = f1 + pp;
      double f2 = EE + pp;
      o->f2 = u * f2;
    }
    for (int64_t j = 1; j < n; ++j) roe_interface(g1, fix, &cell[j - 1], &cell[j], &F[3 * j], NULL);
    if (p->bc == OFQ_BC_PERIODIC) {
      roe_interface(g1, fix, &cell[n - 1], &cell[0], &F[0], NULL);
      for (int c = 0; c < 3; ++c) F[3 * n + c] = F[c];
    } else {
      roe_interface(g1, fix, &cell[0], &cell[0], &F[0], NULL);
      roe_interface(g1, fix, &cell[n - 1], &cell[n - 1], &F[3 * n], NULL);
    }
    for (int64_t j = 0; j <= n; ++j) {
      double v = F[3 * j] * p->lambda;
      v = v / p->delta;
      if ((st = round_to_int(v, &T[j]))) break;
      if (!fits(p, T[j])) { st = OFQ_E_RANGE; break; }
    }
    if (st) break;
    for (int64_t i = 0; i < n; ++i) {
      const int64_t d = T[i + 1] - T[i];
      const int64_t v = qr[i] - d;
      if (!fits(p, d) || !fits(p, v)) { st = OFQ_E_RANGE; break; }
      qr[i] = v;
      m[i] = m[i] - p->lambda * (F[3 * (i + 1) + 1] - F[3 * i + 1]);
      E[i] = E[i] - p->lambda * (F[3 * (i + 1) + 2] - F[3 * i + 2]);
    }
    if (!st && ledger) *ledger += T[0] - T[n];
  }
  free(cell);
  free(F);
  free(T);
  return st;
}

/* ---------------------------------------------------------------------------
 * Level statistics (Supplementary Information): occupancy c_k, Shannon entropy
 * S = -sum p_k log p_k, and the one-step level-transition counts N_{k'k}.
 * Plain O(n log n) sort-based counting.
 * ------------------------------------------------------------------------- */
static int cmp_i64(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return (x > y) - (x < y);
}

/* Returns the number of occupied levels; levels/counts must hold n entries. */
int64_t ofq_level_histogram(const int64_t* q, int64_t n, int64_t* levels, int64_t* counts) {
  int64_t* s = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  if (!s) return -1;
  memcpy(s, q, sizeof(int64_t) * (size_t)n);
  qsort(s, (size_t)n, sizeof(int64_t), cmp_i64);
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (m > 0 && levels[m - 1] == s[i]) {
      counts[m - 1]++;
    } else {
      levels[m] = s[i];
      counts[m] = 1;
      m++;
    }
  }
  free(s);
  return m;
}

double ofq_entropy(const int64_t* q, int64_t n) {
  int64_t* lv = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int64_t* ct = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  if (!lv || !ct) { free(lv); free(ct); return NAN; }
  int64_t m = ofq_level_histogram(q, n, lv, ct);
  double S = 0.0;
  for (int64_t k = 0; k < m; ++k) {
    double pk = (double)ct[k] / (double)n;
    S -= pk * log(pk);
  }
  free(lv);
  free(ct);
  return S;
}

static int cmp_pair(const void* a, const void* b) {
  const int64_t* x = (const int64_t*)a;
  const int64_t* y = (const int64_t*)b;
  if (x[0] != y[0]) return (x[0] > y[0]) - (x[0] < y[0]);
  return (x[1] > y[1]) - (x[1] < y[1]);
}

/* Transition counts N_{k'k} = #{i : q0_i = k and q1_i = k'} as sorted unique
 * (k, k', count) triples.  Returns the number of triples written. */
int64_t ofq_level_transitions(const int64_t* q0, const int64_t* q1, int64_t n, int64_t* from,
                              int64_t* to, int64_t* count) {
  int64_t* pairs = (int64_t*)malloc(sizeof(int64_t) * 2 * (size_t)n);
  if (!pairs) return -1;
  for (int64_t i = 0; i < n; ++i) {
    pairs[2 * i] = q0[i];
    pairs[2 * i + 1] = q1[i];
  }
  qsort(pairs, (size_t)n, 2 * sizeof(int64_t), cmp_pair);
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i) {
    int64_t k = pairs[2 * i], k2 = pairs[2 * i + 1];
    if (m > 0 && from[m - 1] == k && to[m - 1] == k2) {
      count[m - 1]++;
    } else {
      from[m] = k;
      to[m] = k2;
      count[m] = 1;
      m++;
    }
  }
  free(pairs);
  return m;
}

/* Row-sum defect of the empirical level-transition matrix (Supplementary
 * Information, eq:empirical_M and Remark doubly_stochastic_condition):
 *   M_{k'k} = N_{k'k} / c_k   (c_k = #{i : q0_i = k}),
 *   rho = max over k' of | sum_k M_{k'k} - 1 |,
 * with k' running over the levels occupied after the step (the rows of M that
 * hold any entry).  Each row is summed in increasing k.  Returns -1.0 on
 * allocation failure and 0.0 for n == 0. */
static int cmp_pair_rev(const void* a, const void* b) {
  const int64_t* x = (const int64_t*)a;
  const int64_t* y = (const int64_t*)b;
  if (x[1] != y[1]) return (x[1] > y[1]) - (x[1] < y[1]);
  return (x[0] > y[0]) - (x[0] < y[0]);
}

double ofq_row_defect(const int64_t* q0, const int64_t* q1, int64_t n) {
  if (n == 0) return 0.0;
  int64_t* lv = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int64_t* ct = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int64_t* f = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int64_t* t = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int64_t* c = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int64_t* trip = (int64_t*)malloc(sizeof(int64_t) * 3 * (size_t)n);
  double rho = -1.0;
  if (!lv || !ct || !f || !t || !c || !trip) goto done;
  {
    const int64_t nl = ofq_level_histogram(q0, n, lv, ct);
    const int64_t m = ofq_level_transitions(q0, q1, n, f, t, c);
    /* triples (k, k', N) ordered by (k', k) */
    for (int64_t r = 0; r < m; ++r) {
      trip[3 * r] = f[r];
      trip[3 * r + 1] = t[r];
      trip[3 * r + 2] = c[r];
    }
    qsort(trip, (size_t)m, 3 * sizeof(int64_t), cmp_pair_rev);
    rho = 0.0;
    int64_t r = 0;
    while (r < m) {
      const int64_t kp = trip[3 * r + 1];
      double row = 0.0;
      for (; r < m && trip[3 * r + 1] == kp; ++r) {
        /* c_k by lookup in the (sorted) histogram of q0 */
        const int64_t* hit =
            (const int64_t*)bsearch(&trip[3 * r], lv, (size_t)nl, sizeof(int64_t), cmp_i64);
        const int64_t ck = ct[hit - lv];
        row += (double)trip[3 * r + 2] / (double)ck;
      }
      const double d = fabs(row - 1.0);
      if (d > rho) rho = d;
    }
  }
done:
  free(lv); free(ct); free(f); free(t); free(c); free(trip);
  return rho;
}
