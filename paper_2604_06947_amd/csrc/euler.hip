// euler.hip -- componentwise quantised Roe transfer for the 1D Euler equations.
//
// Sec. 3.3 runs the Sod shock tube with a Roe-type flux and names the variant
// in which all conserved components (rho, m, E) are quantised; that variant is
// implemented here.  Per step and interface the Roe flux F(U_L, U_R) is
// evaluated in FP64 on the reconstructed states U = delta*q, in one fixed
// sequence of IEEE operations (compiled without contraction), and each
// component is rounded once: T_c = rint((F_c*lambda)/delta).  Each cell then
// applies the integer telescoping update of eq:update_rule_conservative_form
// to each component, so sum(q_c) changes only by the boundary counts.
//
// The density-only prototype the paper actually runs is the same kernel with
// EulerParams::dens set: component 0 holds the integer density counts, and
// components 1 and 2 hold FP64 momentum and energy (their bit patterns in the
// 8-byte slots).  Only the density flux is rounded, T_rho = rint((F_rho*lambda)/
// delta); m and E take the classical update U - lambda*(F_R - F_L).
//
// Layout: three 8-byte arrays of n cells (rho, m, E) back to back, ping-pong.
// A 256-thread block loads positions [b0-8, b0+248) and advances them up to 8
// steps per launch: each step computes the per-cell primitives once into LDS,
// evaluates the 255 interfaces between them and updates the 254 positions
// that have both neighbours.  After step s the positions [s, 255-s] are exact,
// so the 240 cells [b0, b0+240) are stored after up to 8 steps.  Positions
// outside [0, n) are ghost copies (periodic wrap, or the outflow copy of the
// end cell, renewed after every step), so the outflow boundary flux is
// F(U_0, U_0) = f(U_0).  Arithmetic per cell-update: one set of
// primitives (1 division, 1-2 square roots) and one Roe interface
// (4 divisions, 1 square root, ~60 other FP64 operations); HBM traffic
// 48 bytes (3 int64 read + 3 written).
#include <hip/hip_runtime.h>

#include "fqnm_internal.h"

namespace fqnm {

namespace {

constexpr int EB = 256;               // threads per block
constexpr int EKS = 8;                // steps per launch at most
constexpr int ECELLS = EB - 2 * EKS;  // cells stored per block

struct Prim {
  double r, u, p, H, s, c, f0, f1, f2;
};

// Primitives of a cell from its conserved values (r, m, en) in FP64.
__device__ __forceinline__ Prim cell_primitives_f(const EulerParams& E, double r, double m,
                                                  double en) {
  Prim o;
  const double u = m / r;
  double t = 0.5 * m;
  t = t * u;
  t = en - t;
  const double p = E.g1 * t;
  double H = en + p;
  H = H / r;
  o.r = r;
  o.u = u;
  o.p = p;
  o.H = H;
  o.s = sqrt(r);
  if (E.fix) {
    double c = E.g1 + 1.0;
    c = c * p;
    c = c / r;
    o.c = sqrt(c);
  } else {
    o.c = 0.0;
  }
  o.f0 = m;
  double f1 = m * u;
  o.f1 = f1 + p;
  double f2 = en + p;
  o.f2 = u * f2;
  return o;
}

// Cell of the 8-byte state slots: counts times delta, or (density-only) the
// density counts with FP64 m and E.
__device__ __forceinline__ Prim cell_primitives(const EulerParams& E, int64_t qr, int64_t qm,
                                                int64_t qE) {
  const double r = E.delta * as_f64<int64_t>(qr);
  if (E.dens)
    return cell_primitives_f(E, r, __builtin_bit_cast(double, qm), __builtin_bit_cast(double, qE));
  const double m = E.delta * as_f64<int64_t>(qm);
  const double en = E.delta * as_f64<int64_t>(qE);
  return cell_primitives_f(E, r, m, en);
}

__device__ __forceinline__ double acoustic_fix(double l, double e, double lLk, double lRk) {
  const double d1 = l - lLk;
  const double d2 = lRk - l;
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

// Roe flux of two cells, then the three quantised transfers (density-only:
// the density transfer and the FP64 fluxes of m and E as bit patterns).
// Returns false when a value to be rounded is not a number or too large for
// the conversion (|v| >= 2^51), i.e. when the transfer is meaningless.
__device__ __forceinline__ bool roe_transfer(const EulerParams& E, const Prim& L, const Prim& R,
                                             int64_t T[3]) {
  const double w = L.s + R.s;
  double ub = L.s * L.u;
  double t = R.s * R.u;
  ub = ub + t;
  ub = ub / w;
  double Hb = L.s * L.H;
  t = R.s * R.H;
  Hb = Hb + t;
  Hb = Hb / w;
  double c2 = ub * ub;
  c2 = 0.5 * c2;
  c2 = Hb - c2;
  c2 = E.g1 * c2;
  const double cb = sqrt(c2);
  const double rb = L.s * R.s;
  const double dr = R.r - L.r;
  const double du = R.u - L.u;
  const double dp = R.p - L.p;
  double k = rb * cb;
  k = k * du;
  const double d2 = 2.0 * c2;
  double a1 = dp - k;
  a1 = a1 / d2;
  double a3 = dp + k;
  a3 = a3 / d2;
  double a2 = dp / c2;
  a2 = dr - a2;
  const double l1 = ub - cb;
  const double l3 = ub + cb;
  double e1 = fabs(l1);
  const double e2 = fabs(ub);
  double e3 = fabs(l3);
  if (E.fix) {
    e1 = acoustic_fix(l1, e1, L.u - L.c, R.u - R.c);
    e3 = acoustic_fix(l3, e3, L.u + L.c, R.u + R.c);
  }
  const double w1 = e1 * a1;
  const double w2 = e2 * a2;
  const double w3 = e3 * a3;
  double D0 = w1 + w2;
  D0 = D0 + w3;
  double D1 = w1 * l1;
  t = w2 * ub;
  D1 = D1 + t;
  t = w3 * l3;
  D1 = D1 + t;
  const double h1 = ub * cb;
  const double hm = Hb - h1;
  const double hp = Hb + h1;
  double kk = ub * ub;
  kk = 0.5 * kk;
  double D2 = w1 * hm;
  t = w2 * kk;
  D2 = D2 + t;
  t = w3 * hp;
  D2 = D2 + t;
  const double fl[3] = {L.f0, L.f1, L.f2};
  const double fr[3] = {R.f0, R.f1, R.f2};
  const double D[3] = {D0, D1, D2};
  bool ok = true;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double F = fl[c] + fr[c];
    F = 0.5 * F;
    const double h = 0.5 * D[c];
    F = F - h;
    if (E.dens && c > 0) {
      T[c] = __builtin_bit_cast(int64_t, F);
    } else {
      double v = F * E.lambda;
      v = v / E.delta;
      ok = ok && fabs(v) < 2251799813685248.0;  // false for NaN
      T[c] = round_to<int64_t>(v);  // exact for |v| < 2^51
    }
  }
  return ok;
}

__device__ __forceinline__ int64_t ghost(int64_t g, int64_t n, int bc) {
  if (g >= 0 && g < n) return g;
  return bc == FQNM_BC_PERIODIC ? wrap_index(g, n) : clamp_index(g, n);
}

// Up to EKS steps (nst) of one tile of cells [b0, b0 + ECELLS) of an n-cell
// problem; the block holds positions [b0 - EKS, b0 - EKS + EB).
__device__ __forceinline__ void euler_tile_step(const int64_t* __restrict__ src,
                                                int64_t* __restrict__ dst, int64_t n, int bc,
                                                const EulerParams& E, int64_t b0, int nst,
                                                long long* __restrict__ ledger, Prim* s_prim,
                                                int64_t (*s_T)[EB], int64_t* s_edge) {
  const int t = threadIdx.x;
  const int64_t g = b0 - EKS + t;  // cell of this thread
  const int64_t gi = ghost(g, n, bc);
  int64_t qr = src[gi], qm = src[n + gi], qE = src[2 * n + gi];
  const bool outflow = bc == FQNM_BC_OUTFLOW;
  const bool stored = t >= EKS && t < EB - EKS && g < n;
  // the block holds outflow ghosts, to be renewed after every step (uniform)
  const bool ghosts = outflow && (b0 - EKS < 0 || b0 - EKS + EB > n);
  const int nled = E.dens ? 1 : 3;  // density-only: only the counts have a ledger
  for (int s = 0; s < nst; ++s) {
    const Prim pc = cell_primitives(E, qr, qm, qE);
    s_prim[t] = pc;
    // positions [s, EB-1-s] hold the exact state after s steps; a cell of the
    // domain there whose density or pressure is not positive (or NaN) makes
    // the flux meaningless: raise the context's sticky flag
    if (E.err && t >= s && t <= EB - 1 - s && g >= 0 && g < n && !(pc.r > 0.0 && pc.p > 0.0))
      __hip_atomic_store(E.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    // interface between positions t and t+1 (t < EB-1)
    int64_t T[3] = {0, 0, 0};
    if (t < EB - 1) {
      const bool ok = roe_transfer(E, s_prim[t], s_prim[t + 1], T);
      // an interface between two exact positions with a cell of the domain
      // on one side (the outflow boundary faces included)
      if (!ok && E.err && t >= s && t + 1 <= EB - 1 - s && g + 1 >= 0 && g < n)
        __hip_atomic_store(E.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    s_T[0][t] = T[0];
    s_T[1][t] = T[1];
    s_T[2][t] = T[2];
    __syncthreads();
    if (t >= 1 && t <= EB - 2) {  // positions with both neighbours
      const int64_t Tl[3] = {s_T[0][t - 1], s_T[1][t - 1], s_T[2][t - 1]};
      qr = qr - (T[0] - Tl[0]);
      if (E.dens) {
        // classical update of the real-valued components
        const double dm = __builtin_bit_cast(double, T[1]) - __builtin_bit_cast(double, Tl[1]);
        const double dE = __builtin_bit_cast(double, T[2]) - __builtin_bit_cast(double, Tl[2]);
        const double tm = E.lambda * dm;
        const double tE = E.lambda * dE;
        qm = __builtin_bit_cast(int64_t, __builtin_bit_cast(double, qm) - tm);
        qE = __builtin_bit_cast(int64_t, __builtin_bit_cast(double, qE) - tE);
      } else {
        qm = qm - (T[1] - Tl[1]);
        qE = qE - (T[2] - Tl[2]);
      }
      if (outflow && stored) {
        if (g == 0) {
          for (int c = 0; c < nled; ++c)
            atomicAdd(reinterpret_cast<unsigned long long*>(ledger + c),
                      static_cast<unsigned long long>(Tl[c]));
        }
        if (g == n - 1) {
          for (int c = 0; c < nled; ++c)
            atomicAdd(reinterpret_cast<unsigned long long*>(ledger + c),
                      static_cast<unsigned long long>(-static_cast<long long>(T[c])));
        }
      }
    }
    if (ghosts && s + 1 < nst) {  // uniform: the ghosts take the end cells' new states
      if (g == 0) {
        s_edge[0] = qr;
        s_edge[1] = qm;
        s_edge[2] = qE;
      }
      if (g == n - 1) {
        s_edge[3] = qr;
        s_edge[4] = qm;
        s_edge[5] = qE;
      }
      __syncthreads();
      if (g < 0) {
        qr = s_edge[0];
        qm = s_edge[1];
        qE = s_edge[2];
      }
      if (g >= n) {
        qr = s_edge[3];
        qm = s_edge[4];
        qE = s_edge[5];
      }
    }
  }
  if (stored) {
    dst[g] = qr;
    dst[n + g] = qm;
    dst[2 * n + g] = qE;
  }
}

__global__ __launch_bounds__(EB) void k_euler_step(const int64_t* __restrict__ src,
                                                   int64_t* __restrict__ dst, int64_t n, int bc,
                                                   EulerParams E, int nst,
                                                   long long* __restrict__ ledger) {
  __shared__ Prim s_prim[EB];
  __shared__ int64_t s_T[3][EB];
  __shared__ int64_t s_edge[6];
  const int64_t b0 = xcd_tile(blockIdx.x, gridDim.x) * ECELLS;
  euler_tile_step(src, dst, n, bc, E, b0, nst, ledger, s_prim, s_T, s_edge);
}

// Many independent problems in one launch: block b advances tile tiles[b] of
// request tiles[b].req by up to EKS steps, if that request still has steps to
// take from this position `s` (a multiple of EKS) of the current tick.  Each
// request has its own ping-pong buffers; every launch writes the other one, so
// its source buffer is given by (parity + s / EKS) & 1.
__global__ __launch_bounds__(EB) void k_euler_multi(const EulerTile* __restrict__ tiles,
                                                    const EulerReq* __restrict__ reqs, int s) {
  __shared__ Prim s_prim[EB];
  __shared__ int64_t s_T[3][EB];
  __shared__ int64_t s_edge[6];
  const EulerTile tl = tiles[blockIdx.x];
  const EulerReq& R = reqs[tl.req];
  if (s >= R.steps) return;  // uniform over the block
  const int nst = R.steps - s < EKS ? R.steps - s : EKS;
  const int par = (R.parity + s / EKS) & 1;
  const int64_t* src = par ? R.buf1 : R.buf0;
  int64_t* dst = par ? R.buf0 : R.buf1;
  euler_tile_step(src, dst, R.n, R.bc, R.E, tl.start, nst, R.ledger, s_prim, s_T, s_edge);
}

}  // namespace

hipError_t launch_euler_step(const int64_t* src, int64_t* dst, int64_t n, int bc,
                             const EulerParams& E, int nsteps, long long* d_ledger, hipStream_t s) {
  if (nsteps < 1 || nsteps > EKS) return hipErrorInvalidValue;
  const int64_t blocks = (n + ECELLS - 1) / ECELLS;
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  k_euler_step<<<dim3((unsigned)blocks), dim3(EB), 0, s>>>(src, dst, n, bc, E, nsteps, d_ledger);
  return hipGetLastError();
}

int64_t euler_tiles(int64_t n) { return (n + ECELLS - 1) / ECELLS; }
int64_t euler_tile_cells() { return ECELLS; }
int euler_steps_per_launch() { return EKS; }

hipError_t launch_euler_multi(const EulerTile* d_tiles, int64_t ntiles, const EulerReq* d_reqs,
                              int s, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  k_euler_multi<<<dim3((unsigned)ntiles), dim3(EB), 0, st>>>(d_tiles, d_reqs, s);
  return hipGetLastError();
}

}  // namespace fqnm

namespace {
__global__ void k_fp64_selfcheck(const double* __restrict__ a, const double* __restrict__ b,
                                 double* __restrict__ s, double* __restrict__ d, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    s[i] = sqrt(a[i]);
    d[i] = a[i] / b[i];
  }
}
}  // namespace

extern "C" fqnm_status fqnm_fp64_selfcheck(const double* d_a, const double* d_b,
                                           double* d_out_sqrt, double* d_out_div, int64_t n,
                                           void* hip_stream) {
  if (!d_a || !d_b || !d_out_sqrt || !d_out_div || n < 0) {
    fqnm::set_error("NULL argument or negative n");
    return FQNM_ERR_ARG;
  }
  if (n == 0) return FQNM_OK;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  k_fp64_selfcheck<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(d_a, d_b, d_out_sqrt, d_out_div, n);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    fqnm::set_error(std::string("fp64 self-check: ") + hipGetErrorString(e));
    return FQNM_ERR_DEVICE;
  }
  return FQNM_OK;
}
