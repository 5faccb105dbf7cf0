// classical.hip -- the FP64 split finite-volume twin of the integer update.
//
// Sec. 2.1 (eq:classical_operator_definition) compares FQNM with the classical
// split finite-volume operator O_h[u]_i = -(F(u_i,u_{i+1}) - F(u_{i-1},u_i))/dx,
// F(uL,uR) = f+(uL) + f-(uR).  This file runs that scheme with the same tiling
// machinery as the integer kernels, on an FP64 state, so the two realisations
// can be timed side by side on the same workload (the paper's arithmetic
// comparison, Sec. 2.4 Table tab:alu_structure and Sec. 3), and so the loss of
// bitwise conservation of an FP update (Remark fp_no_exact_invariance) can be
// observed.  Every floating-point operation is one IEEE op in a fixed order:
//   F = f+(uL) + f-(uR);  u_i <- u_i - lambda*(F_{i+1/2} - F_{i-1/2})
// with f+- per kind:
//   UPWIND   f+ = (a >= 0 ? a*u : 0),  f- = (a < 0 ? a*u : 0)
//   EO       f+ = (s*s)*0.5, s = max(u,0);  f- = (s*s)*0.5, s = min(u,0)
//   LF       f+- = (f(u) +- alpha*u)*0.5,  f = a*u or (u*u)*0.5
//   Godunov / Murman-Roe: F = (s*s)*0.5 for the state s the flux selects.
#include <hip/hip_runtime.h>

#include "fqnm_internal.h"

namespace fqnm {
namespace {

template <int POL>
__device__ __forceinline__ double cl_fplus(const XParams& P, double u) {
  if constexpr (POL == P_UPWIND_POS || POL == P_UPWIND_NEG) {
    return P.a >= 0.0 ? P.a * u : 0.0;
  } else if constexpr (POL == P_EO) {
    const double s = u > 0.0 ? u : 0.0;
    return (s * s) * 0.5;
  } else if constexpr (POL == P_LF_LINEAR) {
    const double f = P.a * u;
    const double g = P.alpha * u;
    return (f + g) * 0.5;
  } else {
    const double f = (u * u) * 0.5;
    const double g = P.alpha * u;
    return (f + g) * 0.5;
  }
}

template <int POL>
__device__ __forceinline__ double cl_fminus(const XParams& P, double u) {
  if constexpr (POL == P_UPWIND_POS || POL == P_UPWIND_NEG) {
    return P.a < 0.0 ? P.a * u : 0.0;
  } else if constexpr (POL == P_EO) {
    const double s = u < 0.0 ? u : 0.0;
    return (s * s) * 0.5;
  } else if constexpr (POL == P_LF_LINEAR) {
    const double f = P.a * u;
    const double g = P.alpha * u;
    return (f - g) * 0.5;
  } else {
    const double f = (u * u) * 0.5;
    const double g = P.alpha * u;
    return (f - g) * 0.5;
  }
}

template <int POL>
__device__ __forceinline__ double cl_flux(const XParams& P, double uL, double uR) {
  if constexpr (POL == P_GODUNOV || POL == P_MURMAN_ROE) {
    double s;
    if constexpr (POL == P_MURMAN_ROE) {
      s = (uL + uR >= 0.0) ? uL : uR;
    } else if (uL <= uR) {
      s = uL > 0.0 ? uL : (uR < 0.0 ? uR : 0.0);
    } else {
      s = (uL * uL >= uR * uR) ? uL : uR;
    }
    return (s * s) * 0.5;
  } else {
    return cl_fplus<POL>(P, uL) + cl_fminus<POL>(P, uR);
  }
}

__device__ __forceinline__ int64_t cl_ghost(int64_t g, int64_t n, int bc) {
  if (g >= 0 && g < n) return g;
  return bc == FQNM_BC_PERIODIC ? wrap_index(g, n) : clamp_index(g, n);
}

// One step per pass; V cells per lane.
template <int POL, int V>
__global__ __launch_bounds__(256) void k_cl_stream(const double* __restrict__ src,
                                                   double* __restrict__ dst, int64_t n, int bc,
                                                   XParams P) {
  const int lane = threadIdx.x & 63;
  const int64_t base = (xcd_tile(blockIdx.x, gridDim.x) * 256 + threadIdx.x) * V;
  double u[V];
#pragma unroll
  for (int j = 0; j < V; ++j) u[j] = src[base + j < n ? base + j : cl_ghost(base + j, n, bc)];
  double un = lane_from_next<double>(u[0]);
  if (lane == 63) un = src[cl_ghost(base + V, n, bc)];
  double F[V];
#pragma unroll
  for (int j = 0; j < V; ++j) F[j] = cl_flux<POL>(P, u[j], j + 1 < V ? u[j + 1] : un);
  double Fl = lane_from_prev<double>(F[V - 1]);
  if (lane == 0) Fl = cl_flux<POL>(P, src[cl_ghost(base - 1, n, bc)], u[0]);
#pragma unroll
  for (int j = 0; j < V; ++j) {
    const double d = F[j] - (j == 0 ? Fl : F[j - 1]);
    const double t = P.lambda * d;
    if (base + j < n) dst[base + j] = u[j] - t;
  }
}

// Temporal blocking in registers, as the integer k_tblock: a wavefront loads
// 64*V cells, advances them `ksteps` steps, stores the interior.  Outflow
// ends: positions outside [0, n) are frozen and the boundary interfaces use
// the in-domain cell on both sides.
template <int POL, int V>
__global__ __launch_bounds__(256) void k_cl_tblock(const double* __restrict__ src,
                                                   double* __restrict__ dst, int64_t n, int bc,
                                                   int ksteps, int khalo, int64_t ntiles,
                                                   XParams P) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x) * 4 + wave;
  if (tile >= ntiles) return;
  const int64_t T = 64 * V - 2 * khalo;
  const int64_t tstart = tile * T;
  const int64_t wstart = tstart - khalo;
  const int64_t g0 = wstart + static_cast<int64_t>(lane) * V;
  const bool edge = bc == FQNM_BC_OUTFLOW && !(wstart >= 0 && wstart + 64 * V <= n);
  double u[V];
#pragma unroll
  for (int j = 0; j < V; ++j) u[j] = src[cl_ghost(g0 + j, n, bc)];
  for (int s = 0; s < ksteps; ++s) {
    const double un = lane_from_next<double>(u[0]);
    double F[V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
      double uL = u[j];
      double uR = j + 1 < V ? u[j + 1] : un;
      if (edge) {
        const int64_t g = g0 + j;
        if (g == -1) uL = uR;
        if (g == n - 1) uR = uL;
      }
      F[j] = cl_flux<POL>(P, uL, uR);
    }
    const double Fl = lane_from_prev<double>(F[V - 1]);
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const double d = F[j] - (j == 0 ? Fl : F[j - 1]);
      const double t = P.lambda * d;
      const double v = u[j] - t;
      if (edge) {
        const int64_t g = g0 + j;
        u[j] = (g >= 0 && g < n) ? v : u[j];
      } else {
        u[j] = v;
      }
    }
  }
  if (lane >= khalo / V && lane < 64 - khalo / V) {
#pragma unroll
    for (int j = 0; j < V; ++j)
      if (g0 + j < n) dst[g0 + j] = u[j];
  }
}

template <int POL, int V>
hipError_t cl_launch(int kernel, const double* a, double* b, int64_t n, int bc, int ksteps,
                     int khalo, const XParams& P, hipStream_t s) {
  if (kernel == K_STREAM) {
    const int64_t blocks = ((n + V - 1) / V + 255) / 256;
    k_cl_stream<POL, V><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(a, b, n, bc, P);
  } else {
    const int64_t T = 64 * V - 2 * khalo;
    const int64_t ntiles = (n + T - 1) / T;
    k_cl_tblock<POL, V><<<dim3((unsigned)((ntiles + 3) / 4)), dim3(256), 0, s>>>(
        a, b, n, bc, ksteps, khalo, ntiles, P);
  }
  return hipGetLastError();
}

template <int POL>
hipError_t cl_by_vec(int kernel, int vec, const double* a, double* b, int64_t n, int bc,
                     int ksteps, int khalo, const XParams& P, hipStream_t s) {
  switch (vec) {
    case 2: return cl_launch<POL, 2>(kernel, a, b, n, bc, ksteps, khalo, P, s);
    case 4: return cl_launch<POL, 4>(kernel, a, b, n, bc, ksteps, khalo, P, s);
    case 8: return cl_launch<POL, 8>(kernel, a, b, n, bc, ksteps, khalo, P, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool classical_variant_available(int pol, int kernel, int vec) {
  if (pol < 0 || pol >= P_LUT) return false;
  if (kernel != K_STREAM && kernel != K_TBLOCK) return false;
  return vec == 2 || vec == 4 || vec == 8;
}

hipError_t launch_classical(int pol, int kernel, int vec, const double* src, double* dst,
                            int64_t n, int bc, int ksteps, int khalo, const XParams& P,
                            hipStream_t s) {
  if (!classical_variant_available(pol, kernel, vec)) return hipErrorInvalidValue;
  if (kernel == K_TBLOCK && (khalo < ksteps || khalo % vec != 0 || 64 * vec - 2 * khalo <= 0))
    return hipErrorInvalidValue;
  switch (pol) {
    case P_UPWIND_POS: return cl_by_vec<P_UPWIND_POS>(kernel, vec, src, dst, n, bc, ksteps, khalo, P, s);
    case P_UPWIND_NEG: return cl_by_vec<P_UPWIND_NEG>(kernel, vec, src, dst, n, bc, ksteps, khalo, P, s);
    case P_EO: return cl_by_vec<P_EO>(kernel, vec, src, dst, n, bc, ksteps, khalo, P, s);
    case P_GODUNOV: return cl_by_vec<P_GODUNOV>(kernel, vec, src, dst, n, bc, ksteps, khalo, P, s);
    case P_MURMAN_ROE: return cl_by_vec<P_MURMAN_ROE>(kernel, vec, src, dst, n, bc, ksteps, khalo, P, s);
    case P_LF_LINEAR: return cl_by_vec<P_LF_LINEAR>(kernel, vec, src, dst, n, bc, ksteps, khalo, P, s);
    case P_LF_BURGERS: return cl_by_vec<P_LF_BURGERS>(kernel, vec, src, dst, n, bc, ksteps, khalo, P, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fqnm
