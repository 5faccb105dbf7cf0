// fqnm_device.h -- device-side transfer maps and cross-lane helpers for gfx950.
//
// Transfer maps follow Sec. 2, eq:flux_table (split kinds: phi+ and phi- are
// rounded separately and F = phi+(qL) + phi-(qR), eq:numerical_count_flux_definition)
// and Sec. 2.2, eq:transfer_operator_equivalence_definition (two-point kinds:
// the interface flux is rounded once).  Every floating-point operation is one
// IEEE double operation in the order written; the library is compiled with
// -ffp-contract=off so no multiply-add is fused.  rint() lowers to
// v_rndne_f64 (round half to even).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fqnm {

// Flux policies (template tags).
enum : int {
  P_UPWIND_POS = 0,  // a >= 0: F = rint(c*qL)
  P_UPWIND_NEG = 1,  // a <  0: F = rint(c*qR)
  P_EO = 2,          // Engquist-Osher, f = u^2/2
  P_GODUNOV = 3,     // two-point Godunov, f = u^2/2
  P_MURMAN_ROE = 4,  // two-point Murman-Roe, f = u^2/2
  P_LF_LINEAR = 5,   // Lax-Friedrichs split, f = a u
  P_LF_BURGERS = 6,  // Lax-Friedrichs split, f = u^2/2
  P_LUT = 7,         // tabulated split maps {phi+, phi-} over [lo, hi]
  P_COUNT = 8
};

// Constants of one scalar problem, passed by value to every kernel.
struct XParams {
  double c;       // UPWIND: a*lambda
  double h;       // Burgers kinds: (delta*lambda)*0.5
  double a;       // LF_LINEAR: advection speed
  double alpha;   // LF kinds
  double delta;
  double lambda;
  const void* lut;  // P_LUT: int2 (I32) or longlong2 (I64) entries {phi+(q), phi-(q)}
  int64_t lut_lo;   // first tabulated state
  int64_t lut_last; // number of entries - 1
  int32_t lut_pol;  // P_LUT: the direct split policy whose maps the table holds
  int32_t lut_mono; // P_LUT: 1 when the table certifies the maximum principle (k_lut_build)
};

// For 64-bit states the conversions use the bias B = 1.5*2^52: for |v| < 2^51
// the double B + v has the integer v in its low mantissa bits, so
// int64 -> double is one integer add and one FP subtraction, both exact, and
// rounding x to an integer is the FP addition x + B, which rounds half to even
// like rint.  States and map values of 64-bit contexts are validated below
// 2^51 in magnitude (map values are at most |q| under the CFL condition); a
// discarded halo lane holding anything else gets a meaningless, never stored,
// value.  32-bit states convert with the hardware instruction and round with
// the same bias addition.
constexpr int64_t F64_BIAS_BITS = 0x4338000000000000LL;  // 1.5*2^52
constexpr double F64_BIAS = 6755399441055744.0;          // 1.5*2^52

template <typename IT>
__device__ __forceinline__ IT round_to(double x) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x + F64_BIAS);
  if constexpr (sizeof(IT) == 8) {
    return static_cast<IT>(b - static_cast<uint64_t>(F64_BIAS_BITS));
  } else {
    // the bias has a zero low word: the low 32 bits are the rounded integer
    // (map values of 32-bit states are validated to fit int32)
    return static_cast<IT>(static_cast<uint32_t>(b));
  }
}

template <typename IT>
__device__ __forceinline__ double as_f64(IT q) {
  if constexpr (sizeof(IT) == 8) {
    const uint64_t b = static_cast<uint64_t>(F64_BIAS_BITS) + static_cast<uint64_t>(q);
    return __builtin_bit_cast(double, b) - F64_BIAS;
  } else {
    return static_cast<double>(q);
  }
}

// s*s for a state s with s^2 < 2^53 (validated at create): the FP64 product of
// the exact conversions equals the conversion of the exact integer square.
template <typename IT>
__device__ __forceinline__ double square_f64(IT s) {
  double d = as_f64<IT>(s);
  return d * d;
}

template <typename IT>
__device__ __forceinline__ IT lf_phi(const XParams& P, IT q, bool plus, bool linear) {
  double x = P.delta * as_f64<IT>(q);
  double fx = linear ? P.a * x : (x * x) * 0.5;
  double ax = P.alpha * x;
  double g = plus ? fx + ax : fx - ax;
  g = g * 0.5;
  g = g * P.lambda;
  g = g / P.delta;
  return round_to<IT>(g);
}

template <typename IT>
struct LutEntry;
template <>
struct LutEntry<int32_t> { using T = int2; };
template <>
struct LutEntry<int64_t> { using T = longlong2; };

template <int POL>
struct IsSplit {
  static constexpr bool value = POL == P_UPWIND_POS || POL == P_UPWIND_NEG || POL == P_EO ||
                                POL == P_LF_LINEAR || POL == P_LF_BURGERS || POL == P_LUT;
};

// One rounded split map phi+ (plus) or phi- of a direct split policy.
template <typename IT, int POL>
__device__ __forceinline__ IT split_phi(const XParams& P, IT q, bool plus) {
  if constexpr (POL == P_UPWIND_POS) {
    return plus ? round_to<IT>(P.c * as_f64<IT>(q)) : IT(0);
  } else if constexpr (POL == P_UPWIND_NEG) {
    return plus ? IT(0) : round_to<IT>(P.c * as_f64<IT>(q));
  } else if constexpr (POL == P_EO) {
    IT s = plus ? (q > IT(0) ? q : IT(0)) : (q < IT(0) ? q : IT(0));
    return round_to<IT>(P.h * square_f64<IT>(s));
  } else if constexpr (POL == P_LF_LINEAR) {
    return lf_phi<IT>(P, q, plus, true);
  } else {
    static_assert(POL == P_LF_BURGERS, "not a direct split policy");
    return lf_phi<IT>(P, q, plus, false);
  }
}

// Both split maps of one state.  For Engquist-Osher only one of them can be
// nonzero (the sign of q decides), so one rounded product serves both: the
// other map is rint(0) = 0, the value its own evaluation gives.
template <typename IT, int POL>
__device__ __forceinline__ void split_maps(const XParams& P, IT q, IT& pp, IT& pm) {
  if constexpr (POL == P_EO) {
    const IT t = round_to<IT>(P.h * square_f64<IT>(q));
    const bool pos = q > IT(0);
    pp = pos ? t : IT(0);
    pm = pos ? IT(0) : t;
  } else {
    pp = split_phi<IT, POL>(P, q, true);
    pm = split_phi<IT, POL>(P, q, false);
  }
}

// Interface transfer T(qL, qR) for policy POL.
template <typename IT, int POL>
__device__ __forceinline__ IT transfer(const XParams& P, IT qL, IT qR) {
  if constexpr (POL == P_GODUNOV) {
    IT s;
    if (qL <= qR) {
      s = qL > IT(0) ? qL : (qR < IT(0) ? qR : IT(0));
    } else {
      // compare squares exactly in FP64 (both below 2^53)
      s = square_f64<IT>(qL) >= square_f64<IT>(qR) ? qL : qR;
    }
    return round_to<IT>(P.h * square_f64<IT>(s));
  } else if constexpr (POL == P_MURMAN_ROE) {
    // sign of the Roe speed (qL + qR)/2, summed in 64 bits
    IT s = (static_cast<int64_t>(qL) + static_cast<int64_t>(qR) >= 0) ? qL : qR;
    return round_to<IT>(P.h * square_f64<IT>(s));
  } else if constexpr (POL == P_LUT) {
    using E = typename LutEntry<IT>::T;
    const E* lut = static_cast<const E*>(P.lut);
    // Indices are clamped so that no lane can read outside the table; states
    // of cells inside the domain never leave [lo, hi] (maximum principle), so
    // the clamp only ever acts on discarded halo lanes.
    int64_t iL = static_cast<int64_t>(qL) - P.lut_lo;
    int64_t iR = static_cast<int64_t>(qR) - P.lut_lo;
    iL = iL < 0 ? 0 : (iL > P.lut_last ? P.lut_last : iL);
    iR = iR < 0 ? 0 : (iR > P.lut_last ? P.lut_last : iR);
    return static_cast<IT>(lut[iL].x) + static_cast<IT>(lut[iR].y);
  } else {
    return split_phi<IT, POL>(P, qL, true) + split_phi<IT, POL>(P, qR, false);
  }
}

// Wrapping integer arithmetic (discarded halo lanes may hold garbage; avoid UB).
template <typename IT>
__device__ __forceinline__ IT wsub(IT a, IT b) {
  using U = typename std::make_unsigned<IT>::type;
  return static_cast<IT>(static_cast<U>(a) - static_cast<U>(b));
}

// Cross-lane moves within a 64-wide wavefront, as DPP wavefront shifts (a
// modifier on a VALU move, no LDS round trip).  gfx9 controls: 0x130 shift
// left (lane l takes lane l+1), 0x138 shift right (lane l takes lane l-1),
// 0x134 / 0x13C the rotating forms.  The end lane of a shift keeps its own
// value.
template <int CTRL>
__device__ __forceinline__ int dpp32(int v) {
  return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xf, 0xf, false);
}

template <int CTRL, typename IT>
__device__ __forceinline__ IT dpp_move(IT v) {
  if constexpr (sizeof(IT) == 4) {
    return __builtin_bit_cast(IT, dpp32<CTRL>(__builtin_bit_cast(int, v)));
  } else {
    // 64-bit values (integers or doubles) move as their bit patterns
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = dpp32<CTRL>(static_cast<int>(static_cast<uint32_t>(u)));
    const int hi = dpp32<CTRL>(static_cast<int>(static_cast<uint32_t>(u >> 32)));
    return __builtin_bit_cast(IT, (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) |
                                      static_cast<uint32_t>(lo));
  }
}

template <typename IT>
__device__ __forceinline__ IT lane_from_next(IT v) {  // lane l receives lane l+1 (lane 63: own)
  return dpp_move<0x130, IT>(v);
}
template <typename IT>
__device__ __forceinline__ IT lane_from_prev(IT v) {  // lane l receives lane l-1 (lane 0: own)
  return dpp_move<0x138, IT>(v);
}
template <typename IT>
__device__ __forceinline__ IT rotate_from_next(IT v) {  // lane l receives lane (l+1) mod 64
  return dpp_move<0x134, IT>(v);
}
template <typename IT>
__device__ __forceinline__ IT rotate_from_prev(IT v) {  // lane l receives lane (l-1) mod 64
  return dpp_move<0x13C, IT>(v);
}

// Map block index to a tile index so that consecutive tiles land on the same
// XCD (blocks are dispatched round-robin over the 8 XCDs).
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nb) {
  const int64_t X = 8;
  int64_t q = nb / X, r = nb % X;
  int64_t x = b % X;
  int64_t start = x * q + (x < r ? x : r);
  return start + b / X;
}

__device__ __forceinline__ int64_t wrap_index(int64_t g, int64_t n) {
  int64_t r = g % n;
  return r < 0 ? r + n : r;
}
__device__ __forceinline__ int64_t clamp_index(int64_t g, int64_t n) {
  return g < 0 ? 0 : (g >= n ? n - 1 : g);
}

}  // namespace fqnm
