// nd_common.h -- pieces shared by the d-dimensional kernels: per-lane vector
// access of a lane's consecutive cells and the split maps of one cell along
// one axis.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "fqnm_internal.h"

namespace fqnm {
namespace {

typedef int v4i_nd __attribute__((ext_vector_type(4)));

typedef int v2i_nd __attribute__((ext_vector_type(2)));

// Bytes per vector access of a lane's V cells: 16, or 8 when they fill less.
template <typename IT, int V>
struct NdVec {
  static constexpr int BYTES = V * sizeof(IT) >= 16 ? 16 : 8;
  static_assert(V * sizeof(IT) % BYTES == 0, "cells per lane must fill whole vectors");
  using T = typename std::conditional<BYTES == 16, v4i_nd, v2i_nd>::type;
};

template <typename IT, int V>
__device__ __forceinline__ void nd_load(const IT* __restrict__ p, IT (&q)[V]) {
  using Vec = NdVec<IT, V>;
  constexpr int PER = Vec::BYTES / sizeof(IT);
  const typename Vec::T* pv = reinterpret_cast<const typename Vec::T*>(p);
#pragma unroll
  for (int c = 0; c < V / PER; ++c) {
    typename Vec::T v = pv[c];
    __builtin_memcpy(&q[c * PER], &v, Vec::BYTES);
  }
}

template <typename IT, int V>
__device__ __forceinline__ void nd_store(IT* __restrict__ p, const IT (&q)[V]) {
  using Vec = NdVec<IT, V>;
  constexpr int PER = Vec::BYTES / sizeof(IT);
  typename Vec::T* pv = reinterpret_cast<typename Vec::T*>(p);
#pragma unroll
  for (int c = 0; c < V / PER; ++c) {
    typename Vec::T v;
    __builtin_memcpy(&v, &q[c * PER], Vec::BYTES);
    pv[c] = v;
  }
}

// Ghost position along an axis of n cells: periodic wrap or outflow copy.
__device__ __forceinline__ int64_t nd_ghost(int64_t g, int64_t n, int bc) {
  if (g >= 0 && g < n) return g;
  return bc == FQNM_BC_PERIODIC ? wrap_index(g, n) : clamp_index(g, n);
}

// Split maps of one cell along one axis.  For UPWIND and Engquist-Osher only
// one of phi+ and phi- can be nonzero for a given state (the sign of a, or of
// q, decides), so one rounded product serves both: the value is the one the
// separate evaluation gives, the other map being rint(+-0) = 0.
template <typename IT, int POL>
__device__ __forceinline__ void axis_maps(const NdAxis& A, IT q, IT& pp, IT& pm) {
  if constexpr (POL == P_UPWIND_POS) {  // UPWIND of either sign
    const IT t = round_to<IT>(A.x.c * as_f64<IT>(q));
    pp = A.x.c >= 0.0 ? t : IT(0);
    pm = A.x.c >= 0.0 ? IT(0) : t;
  } else if constexpr (POL == P_EO) {
    // t = 0 for q = 0, so one comparison places t in the map that holds it
    const IT t = round_to<IT>(A.x.h * square_f64<IT>(q));
    const bool pos = q > IT(0);
    pp = pos ? t : IT(0);
    pm = pos ? IT(0) : t;
  } else {
    pp = split_phi<IT, POL>(A.x, q, true);
    pm = split_phi<IT, POL>(A.x, q, false);
  }
}

template <int POL>
struct NdSplit {
  static constexpr bool value = POL == P_UPWIND_POS || POL == P_EO || POL == P_LF_LINEAR ||
                                POL == P_LF_BURGERS;
};

// Two axes with the same one-dimensional map constants evaluate the same maps.
__device__ __forceinline__ bool nd_same_axis(const NdAxis& a, const NdAxis& b) {
  return a.x.c == b.x.c && a.x.h == b.x.h && a.x.a == b.x.a && a.x.alpha == b.x.alpha &&
         a.x.delta == b.x.delta && a.x.lambda == b.x.lambda;
}

}  // namespace
}  // namespace fqnm
