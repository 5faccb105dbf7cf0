// nd_tb.hip -- 2-D periodic grids, several steps of eq:nd_transfer_rule per
// pass (temporal blocking of the directional composition, Thm
// dimension_extension).
//
// k_nd_tb: a wavefront owns a strip of 64*V consecutive cells of axis 0 (V per
// lane) that overlaps each neighbouring strip by H cells (H = K rounded up to
// a multiple of V), and marches along axis 1 over a block of R rows plus K
// rows on each side.  The K time levels of the pass are chained in registers:
// when a row of level s-1 arrives, level s turns the row before it into level
// s.  Each level keeps, for the row it last received, the state, the axis-0
// flux divergence and phi+ along axis 1 (or the state alone for two-point
// rules), and the axis-1 flux on that row's lower face.  Axis-0 neighbours come
// from the adjacent lanes by cross-lane moves.  A level-s value is exact on
// cells at least s cells from the strip's ends and on rows at least s rows from
// the first and last loaded row; the cells stored (the strip's middle 64V - 2H,
// the block's R rows) are K away from both.  Values outside that region are
// computed but never stored; the integer arithmetic wraps there.
//
// A level keeps two values per cell for the row it received last: e = q - (its
// axis-0 flux divergence) + (the axis-1 flux on its lower face), and aux = its
// phi+ along axis 1 (split rules) or its state (two-point rules).  When the
// next row arrives, the flux F between the two rows follows from aux and the
// new row, the older row leaves the level as e - F, and the new row's e is its
// q - divergence + F.
#include <hip/hip_runtime.h>

#include "nd_common.h"

namespace fqnm {
namespace {

template <typename IT>
__device__ __forceinline__ IT wadd(IT a, IT b) {
  using U = typename std::make_unsigned<IT>::type;
  return static_cast<IT>(static_cast<U>(a) + static_cast<U>(b));
}

// Wavefront shifts by one lane that fill the end lane with 0 (lane l receives
// lane l+1, or lane l-1).  The ends belong to the strip's halo, whose values
// are never stored; the zero fill lets the compiler fold a 32-bit move into
// the instruction that consumes it.  64-bit values move as two halves.
template <int CTRL>
__device__ __forceinline__ int tb_dpp0(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, true);
}
template <int CTRL, typename IT>
__device__ __forceinline__ IT tb_shift(IT v) {
  if constexpr (sizeof(IT) == 4) {
    return __builtin_bit_cast(IT, tb_dpp0<CTRL>(__builtin_bit_cast(int, v)));
  } else {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = static_cast<uint32_t>(tb_dpp0<CTRL>(static_cast<int>(u)));
    const uint32_t hi = static_cast<uint32_t>(tb_dpp0<CTRL>(static_cast<int>(u >> 32)));
    return __builtin_bit_cast(IT, (static_cast<uint64_t>(hi) << 32) | lo);
  }
}
template <typename IT>
__device__ __forceinline__ IT tb_from_next(IT v) {
  return tb_shift<0x130, IT>(v);
}
template <typename IT>
__device__ __forceinline__ IT tb_from_prev(IT v) {
  return tb_shift<0x138, IT>(v);
}

// One time level's registers (see the file comment).
template <typename IT, int V>
struct TbLevel {
  IT e[V];
  IT aux[V];
};

// The axis-0 fluxes of a row (Fx[k] on the right face of cell k, Fl on the
// left face of cell 0) and its maps along axis 1.
template <typename IT, int POL, int V, bool SAME>
__device__ __forceinline__ void tb_row(const NdParams& P, const IT (&q)[V], IT (&Fx)[V], IT& Fl,
                                       IT (&ppy)[V], IT (&pmy)[V]) {
  const NdAxis& AX = P.ax[0];
  if constexpr (NdSplit<POL>::value) {
    IT ppx[V], pmx[V];
#pragma unroll
    for (int k = 0; k < V; ++k) axis_maps<IT, POL>(AX, q[k], ppx[k], pmx[k]);
#pragma unroll
    for (int k = 0; k < V; ++k)
      Fx[k] = wadd<IT>(k + 1 < V ? pmx[k + 1] : tb_from_next<IT>(pmx[0]), ppx[k]);
    if constexpr (SAME) {
#pragma unroll
      for (int k = 0; k < V; ++k) {
        ppy[k] = ppx[k];
        pmy[k] = pmx[k];
      }
    } else {
#pragma unroll
      for (int k = 0; k < V; ++k) axis_maps<IT, POL>(P.ax[1], q[k], ppy[k], pmy[k]);
    }
  } else {
    const IT qn = tb_from_next<IT>(q[0]);
#pragma unroll
    for (int k = 0; k < V; ++k) {
      Fx[k] = transfer<IT, POL>(AX.x, q[k], k + 1 < V ? q[k + 1] : qn);
      ppy[k] = IT(0);
      pmy[k] = IT(0);
    }
  }
  Fl = tb_from_prev<IT>(Fx[V - 1]);
}

// One row through level s: `in` is the incoming row of level s-1 and X holds
// the row before it.  Fills Y for the incoming row and writes level s of X's
// row to out (exact once the level has received three rows).  Successive rows
// alternate between two register sets, so nothing is copied.
template <typename IT, int POL, int V, bool SAME>
__device__ __forceinline__ void tb_feed(const NdParams& P, const TbLevel<IT, V>& X,
                                        TbLevel<IT, V>& Y, const IT (&in)[V], IT (&out)[V]) {
  IT Fx[V], Fl, pp[V], pm[V];
  tb_row<IT, POL, V, SAME>(P, in, Fx, Fl, pp, pm);
#pragma unroll
  for (int k = 0; k < V; ++k) {
    IT f;
    if constexpr (NdSplit<POL>::value) f = wadd<IT>(X.aux[k], pm[k]);
    else f = transfer<IT, POL>(P.ax[1].x, X.aux[k], in[k]);
    out[k] = wsub<IT>(X.e[k], f);
    // q - (Fx[k] - Fx[k-1]) + f
    Y.e[k] = wadd<IT>(wadd<IT>(k == 0 ? Fl : Fx[k - 1], f), wsub<IT>(in[k], Fx[k]));
    Y.aux[k] = NdSplit<POL>::value ? pp[k] : in[k];
  }
}

template <int V>
constexpr int tb_halo(int K) {
  return (K + V - 1) / V * V;
}

// SAME: both axes have the same map constants, so axis 1 reuses axis 0's maps.
template <typename IT, int POL, int V, int K, bool SAME>
__global__ __launch_bounds__(256) void k_nd_tb(const IT* __restrict__ src, IT* __restrict__ dst,
                                               NdParams P, int rows, int64_t nstrips,
                                               int64_t nwaves) {
  constexpr int H = tb_halo<V>(K);
  constexpr int W = 64 * V - 2 * H;  // cells stored per strip
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int64_t w = xcd_tile(blockIdx.x, gridDim.x) * 4 + wave;
  if (w >= nwaves) return;
  const int64_t nx = P.ax[0].n, ny = P.ax[1].n;
  const int64_t xs = (w % nstrips) * W;  // first stored cell of the strip
  const int64_t j0 = (w / nstrips) * rows;
  const int64_t jend = j0 + rows < ny ? j0 + rows : ny;
  // this lane's V cells start at x (unwrapped); nx is a multiple of V, so the
  // V cells wrap together
  const int64_t x = xs - H + static_cast<int64_t>(lane) * V;
  const int64_t xw = wrap_index(x, nx);
  const bool store = lane >= H / V && lane < 64 - H / V && x < nx;

  TbLevel<IT, V> A[K], B[K];
#pragma unroll
  for (int s = 0; s < K; ++s)
#pragma unroll
    for (int k = 0; k < V; ++k) A[s].e[k] = A[s].aux[k] = B[s].e[k] = B[s].aux[k] = IT(0);

  // rows j0 - K .. jend + K - 1 are loaded; iteration p loads row j0 - K + p
  // and level K leaves row j0 + p - 2K
  // (np >= 2K + 1 >= 3; the wrapped row index advances by one per load)
  const int64_t np = (jend - j0) + 2 * K;
  int64_t rw = wrap_index(j0 - K, ny);
  auto next_row = [&]() { rw = rw + 1 == ny ? 0 : rw + 1; };
  IT a[V], b[V];
  nd_load<IT, V>(src + rw * nx + xw, a);
  next_row();
  nd_load<IT, V>(src + rw * nx + xw, b);
  // iteration p: X holds each level's previous row, Y receives the new one
  auto iteration = [&](int64_t p, TbLevel<IT, V>(&X)[K], TbLevel<IT, V>(&Y)[K]) {
    IT cur[V];
#pragma unroll
    for (int k = 0; k < V; ++k) {
      cur[k] = a[k];
      a[k] = b[k];
    }
    if (p + 2 < np) {  // uniform
      next_row();
      nd_load<IT, V>(src + rw * nx + xw, b);
    }
    // level s + 1 receives exact rows from iteration 2s on (what it held
    // before then flushes out of its registers)
#pragma unroll
    for (int s = 0; s < K; ++s) {
      if (p < 2 * s) break;  // uniform
      IT out[V];
      tb_feed<IT, POL, V, SAME>(P, X[s], Y[s], cur, out);
#pragma unroll
      for (int k = 0; k < V; ++k) cur[k] = out[k];
    }
    if (p >= 2 * K && store) nd_store<IT, V>(dst + (j0 + p - 2 * K) * nx + x, cur);
  };
  for (int64_t p = 0; p < np; p += 2) {
    iteration(p, A, B);
    if (p + 1 < np) iteration(p + 1, B, A);
  }
}

template <typename IT, int POL, int V, int K>
hipError_t tb_launch(const void* src, void* dst, const NdParams& P, int rows, hipStream_t s) {
  constexpr int W = 64 * V - 2 * tb_halo<V>(K);
  const int64_t nstrips = (P.ax[0].n + W - 1) / W;
  const int64_t nwaves = nstrips * ((P.ax[1].n + rows - 1) / rows);
  const int64_t blocks = (nwaves + 3) / 4;
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  const dim3 g(static_cast<unsigned>(blocks)), b(256);
  const IT* a = static_cast<const IT*>(src);
  IT* d = static_cast<IT*>(dst);
  const NdAxis &X = P.ax[0], &Y = P.ax[1];
  const bool same = X.x.c == Y.x.c && X.x.h == Y.x.h && X.x.a == Y.x.a &&
                    X.x.alpha == Y.x.alpha && X.x.delta == Y.x.delta && X.x.lambda == Y.x.lambda;
  if constexpr (NdSplit<POL>::value) {
    if (same) {
      k_nd_tb<IT, POL, V, K, true><<<g, b, 0, s>>>(a, d, P, rows, nstrips, nwaves);
      return hipGetLastError();
    }
  }
  k_nd_tb<IT, POL, V, K, false><<<g, b, 0, s>>>(a, d, P, rows, nstrips, nwaves);
  return hipGetLastError();
}

template <typename IT, int POL, int V>
hipError_t tb_by_k(int K, const void* src, void* dst, const NdParams& P, int rows,
                   hipStream_t s) {
  switch (K) {
    case 1: return tb_launch<IT, POL, V, 1>(src, dst, P, rows, s);
    case 2: return tb_launch<IT, POL, V, 2>(src, dst, P, rows, s);
    case 4: return tb_launch<IT, POL, V, 4>(src, dst, P, rows, s);
    case 8: return tb_launch<IT, POL, V, 8>(src, dst, P, rows, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename IT, int POL>
hipError_t tb_by_vec(int vec, int K, const void* src, void* dst, const NdParams& P, int rows,
                     hipStream_t s) {
  if (vec == 2) return tb_by_k<IT, POL, 2>(K, src, dst, P, rows, s);
  if constexpr (sizeof(IT) == 4) {
    if (vec == 4) return tb_by_k<IT, POL, 4>(K, src, dst, P, rows, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

bool nd_tb_valid(int itype, int pol, int vec, const NdParams& P) {
  if (P.dim != 2) return false;
  if (itype == FQNM_I32 ? (vec != 2 && vec != 4) : vec != 2) return false;
  if (P.ax[0].bc != FQNM_BC_PERIODIC || P.ax[1].bc != FQNM_BC_PERIODIC) return false;
  if (pol != P_UPWIND_POS && pol != P_EO && pol != P_GODUNOV && pol != P_MURMAN_ROE &&
      pol != P_LF_LINEAR && pol != P_LF_BURGERS)
    return false;
  return P.ax[0].n % vec == 0;
}

int nd_tb_step_depth(int max_depth) {
  for (int k : {8, 4, 2})
    if (k <= max_depth) return k;
  return 1;
}

template <typename IT>
hipError_t tb_by_pol(int pol, int vec, int depth, const void* src, void* dst, const NdParams& P,
                     int rows, hipStream_t s) {
  switch (pol) {
    case P_UPWIND_POS: return tb_by_vec<IT, P_UPWIND_POS>(vec, depth, src, dst, P, rows, s);
    case P_EO: return tb_by_vec<IT, P_EO>(vec, depth, src, dst, P, rows, s);
    case P_GODUNOV: return tb_by_vec<IT, P_GODUNOV>(vec, depth, src, dst, P, rows, s);
    case P_MURMAN_ROE: return tb_by_vec<IT, P_MURMAN_ROE>(vec, depth, src, dst, P, rows, s);
    case P_LF_LINEAR: return tb_by_vec<IT, P_LF_LINEAR>(vec, depth, src, dst, P, rows, s);
    case P_LF_BURGERS: return tb_by_vec<IT, P_LF_BURGERS>(vec, depth, src, dst, P, rows, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_nd_tb(int itype, int pol, int vec, int depth, int rows, const void* src,
                        void* dst, const NdParams& P, hipStream_t s) {
  if (!nd_tb_valid(itype, pol, vec, P) || rows < 1 || nd_tb_step_depth(depth) != depth)
    return hipErrorInvalidValue;
  if (itype == FQNM_I32) return tb_by_pol<int32_t>(pol, vec, depth, src, dst, P, rows, s);
  return tb_by_pol<int64_t>(pol, vec, depth, src, dst, P, rows, s);
}

}  // namespace fqnm
