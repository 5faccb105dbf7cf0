// nd_tb.hip -- 2-D grids, several steps of eq:nd_transfer_rule per
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
// Outflow ends (OUT variants, either axis outflow): loads clamp to the grid.
// The faces at the ends of an outflow axis take the end cell's own transfer
// at every level: the lanes holding the first or last cell of axis 0 select
// it for their outer face, and along axis 1 the face below row 0 is computed
// from row 0 itself and the face above the last row from that row's own
// transfer, kept per level until the row above it passes.  Cells and rows
// outside the grid are never stored, and no stored value reads them.  The
// counts crossing those faces go to the ledger, each counted by the
// wavefront that owns the row and stores the cell.
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

// This lane's place at the ends of an outflow axis 0 (cell 0 is its first
// cell, cell nx - 1 its last), whether it stores its cells, and whether axis 1
// is outflow.
struct TbEdges {
  bool xl, xr, store, oy;
};

// One time level's registers (see the file comment).
template <typename IT, int V>
struct TbLevel {
  IT e[V];
  IT aux[V];
};

// The axis-0 fluxes of a row (Fx[k] on the right face of cell k, Fl on the
// left face of cell 0) and its maps along axis 1.
template <typename IT, int POL, int V, bool SAME, bool OUT>
__device__ __forceinline__ void tb_row(const NdParams& P, const TbEdges& E, const IT (&q)[V],
                                       IT (&Fx)[V], IT& Fl, IT (&ppy)[V], IT (&pmy)[V]) {
  const NdAxis& AX = P.ax[0];
  if constexpr (NdSplit<POL>::value) {
    IT ppx[V], pmx[V];
#pragma unroll
    for (int k = 0; k < V; ++k) axis_maps<IT, POL>(AX, q[k], ppx[k], pmx[k]);
#pragma unroll
    for (int k = 0; k < V; ++k)
      Fx[k] = wadd<IT>(k + 1 < V ? pmx[k + 1] : tb_from_next<IT>(pmx[0]), ppx[k]);
    Fl = tb_from_prev<IT>(Fx[V - 1]);
    if constexpr (OUT) {  // the end cells' own transfers on the outer faces
      Fl = E.xl ? wadd<IT>(ppx[0], pmx[0]) : Fl;
      Fx[V - 1] = E.xr ? wadd<IT>(ppx[V - 1], pmx[V - 1]) : Fx[V - 1];
    }
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
    IT qn = tb_from_next<IT>(q[0]);
    if constexpr (OUT) qn = E.xr ? q[V - 1] : qn;
#pragma unroll
    for (int k = 0; k < V; ++k) {
      Fx[k] = transfer<IT, POL>(AX.x, q[k], k + 1 < V ? q[k + 1] : qn);
      ppy[k] = IT(0);
      pmy[k] = IT(0);
    }
    Fl = tb_from_prev<IT>(Fx[V - 1]);
    if constexpr (OUT) Fl = E.xl ? transfer<IT, POL>(AX.x, q[0], q[0]) : Fl;
  }
}

// One row through level s: `in` is the incoming row of level s-1 and X holds
// the row before it.  Fills Y for the incoming row and writes level s of X's
// row to out (exact once the level has received three rows).  Successive rows
// alternate between two register sets, so nothing is copied.
//
// OUT: m is the incoming row's index, [j0, jend) the rows this wavefront
// owns, ynear whether this iteration's rows reach row 0 or the last row, ftop
// the level's kept transfer above the last row, led the ledger.
template <typename IT, int POL, int V, bool SAME, bool OUT>
__device__ __forceinline__ void tb_feed(const NdParams& P, const TbEdges& E,
                                        const TbLevel<IT, V>& X, TbLevel<IT, V>& Y,
                                        const IT (&in)[V], IT (&out)[V], int64_t m, int64_t j0,
                                        int64_t jend, bool ynear, IT (&ftop)[V], long long& led) {
  IT Fx[V], Fl, pp[V], pm[V];
  tb_row<IT, POL, V, SAME, OUT>(P, E, in, Fx, Fl, pp, pm);
  const int64_t ny = P.ax[1].n;
  if constexpr (OUT) {
    // only the (at most two) lanes at the ends of axis 0 take this branch
    if ((E.xl || E.xr) && E.store && m >= j0 && m < jend) {
      led += E.xl ? static_cast<long long>(Fl) : 0;
      led -= E.xr ? static_cast<long long>(Fx[V - 1]) : 0;
    }
  }
#pragma unroll
  for (int k = 0; k < V; ++k) {
    IT f;
    if constexpr (NdSplit<POL>::value) f = wadd<IT>(X.aux[k], pm[k]);
    else f = transfer<IT, POL>(P.ax[1].x, X.aux[k], in[k]);
    if constexpr (OUT) {
      if (E.oy && ynear) {  // uniform, as are the row tests
        if (m == 0 || m == ny - 1) {
          IT self;
          if constexpr (NdSplit<POL>::value) self = wadd<IT>(pp[k], pm[k]);
          else self = transfer<IT, POL>(P.ax[1].x, in[k], in[k]);
          if (m == 0) {
            f = self;
            if (j0 == 0 && E.store) led += static_cast<long long>(self);
          }
          if (m == ny - 1) ftop[k] = self;
        }
        if (m == ny) {
          f = ftop[k];
          if (jend == ny && E.store) led -= static_cast<long long>(f);
        }
      }
    }
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

// The march of one wavefront over its strip [xs - H, xs - H + 64V) and rows
// [j0 - K, jend + K).  EDGES: that range reaches past an end of an outflow
// axis, so the faces at the grid's ends take the end cells' own transfers and
// the counts crossing them go to the ledger.  Without EDGES every load is
// inside the grid or wraps, and no stored cell depends on an end face.
template <typename IT, int POL, int V, int K, bool SAME, bool EDGES>
__device__ __forceinline__ void tb_march(const IT* __restrict__ src, IT* __restrict__ dst,
                                         const NdParams& P, int64_t xs, int64_t j0,
                                         int64_t jend, int lane, long long* __restrict__ ledger) {
  constexpr int H = tb_halo<V>(K);
  const int64_t nx = P.ax[0].n, ny = P.ax[1].n;
  // this lane's V cells start at x (unwrapped); nx is a multiple of V, so the
  // V cells wrap (or clamp) together
  const int64_t x = xs - H + static_cast<int64_t>(lane) * V;
  const bool ox = P.ax[0].bc == FQNM_BC_OUTFLOW;
  const bool oy = P.ax[1].bc == FQNM_BC_OUTFLOW;
  const int64_t xw = ox ? (x < 0 ? 0 : (x > nx - V ? nx - V : x)) : wrap_index(x, nx);
  const bool store = lane >= H / V && lane < 64 - H / V && x < nx;
  const TbEdges E{EDGES && ox && x == 0, EDGES && ox && x == nx - V, store, EDGES && oy};
  IT ftop[K][V];
#pragma unroll
  for (int s = 0; s < K; ++s)
#pragma unroll
    for (int k = 0; k < V; ++k) ftop[s][k] = IT(0);
  long long led = 0;

  TbLevel<IT, V> A[K], B[K];
#pragma unroll
  for (int s = 0; s < K; ++s)
#pragma unroll
    for (int k = 0; k < V; ++k) A[s].e[k] = A[s].aux[k] = B[s].e[k] = B[s].aux[k] = IT(0);

  // rows j0 - K .. jend + K - 1 are loaded; iteration p loads row j0 - K + p
  // and level K leaves row j0 + p - 2K
  // (np >= 2K + 1 >= 3; the row index advances by one per load)
  const int64_t np = (jend - j0) + 2 * K;
  int64_t r = j0 - K;  // row of the latest load (unwrapped)
  int64_t rw = oy ? (r < 0 ? 0 : r) : wrap_index(r, ny);
  auto next_row = [&]() {
    ++r;
    if (oy) rw = r < 0 ? 0 : (r >= ny ? ny - 1 : r);
    else rw = rw + 1 == ny ? 0 : rw + 1;
  };
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
    // before then flushes out of its registers); its incoming row is
    // j0 - K + p - s
    const int64_t sb = j0 - K + p;
    const bool ynear = EDGES && oy && ((sb - (K - 1) <= 0 && sb >= 0) ||
                                       (sb - (K - 1) <= ny && sb >= ny - 1));
#pragma unroll
    for (int s = 0; s < K; ++s) {
      if (p < 2 * s) break;  // uniform
      IT out[V];
      tb_feed<IT, POL, V, SAME, EDGES>(P, E, X[s], Y[s], cur, out, sb - s, j0, jend, ynear,
                                       ftop[s], led);
#pragma unroll
      for (int k = 0; k < V; ++k) cur[k] = out[k];
    }
    if (p >= 2 * K && store) nd_store<IT, V>(dst + (j0 + p - 2 * K) * nx + x, cur);
  };
  for (int64_t p = 0; p < np; p += 2) {
    iteration(p, A, B);
    if (p + 1 < np) iteration(p + 1, B, A);
  }
  if constexpr (EDGES) {
    // one atomic per wavefront: the lanes' counts are summed across the
    // wavefront first (every lane is active here)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) led += __shfl_xor(led, off, 64);
    if (lane == 0 && led != 0)
      atomicAdd(reinterpret_cast<unsigned long long*>(ledger), static_cast<unsigned long long>(led));
  }
}

// Wavefronts to (strip, row block).  The ni interior strips [first, first + ni)
// come first, `rows` rows per wavefront; then the ne strips whose loaded range
// reaches past an end of an outflow axis 0 (strip 0 and strips te and above),
// rows_e rows per wavefront: they run the slower boundary code, and shorter
// marches keep them from setting the launch's length.  Without outflow along
// axis 0 every strip is interior.
struct TbMap {
  int64_t ni, first, te, ne, nblk, nblk_e;
  int32_t rows, rows_e;
};

// SAME: both axes have the same map constants, so axis 1 reuses axis 0's maps.
// OUT: at least one axis is outflow.
template <typename IT, int POL, int V, int K, bool SAME, bool OUT>
__global__ __launch_bounds__(256) void k_nd_tb(const IT* __restrict__ src, IT* __restrict__ dst,
                                               NdParams P, TbMap M, int64_t nwaves,
                                               long long* __restrict__ ledger) {
  constexpr int H = tb_halo<V>(K);
  constexpr int W = 64 * V - 2 * H;  // cells stored per strip
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int64_t w = xcd_tile(blockIdx.x, gridDim.x) * 4 + wave;
  if (w >= nwaves) return;
  const int64_t nx = P.ax[0].n, ny = P.ax[1].n;
  int64_t strip, j0, rws;
  if (w < M.ni * M.nblk) {
    strip = M.first + w % M.ni;
    j0 = (w / M.ni) * M.rows;
    rws = M.rows;
  } else {
    const int64_t w2 = w - M.ni * M.nblk;
    const int64_t e = w2 % M.ne;
    strip = (M.first == 1 && e == 0) ? 0 : M.te + e - M.first;
    j0 = (w2 / M.ne) * M.rows_e;
    rws = M.rows_e;
  }
  const int64_t xs = strip * W;  // first stored cell of the strip
  const int64_t jend = j0 + rws < ny ? j0 + rws : ny;
  if constexpr (OUT) {
    const bool edges =
        (P.ax[0].bc == FQNM_BC_OUTFLOW && (xs - H < 0 || xs - H + 64 * V > nx)) ||
        (P.ax[1].bc == FQNM_BC_OUTFLOW && (j0 - K < 0 || jend + K > ny));
    if (edges) {  // uniform
      tb_march<IT, POL, V, K, SAME, true>(src, dst, P, xs, j0, jend, lane, ledger);
      return;
    }
  }
  tb_march<IT, POL, V, K, SAME, false>(src, dst, P, xs, j0, jend, lane, ledger);
}

template <typename IT, int POL, int V, int K, bool SAME>
void tb_go(dim3 g, const IT* a, IT* d, const NdParams& P, const TbMap& M, int64_t nwaves,
           long long* led, hipStream_t s) {
  if (P.ax[0].bc == FQNM_BC_OUTFLOW || P.ax[1].bc == FQNM_BC_OUTFLOW)
    k_nd_tb<IT, POL, V, K, SAME, true><<<g, dim3(256), 0, s>>>(a, d, P, M, nwaves, led);
  else
    k_nd_tb<IT, POL, V, K, SAME, false><<<g, dim3(256), 0, s>>>(a, d, P, M, nwaves, led);
}

template <typename IT, int POL, int V, int K>
hipError_t tb_launch(const void* src, void* dst, const NdParams& P, int rows, long long* led,
                     hipStream_t s) {
  constexpr int H = tb_halo<V>(K);
  constexpr int W = 64 * V - 2 * H;
  const int64_t nx = P.ax[0].n, ny = P.ax[1].n;
  const int64_t nstrips = (nx + W - 1) / W;
  TbMap M;
  M.rows = rows;
  M.rows_e = rows > 1 ? rows / 2 : 1;
  M.nblk = (ny + rows - 1) / rows;
  M.nblk_e = (ny + M.rows_e - 1) / M.rows_e;
  if (P.ax[0].bc == FQNM_BC_OUTFLOW) {
    // strip t loads cells [tW - H, tW - H + 64V): strip 0 and the strips with
    // tW + W + H > nx reach past an end
    M.first = 1;
    const int64_t last_in = nx - W - H >= 0 ? (nx - W - H) / W : 0;  // last t inside
    M.te = last_in + 1 > nstrips ? nstrips : (last_in + 1 < 1 ? 1 : last_in + 1);
    M.ni = M.te - 1;
    M.ne = nstrips - M.ni;
  } else {
    M.first = 0;
    M.te = nstrips;
    M.ni = nstrips;
    M.ne = 0;
  }
  const int64_t nwaves = M.ni * M.nblk + M.ne * M.nblk_e;
  const int64_t blocks = (nwaves + 3) / 4;
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  const dim3 g(static_cast<unsigned>(blocks));
  const IT* a = static_cast<const IT*>(src);
  IT* d = static_cast<IT*>(dst);
  const NdAxis &X = P.ax[0], &Y = P.ax[1];
  const bool same = X.x.c == Y.x.c && X.x.h == Y.x.h && X.x.a == Y.x.a &&
                    X.x.alpha == Y.x.alpha && X.x.delta == Y.x.delta && X.x.lambda == Y.x.lambda;
  if constexpr (NdSplit<POL>::value) {
    if (same) {
      tb_go<IT, POL, V, K, true>(g, a, d, P, M, nwaves, led, s);
      return hipGetLastError();
    }
  }
  tb_go<IT, POL, V, K, false>(g, a, d, P, M, nwaves, led, s);
  return hipGetLastError();
}

template <typename IT, int POL, int V>
hipError_t tb_by_k(int K, const void* src, void* dst, const NdParams& P, int rows,
                   long long* led, hipStream_t s) {
  switch (K) {
    case 1: return tb_launch<IT, POL, V, 1>(src, dst, P, rows, led, s);
    case 2: return tb_launch<IT, POL, V, 2>(src, dst, P, rows, led, s);
    case 4: return tb_launch<IT, POL, V, 4>(src, dst, P, rows, led, s);
    case 8: return tb_launch<IT, POL, V, 8>(src, dst, P, rows, led, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename IT, int POL>
hipError_t tb_by_vec(int vec, int K, const void* src, void* dst, const NdParams& P, int rows,
                     long long* led, hipStream_t s) {
  if (vec == 2) return tb_by_k<IT, POL, 2>(K, src, dst, P, rows, led, s);
  if constexpr (sizeof(IT) == 4) {
    if (vec == 4) return tb_by_k<IT, POL, 4>(K, src, dst, P, rows, led, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

bool nd_tb_valid(int itype, int pol, int vec, const NdParams& P) {
  if (P.dim != 2) return false;
  if (itype == FQNM_I32 ? (vec != 2 && vec != 4) : vec != 2) return false;
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
                     int rows, long long* led, hipStream_t s) {
  switch (pol) {
    case P_UPWIND_POS: return tb_by_vec<IT, P_UPWIND_POS>(vec, depth, src, dst, P, rows, led, s);
    case P_EO: return tb_by_vec<IT, P_EO>(vec, depth, src, dst, P, rows, led, s);
    case P_GODUNOV: return tb_by_vec<IT, P_GODUNOV>(vec, depth, src, dst, P, rows, led, s);
    case P_MURMAN_ROE: return tb_by_vec<IT, P_MURMAN_ROE>(vec, depth, src, dst, P, rows, led, s);
    case P_LF_LINEAR: return tb_by_vec<IT, P_LF_LINEAR>(vec, depth, src, dst, P, rows, led, s);
    case P_LF_BURGERS: return tb_by_vec<IT, P_LF_BURGERS>(vec, depth, src, dst, P, rows, led, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_nd_tb(int itype, int pol, int vec, int depth, int rows, const void* src,
                        void* dst, const NdParams& P, long long* d_ledger, hipStream_t s) {
  if (!nd_tb_valid(itype, pol, vec, P) || rows < 1 || nd_tb_step_depth(depth) != depth)
    return hipErrorInvalidValue;
  if (itype == FQNM_I32)
    return tb_by_pol<int32_t>(pol, vec, depth, src, dst, P, rows, d_ledger, s);
  return tb_by_pol<int64_t>(pol, vec, depth, src, dst, P, rows, d_ledger, s);
}

}  // namespace fqnm
