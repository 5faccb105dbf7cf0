// scalar.hip -- single-grid kernels of the scalar integer transfer update.
//
// One step of Sec. 2 (eq:update_rule_conservative_form) is two phases: form the
// interface count fluxes F_{i+1/2} = T(q_i, q_{i+1}), then q_i -= F_{i+1/2} - F_{i-1/2}
// (Sec. 2.4).  Both phases are fused here; F never touches memory.
//
// Data layout: a state is a dense array of n integers (int32 or int64) in HBM,
// 256-byte aligned, with a second array of the same size for ping-pong.  Each
// lane owns `V` consecutive cells (16-byte vector loads/stores), a wavefront
// owns 64*V consecutive cells, and the neighbour cells of a lane's first and
// last cell arrive from the adjacent lanes by cross-lane moves.
//
// k_stream : one step per pass over memory.  Algorithmic traffic per
//            cell-update: one state read + one state write (2*sizeof(IT) bytes).
// k_tblock : temporal blocking.  A wavefront loads 64*V cells (its tile plus a
//            halo of `khalo` cells on each side), advances them `ksteps` <= khalo
//            steps in registers (the valid region shrinks by one cell per side
//            per step), and stores the 64*V - 2*khalo interior cells.  Traffic
//            per pass is that of one step; the redundant halo work is
//            2*khalo/(64*V) of the tile.
//
// Boundaries (Sec. 2 grid; outflow by copied ghost cells):
//   periodic: tile positions outside [0, n) load the wrapped cell, so a tile
//             evolves a contiguous piece of the periodic extension.
//   outflow : F_{-1/2} = T(q_0, q_0), F_{n-1/2} = T(q_{n-1}, q_{n-1}).  In k_tblock
//             positions outside [0, n) are frozen (never updated) and the two
//             boundary interfaces are evaluated from the in-domain cell.  The
//             net boundary count F_{-1/2} - F_{n-1/2} of every step is added to a
//             device ledger, so sum(q) - sum(q0) == ledger exactly.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fqnm_internal.h"

namespace fqnm {

typedef int v4i __attribute__((ext_vector_type(4)));

template <typename IT, int V>
__device__ __forceinline__ void load_vec(const IT* __restrict__ p, IT (&q)[V]) {
  constexpr int PER = 16 / sizeof(IT);
  static_assert(V % PER == 0, "V must fill whole 16-byte vectors");
  const v4i* p4 = reinterpret_cast<const v4i*>(p);
#pragma unroll
  for (int c = 0; c < V / PER; ++c) {
    v4i v = p4[c];
    __builtin_memcpy(&q[c * PER], &v, 16);
  }
}

template <typename IT, int V>
__device__ __forceinline__ void store_vec(IT* __restrict__ p, const IT (&q)[V]) {
  constexpr int PER = 16 / sizeof(IT);
  v4i* p4 = reinterpret_cast<v4i*>(p);
#pragma unroll
  for (int c = 0; c < V / PER; ++c) {
    v4i v;
    __builtin_memcpy(&v, &q[c * PER], 16);
    p4[c] = v;
  }
}

// Ghost-cell index of position g for a one-step pass: periodic wrap or outflow copy.
__device__ __forceinline__ int64_t ghost_index(int64_t g, int64_t n, int bc) {
  if (g >= 0 && g < n) return g;
  return bc == FQNM_BC_PERIODIC ? wrap_index(g, n) : clamp_index(g, n);
}

// Split maps of one cell: {phi+(q), phi-(q)}; a single 8- or 16-byte table
// read in LUT mode.  For int32 states the read is a raw buffer load whose
// resource holds the table size, so the hardware range check returns zeros
// for any offset past the table instead of touching other memory; states of
// cells inside the domain never leave [lo, hi] (maximum principle), so only
// discarded halo lanes can ever be out of range.
struct LutView {
  __amdgpu_buffer_rsrc_t rsrc;
  uint32_t bias;  // -8*lo modulo 2^32
};

__device__ __forceinline__ LutView lut_view(const XParams& P) {
  LutView v;
  const int64_t bytes = (P.lut_last + 1) * 8;
  v.rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(P.lut), static_cast<short>(0),
                                             static_cast<int>(bytes), 0x00020000);
  v.bias = 0u - (static_cast<uint32_t>(P.lut_lo) << 3);
  return v;
}

template <typename IT, int POL>
__device__ __forceinline__ void cell_maps(const XParams& P, const LutView& L, IT q, IT& pp,
                                          IT& pm) {
  if constexpr (POL == P_LUT) {
    if constexpr (sizeof(IT) == 4) {
      // byte offset 8*(q - lo), in 32-bit wrapping arithmetic: one shift-add
      const uint32_t off = (static_cast<uint32_t>(q) << 3) + L.bias;
      const auto e = __builtin_amdgcn_raw_buffer_load_b64(L.rsrc, off, 0, 0);
      pp = static_cast<IT>(e[0]);
      pm = static_cast<IT>(e[1]);
    } else {
      using E = typename LutEntry<IT>::T;
      uint64_t i = static_cast<uint64_t>(q) - static_cast<uint64_t>(P.lut_lo);
      const uint64_t last = static_cast<uint64_t>(P.lut_last);
      i = i < last ? i : last;  // clamped: never outside the table
      const E e = static_cast<const E*>(P.lut)[i];
      pp = static_cast<IT>(e.x);
      pm = static_cast<IT>(e.y);
    }
  } else {
    split_maps<IT, POL>(P, q, pp, pm);
  }
}

// A wavefront-private slice of the int32 table in LDS: entries for states
// [lo, lo + last].  Indices are clamped into the slice, so a discarded halo
// lane holding any value reads inside it.
constexpr int TB_WIN = 512;

typedef __attribute__((address_space(3))) int2 lds_int2;
typedef __attribute__((address_space(3))) const uint64_t lds_u64;

struct LdsWindow {
  uint32_t bias;  // LDS byte address of the slice minus 8*lo, modulo 2^32
  uint32_t end;   // LDS byte address of the slice's last entry
};

template <typename IT, int POL, bool WIN>
__device__ __forceinline__ void cell_maps_w(const XParams& P, const LutView& L,
                                            const LdsWindow& Wn, IT q, IT& pp, IT& pm) {
  if constexpr (WIN) {
    // LDS byte address of entry q: one shift-add, then one unsigned min.  A
    // state past the slice clamps to its last entry; one below it lands lower
    // in this workgroup's LDS (or wraps high and clamps): always inside the
    // allocation, and only discarded halo lanes can hold such states.
    uint32_t a = (static_cast<uint32_t>(q) << 3) + Wn.bias;
    a = a < Wn.end ? a : Wn.end;
    const uint64_t e = *(lds_u64*)(static_cast<uintptr_t>(a));
    pp = static_cast<IT>(static_cast<int32_t>(static_cast<uint32_t>(e)));
    pm = static_cast<IT>(static_cast<int32_t>(static_cast<uint32_t>(e >> 32)));
  } else {
    cell_maps<IT, POL>(P, L, q, pp, pm);
  }
}

// ---------------------------------------------------------------------------
// K1: one step per pass.
// ---------------------------------------------------------------------------
template <typename IT, int POL, int V>
__global__ __launch_bounds__(256) void k_stream(const IT* __restrict__ src, IT* __restrict__ dst,
                                                int64_t n, int bc, XParams P,
                                                long long* __restrict__ ledger) {
  const int lane = threadIdx.x & 63;
  const int64_t blk = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t base = (blk * 256 + threadIdx.x) * V;
  const bool full = base + V <= n;
  IT q[V];
  if (full) {
    load_vec<IT, V>(src + base, q);
  } else {
#pragma unroll
    for (int j = 0; j < V; ++j) q[j] = src[ghost_index(base + j, n, bc)];
  }
  IT F[V];
  IT Fl;
  if constexpr (IsSplit<POL>::value) {
    const LutView L = lut_view(P);
    IT pp[V], pm[V];
#pragma unroll
    for (int j = 0; j < V; ++j) cell_maps<IT, POL>(P, L, q[j], pp[j], pm[j]);
    IT pmn = lane_from_next<IT>(pm[0]);
    if (lane == 63) {
      IT a, b;
      cell_maps<IT, POL>(P, L, src[ghost_index(base + V, n, bc)], a, b);
      pmn = b;
    }
#pragma unroll
    for (int j = 0; j < V; ++j) F[j] = pp[j] + (j + 1 < V ? pm[j + 1] : pmn);
    Fl = lane_from_prev<IT>(F[V - 1]);
    if (lane == 0) {
      IT a, b;
      cell_maps<IT, POL>(P, L, src[ghost_index(base - 1, n, bc)], a, b);
      Fl = a + pm[0];
    }
  } else {
    IT qn = lane_from_next<IT>(q[0]);
    if (lane == 63) qn = src[ghost_index(base + V, n, bc)];
#pragma unroll
    for (int j = 0; j < V; ++j) F[j] = transfer<IT, POL>(P, q[j], j + 1 < V ? q[j + 1] : qn);
    Fl = lane_from_prev<IT>(F[V - 1]);
    if (lane == 0) Fl = transfer<IT, POL>(P, src[ghost_index(base - 1, n, bc)], q[0]);
  }
  IT out[V];
  out[0] = wsub<IT>(q[0], wsub<IT>(F[0], Fl));
#pragma unroll
  for (int j = 1; j < V; ++j) out[j] = wsub<IT>(q[j], wsub<IT>(F[j], F[j - 1]));
  if (full) {
    store_vec<IT, V>(dst + base, out);
  } else {
#pragma unroll
    for (int j = 0; j < V; ++j)
      if (base + j < n) dst[base + j] = out[j];
  }
  if (bc == FQNM_BC_OUTFLOW) {
    long long led = 0;
    if (base == 0) led += static_cast<long long>(Fl);
    if (base <= n - 1 && n - 1 < base + V) {
#pragma unroll
      for (int j = 0; j < V; ++j)
        if (base + j == n - 1) led -= static_cast<long long>(F[j]);
    }
    if (led != 0) atomicAdd(reinterpret_cast<unsigned long long*>(ledger),
                            static_cast<unsigned long long>(led));
  }
}

// ---------------------------------------------------------------------------
// K2: temporal blocking in registers, lane-contiguous cells.
// ---------------------------------------------------------------------------
// Interface fluxes of one step for the cells q[0..V) of every lane; the last
// interface of a lane needs the next lane's first cell, the first cell's left
// interface arrives from the previous lane.  With `edge` the outflow rules of
// the domain ends apply at global positions g0+j (frozen outside [0, n)), and
// the transfers across the two ends go to the ledger from the tiles that hold
// cell 0 (own_left) and cell n-1 (own_right) only: a pass deeper than a tile
// is wide reaches an end from several windows.
template <typename IT, int POL, int V, bool EDGE, bool WIN = false>
__device__ __forceinline__ void tb_step(const XParams& P, const LutView& L, const LdsWindow& Wn,
                                        IT (&q)[V], int64_t g0, int64_t n, bool own_left,
                                        bool own_right, long long& led) {
  IT F[V];
  if constexpr (IsSplit<POL>::value) {
    IT pp[V], pm[V];
#pragma unroll
    for (int j = 0; j < V; ++j) cell_maps_w<IT, POL, WIN>(P, L, Wn, q[j], pp[j], pm[j]);
    const IT pmn = lane_from_next<IT>(pm[0]);
    if constexpr (!EDGE) {
#pragma unroll
      for (int j = 0; j < V; ++j) F[j] = pp[j] + (j + 1 < V ? pm[j + 1] : pmn);
    } else {
      const IT ppn = lane_from_next<IT>(pp[0]);
#pragma unroll
      for (int j = 0; j < V; ++j) {
        const int64_t g = g0 + j;
        const IT ppR = j + 1 < V ? pp[j + 1] : ppn;
        const IT pmR = j + 1 < V ? pm[j + 1] : pmn;
        IT f = pp[j] + pmR;
        if (g == -1) f = ppR + pmR;        // F_{-1/2} = T(q_0, q_0)
        if (g == n - 1) f = pp[j] + pm[j]; // F_{n-1/2} = T(q_{n-1}, q_{n-1})
        F[j] = f;
        if (g == -1 && own_left) led += static_cast<long long>(f);
        if (g == n - 1 && own_right) led -= static_cast<long long>(f);
      }
    }
  } else {
    const IT qn = lane_from_next<IT>(q[0]);
#pragma unroll
    for (int j = 0; j < V; ++j) {
      IT qL = q[j];
      IT qR = j + 1 < V ? q[j + 1] : qn;
      if constexpr (EDGE) {
        const int64_t g = g0 + j;
        if (g == -1) qL = qR;
        if (g == n - 1) qR = qL;
        F[j] = transfer<IT, POL>(P, qL, qR);
        if (g == -1 && own_left) led += static_cast<long long>(F[j]);
        if (g == n - 1 && own_right) led -= static_cast<long long>(F[j]);
      } else {
        F[j] = transfer<IT, POL>(P, qL, qR);
      }
    }
  }
  const IT Fl = lane_from_prev<IT>(F[V - 1]);
#pragma unroll
  for (int j = 0; j < V; ++j) {
    const IT d = wsub<IT>(F[j], j == 0 ? Fl : F[j - 1]);
    if constexpr (EDGE) {
      const int64_t g = g0 + j;
      if (g >= 0 && g < n) q[j] = wsub<IT>(q[j], d);
    } else {
      q[j] = wsub<IT>(q[j], d);
    }
  }
}

// Wavefront shifts by one lane that fill the end lane with 0 (lane l receives
// lane l+1, or lane l-1).  Used where both end cells of the tile are halo, so
// their values are never stored; the zero fill lets the compiler fold the
// move into the add or subtract that consumes it.
__device__ __forceinline__ uint32_t tb_from_next_z(uint32_t v) {
  return static_cast<uint32_t>(
      __builtin_amdgcn_mov_dpp(static_cast<int>(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ uint32_t tb_from_prev_z(uint32_t v) {
  return static_cast<uint32_t>(
      __builtin_amdgcn_mov_dpp(static_cast<int>(v), 0x138, 0xf, 0xf, true));
}

// One step of a tile whose cells are held as their table addresses in the
// wavefront's LDS slice: a = base + 8*(q - lo).  The update q - (F - F_left)
// becomes a + 8*(F_left - F), so a step costs one clamp, one LDS read, one
// add, one subtraction and one shift-add per cell.  The clamp keeps every
// read inside the slice; in-domain cells never need it (maximum principle),
// only discarded halo lanes can drift.  Int32 tables, interior tiles.
template <int V>
__device__ __forceinline__ void tb_step_addr(uint32_t (&a)[V], uint32_t end) {
  uint32_t pp[V], pm[V];
#pragma unroll
  for (int j = 0; j < V; ++j) {
    const uint32_t x = a[j] < end ? a[j] : end;
    const uint64_t e = *(lds_u64*)(static_cast<uintptr_t>(x));
    pp[j] = static_cast<uint32_t>(e);
    pm[j] = static_cast<uint32_t>(e >> 32);
  }
  uint32_t F[V];
#pragma unroll
  for (int j = 0; j < V; ++j) F[j] = (j + 1 < V ? pm[j + 1] : tb_from_next_z(pm[0])) + pp[j];
  const uint32_t Fl = tb_from_prev_z(F[V - 1]);
#pragma unroll
  for (int j = 0; j < V; ++j) a[j] += ((j == 0 ? Fl : F[j - 1]) - F[j]) << 3;
}

// ksteps upwind steps of a plain window of 64-bit states, carried as exact
// doubles.  With B = 1.5*2^52, fb = (c*x) + B is B + rint(c*x) exactly (the
// same two roundings as the integer path, |c*x| < 2^51), the difference of
// two such values is the exact integer flux difference, and x minus it is the
// exact new state (states are validated below 2^51 in magnitude and the
// upwind update keeps them in their initial range).  Four FP64 operations per
// cell and step replace the per-step conversions and 64-bit integer
// arithmetic; the states are converted once per pass in each direction.
template <int POL, int V>
__device__ __forceinline__ void tb_steps_upwind_f64(double c, int64_t (&q)[V], int ksteps) {
  double x[V];
#pragma unroll
  for (int j = 0; j < V; ++j) x[j] = as_f64<int64_t>(q[j]);
  for (int s = 0; s < ksteps; ++s) {
    double fb[V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const double y = c * x[j];
      fb[j] = y + F64_BIAS;
    }
    if constexpr (POL == P_UPWIND_POS) {  // F_{j+1/2} = rint(c q_j)
      const double fl = lane_from_prev<double>(fb[V - 1]);
#pragma unroll
      for (int j = 0; j < V; ++j) x[j] = x[j] - (fb[j] - (j == 0 ? fl : fb[j - 1]));
    } else {  // F_{j+1/2} = rint(c q_{j+1})
      const double fn = lane_from_next<double>(fb[0]);
#pragma unroll
      for (int j = 0; j < V; ++j) x[j] = x[j] - ((j + 1 < V ? fb[j + 1] : fn) - fb[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < V; ++j) q[j] = round_to<int64_t>(x[j]);
}

// One step in the update's per-cell form.  Regrouping the telescoping sum by
// cell (Sec. 2.3), the new state is g(q_i) + phi+(q_{i-1}) - phi-(q_{i+1}) with
// g(q) = q - phi+(q) + phi-(q), exactly in integers.  For a certified table
// (XParams lut_mono) the wavefront's slice holds, for each state q of
// [lo, lo + span], the pair
//   x: the slice address of g(q) + phi+(lo) - phi-(lo),
//   y: 8*(phi+(q) - phi+(lo)) in the low half, 8*(phi-(lo) - phi-(q)) in the
//      high half,
// both halves in [0, 8*span]: the certificate bounds each map's change
// between consecutive states by one.  A step is one LDS read and two
// instructions per cell, plus one cross-lane move for each of a lane's two
// end cells.  The zero-filled moves make a missing neighbour at the window's
// ends read as state lo; the certified update is non-decreasing in each of
// its three states and fixes constant states, so every state stays in
// [lo, lo + span] and no read leaves the slice.  The ends' wrong values are
// halo and reach the stored interior no sooner than the clamped step's.
template <int V>
__device__ __forceinline__ void tb_step_addr3(uint32_t (&a)[V]) {
  uint32_t G[V], O[V];
#pragma unroll
  for (int j = 0; j < V; ++j) {
    const uint64_t e = *(lds_u64*)(static_cast<uintptr_t>(a[j]));
    G[j] = static_cast<uint32_t>(e);
    O[j] = static_cast<uint32_t>(e >> 32);
  }
  const uint32_t Ol = tb_from_prev_z(O[V - 1]), On = tb_from_next_z(O[0]);
#pragma unroll
  for (int j = 0; j < V; ++j) {
    const uint32_t left = j == 0 ? Ol : O[j - 1], right = j + 1 < V ? O[j + 1] : On;
    // G + low half of left + high half of right: one bit-field insert and one
    // sum of 16-bit halves, in place of two extractions and a 3-way add
    a[j] = __builtin_amdgcn_sad_u16((left & 0xffffu) | (right & 0xffff0000u), 0u, G[j]);
  }
}

// ksteps steps of a wavefront window with no LDS table slice.
template <typename IT, int POL, int V>
__device__ __forceinline__ void tb_steps_direct(const XParams& P, const LutView& L, IT (&q)[V],
                                                int64_t g0, int64_t n, bool plain, bool own_left,
                                                bool own_right, int ksteps, long long& led) {
  const LdsWindow Wn{0u, 0u};
  if constexpr (sizeof(IT) == 8 && (POL == P_UPWIND_POS || POL == P_UPWIND_NEG)) {
    if (plain) {
      tb_steps_upwind_f64<POL, V>(P.c, q, ksteps);
      return;
    }
  }
  if (plain) {
    for (int s = 0; s < ksteps; ++s)
      tb_step<IT, POL, V, false>(P, L, Wn, q, g0, n, false, false, led);
  } else {
    for (int s = 0; s < ksteps; ++s)
      tb_step<IT, POL, V, true>(P, L, Wn, q, g0, n, own_left, own_right, led);
  }
}

// One wavefront's pass over tile `tile` of a grid (the body of K2, shared
// with the batch's tiled work items): load the window, advance it ksteps
// steps, store the tile interior, add the boundary counts to the ledger.
template <typename IT, int POL, int V>
__device__ __forceinline__ void tblock_tile(const IT* __restrict__ src, IT* __restrict__ dst,
                                            int64_t n, int bc, int ksteps, int khalo, int64_t tile,
                                            const XParams& P, long long* __restrict__ ledger,
                                            int wave, int lane) {
  const int64_t T = 64 * V - 2 * khalo;
  const int64_t tstart = tile * T;
  const int64_t wstart = tstart - khalo;
  const int64_t g0 = wstart + static_cast<int64_t>(lane) * V;
  const bool inside = wstart >= 0 && wstart + 64 * V <= n;  // wavefront-uniform
  IT q[V];
  if (inside) {
    load_vec<IT, V>(src + g0, q);
  } else {
#pragma unroll
    for (int j = 0; j < V; ++j) q[j] = src[ghost_index(g0 + j, n, bc)];
  }
  long long led = 0;
  const LutView L = lut_view(P);
  const bool plain = inside || bc == FQNM_BC_PERIODIC;
  // the tiles holding cells 0 and n-1 count the boundary transfers (with
  // passes deeper than a tile is wide, other windows reach past the ends too)
  const bool own_left = tstart == 0;
  const bool own_right = tstart <= n - 1 && n - 1 < tstart + T;
  bool done = false;
  if constexpr (POL == P_LUT && sizeof(IT) == 4) {
    // Every in-domain state of this tile stays inside the tile's initial
    // range for the whole launch (each update is a monotone function of its
    // three-cell stencil), so that slice of the table is all it reads.
    __shared__ int2 s_win[4][TB_WIN];
    int32_t mn = static_cast<int32_t>(q[0]), mx = mn;
#pragma unroll
    for (int j = 1; j < V; ++j) {
      mn = q[j] < mn ? static_cast<int32_t>(q[j]) : mn;
      mx = q[j] > mx ? static_cast<int32_t>(q[j]) : mx;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const int32_t a = __shfl_xor(mn, off, 64), b = __shfl_xor(mx, off, 64);
      mn = a < mn ? a : mn;
      mx = b > mx ? b : mx;
    }
    const int64_t span = static_cast<int64_t>(mx) - mn;
    if (span < TB_WIN) {  // wavefront-uniform
      int2* w = s_win[wave];
      const uint32_t base =
          static_cast<uint32_t>(reinterpret_cast<uintptr_t>((lds_int2*)(w)));
      const uint32_t off0 = (static_cast<uint32_t>(mn) - static_cast<uint32_t>(P.lut_lo)) << 3;
      if (plain && P.lut_mono) {
        // the per-cell form's entries (tb_step_addr3), relative to state mn
        const auto e0 = __builtin_amdgcn_raw_buffer_load_b64(L.rsrc, off0, 0, 0);
        const uint32_t p0 = static_cast<uint32_t>(e0[0]), m0 = static_cast<uint32_t>(e0[1]);
        for (int i = lane; i <= span; i += 64) {
          const uint32_t off = off0 + (static_cast<uint32_t>(i) << 3);
          const auto e = __builtin_amdgcn_raw_buffer_load_b64(L.rsrc, off, 0, 0);
          const uint32_t pp = static_cast<uint32_t>(e[0]), pm = static_cast<uint32_t>(e[1]);
          // g(q) - mn + phi+(mn) - phi-(mn) with q = mn + i
          const uint32_t gr = static_cast<uint32_t>(i) - (pp - p0) - (m0 - pm);
          w[i] = make_int2(static_cast<int>(base + (gr << 3)),
                           static_cast<int>(((pp - p0) << 3) | (((m0 - pm) << 3) << 16)));
        }
      } else {
        for (int i = lane; i <= span; i += 64) {
          const uint32_t off = off0 + (static_cast<uint32_t>(i) << 3);
          const auto e = __builtin_amdgcn_raw_buffer_load_b64(L.rsrc, off, 0, 0);
          w[i] = make_int2(e[0], e[1]);
        }
      }
      // the slice written by some lanes is read by all lanes of this wavefront
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const LdsWindow Wn{base - (static_cast<uint32_t>(mn) << 3),
                         base + (static_cast<uint32_t>(span) << 3)};
      if (plain) {
        const uint32_t end = base + (static_cast<uint32_t>(span) << 3);
        uint32_t a[V];
#pragma unroll
        for (int j = 0; j < V; ++j)
          a[j] = base + ((static_cast<uint32_t>(q[j]) - static_cast<uint32_t>(mn)) << 3);
        if (P.lut_mono) {
          for (int s = 0; s < ksteps; ++s) tb_step_addr3<V>(a);
        } else {
          for (int s = 0; s < ksteps; ++s) tb_step_addr<V>(a, end);
        }
#pragma unroll
        for (int j = 0; j < V; ++j)
          q[j] = static_cast<IT>(static_cast<uint32_t>(mn) +
                                 static_cast<uint32_t>(static_cast<int32_t>(a[j] - base) >> 3));
      } else {
        for (int s = 0; s < ksteps; ++s)
          tb_step<IT, POL, V, true, true>(P, L, Wn, q, g0, n, own_left, own_right, led);
      }
      done = true;
    }
  }
  if (!done) {
    if constexpr (POL == P_LUT) {
      // The tile's states span more than the window (a shock inside it), or
      // the states are 64-bit (no LDS slice): the split maps the table was
      // built from give the same entries without a dependent L2 read on every
      // step.
      switch (P.lut_pol) {
        case P_UPWIND_POS:
          tb_steps_direct<IT, P_UPWIND_POS, V>(P, L, q, g0, n, plain, own_left, own_right,
                                               ksteps, led);
          break;
        case P_UPWIND_NEG:
          tb_steps_direct<IT, P_UPWIND_NEG, V>(P, L, q, g0, n, plain, own_left, own_right,
                                               ksteps, led);
          break;
        default:
          tb_steps_direct<IT, P_EO, V>(P, L, q, g0, n, plain, own_left, own_right,
                                       ksteps, led);
          break;
      }
    } else {
      tb_steps_direct<IT, POL, V>(P, L, q, g0, n, plain, own_left, own_right, ksteps, led);
    }
  }
  const int lane_lo = khalo / V, lane_hi = 64 - khalo / V;
  if (lane >= lane_lo && lane < lane_hi) {
    if (g0 + V <= n) {
      store_vec<IT, V>(dst + g0, q);
    } else {
#pragma unroll
      for (int j = 0; j < V; ++j)
        if (g0 + j < n) dst[g0 + j] = q[j];
    }
  }
  if (led != 0)
    atomicAdd(reinterpret_cast<unsigned long long*>(ledger), static_cast<unsigned long long>(led));
}

template <typename IT, int POL, int V>
__global__ __launch_bounds__(256) void k_tblock(const IT* __restrict__ src, IT* __restrict__ dst,
                                                int64_t n, int bc, int ksteps, int khalo,
                                                int64_t ntiles, XParams P,
                                                long long* __restrict__ ledger) {
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x) * 4 + wave;
  if (tile >= ntiles) return;  // the whole wavefront leaves together
  tblock_tile<IT, POL, V>(src, dst, n, bc, ksteps, khalo, tile, P, ledger, wave, lane);
}

// Tiled work items of many grids (the batch's instances outside the
// register-resident envelope): one launch runs one step block of every grid
// listed for it, one wavefront per (grid, tile) item, each item K2 on that
// tile for the grid's steps of this block.  The grids of a launch share the
// storage type, policy and cells per lane; each has its own buffers,
// constants and halo.  entries[e] covers the launch's items
// [entries[e].first, entries[e+1].first); a wavefront finds its entry by
// binary search (the same for every lane).  The launch boundary is the
// barrier between a grid's step blocks.
template <typename IT, int POL, int V>
__global__ __launch_bounds__(256) void k_tblock_items(const BlockGrid* __restrict__ entries,
                                                      int32_t nentries, int64_t nitems,
                                                      const TileGrid* __restrict__ grids) {
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t w = static_cast<int64_t>(blockIdx.x) * 4 + wave;
  if (w >= nitems) return;  // the whole wavefront leaves together
  int32_t lo = 0, hi = nentries - 1;  // last entry with first <= w
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (entries[mid].first <= w) lo = mid;
    else hi = mid - 1;
  }
  const BlockGrid e = entries[lo];
  const TileGrid& g = grids[e.grid];
  const IT* src = static_cast<const IT*>(e.parity ? g.buf1 : g.buf0);
  IT* dst = static_cast<IT*>(const_cast<void*>(e.parity ? g.buf0 : g.buf1));
  tblock_tile<IT, POL, V>(src, dst, g.n, g.bc, e.ksteps, g.khalo, w - e.first, g.P, g.ledger,
                          wave, lane);
}

// ---------------------------------------------------------------------------
// K10: persistent temporal blocking on periodic grids.  One launch runs every
// pass of a k_tblock-style plan (64*V positions per wavefront, `depth` steps
// per pass, a halo of `khalo` >= depth cells on each side), but a wavefront
// keeps its tile in registers from one pass to the next instead of storing
// it and ending the launch: between passes it hands the `khalo` cells at each
// end of its tile to its two neighbouring tiles through memory and takes
// theirs as its new halo.  Each exchanged cell is one 64-bit word holding the
// value and the pass it belongs to, written and read with relaxed
// device-scope atomics: the tag alone tells a reader that a word is the one
// it waits for, so no other ordering between the words is needed.  Two
// buffers alternate by pass parity; a tile can only overwrite a buffer again
// after both neighbours have read it (they need this tile's next exchange
// before they can produce theirs).
//
// Tiles: tile t holds the cells [s(t), s(t+1)), s(t) = floor(t*n/ntiles)
// rounded down to a multiple of V (s(ntiles) = n); the host checks that every
// tile holds between khalo and 64*V - 2*khalo cells.  At the start of a pass
// the window positions [0, 2*khalo + T) hold exact states (halo refreshed,
// tile interior carried over); the positions behind them are never read by
// the valid region and are reset to an in-range state.
//
// The launch is cooperative (every workgroup resident at once, checked by the
// host and by the runtime), and every wait is bounded: a wavefront that polls
// more than `spin` times raises the error flag, and every waiting wavefront
// leaves once it sees the flag, so the launch always ends; the host reports
// FQNM_ERR_DEVICE.  Int32 states, split or two-point policies, and table
// slices in LDS as in K2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t persist_tile_start(int64_t t, int64_t n, int64_t ntiles,
                                                      int V) {
  if (t >= ntiles) return n;
  const int64_t s = t * (n / ntiles) + (t * (n % ntiles)) / ntiles;
  return s & ~static_cast<int64_t>(V - 1);
}

__device__ __forceinline__ uint64_t persist_pack(int32_t v, uint32_t tag) {
  return (static_cast<uint64_t>(tag) << 32) | static_cast<uint32_t>(v);
}

template <int POL, int V>
__global__ __launch_bounds__(256) void k_persist(const int32_t* __restrict__ src,
                                                 int32_t* __restrict__ dst, int64_t n,
                                                 int nsteps, int depth, int khalo, int ntiles,
                                                 XParams P, uint64_t* __restrict__ exch,
                                                 uint32_t tag0, int* __restrict__ err, int spin) {
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x) * 4 + wave;
  if (tile >= ntiles) return;  // the whole wavefront leaves together
  const int64_t s0 = persist_tile_start(tile, n, ntiles, V);
  const int T = static_cast<int>(persist_tile_start(tile + 1, n, ntiles, V) - s0);
  const int64_t w = s0 - khalo;
  const int off0 = lane * V;
  int32_t q[V];
  if (w >= 0 && w + 64 * V <= n) {
    load_vec<int32_t, V>(src + w + off0, q);
  } else {
#pragma unroll
    for (int j = 0; j < V; ++j) q[j] = src[wrap_index(w + off0 + j, n)];
  }
  const LutView L = lut_view(P);
  const int lim = 2 * khalo + T;  // exact positions at the start of a pass
  const int64_t left = tile > 0 ? tile - 1 : ntiles - 1;
  const int64_t right = tile + 1 < ntiles ? tile + 1 : 0;
  __shared__ int2 s_win[4][TB_WIN];
  int32_t slo = 1, shi = 0;  // range of the staged table slice (empty)
  long long led = 0;
  bool failed = false;
  int done = 0;
  uint32_t pass = 0;
  while (done < nsteps) {
    const int ks = nsteps - done < depth ? nsteps - done : depth;
    // range of the exact positions; the ones behind take an in-range state
    int32_t mn = INT32_MAX, mx = INT32_MIN;
#pragma unroll
    for (int j = 0; j < V; ++j) {
      if (off0 + j < lim) {
        mn = q[j] < mn ? q[j] : mn;
        mx = q[j] > mx ? q[j] : mx;
      }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const int32_t a = __shfl_xor(mn, o, 64), b = __shfl_xor(mx, o, 64);
      mn = a < mn ? a : mn;
      mx = b > mx ? b : mx;
    }
#pragma unroll
    for (int j = 0; j < V; ++j)
      if (off0 + j >= lim) q[j] = mn;
    bool stepped = false;
    if constexpr (POL == P_LUT) {
      const int64_t span = static_cast<int64_t>(mx) - mn;
      if (span < TB_WIN) {  // wavefront-uniform
        int2* win = s_win[wave];
        if (mn < slo || mx > shi) {
          // restage: the slice of TB_WIN entries centred on the tile's range
          // (clamped to the table), so that later passes can reuse it
          int64_t lo = static_cast<int64_t>(mn) - (TB_WIN - 1 - span) / 2;
          const int64_t tlo = P.lut_lo, thi = P.lut_lo + P.lut_last;
          if (lo + TB_WIN - 1 > thi) lo = thi - (TB_WIN - 1);
          if (lo < tlo) lo = tlo;
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          const uint32_t off0 = (static_cast<uint32_t>(lo) - static_cast<uint32_t>(P.lut_lo)) << 3;
          if (P.lut_mono) {
            // the per-cell form's entries (tb_step_addr3), relative to state
            // lo; entries past the table's end are never reached
            const uint32_t wbase =
                static_cast<uint32_t>(reinterpret_cast<uintptr_t>((lds_int2*)(win)));
            const auto e0 = __builtin_amdgcn_raw_buffer_load_b64(L.rsrc, off0, 0, 0);
            const uint32_t p0 = static_cast<uint32_t>(e0[0]), m0 = static_cast<uint32_t>(e0[1]);
            for (int i = lane; i < TB_WIN; i += 64) {
              const auto e = __builtin_amdgcn_raw_buffer_load_b64(
                  L.rsrc, off0 + (static_cast<uint32_t>(i) << 3), 0, 0);
              const uint32_t pp = static_cast<uint32_t>(e[0]), pm = static_cast<uint32_t>(e[1]);
              const uint32_t gr = static_cast<uint32_t>(i) - (pp - p0) - (m0 - pm);
              win[i] = make_int2(static_cast<int>(wbase + (gr << 3)),
                                 static_cast<int>(((pp - p0) << 3) | (((m0 - pm) << 3) << 16)));
            }
          } else {
            for (int i = lane; i < TB_WIN; i += 64) {
              const auto e = __builtin_amdgcn_raw_buffer_load_b64(
                  L.rsrc, off0 + (static_cast<uint32_t>(i) << 3), 0, 0);
              win[i] = make_int2(e[0], e[1]);
            }
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          slo = static_cast<int32_t>(lo);
          shi = static_cast<int32_t>(lo + TB_WIN - 1);
        }
        const uint32_t base = static_cast<uint32_t>(reinterpret_cast<uintptr_t>((lds_int2*)(win)));
        const uint32_t end = base + (static_cast<uint32_t>(shi - slo) << 3);
        uint32_t a[V];
#pragma unroll
        for (int j = 0; j < V; ++j)
          a[j] = base + ((static_cast<uint32_t>(q[j]) - static_cast<uint32_t>(slo)) << 3);
        if (P.lut_mono) {
          for (int s = 0; s < ks; ++s) tb_step_addr3<V>(a);
        } else {
          for (int s = 0; s < ks; ++s) tb_step_addr<V>(a, end);
        }
#pragma unroll
        for (int j = 0; j < V; ++j)
          q[j] = static_cast<int32_t>(static_cast<uint32_t>(slo) +
                                      static_cast<uint32_t>(static_cast<int32_t>(a[j] - base) >> 3));
        stepped = true;
      }
    }
    if (!stepped) {
      if constexpr (POL == P_LUT) {
        switch (P.lut_pol) {
          case P_UPWIND_POS:
            tb_steps_direct<int32_t, P_UPWIND_POS, V>(P, L, q, w + off0, n, true, false, false,
                                                      ks, led);
            break;
          case P_UPWIND_NEG:
            tb_steps_direct<int32_t, P_UPWIND_NEG, V>(P, L, q, w + off0, n, true, false, false,
                                                      ks, led);
            break;
          default:
            tb_steps_direct<int32_t, P_EO, V>(P, L, q, w + off0, n, true, false, false, ks, led);
            break;
        }
      } else {
        tb_steps_direct<int32_t, POL, V>(P, L, q, w + off0, n, true, false, false, ks, led);
      }
    }
    done += ks;
    ++pass;
    if (done >= nsteps) break;
    // hand the first and last khalo cells of the tile to the neighbours and
    // take their cells as the new halo
    const uint32_t tag = tag0 + pass;
    const int64_t par = pass & 1;
    uint64_t* mine = exch + (par * ntiles + tile) * 2 * khalo;
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const int o = off0 + j;
      if (o >= khalo && o < 2 * khalo)
        __hip_atomic_store(mine + (o - khalo), persist_pack(q[j], tag), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      if (o >= T && o < T + khalo)
        __hip_atomic_store(mine + khalo + (o - T), persist_pack(q[j], tag), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    const uint64_t* from_left = exch + ((par * ntiles + left) * 2 + 1) * khalo;
    const uint64_t* from_right = exch + (par * ntiles + right) * 2 * khalo;
    uint32_t need = 0;  // bit j: cell j still waits for its word
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const int o = off0 + j;
      if (o < khalo || (o >= khalo + T && o < lim)) need |= 1u << j;
    }
    for (int it = 0;; ++it) {
#pragma unroll
      for (int j = 0; j < V; ++j) {
        if (need & (1u << j)) {
          const int o = off0 + j;
          const uint64_t* p = o < khalo ? from_left + o : from_right + (o - khalo - T);
          const uint64_t v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (static_cast<uint32_t>(v >> 32) == tag) {
            q[j] = static_cast<int32_t>(static_cast<uint32_t>(v));
            need &= ~(1u << j);
          }
        }
      }
      if (!__any(need != 0)) break;
      if ((it & 63) == 63) {
        const int e = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (e != 0 || it >= spin) {
          if (e == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          failed = true;
          break;
        }
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (failed) break;  // wavefront-uniform
  }
  if (failed) return;
#pragma unroll
  for (int j = 0; j < V; ++j) {
    const int o = off0 + j;
    if (o >= khalo && o < khalo + T) dst[s0 + (o - khalo)] = q[j];
  }
}

// ---------------------------------------------------------------------------
// K5: workgroup tiles with overlapping wavefront windows (int32 tables,
// periodic grids).  The NW wavefronts of a workgroup hold windows of 64*V
// cells that overlap their neighbours by 2*WG_H cells; every WG_H steps each
// wavefront refreshes the WG_H cells at each end of its window from the
// neighbour's cells that are still valid there (LDS, double-buffered, one
// barrier per refresh).  Only the workgroup's two outer ends pay the deep halo
// of `khalo` >= ksteps cells, so about 1 - 2*khalo/(NW*64*V) of the work is
// stored instead of 1 - 2*khalo/(64*V).  The table slice the tile can reach is
// shared by the workgroup; cells are carried as their slice addresses.
// ---------------------------------------------------------------------------
constexpr int WG_H = 8;       // refresh period, and half the overlap of two windows
constexpr int WG_WIN = 2048;  // table entries one workgroup can stage

template <int V>
__device__ __forceinline__ void wg_load(const int32_t* __restrict__ p, int32_t (&q)[V]) {
  if constexpr (V == 2) {
    typedef int v2 __attribute__((ext_vector_type(2)));
    const v2 v = *reinterpret_cast<const v2*>(p);
    q[0] = v[0];
    q[1] = v[1];
  } else {
    load_vec<int32_t, V>(p, q);
  }
}

template <int V, int NW>
__global__ __launch_bounds__(NW * 64) void k_tblock_wg(const int32_t* __restrict__ src,
                                                       int32_t* __restrict__ dst, int64_t n,
                                                       int ksteps, int khalo, XParams P) {
  constexpr int W = 64 * V;
  constexpr int WTOT = NW * W - (NW - 1) * 2 * WG_H;
  __shared__ int2 s_win[WG_WIN];
  __shared__ uint32_t s_xch[2][NW][2][WG_H];
  __shared__ int32_t s_mn[NW], s_mx[NW];
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int64_t TS = WTOT - 2 * khalo;  // cells stored per workgroup
  const int64_t S = xcd_tile(blockIdx.x, gridDim.x) * TS - khalo;
  const int64_t g0 = S + wave * (W - 2 * WG_H) + lane * V;
  const bool inside = S >= 0 && S + WTOT <= n;  // uniform over the workgroup
  int32_t q[V];
  if (inside) {
    wg_load<V>(src + g0, q);
  } else {
#pragma unroll
    for (int j = 0; j < V; ++j) q[j] = src[wrap_index(g0 + j, n)];
  }
  // range of the tile's initial states
  int32_t mn = q[0], mx = q[0];
#pragma unroll
  for (int j = 1; j < V; ++j) {
    mn = q[j] < mn ? q[j] : mn;
    mx = q[j] > mx ? q[j] : mx;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const int32_t a = __shfl_xor(mn, off, 64), b = __shfl_xor(mx, off, 64);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
  }
  if (lane == 0) {
    s_mn[wave] = mn;
    s_mx[wave] = mx;
  }
  __syncthreads();
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    mn = s_mn[w] < mn ? s_mn[w] : mn;
    mx = s_mx[w] > mx ? s_mx[w] : mx;
  }
  const int64_t span = static_cast<int64_t>(mx) - mn;
  const LutView L = lut_view(P);
  // Exchange the window ends with the neighbouring wavefronts: a wavefront
  // sends its cells at positions [WG_H, 2*WG_H) and [W - 2*WG_H, W - WG_H)
  // (position = lane*V + j) and receives [0, WG_H) and [W - WG_H, W).  The
  // buffer alternates between refreshes, so one barrier per refresh suffices.
  auto refresh = [&](auto (&x)[V], int par) {
    using T = typename std::remove_reference<decltype(x[0])>::type;
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const int p = lane * V + j;
      if (p >= WG_H && p < 2 * WG_H) s_xch[par][wave][0][p - WG_H] = static_cast<uint32_t>(x[j]);
      if (p >= W - 2 * WG_H && p < W - WG_H)
        s_xch[par][wave][1][p - (W - 2 * WG_H)] = static_cast<uint32_t>(x[j]);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const int p = lane * V + j;
      if (wave > 0 && p < WG_H) x[j] = static_cast<T>(s_xch[par][wave - 1][1][p]);
      if (wave < NW - 1 && p >= W - WG_H) x[j] = static_cast<T>(s_xch[par][wave + 1][0][p - (W - WG_H)]);
    }
  };
  if (span < WG_WIN) {  // uniform over the workgroup
    for (int i = threadIdx.x; i <= span; i += NW * 64) {
      const uint32_t off =
          (static_cast<uint32_t>(mn) + static_cast<uint32_t>(i) - static_cast<uint32_t>(P.lut_lo))
          << 3;
      const auto e = __builtin_amdgcn_raw_buffer_load_b64(L.rsrc, off, 0, 0);
      s_win[i] = make_int2(e[0], e[1]);
    }
    __syncthreads();
    const uint32_t base = static_cast<uint32_t>(reinterpret_cast<uintptr_t>((lds_int2*)(s_win)));
    const uint32_t end = base + (static_cast<uint32_t>(span) << 3);
    uint32_t a[V];
#pragma unroll
    for (int j = 0; j < V; ++j)
      a[j] = base + ((static_cast<uint32_t>(q[j]) - static_cast<uint32_t>(mn)) << 3);
    for (int s = 0; s < ksteps; ++s) {
      tb_step_addr<V>(a, end);
      if ((s + 1) % WG_H == 0 && s + 1 < ksteps) refresh(a, ((s + 1) / WG_H) & 1);
    }
#pragma unroll
    for (int j = 0; j < V; ++j)
      q[j] = static_cast<int32_t>(static_cast<uint32_t>(mn) +
                                  static_cast<uint32_t>(static_cast<int32_t>(a[j] - base) >> 3));
  } else {
    // The workgroup's states span more than the staged slice: the split maps
    // the table was built from give the same entries without a dependent L2
    // read on every step.  (The switch is uniform over the workgroup, so
    // every wavefront reaches the refresh barriers.)
    const LdsWindow Wn{0u, 0u};
    long long led = 0;
    auto run = [&](auto pol) {
      constexpr int PD = decltype(pol)::value;
      for (int s = 0; s < ksteps; ++s) {
        tb_step<int32_t, PD, V, false>(P, L, Wn, q, g0, n, false, false, led);
        if ((s + 1) % WG_H == 0 && s + 1 < ksteps) refresh(q, ((s + 1) / WG_H) & 1);
      }
    };
    switch (P.lut_pol) {
      case P_UPWIND_POS: run(std::integral_constant<int, P_UPWIND_POS>{}); break;
      case P_UPWIND_NEG: run(std::integral_constant<int, P_UPWIND_NEG>{}); break;
      default: run(std::integral_constant<int, P_EO>{}); break;
    }
  }
  // this wavefront's share of the stored cells
  const int lo_p = wave == 0 ? khalo : WG_H;
  const int hi_p = wave == NW - 1 ? W - khalo : W - WG_H;
#pragma unroll
  for (int j = 0; j < V; ++j) {
    const int p = lane * V + j;
    if (p >= lo_p && p < hi_p && g0 + j < n) dst[g0 + j] = q[j];
  }
}

// ---------------------------------------------------------------------------
// K4: temporal blocking with a workgroup tile.  The NW wavefronts of a
// workgroup hold one contiguous tile of NW*64*V cells (V per lane, lanes in
// order), so the halo is paid once per workgroup instead of once per
// wavefront.  Each step every wavefront publishes its first and last cell in
// LDS (double buffered by step parity, one barrier per step); the edge lanes
// evaluate the one extra map or transfer they need from those cells.  For
// int32 tables the workgroup stages the slice of the table its tile can reach
// in LDS, as K2 does per wavefront.
// ---------------------------------------------------------------------------
constexpr int TBB_WIN = 2048;

template <typename IT, int POL, bool WIN>
__device__ __forceinline__ IT map_plus(const XParams& P, const LutView& L, const LdsWindow& Wn,
                                       IT q) {
  IT a, b;
  cell_maps_w<IT, POL, WIN>(P, L, Wn, q, a, b);
  return a;
}
template <typename IT, int POL, bool WIN>
__device__ __forceinline__ IT map_minus(const XParams& P, const LutView& L, const LdsWindow& Wn,
                                        IT q) {
  IT a, b;
  cell_maps_w<IT, POL, WIN>(P, L, Wn, q, a, b);
  return b;
}

// Edge cells of every wavefront, in LDS: [parity][first, last][wave].
template <typename IT>
using lds_ptr = __attribute__((address_space(3))) IT*;

template <typename IT, int POL, int V, int NW, bool EDGE, bool WIN>
__device__ __forceinline__ void blk_step(const XParams& P, const LutView& L, const LdsWindow& Wn,
                                         IT (&q)[V], lds_ptr<IT> s_edge, int s, int wave,
                                         int lane, int64_t g0, int64_t n, bool own_left,
                                         bool own_right, long long& led) {
  const int b = s & 1;
  if (lane == 0) s_edge[(b * 2 + 0) * NW + wave] = q[0];
  if (lane == 63) s_edge[(b * 2 + 1) * NW + wave] = q[V - 1];
  __syncthreads();
  // neighbours across wavefronts (the tile's two ends are halo and may hold anything)
  const IT q_next = (wave + 1 < NW) ? s_edge[(b * 2 + 0) * NW + wave + 1] : q[V - 1];
  const IT q_prev = (wave > 0) ? s_edge[(b * 2 + 1) * NW + wave - 1] : q[0];
  IT F[V];
  IT Fl;
  if constexpr (IsSplit<POL>::value) {
    IT pp[V], pm[V];
#pragma unroll
    for (int j = 0; j < V; ++j) cell_maps_w<IT, POL, WIN>(P, L, Wn, q[j], pp[j], pm[j]);
    IT pmn = lane_from_next<IT>(pm[0]);
    IT ppn = EDGE ? lane_from_next<IT>(pp[0]) : IT(0);
    if (lane == 63) {
      IT a, c;
      cell_maps_w<IT, POL, WIN>(P, L, Wn, q_next, a, c);
      pmn = c;
      ppn = a;
    }
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const IT pmR = j + 1 < V ? pm[j + 1] : pmn;
      IT f = pp[j] + pmR;
      if constexpr (EDGE) {
        const int64_t g = g0 + j;
        const IT ppR = j + 1 < V ? pp[j + 1] : ppn;
        if (g == -1) f = ppR + pmR;         // F_{-1/2} = T(q_0, q_0)
        if (g == n - 1) f = pp[j] + pm[j];  // F_{n-1/2} = T(q_{n-1}, q_{n-1})
        if (g == -1 && own_left) led += static_cast<long long>(f);
        if (g == n - 1 && own_right) led -= static_cast<long long>(f);
      }
      F[j] = f;
    }
    Fl = lane_from_prev<IT>(F[V - 1]);
    if (lane == 0) Fl = map_plus<IT, POL, WIN>(P, L, Wn, q_prev) + pm[0];
    if constexpr (EDGE) {
      // the interface in front of this lane's first cell, if it is F_{-1/2}
      if (lane == 0 && g0 - 1 == -1) Fl = pp[0] + pm[0];
    }
  } else {
    IT qn = lane_from_next<IT>(q[0]);
    if (lane == 63) qn = q_next;
#pragma unroll
    for (int j = 0; j < V; ++j) {
      IT qL = q[j];
      IT qR = j + 1 < V ? q[j + 1] : qn;
      if constexpr (EDGE) {
        const int64_t g = g0 + j;
        if (g == -1) qL = qR;
        if (g == n - 1) qR = qL;
        F[j] = transfer<IT, POL>(P, qL, qR);
        if (g == -1 && own_left) led += static_cast<long long>(F[j]);
        if (g == n - 1 && own_right) led -= static_cast<long long>(F[j]);
      } else {
        F[j] = transfer<IT, POL>(P, qL, qR);
      }
    }
    Fl = lane_from_prev<IT>(F[V - 1]);
    if (lane == 0) Fl = transfer<IT, POL>(P, q_prev, q[0]);
    if constexpr (EDGE) {
      if (lane == 0 && g0 - 1 == -1) Fl = transfer<IT, POL>(P, q[0], q[0]);
    }
  }
#pragma unroll
  for (int j = 0; j < V; ++j) {
    const IT d = wsub<IT>(F[j], j == 0 ? Fl : F[j - 1]);
    if constexpr (EDGE) {
      const int64_t g = g0 + j;
      if (g >= 0 && g < n) q[j] = wsub<IT>(q[j], d);
    } else {
      q[j] = wsub<IT>(q[j], d);
    }
  }
}

template <typename IT, int POL, int V, int NW>
__global__ __launch_bounds__(NW * 64) void k_tblock_blk(const IT* __restrict__ src,
                                                        IT* __restrict__ dst, int64_t n, int bc,
                                                        int ksteps, int khalo, int64_t ntiles,
                                                        XParams P,
                                                        long long* __restrict__ ledger) {
  __shared__ IT s_edge_mem[2 * 2 * NW];
  const lds_ptr<IT> s_edge = (lds_ptr<IT>)(s_edge_mem);
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= ntiles) return;  // uniform over the workgroup
  constexpr int PW = NW * 64 * V;
  const int64_t T = PW - 2 * khalo;
  const int64_t tstart = tile * T;
  const int64_t wstart = tstart - khalo;
  const int64_t g0 = wstart + static_cast<int64_t>(threadIdx.x) * V;
  const bool inside = wstart >= 0 && wstart + PW <= n;  // workgroup-uniform
  IT q[V];
  if (inside) {
    load_vec<IT, V>(src + g0, q);
  } else {
#pragma unroll
    for (int j = 0; j < V; ++j) q[j] = src[ghost_index(g0 + j, n, bc)];
  }
  long long led = 0;
  const LutView L = lut_view(P);
  const bool plain = inside || bc == FQNM_BC_PERIODIC;
  const bool own_left = tstart == 0;
  const bool own_right = tstart <= n - 1 && n - 1 < tstart + T;
  bool done = false;
  if constexpr (POL == P_LUT && sizeof(IT) == 4) {
    __shared__ int2 s_win[TBB_WIN];
    __shared__ int32_t s_mm[2][NW];
    int32_t mn = static_cast<int32_t>(q[0]), mx = mn;
#pragma unroll
    for (int j = 1; j < V; ++j) {
      mn = q[j] < mn ? static_cast<int32_t>(q[j]) : mn;
      mx = q[j] > mx ? static_cast<int32_t>(q[j]) : mx;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const int32_t a = __shfl_xor(mn, off, 64), c = __shfl_xor(mx, off, 64);
      mn = a < mn ? a : mn;
      mx = c > mx ? c : mx;
    }
    if (lane == 0) {
      s_mm[0][wave] = mn;
      s_mm[1][wave] = mx;
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      mn = s_mm[0][w] < mn ? s_mm[0][w] : mn;
      mx = s_mm[1][w] > mx ? s_mm[1][w] : mx;
    }
    const int64_t span = static_cast<int64_t>(mx) - mn;
    if (span < TBB_WIN) {  // workgroup-uniform
      for (int i = threadIdx.x; i <= span; i += NW * 64) {
        const uint32_t off = ((static_cast<uint32_t>(mn) + static_cast<uint32_t>(i)) << 3) + L.bias;
        const auto e = __builtin_amdgcn_raw_buffer_load_b64(L.rsrc, off, 0, 0);
        s_win[i] = make_int2(e[0], e[1]);
      }
      __syncthreads();
      const uint32_t base =
          static_cast<uint32_t>(reinterpret_cast<uintptr_t>((lds_int2*)(s_win)));
      const LdsWindow Wn{base - (static_cast<uint32_t>(mn) << 3),
                         base + (static_cast<uint32_t>(span) << 3)};
      if (plain) {
        for (int s = 0; s < ksteps; ++s)
          blk_step<IT, POL, V, NW, false, true>(P, L, Wn, q, s_edge, s, wave, lane, g0, n, false,
                                                false, led);
      } else {
        for (int s = 0; s < ksteps; ++s)
          blk_step<IT, POL, V, NW, true, true>(P, L, Wn, q, s_edge, s, wave, lane, g0, n,
                                               own_left, own_right, led);
      }
      done = true;
    }
  }
  if (!done) {
    const LdsWindow Wn{0u, 0u};
    auto run = [&](auto pol) {
      constexpr int PD = decltype(pol)::value;
      if (plain) {
        for (int s = 0; s < ksteps; ++s)
          blk_step<IT, PD, V, NW, false, false>(P, L, Wn, q, s_edge, s, wave, lane, g0, n, false,
                                                false, led);
      } else {
        for (int s = 0; s < ksteps; ++s)
          blk_step<IT, PD, V, NW, true, false>(P, L, Wn, q, s_edge, s, wave, lane, g0, n,
                                               own_left, own_right, led);
      }
    };
    if constexpr (POL == P_LUT) {
      // The tile's states span more than the staged slice, or the states are
      // 64-bit (no staged slice): the split maps the table was built from give
      // the same entries without a dependent L2 read on every step (the
      // switch is uniform over the workgroup, so every wavefront reaches the
      // per-step barriers).
      switch (P.lut_pol) {
        case P_UPWIND_POS: run(std::integral_constant<int, P_UPWIND_POS>{}); break;
        case P_UPWIND_NEG: run(std::integral_constant<int, P_UPWIND_NEG>{}); break;
        default: run(std::integral_constant<int, P_EO>{}); break;
      }
    } else {
      run(std::integral_constant<int, POL>{});
    }
  }
  const int lo_t = khalo / V, hi_t = NW * 64 - khalo / V;
  if (static_cast<int>(threadIdx.x) >= lo_t && static_cast<int>(threadIdx.x) < hi_t) {
    if (g0 + V <= n) {
      store_vec<IT, V>(dst + g0, q);
    } else {
#pragma unroll
      for (int j = 0; j < V; ++j)
        if (g0 + j < n) dst[g0 + j] = q[j];
    }
  }
  if (led != 0)
    atomicAdd(reinterpret_cast<unsigned long long*>(ledger), static_cast<unsigned long long>(led));
}

// ---------------------------------------------------------------------------
// K3: temporal blocking in registers, lane-interleaved cells (split kinds).
// Position p = j*64 + lane of the wavefront tile holds slot j of that lane, so
// a table read of slot j touches the maps of 64 consecutive cells (a few cache
// lines) instead of 64 cells spread V apart.  Every neighbour is one lane
// away: values move by a rotation of the wavefront (DPP), and the lane at the
// end of a slot takes the value rotated out of the adjacent slot.
// The halo is a whole number of slots (khalo % 64 == 0).
// ---------------------------------------------------------------------------
template <typename IT, int POL, int V, bool EDGE>
__device__ __forceinline__ void il_step(const XParams& P, const LutView& L, IT (&q)[V], int lane,
                                        int a_next,
                                        int a_prev, int64_t wstart, int64_t n, bool own_left,
                                        bool own_right,
                                        long long& led) {
  IT pp[V], pm[V], F[V];
#pragma unroll
  for (int j = 0; j < V; ++j) cell_maps<IT, POL>(P, L, q[j], pp[j], pm[j]);
  // pm of the right neighbour: lane l+1 of the same slot, or lane 0 of slot j+1
  IT rm[V];
#pragma unroll
  for (int j = 0; j < V; ++j) rm[j] = rotate_from_next<IT>(pm[j]);
  if constexpr (!EDGE) {
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const IT pmR = (lane == 63 && j + 1 < V) ? rm[j + 1] : rm[j];
      F[j] = pp[j] + pmR;
    }
  } else {
    IT rp[V];
#pragma unroll
    for (int j = 0; j < V; ++j) rp[j] = rotate_from_next<IT>(pp[j]);
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const int64_t g = wstart + j * 64 + lane;
      const IT pmR = (lane == 63 && j + 1 < V) ? rm[j + 1] : rm[j];
      const IT ppR = (lane == 63 && j + 1 < V) ? rp[j + 1] : rp[j];
      IT f = pp[j] + pmR;
      if (g == -1) f = ppR + pmR;
      if (g == n - 1) f = pp[j] + pm[j];
      F[j] = f;
      if (g == -1 && own_left) led += static_cast<long long>(f);
      if (g == n - 1 && own_right) led -= static_cast<long long>(f);
    }
  }
  // F of the left interface: lane l-1 of the same slot, or lane 63 of slot j-1
  IT rf[V];
#pragma unroll
  for (int j = 0; j < V; ++j) rf[j] = rotate_from_prev<IT>(F[j]);
#pragma unroll
  for (int j = 0; j < V; ++j) {
    const IT Fl = (lane == 0 && j > 0) ? rf[j - 1] : rf[j];
    const IT d = wsub<IT>(F[j], Fl);
    if constexpr (EDGE) {
      const int64_t g = wstart + j * 64 + lane;
      if (g >= 0 && g < n) q[j] = wsub<IT>(q[j], d);
    } else {
      q[j] = wsub<IT>(q[j], d);
    }
  }
}

template <typename IT, int POL, int V>
__global__ __launch_bounds__(256) void k_tblock_il(const IT* __restrict__ src,
                                                   IT* __restrict__ dst, int64_t n, int bc,
                                                   int ksteps, int khalo, int64_t ntiles,
                                                   XParams P, long long* __restrict__ ledger) {
  static_assert(IsSplit<POL>::value, "interleaved tiles serve split kinds");
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x) * 4 + wave;
  if (tile >= ntiles) return;
  const int64_t T = 64 * V - 2 * khalo;
  const int64_t tstart = tile * T;
  const int64_t wstart = tstart - khalo;
  const bool inside = wstart >= 0 && wstart + 64 * V <= n;
  IT q[V];
#pragma unroll
  for (int j = 0; j < V; ++j) {
    const int64_t g = wstart + j * 64 + lane;
    q[j] = src[inside ? g : ghost_index(g, n, bc)];
  }
  const int a_next = ((lane + 1) & 63) << 2;
  const int a_prev = ((lane + 63) & 63) << 2;
  const LutView L = lut_view(P);
  long long led = 0;
  if (inside || bc == FQNM_BC_PERIODIC) {
    for (int s = 0; s < ksteps; ++s)
      il_step<IT, POL, V, false>(P, L, q, lane, a_next, a_prev, wstart, n, false, false, led);
  } else {
    const bool own_left = tstart == 0;
    const bool own_right = tstart <= n - 1 && n - 1 < tstart + T;
    for (int s = 0; s < ksteps; ++s)
      il_step<IT, POL, V, true>(P, L, q, lane, a_next, a_prev, wstart, n, own_left, own_right,
                                led);
  }
  const int jlo = khalo / 64, jhi = V - khalo / 64;
#pragma unroll
  for (int j = 0; j < V; ++j) {
    const int64_t g = wstart + j * 64 + lane;
    if (j >= jlo && j < jhi && g < n) dst[g] = q[j];
  }
  if (led != 0)
    atomicAdd(reinterpret_cast<unsigned long long*>(ledger), static_cast<unsigned long long>(led));
}

// ---------------------------------------------------------------------------
// Off-loop kernels: LUT construction, quantisation, reconstruction, reduction.
// ---------------------------------------------------------------------------
// Builds the table {phi+(q), phi-(q)} for q in [lo, lo + count) and checks, for
// every pair of consecutive states, that phi+ does not decrease, phi- does not
// increase and g(q) = q - phi+(q) + phi-(q) does not decrease.  Then the
// update H(a, b, c) = g(b) + phi+(a) - phi-(c) of a cell b between a and c is
// non-decreasing in each argument and H(x, x, x) = x, so it lies between the
// least and the largest of a, b, c: the maximum principle holds exactly, for
// any three states of the table's range (Lemma cfl_monotone, checked on the
// rounded maps themselves).  A violation sets *violation to 1.
template <typename IT, int POL>
__global__ void k_lut_build(XParams P, typename LutEntry<IT>::T* __restrict__ lut, int64_t lo,
                            int64_t count, int* __restrict__ violation) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    IT q = static_cast<IT>(lo + i);
    typename LutEntry<IT>::T e;
    e.x = split_phi<IT, POL>(P, q, true);
    e.y = split_phi<IT, POL>(P, q, false);
    lut[i] = e;
    if (i + 1 < count) {
      const IT q1 = static_cast<IT>(lo + i + 1);
      const int64_t p0 = e.x, m0 = e.y;
      const int64_t p1 = split_phi<IT, POL>(P, q1, true);
      const int64_t m1 = split_phi<IT, POL>(P, q1, false);
      if (p1 < p0 || m1 > m0 || 1 - (p1 - p0) + (m1 - m0) < 0) *violation = 1;
    }
  }
}

// q_i = rint(u_i / delta) (eq:quantisation); IEEE division.  Values outside
// the storage range (or not exactly convertible to FP64) raise *err.
template <typename IT>
__global__ void k_quantise(const double* __restrict__ u, IT* __restrict__ q, int64_t n,
                           double delta, double lim, int* err) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double r = rint(u[i] / delta);
    bool ok = fabs(r) <= lim;
    if (!ok) atomicOr(err, 1);
    q[i] = ok ? static_cast<IT>(r) : IT(0);
  }
}

// u_i = delta * q_i (eq:reconstruction_operator).
template <typename IT>
__global__ void k_reconstruct(const IT* __restrict__ q, double* __restrict__ u, int64_t n,
                              double delta) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    u[i] = delta * static_cast<double>(q[i]);
}

constexpr int RED_THREADS = 256;
constexpr int64_t RED_CELLS_PER_BLOCK = 256 * 64;

// Exact sum (128-bit), min, max and total variation of one state: block b
// reduces cells [b*cpb, min((b+1)*cpb, n)) into out[b].
template <typename IT>
__global__ __launch_bounds__(RED_THREADS) void k_reduce(const IT* __restrict__ q, int64_t n,
                                                        int periodic, int64_t cpb,
                                                        ReducePartial* __restrict__ out) {
  __shared__ __int128 s_sum[RED_THREADS];
  __shared__ __int128 s_tv[RED_THREADS];
  __shared__ int64_t s_min[RED_THREADS];
  __shared__ int64_t s_max[RED_THREADS];
  const int64_t b0 = blockIdx.x * cpb;
  const int64_t b1 = b0 + cpb < n ? b0 + cpb : n;
  __int128 sum = 0, tv = 0;
  int64_t mn = INT64_MAX, mx = INT64_MIN;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += RED_THREADS) {
    int64_t v = static_cast<int64_t>(q[i]);
    sum += v;
    mn = v < mn ? v : mn;
    mx = v > mx ? v : mx;
    int64_t w;
    bool has = true;
    if (i + 1 < n) w = static_cast<int64_t>(q[i + 1]);
    else if (periodic && n > 1) w = static_cast<int64_t>(q[0]);
    else { has = false; w = v; }
    if (has) {
      __int128 d = static_cast<__int128>(w) - v;
      tv += d < 0 ? -d : d;
    }
  }
  s_sum[threadIdx.x] = sum;
  s_tv[threadIdx.x] = tv;
  s_min[threadIdx.x] = mn;
  s_max[threadIdx.x] = mx;
  __syncthreads();
  for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s_sum[threadIdx.x] += s_sum[threadIdx.x + w];
      s_tv[threadIdx.x] += s_tv[threadIdx.x + w];
      s_min[threadIdx.x] = s_min[threadIdx.x + w] < s_min[threadIdx.x] ? s_min[threadIdx.x + w]
                                                                       : s_min[threadIdx.x];
      s_max[threadIdx.x] = s_max[threadIdx.x + w] > s_max[threadIdx.x] ? s_max[threadIdx.x + w]
                                                                       : s_max[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    ReducePartial r;
    r.sum_lo = static_cast<uint64_t>(s_sum[0]);
    r.sum_hi = static_cast<int64_t>(s_sum[0] >> 64);
    r.tv_lo = static_cast<uint64_t>(s_tv[0]);
    r.tv_hi = static_cast<int64_t>(s_tv[0] >> 64);
    r.qmin = s_min[0];
    r.qmax = s_max[0];
    out[blockIdx.x] = r;
  }
}

// Combines count >= 1 partial records into out[0] (one block; exact integer
// sums, so the order does not matter).
__global__ __launch_bounds__(RED_THREADS) void k_reduce_final(const ReducePartial* __restrict__ in,
                                                              int count,
                                                              ReducePartial* __restrict__ out) {
  __shared__ __int128 s_sum[RED_THREADS];
  __shared__ __int128 s_tv[RED_THREADS];
  __shared__ int64_t s_min[RED_THREADS];
  __shared__ int64_t s_max[RED_THREADS];
  __int128 sum = 0, tv = 0;
  int64_t mn = INT64_MAX, mx = INT64_MIN;
  for (int i = threadIdx.x; i < count; i += RED_THREADS) {
    const ReducePartial r = in[i];
    sum += (static_cast<__int128>(r.sum_hi) << 64) | r.sum_lo;
    tv += (static_cast<__int128>(r.tv_hi) << 64) | r.tv_lo;
    mn = r.qmin < mn ? r.qmin : mn;
    mx = r.qmax > mx ? r.qmax : mx;
  }
  s_sum[threadIdx.x] = sum;
  s_tv[threadIdx.x] = tv;
  s_min[threadIdx.x] = mn;
  s_max[threadIdx.x] = mx;
  __syncthreads();
  for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s_sum[threadIdx.x] += s_sum[threadIdx.x + w];
      s_tv[threadIdx.x] += s_tv[threadIdx.x + w];
      s_min[threadIdx.x] = s_min[threadIdx.x + w] < s_min[threadIdx.x] ? s_min[threadIdx.x + w]
                                                                       : s_min[threadIdx.x];
      s_max[threadIdx.x] = s_max[threadIdx.x + w] > s_max[threadIdx.x] ? s_max[threadIdx.x + w]
                                                                       : s_max[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    ReducePartial r;
    r.sum_lo = static_cast<uint64_t>(s_sum[0]);
    r.sum_hi = static_cast<int64_t>(s_sum[0] >> 64);
    r.tv_lo = static_cast<uint64_t>(s_tv[0]);
    r.tv_hi = static_cast<int64_t>(s_tv[0] >> 64);
    r.qmin = s_min[0];
    r.qmax = s_max[0];
    out[0] = r;
  }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
namespace {

template <typename IT, int POL, int V>
hipError_t do_launch(int kernel, const void* src, void* dst, int64_t n, int bc, int ksteps,
                     int khalo, const XParams& P, long long* d_ledger, hipStream_t s) {
  const IT* a = static_cast<const IT*>(src);
  IT* b = static_cast<IT*>(dst);
  if (kernel == K_STREAM) {
    const int64_t threads = (n + V - 1) / V;
    const int64_t blocks = (threads + 255) / 256;
    k_stream<IT, POL, V><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(a, b, n, bc, P, d_ledger);
  } else {
    const int64_t T = 64 * V - 2 * khalo;
    const int64_t ntiles = (n + T - 1) / T;
    const int64_t blocks = (ntiles + 3) / 4;
    if (kernel == K_TBLOCK) {
      k_tblock<IT, POL, V><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(a, b, n, bc, ksteps,
                                                                         khalo, ntiles, P, d_ledger);
    } else if (kernel == K_TBLOCK_B2 || kernel == K_TBLOCK_B4 || kernel == K_TBLOCK_B8) {
      const int nw = kernel == K_TBLOCK_B2 ? 2 : (kernel == K_TBLOCK_B4 ? 4 : 8);
      const int64_t Tb = int64_t(nw) * 64 * V - 2 * khalo;
      const int64_t nt = (n + Tb - 1) / Tb;
      if (nw == 2)
        k_tblock_blk<IT, POL, V, 2><<<dim3((unsigned)nt), dim3(128), 0, s>>>(a, b, n, bc, ksteps,
                                                                             khalo, nt, P, d_ledger);
      else if (nw == 4)
        k_tblock_blk<IT, POL, V, 4><<<dim3((unsigned)nt), dim3(256), 0, s>>>(a, b, n, bc, ksteps,
                                                                             khalo, nt, P, d_ledger);
      else
        k_tblock_blk<IT, POL, V, 8><<<dim3((unsigned)nt), dim3(512), 0, s>>>(a, b, n, bc, ksteps,
                                                                             khalo, nt, P, d_ledger);
    } else {
      if constexpr (IsSplit<POL>::value) {
        k_tblock_il<IT, POL, V><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(
            a, b, n, bc, ksteps, khalo, ntiles, P, d_ledger);
      } else {
        return hipErrorInvalidValue;
      }
    }
  }
  return hipGetLastError();
}

template <typename IT, int POL>
hipError_t by_vec(int kernel, int vec, const void* src, void* dst, int64_t n, int bc, int ksteps,
                  int khalo, const XParams& P, long long* d_ledger, hipStream_t s) {
  if constexpr (sizeof(IT) == 4) {
    switch (vec) {
      case 4: return do_launch<IT, POL, 4>(kernel, src, dst, n, bc, ksteps, khalo, P, d_ledger, s);
      case 8: return do_launch<IT, POL, 8>(kernel, src, dst, n, bc, ksteps, khalo, P, d_ledger, s);
      case 16: return do_launch<IT, POL, 16>(kernel, src, dst, n, bc, ksteps, khalo, P, d_ledger, s);
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (vec) {
      case 2: return do_launch<IT, POL, 2>(kernel, src, dst, n, bc, ksteps, khalo, P, d_ledger, s);
      case 4: return do_launch<IT, POL, 4>(kernel, src, dst, n, bc, ksteps, khalo, P, d_ledger, s);
      case 8: return do_launch<IT, POL, 8>(kernel, src, dst, n, bc, ksteps, khalo, P, d_ledger, s);
      case 16:
        // 64-bit upwind windows step as exact doubles (four FP64 operations
        // per cell and step), light enough on registers for 16 cells per lane
        if constexpr (POL == P_UPWIND_POS || POL == P_UPWIND_NEG) {
          if (kernel != K_TBLOCK) return hipErrorInvalidValue;
          const int64_t T = 64 * 16 - 2 * khalo;
          const int64_t ntiles = (n + T - 1) / T;
          k_tblock<IT, POL, 16><<<dim3((unsigned)((ntiles + 3) / 4)), dim3(256), 0, s>>>(
              static_cast<const IT*>(src), static_cast<IT*>(dst), n, bc, ksteps, khalo, ntiles,
              P, d_ledger);
          return hipGetLastError();
        }
        return hipErrorInvalidValue;
      default: return hipErrorInvalidValue;
    }
  }
}

template <typename IT>
hipError_t by_pol(int pol, int kernel, int vec, const void* src, void* dst, int64_t n, int bc,
                  int ksteps, int khalo, const XParams& P, long long* d_ledger, hipStream_t s) {
#define FQNM_POL_CASE(p) \
  case p: return by_vec<IT, p>(kernel, vec, src, dst, n, bc, ksteps, khalo, P, d_ledger, s);
  switch (pol) {
    FQNM_POL_CASE(P_UPWIND_POS)
    FQNM_POL_CASE(P_UPWIND_NEG)
    FQNM_POL_CASE(P_EO)
    FQNM_POL_CASE(P_GODUNOV)
    FQNM_POL_CASE(P_MURMAN_ROE)
    FQNM_POL_CASE(P_LF_LINEAR)
    FQNM_POL_CASE(P_LF_BURGERS)
    FQNM_POL_CASE(P_LUT)
    default: return hipErrorInvalidValue;
  }
#undef FQNM_POL_CASE
}

unsigned grid_for(int64_t n, int threads) {
  int64_t b = (n + threads - 1) / threads;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return static_cast<unsigned>(b);
}

}  // namespace

bool scalar_variant_available(int itype, int pol, int kernel, int vec) {
  if (pol < 0 || pol >= P_COUNT) return false;
  if (kernel < K_STREAM || kernel > K_TBLOCK_B8) return false;
  if (kernel == K_TBLOCK_IL && (pol == P_GODUNOV || pol == P_MURMAN_ROE)) return false;
  if (itype == FQNM_I32) return vec == 4 || vec == 8 || vec == 16;
  if (itype == FQNM_I64)
    return vec == 2 || vec == 4 || vec == 8 ||
           (vec == 16 && kernel == K_TBLOCK && (pol == P_UPWIND_POS || pol == P_UPWIND_NEG));
  return false;
}

int scalar_tile_positions(int kernel, int vec) {
  const int nw = kernel == K_TBLOCK_B2 ? 2 : (kernel == K_TBLOCK_B4 ? 4 : (kernel == K_TBLOCK_B8 ? 8 : 1));
  return nw * 64 * vec;
}

int scalar_halo(int kernel, int vec, int ksteps) {
  // whole halo lanes (lane-contiguous tiles) or whole halo slots (interleaved)
  const int unit = kernel == K_TBLOCK_IL ? 64 : vec;
  return ((ksteps + unit - 1) / unit) * unit;
}

hipError_t launch_scalar(int itype, int pol, int kernel, int vec, const void* src, void* dst,
                         int64_t n, int bc, int ksteps, int khalo, const XParams& P,
                         long long* d_ledger, hipStream_t s) {
  if (!scalar_variant_available(itype, pol, kernel, vec)) return hipErrorInvalidValue;
  if (kernel == K_STREAM && ksteps != 1) return hipErrorInvalidValue;
  if (kernel == K_TBLOCK && (khalo < ksteps || khalo % vec != 0 || 64 * vec - 2 * khalo <= 0))
    return hipErrorInvalidValue;
  if (kernel == K_TBLOCK_IL && (khalo < ksteps || khalo % 64 != 0 || 64 * vec - 2 * khalo <= 0))
    return hipErrorInvalidValue;
  if (kernel >= K_TBLOCK_B2 &&
      (khalo < ksteps || khalo % vec != 0 || scalar_tile_positions(kernel, vec) - 2 * khalo <= 0))
    return hipErrorInvalidValue;
  if (itype == FQNM_I32)
    return by_pol<int32_t>(pol, kernel, vec, src, dst, n, bc, ksteps, khalo, P, d_ledger, s);
  return by_pol<int64_t>(pol, kernel, vec, src, dst, n, bc, ksteps, khalo, P, d_ledger, s);
}

// ---------------------------------------------------------------------------
// Tiled work items of several grids (the batch).
// ---------------------------------------------------------------------------
namespace {
template <typename IT, int POL>
hipError_t items_by_vec(int vec, const BlockGrid* entries, int32_t nentries, int64_t nitems,
                        const TileGrid* grids, hipStream_t s) {
  const dim3 g(static_cast<unsigned>((nitems + 3) / 4)), b(256);
  if (vec == 4) k_tblock_items<IT, POL, 4><<<g, b, 0, s>>>(entries, nentries, nitems, grids);
  else if (vec == 8) k_tblock_items<IT, POL, 8><<<g, b, 0, s>>>(entries, nentries, nitems, grids);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}
}  // namespace

namespace {
__global__ void k_copy_words(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst,
                             int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}
}  // namespace

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
  if (bytes % 4 != 0) return hipErrorInvalidValue;
  const int64_t n = static_cast<int64_t>(bytes / 4);
  if (n == 0) return hipSuccess;
  k_copy_words<<<grid_for(n, 256), 256, 0, s>>>(static_cast<const uint32_t*>(src),
                                                static_cast<uint32_t*>(dst), n);
  return hipGetLastError();
}

bool items_variant_available(int itype, int pol, int vec) {
  return (vec == 4 || vec == 8) && pol >= 0 && pol < P_COUNT && (itype == FQNM_I32 || itype == FQNM_I64);
}

hipError_t launch_tile_items(int itype, int pol, int vec, const BlockGrid* entries,
                             int32_t nentries, int64_t nitems, const TileGrid* grids,
                             hipStream_t s) {
  if (nitems <= 0 || nentries <= 0) return hipSuccess;
  if (!items_variant_available(itype, pol, vec) || (nitems + 3) / 4 > INT32_MAX)
    return hipErrorInvalidValue;
#define FQNM_ITEMS_CASE(p)                                                                   \
  case p:                                                                                    \
    return itype == FQNM_I32 ? items_by_vec<int32_t, p>(vec, entries, nentries, nitems, grids, s) \
                             : items_by_vec<int64_t, p>(vec, entries, nentries, nitems, grids, s);
  switch (pol) {
    FQNM_ITEMS_CASE(P_UPWIND_POS)
    FQNM_ITEMS_CASE(P_UPWIND_NEG)
    FQNM_ITEMS_CASE(P_EO)
    FQNM_ITEMS_CASE(P_GODUNOV)
    FQNM_ITEMS_CASE(P_MURMAN_ROE)
    FQNM_ITEMS_CASE(P_LF_LINEAR)
    FQNM_ITEMS_CASE(P_LF_BURGERS)
    FQNM_ITEMS_CASE(P_LUT)
    default: return hipErrorInvalidValue;
  }
#undef FQNM_ITEMS_CASE
}

// ---------------------------------------------------------------------------
// Persistent temporal blocking (K_TBLOCK_PERSIST).
// ---------------------------------------------------------------------------
namespace {
template <int POL, int V>
const void* persist_fn() {
  return reinterpret_cast<const void*>(&k_persist<POL, V>);
}
const void* persist_kernel(int pol, int vec) {
#define FQNM_PERSIST_CASE(p)                                     \
  case p:                                                        \
    return vec == 4 ? persist_fn<p, 4>() : (vec == 8 ? persist_fn<p, 8>() : nullptr);
  switch (pol) {
    FQNM_PERSIST_CASE(P_LUT)
    FQNM_PERSIST_CASE(P_EO)
    FQNM_PERSIST_CASE(P_UPWIND_POS)
    FQNM_PERSIST_CASE(P_UPWIND_NEG)
    default: return nullptr;
  }
#undef FQNM_PERSIST_CASE
}
}  // namespace

bool persist_geometry(int64_t n, int vec, int depth, int* khalo, int64_t* ntiles) {
  if (vec != 4 && vec != 8) return false;
  if (depth < 1 || n < 1) return false;
  const int kh = scalar_halo(K_TBLOCK, vec, depth);
  const int64_t tmax = 64 * vec - 2 * kh - vec;
  if (tmax < kh) return false;
  const int64_t nt = (n + tmax - 1) / tmax;
  if (nt > INT32_MAX / 2) return false;
  // the smallest tile: floor(n/nt) rounded down to vec, minus up to vec
  if (n / nt - vec < kh) return false;
  *khalo = kh;
  *ntiles = nt;
  return true;
}

bool persist_available(int itype, int pol, int vec, int bc) {
  return itype == FQNM_I32 && bc == FQNM_BC_PERIODIC && persist_kernel(pol, vec) != nullptr;
}

hipError_t persist_fits(int pol, int vec, int64_t ntiles, bool* fits) {
  const void* f = persist_kernel(pol, vec);
  if (!f) return hipErrorInvalidValue;
  int per_cu = 0, dev = 0, cus = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, 256, 0);
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  *fits = (ntiles + 3) / 4 <= static_cast<int64_t>(per_cu) * cus;
  return hipSuccess;
}

hipError_t launch_persist(int pol, int vec, const int32_t* src, int32_t* dst, int64_t n,
                          int nsteps, int depth, const XParams& P, uint64_t* exch, uint32_t tag0,
                          int* err, int spin, hipStream_t s) {
  int khalo = 0;
  int64_t ntiles = 0;
  const void* f = persist_kernel(pol, vec);
  if (!f || !persist_geometry(n, vec, depth, &khalo, &ntiles)) return hipErrorInvalidValue;
  int nt32 = static_cast<int>(ntiles);
  XParams Pc = P;
  void* args[] = {const_cast<int32_t**>(&src), &dst, &n, &nsteps, &depth, &khalo, &nt32,
                  &Pc, &exch, &tag0, &err, &spin};
  const dim3 g(static_cast<unsigned>((ntiles + 3) / 4)), b(256);
  return hipLaunchCooperativeKernel(f, g, b, args, 0, s);
}

int tblock_wg_positions(int nw, int vec) { return nw * 64 * vec - (nw - 1) * 2 * WG_H; }

bool tblock_wg_valid(int nw, int vec, int ksteps) {
  if ((nw != 4 && nw != 8) || (vec != 2 && vec != 4) || ksteps < 1) return false;
  const int kh = scalar_halo(K_TBLOCK, vec, ksteps);
  return kh <= 64 * vec - 2 * WG_H && tblock_wg_positions(nw, vec) - 2 * kh > 0;
}

hipError_t launch_tblock_wg(int nw, int vec, const int32_t* src, int32_t* dst, int64_t n,
                            int ksteps, const XParams& P, hipStream_t s) {
  if (!tblock_wg_valid(nw, vec, ksteps)) return hipErrorInvalidValue;
  const int kh = scalar_halo(K_TBLOCK, vec, ksteps);
  const int64_t ts = tblock_wg_positions(nw, vec) - 2 * kh;
  const int64_t blocks = (n + ts - 1) / ts;
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  const dim3 g(static_cast<unsigned>(blocks));
  if (nw == 4 && vec == 2) k_tblock_wg<2, 4><<<g, 256, 0, s>>>(src, dst, n, ksteps, kh, P);
  else if (nw == 4) k_tblock_wg<4, 4><<<g, 256, 0, s>>>(src, dst, n, ksteps, kh, P);
  else if (vec == 2) k_tblock_wg<2, 8><<<g, 512, 0, s>>>(src, dst, n, ksteps, kh, P);
  else k_tblock_wg<4, 8><<<g, 512, 0, s>>>(src, dst, n, ksteps, kh, P);
  return hipGetLastError();
}

hipError_t launch_lut_build(int itype, int pol, const XParams& P, void* lut, int64_t lo,
                            int64_t count, int* violation, hipStream_t s) {
  const unsigned g = grid_for(count, 256);
#define FQNM_LUT_CASE(IT, p)                                                                 \
  case p:                                                                                    \
    k_lut_build<IT, p><<<g, 256, 0, s>>>(P, static_cast<typename LutEntry<IT>::T*>(lut), lo, \
                                         count, violation);                                  \
    return hipGetLastError();
  if (itype == FQNM_I32) {
    switch (pol) {
      FQNM_LUT_CASE(int32_t, P_UPWIND_POS)
      FQNM_LUT_CASE(int32_t, P_UPWIND_NEG)
      FQNM_LUT_CASE(int32_t, P_EO)
      default: return hipErrorInvalidValue;
    }
  }
  switch (pol) {
    FQNM_LUT_CASE(int64_t, P_UPWIND_POS)
    FQNM_LUT_CASE(int64_t, P_UPWIND_NEG)
    FQNM_LUT_CASE(int64_t, P_EO)
    default: return hipErrorInvalidValue;
  }
#undef FQNM_LUT_CASE
}

hipError_t launch_quantise(int itype, const double* u, void* q, int64_t n, double delta,
                           int* d_err, hipStream_t s) {
  const unsigned g = grid_for(n, 256);
  if (itype == FQNM_I32)
    k_quantise<int32_t><<<g, 256, 0, s>>>(u, static_cast<int32_t*>(q), n, delta, 2147483647.0,
                                          d_err);
  else
    k_quantise<int64_t><<<g, 256, 0, s>>>(u, static_cast<int64_t*>(q), n, delta,
                                          4503599627370495.0, d_err);
  return hipGetLastError();
}

hipError_t launch_reconstruct(int itype, const void* q, double* u, int64_t n, double delta,
                              hipStream_t s) {
  const unsigned g = grid_for(n, 256);
  if (itype == FQNM_I32)
    k_reconstruct<int32_t><<<g, 256, 0, s>>>(static_cast<const int32_t*>(q), u, n, delta);
  else
    k_reconstruct<int64_t><<<g, 256, 0, s>>>(static_cast<const int64_t*>(q), u, n, delta);
  return hipGetLastError();
}

int64_t reduce_blocks(int64_t n) { return (n + RED_CELLS_PER_BLOCK - 1) / RED_CELLS_PER_BLOCK; }

hipError_t launch_reduce(int itype, const void* q, int64_t n, int periodic, ReducePartial* out,
                         hipStream_t s) {
  return launch_reduce_cpb(itype, q, n, periodic, RED_CELLS_PER_BLOCK, out, s);
}

int64_t reduce_min_cells_per_block() { return RED_CELLS_PER_BLOCK; }

hipError_t launch_reduce_cpb(int itype, const void* q, int64_t n, int periodic, int64_t cpb,
                             ReducePartial* out, hipStream_t s) {
  if (cpb < 1) return hipErrorInvalidValue;
  const unsigned g = static_cast<unsigned>((n + cpb - 1) / cpb);
  if (itype == FQNM_I32)
    k_reduce<int32_t><<<g, RED_THREADS, 0, s>>>(static_cast<const int32_t*>(q), n, periodic, cpb,
                                                out);
  else
    k_reduce<int64_t><<<g, RED_THREADS, 0, s>>>(static_cast<const int64_t*>(q), n, periodic, cpb,
                                                out);
  return hipGetLastError();
}

hipError_t launch_reduce_final(const ReducePartial* in, int count, ReducePartial* out,
                               hipStream_t s) {
  if (count < 1) return hipErrorInvalidValue;
  k_reduce_final<<<1, RED_THREADS, 0, s>>>(in, count, out);
  return hipGetLastError();
}

}  // namespace fqnm
