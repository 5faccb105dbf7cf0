// levels.hip -- level statistics of an integer state (Supplementary Information).
//
// The entropy construction of the Supplementary Information counts how many
// cells sit on each quantised level k: c_k = #{i : q_i = k}, p_k = c_k/N
// (eq:pk_definition), S = -sum_k p_k log p_k (eq:discrete_entropy),
// N_eff = exp S (eq:neff); and, between two consecutive steps, the transition
// counts N_{k'k} = #{i : q_i^n = k, q_i^{n+1} = k'} (Definition
// level_transition) with the row-sum defect
// rho^n = max_k' |sum_k N_{k'k}/c_k - 1| (eq:empirical_M, Remark
// doubly_stochastic_condition), k' over the levels occupied after the step.
//
// Device side: levels are offset by the state's minimum and radix-sorted as
// unsigned keys of just the bits the range needs; a (k, k') pair packs into one
// 64-bit key (k - min k) << b' | (k' - min k') whenever the two ranges fit,
// else two stable sorts order the pairs by k' and then by k.  Run-length
// encoding gives the occupied levels / nonzero transitions.  Row sums of M are
// formed on the device, each by one thread adding its row's terms in
// increasing k, so the value is the same double a sequential sum in that order
// gives.  The entropy sum (one log per occupied level) runs on the host, in
// increasing level order.  A workspace is kept per context and grown on demand.
//
// The sort, the scans and the reductions are written here for the wavefront:
// a stable least-significant-digit radix sort with 8-bit digits, three
// kernels per digit (per-tile digit counts; an exclusive scan of the counts,
// digit-major, which gives every (digit, tile) its output offset; a stable
// scatter in which each wavefront ranks its 64 keys among equal digits with
// eight ballots, and the four wavefronts of a tile add up through LDS).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "runtime.h"

namespace fqnm {
namespace {

unsigned grid_of(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return static_cast<unsigned>(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

#define GRID_STRIDE(i, n)                                                   \
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (n); \
       i += (int64_t)gridDim.x * blockDim.x)

int bit_length(uint64_t r) { return r ? 64 - __builtin_clzll(r) : 0; }

// ---------------------------------------------------------------------------
// Exclusive (or inclusive) scan of int32 values.  A tile of TS = 256 x 16
// values per block: each thread adds its 16 consecutive values, the block
// scans the 256 thread sums, each thread writes its values' prefixes, and the
// tile total goes to a partials array; the partials are scanned the same way
// (recursively) and added back.
// ---------------------------------------------------------------------------
constexpr int SCAN_T = 256, SCAN_R = 16, SCAN_TILE = SCAN_T * SCAN_R;

__device__ __forceinline__ int32_t block_exclusive_sum(int32_t v, int32_t* s_wave, int32_t* total) {
  // wavefront inclusive scan by shifts, then the wavefronts' sums through LDS
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int32_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) s_wave[wave] = x;
  __syncthreads();
  int32_t before = 0, all = 0;
  for (int w = 0; w < SCAN_T / 64; ++w) {
    before += w < wave ? s_wave[w] : 0;
    all += s_wave[w];
  }
  *total = all;
  return before + x - v;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_tiles(const int32_t* __restrict__ in,
                                                       int32_t* __restrict__ out, int64_t n,
                                                       int32_t* __restrict__ partials,
                                                       int inclusive) {
  __shared__ int32_t s_wave[SCAN_T / 64];
  const int64_t base = blockIdx.x * static_cast<int64_t>(SCAN_TILE) + threadIdx.x * SCAN_R;
  int32_t v[SCAN_R];
  int32_t sum = 0;
#pragma unroll
  for (int r = 0; r < SCAN_R; ++r) {
    v[r] = base + r < n ? in[base + r] : 0;
    sum += v[r];
  }
  int32_t total = 0;
  int32_t run = block_exclusive_sum(sum, s_wave, &total);
#pragma unroll
  for (int r = 0; r < SCAN_R; ++r) {
    if (base + r < n) out[base + r] = inclusive ? run + v[r] : run;
    run += v[r];
  }
  if (threadIdx.x == 0 && partials) partials[blockIdx.x] = total;
}

__global__ void k_scan_add(int32_t* __restrict__ out, int64_t n,
                           const int32_t* __restrict__ tile_prefix) {
  GRID_STRIDE(i, n) out[i] += tile_prefix[i / SCAN_TILE];
}

// Scratch of a scan of n values: the partials of every level of the recursion.
size_t scan_scratch(int64_t n) {
  size_t t = 0;
  while (n > SCAN_TILE) {
    n = (n + SCAN_TILE - 1) / SCAN_TILE;
    t += 2 * static_cast<size_t>(n);
  }
  return t;
}

hipError_t scan_i32(const int32_t* in, int32_t* out, int64_t n, bool inclusive, int32_t* scratch,
                    hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
  int32_t* part = tiles > 1 ? scratch : nullptr;
  k_scan_tiles<<<static_cast<unsigned>(tiles), SCAN_T, 0, s>>>(in, out, n, part, inclusive ? 1 : 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || tiles == 1) return e;
  int32_t* pref = scratch + tiles;
  e = scan_i32(part, pref, tiles, false, scratch + 2 * tiles, s);
  if (e != hipSuccess) return e;
  k_scan_add<<<grid_of(n), 256, 0, s>>>(out, n, pref);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of 64-bit unsigned keys whose set bits are all below
// `bits`, carrying an optional value per key.  Tiles of ST = 256 x 16 keys,
// read in rounds of 256 consecutive keys (round r of tile b: keys
// b*ST + r*256 + thread), so rounds and threads follow the input order.
// ---------------------------------------------------------------------------
constexpr int RS_T = 256, RS_R = 16, RS_TILE = RS_T * RS_R, RS_D = 256;
static_assert(RS_T == RS_D, "one thread per digit in the count and scatter kernels");

__global__ __launch_bounds__(RS_T) void k_digit_counts(const uint64_t* __restrict__ keys,
                                                       int64_t n, int shift, int64_t ntiles,
                                                       int32_t* __restrict__ counts) {
  __shared__ int32_t s_cnt[RS_D];
  s_cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = blockIdx.x * static_cast<int64_t>(RS_TILE);
#pragma unroll
  for (int r = 0; r < RS_R; ++r) {
    const int64_t i = base + r * RS_T + threadIdx.x;
    if (i < n) atomicAdd(&s_cnt[(keys[i] >> shift) & (RS_D - 1)], 1);
  }
  __syncthreads();
  // digit-major: the scan of all counts is then each (digit, tile)'s offset
  counts[threadIdx.x * ntiles + blockIdx.x] = s_cnt[threadIdx.x];
}

template <typename VT, bool VALS>
__global__ __launch_bounds__(RS_T) void k_digit_scatter(const uint64_t* __restrict__ keys,
                                                        const VT* __restrict__ vals,
                                                        uint64_t* __restrict__ keys_out,
                                                        VT* __restrict__ vals_out, int64_t n,
                                                        int shift, int64_t ntiles,
                                                        const int32_t* __restrict__ offsets) {
  __shared__ int32_t s_run[RS_D];                // keys of each digit placed so far
  __shared__ int32_t s_wave[RS_T / 64][RS_D];    // this round's keys per wavefront and digit
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  s_run[t] = 0;
  for (int w = 0; w < RS_T / 64; ++w) s_wave[w][t] = 0;
  __syncthreads();
  const uint64_t below = (uint64_t(1) << lane) - 1;
  const int64_t base = blockIdx.x * static_cast<int64_t>(RS_TILE);
  for (int r = 0; r < RS_R; ++r) {
    const int64_t i = base + r * RS_T + t;
    const bool valid = i < n;
    const uint64_t key = valid ? keys[i] : 0;
    const int d = static_cast<int>((key >> shift) & (RS_D - 1));
    // lanes of this wavefront holding a key with the same digit
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const int rank = __popcll(peers & below);
    if (valid && rank == 0) s_wave[wave][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int32_t pos = s_run[d] + rank;
      for (int w = 0; w < wave; ++w) pos += s_wave[w][d];
      const int64_t o = static_cast<int64_t>(offsets[d * ntiles + blockIdx.x]) + pos;
      keys_out[o] = key;
      if constexpr (VALS) vals_out[o] = vals[i];
    }
    __syncthreads();
    int32_t add = 0;
    for (int w = 0; w < RS_T / 64; ++w) {
      add += s_wave[w][t];
      s_wave[w][t] = 0;
    }
    s_run[t] += add;
    __syncthreads();
  }
}

struct SortScratch {
  int32_t* counts;   // RS_D * ntiles
  int32_t* offsets;  // RS_D * ntiles
  int32_t* scan;     // scan_scratch(RS_D * ntiles)
};

int64_t sort_tiles(int64_t n) { return (n + RS_TILE - 1) / RS_TILE; }

// Sorts keys a (and values va) by their low `bits` bits, using b / vb as the
// other buffers of the passes; *in_b tells which buffer holds the result.
template <typename VT, bool VALS>
hipError_t radix_sort(uint64_t* a, uint64_t* b, VT* va, VT* vb, int64_t n, int bits,
                      const SortScratch& sc, hipStream_t s, bool* in_b) {
  *in_b = false;
  if (n <= 1 || bits <= 0) return hipSuccess;
  const int64_t ntiles = sort_tiles(n);
  for (int shift = 0; shift < bits; shift += 8) {
    k_digit_counts<<<static_cast<unsigned>(ntiles), RS_T, 0, s>>>(a, n, shift, ntiles, sc.counts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_i32(sc.counts, sc.offsets, RS_D * ntiles, false, sc.scan, s);
    if (e != hipSuccess) return e;
    k_digit_scatter<VT, VALS><<<static_cast<unsigned>(ntiles), RS_T, 0, s>>>(
        a, va, b, vb, n, shift, ntiles, sc.offsets);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    std::swap(a, b);
    std::swap(va, vb);
    *in_b = !*in_b;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Runs of equal keys in a sorted sequence (one or two key arrays), and the
// largest of n non-negative doubles.
// ---------------------------------------------------------------------------
__global__ void k_heads_u64(const uint64_t* __restrict__ k, const uint64_t* __restrict__ k2,
                            int32_t* __restrict__ head, int64_t n) {
  GRID_STRIDE(i, n)
  head[i] = (i == 0 || k[i] != k[i - 1] || (k2 && k2[i] != k2[i - 1])) ? 1 : 0;
}

__global__ void k_runs_u64(const uint64_t* __restrict__ k, const uint64_t* __restrict__ k2,
                           const int32_t* __restrict__ head, const int32_t* __restrict__ seg,
                           int64_t lo, int64_t lo2, int64_t* __restrict__ rk,
                           int64_t* __restrict__ rk2, int32_t* __restrict__ rstart, int64_t n) {
  GRID_STRIDE(i, n) {
    if (head[i]) {
      const int32_t r = seg[i];
      rk[r] = static_cast<int64_t>(k[i]) + lo;
      if (k2) rk2[r] = static_cast<int64_t>(k2[i]) + lo2;
      rstart[r] = static_cast<int32_t>(i);
    }
  }
}

__global__ __launch_bounds__(256) void k_max_partial(const double* __restrict__ v, int64_t n,
                                                     double* __restrict__ out) {
  __shared__ double s_m[256];
  double m = 0.0;
  GRID_STRIDE(i, n) m = v[i] > m ? v[i] : m;
  s_m[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w && s_m[threadIdx.x + w] > s_m[threadIdx.x])
      s_m[threadIdx.x] = s_m[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = s_m[0];
}

template <typename IT>
__global__ void k_widen(const IT* __restrict__ q, int64_t* __restrict__ out, int64_t n) {
  GRID_STRIDE(i, n) out[i] = static_cast<int64_t>(q[i]);
}

template <typename IT>
__global__ void k_offset_keys(const IT* __restrict__ q, int64_t lo, uint64_t* __restrict__ out,
                              int64_t n) {
  GRID_STRIDE(i, n) out[i] = static_cast<uint64_t>(static_cast<int64_t>(q[i]) - lo);
}

template <typename IT>
__global__ void k_pair_keys(const int64_t* __restrict__ k0, const IT* __restrict__ q1, int64_t lo0,
                            int64_t lo1, int b1, uint64_t* __restrict__ out, int64_t n) {
  GRID_STRIDE(i, n) {
    const uint64_t a = static_cast<uint64_t>(k0[i] - lo0);
    const uint64_t b = static_cast<uint64_t>(static_cast<int64_t>(q1[i]) - lo1);
    out[i] = (a << b1) | b;
  }
}

// Packed run keys (k - lo0) << b1 | (k' - lo1), back to the levels k and k'.
__global__ void k_unpack_runs(int64_t* __restrict__ rk, int64_t lo0, int64_t lo1, int b1,
                              int64_t* __restrict__ rk2, int64_t m) {
  const uint64_t mask = b1 <= 0 ? 0 : (b1 >= 64 ? ~uint64_t(0) : ~uint64_t(0) >> (64 - b1));
  GRID_STRIDE(r, m) {
    const uint64_t key = static_cast<uint64_t>(rk[r]);
    rk2[r] = static_cast<int64_t>(key & mask) + lo1;
    rk[r] = static_cast<int64_t>(b1 >= 64 ? 0 : key >> b1) + lo0;
  }
}

__global__ void k_run_counts(const int32_t* __restrict__ rstart, int32_t* __restrict__ cnt,
                             int64_t m, int64_t n) {
  GRID_STRIDE(r, m) cnt[r] = static_cast<int32_t>((r + 1 < m ? rstart[r + 1] : n) - rstart[r]);
}

// ---------------------------------------------------------------------------
// Direct level histogram, for states spanning a moderate range [lo, hi]: a
// block counts its HIST_CELLS cells in an LDS histogram over the block's own
// range when that fits (states of neighbouring cells are close), then adds
// its non-zero bins to the global histogram; otherwise it counts straight
// into the global histogram.  The non-zero bins, in increasing level order,
// are the levels; their bins the counts.
// ---------------------------------------------------------------------------
constexpr int HIST_T = 256, HIST_R = 16, HIST_CELLS = HIST_T * HIST_R, HIST_LDS = 8192;

template <typename IT>
__global__ __launch_bounds__(HIST_T) void k_hist(const IT* __restrict__ q, int64_t n, int64_t lo,
                                                 int32_t* __restrict__ hist) {
  __shared__ int32_t s_h[HIST_LDS];
  __shared__ int64_t s_mn[HIST_T / 64], s_mx[HIST_T / 64];
  const int64_t c0 = static_cast<int64_t>(blockIdx.x) * HIST_CELLS;
  const int64_t c1 = c0 + HIST_CELLS < n ? c0 + HIST_CELLS : n;
  int64_t v[HIST_R];
  int64_t mn = INT64_MAX, mx = INT64_MIN;
#pragma unroll
  for (int r = 0; r < HIST_R; ++r) {  // coalesced: consecutive threads, consecutive cells
    const int64_t i = c0 + r * HIST_T + threadIdx.x;
    v[r] = i < c1 ? static_cast<int64_t>(q[i]) - lo : -1;
    if (i < c1) {
      mn = v[r] < mn ? v[r] : mn;
      mx = v[r] > mx ? v[r] : mx;
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const int64_t a = __shfl_xor(mn, off, 64), b = __shfl_xor(mx, off, 64);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
  }
  if ((threadIdx.x & 63) == 0) {
    s_mn[threadIdx.x >> 6] = mn;
    s_mx[threadIdx.x >> 6] = mx;
  }
  __syncthreads();
  for (int w = 0; w < HIST_T / 64; ++w) {
    mn = s_mn[w] < mn ? s_mn[w] : mn;
    mx = s_mx[w] > mx ? s_mx[w] : mx;
  }
  if (mx - mn < HIST_LDS) {  // block-uniform
    const int span = static_cast<int>(mx - mn) + 1;
    for (int b = threadIdx.x; b < span; b += HIST_T) s_h[b] = 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < HIST_R; ++r)
      if (v[r] >= 0) atomicAdd(&s_h[v[r] - mn], 1);
    __syncthreads();
    for (int b = threadIdx.x; b < span; b += HIST_T)
      if (s_h[b] != 0) atomicAdd(&hist[mn + b], s_h[b]);
  } else {
#pragma unroll
    for (int r = 0; r < HIST_R; ++r)
      if (v[r] >= 0) atomicAdd(&hist[v[r]], 1);
  }
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n) { GRID_STRIDE(i, n) p[i] = 0; }

__global__ void k_nonzero(const int32_t* __restrict__ h, int32_t* __restrict__ flag, int64_t n) {
  GRID_STRIDE(i, n) flag[i] = h[i] != 0 ? 1 : 0;
}

// The non-zero bins in order: level lo + b and its count, at their rank.
__global__ void k_bins_out(const int32_t* __restrict__ h, const int32_t* __restrict__ rank,
                           int64_t lo, int64_t* __restrict__ lev, int32_t* __restrict__ cnt,
                           int64_t n) {
  GRID_STRIDE(b, n) {
    if (h[b] != 0) {
      lev[rank[b]] = lo + b;
      cnt[rank[b]] = h[b];
    }
  }
}

// v[r] = N_{k'k} / c_k for run r = (k, k'); runs are sorted by k, so c_k is the
// sum of the counts of k's block, read off the inclusive prefix sums P.
__global__ void k_row_terms(const int64_t* __restrict__ rk, const int32_t* __restrict__ cnt,
                            const int32_t* __restrict__ P, double* __restrict__ v,
                            int32_t* __restrict__ idx, int64_t m) {
  GRID_STRIDE(r, m) {
    const int64_t k = rk[r];
    int64_t lo = 0, hi = r;  // first run with level k
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (rk[mid] < k) lo = mid + 1; else hi = mid;
    }
    int64_t lo2 = r + 1, hi2 = m;  // one past the last run with level k
    while (lo2 < hi2) {
      const int64_t mid = (lo2 + hi2) >> 1;
      if (rk[mid] <= k) lo2 = mid + 1; else hi2 = mid;
    }
    const int32_t ck = P[lo2 - 1] - (lo > 0 ? P[lo - 1] : 0);
    v[r] = static_cast<double>(cnt[r]) / static_cast<double>(ck);
    idx[r] = static_cast<int32_t>(r);
  }
}

// After a stable sort of the runs by k', each row k' is a contiguous block in
// increasing k; its first thread sums the block in order.
__global__ void k_row_defects(const uint64_t* __restrict__ skey, const int32_t* __restrict__ idx,
                              const double* __restrict__ v, double* __restrict__ d, int64_t m) {
  GRID_STRIDE(j, m) {
    double out = 0.0;
    if (j == 0 || skey[j] != skey[j - 1]) {
      double s = 0.0;
      for (int64_t t = j; t < m && skey[t] == skey[j]; ++t) s += v[idx[t]];
      out = std::fabs(s - 1.0);
    }
    d[j] = out;
  }
}

// Carves typed arrays out of one allocation; a first pass with base == nullptr
// only measures.
struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += sizeof(T) * (count ? count : 1);
    return p;
  }
};

fqnm_status workspace(fqnm_ctx* ctx, size_t bytes, char** out) {
  if (ctx->ws_bytes < bytes) {
    if (ctx->d_ws) {
      (void)hipStreamSynchronize(ctx->stream);
      (void)hipFree(ctx->d_ws);
      ctx->d_ws = nullptr;
      ctx->ws_bytes = 0;
    }
    if (hipMalloc(&ctx->d_ws, bytes) != hipSuccess) {
      ctx->d_ws = nullptr;
      return fail(FQNM_ERR_OOM, "level statistics workspace");
    }
    ctx->ws_bytes = bytes;
  }
  *out = static_cast<char*>(ctx->d_ws);
  return FQNM_OK;
}

#define LV_HIP(expr, what)       \
  do {                           \
    hipError_t e_ = (expr);      \
    if (e_ != hipSuccess) {      \
      ctx->poisoned = true;      \
      return hip_fail(e_, what); \
    }                            \
  } while (0)

fqnm_status check_levels_ctx(fqnm_ctx* ctx) {
  if (!ctx) return fail(FQNM_ERR_ARG, "ctx is NULL");
  if (ctx->poisoned) return fail(FQNM_ERR_DEVICE, "context is poisoned");
  if (ctx->euler || ctx->classical)
    return fail(FQNM_ERR_UNSUPPORTED, "level statistics are defined for scalar integer states");
  if (ctx->prob.n > INT32_MAX) return fail(FQNM_ERR_UNSUPPORTED, "state too large");
  return FQNM_OK;
}

// Sort scratch of n keys carved from the workspace.
void take_sort_scratch(Carver& c, int64_t n, SortScratch* sc) {
  const int64_t cn = RS_D * sort_tiles(n);
  sc->counts = c.take<int32_t>(cn);
  sc->offsets = c.take<int32_t>(cn);
  sc->scan = c.take<int32_t>(scan_scratch(cn));
}

// Sorted distinct levels and their counts of the current state.
fqnm_status levels_of(fqnm_ctx* ctx, std::vector<int64_t>& lv, std::vector<int64_t>& ct) {
  const int64_t n = ctx->prob.n;
  hipStream_t s = ctx->stream;
  int64_t lo = 0, hi = 0;
  fqnm_status st = ctx_minmax(ctx, 0, &lo, &hi);
  if (st) return st;
  if (lo == hi) {
    lv.assign(1, lo);
    ct.assign(1, n);
    return FQNM_OK;
  }
  // a range of at most max(4n, 2^16) levels (and 2^24): count them directly
  const int64_t R = hi - lo + 1;
  if (R <= (int64_t(1) << 24) && R <= std::max<int64_t>(4 * n, int64_t(1) << 16)) {
    int32_t *hist = nullptr, *flag = nullptr, *rank = nullptr, *cnt = nullptr, *scan = nullptr;
    int64_t* lev = nullptr;
    auto hlayout = [&](char* base) {
      Carver c{base};
      hist = c.take<int32_t>(R);
      flag = c.take<int32_t>(R);
      rank = c.take<int32_t>(R);
      cnt = c.take<int32_t>(R);
      lev = c.take<int64_t>(R);
      scan = c.take<int32_t>(scan_scratch(R));
      return c.off;
    };
    char* hbase = nullptr;
    st = workspace(ctx, hlayout(nullptr), &hbase);
    if (st) return st;
    hlayout(hbase);
    k_fill_i32<<<grid_of(R), 256, 0, s>>>(hist, R);
    LV_HIP(hipGetLastError(), "histogram reset");
    const unsigned hb = static_cast<unsigned>((n + HIST_CELLS - 1) / HIST_CELLS);
    if (ctx->prob.itype == FQNM_I32)
      k_hist<int32_t><<<hb, HIST_T, 0, s>>>(static_cast<const int32_t*>(ctx->buf[ctx->cur]), n,
                                             lo, hist);
    else
      k_hist<int64_t><<<hb, HIST_T, 0, s>>>(static_cast<const int64_t*>(ctx->buf[ctx->cur]), n,
                                             lo, hist);
    LV_HIP(hipGetLastError(), "histogram");
    k_nonzero<<<grid_of(R), 256, 0, s>>>(hist, flag, R);
    LV_HIP(hipGetLastError(), "occupied bins");
    LV_HIP(scan_i32(flag, rank, R, false, scan, s), "scan");
    k_bins_out<<<grid_of(R), 256, 0, s>>>(hist, rank, lo, lev, cnt, R);
    LV_HIP(hipGetLastError(), "levels");
    int32_t last_rank = 0, last_flag = 0;
    LV_HIP(hipMemcpyAsync(&last_rank, rank + (R - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s),
           "copy");
    LV_HIP(hipMemcpyAsync(&last_flag, flag + (R - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s),
           "copy");
    LV_HIP(hipStreamSynchronize(s), "sync");
    const int32_t m = last_rank + last_flag;
    std::vector<int32_t> c32(m);
    lv.resize(m);
    LV_HIP(hipMemcpyAsync(lv.data(), lev, sizeof(int64_t) * m, hipMemcpyDeviceToHost, s),
           "copy levels");
    LV_HIP(hipMemcpyAsync(c32.data(), cnt, sizeof(int32_t) * m, hipMemcpyDeviceToHost, s),
           "copy counts");
    LV_HIP(hipStreamSynchronize(s), "sync");
    ct.resize(m);
    for (int32_t j = 0; j < m; ++j) ct[j] = c32[j];
    return FQNM_OK;
  }
  const int bits = bit_length(static_cast<uint64_t>(hi - lo));
  struct Bufs {
    uint64_t *keys, *alt;
    int32_t *head, *seg, *start, *cnt;
    int64_t* lev;
    SortScratch sc;
  } b{};
  auto layout = [&](char* base, Bufs* o) {
    Carver c{base};
    o->keys = c.take<uint64_t>(n);
    o->alt = c.take<uint64_t>(n);
    o->head = c.take<int32_t>(n);
    o->seg = c.take<int32_t>(n);
    o->start = c.take<int32_t>(n);
    o->cnt = c.take<int32_t>(n);
    o->lev = c.take<int64_t>(n);
    take_sort_scratch(c, n, &o->sc);
    return c.off;
  };
  char* base = nullptr;
  st = workspace(ctx, layout(nullptr, &b), &base);
  if (st) return st;
  layout(base, &b);
  if (ctx->prob.itype == FQNM_I32)
    k_offset_keys<int32_t><<<grid_of(n), 256, 0, s>>>(
        static_cast<const int32_t*>(ctx->buf[ctx->cur]), lo, b.keys, n);
  else
    k_offset_keys<int64_t><<<grid_of(n), 256, 0, s>>>(
        static_cast<const int64_t*>(ctx->buf[ctx->cur]), lo, b.keys, n);
  LV_HIP(hipGetLastError(), "offset keys");
  bool in_b = false;
  LV_HIP((radix_sort<int32_t, false>(b.keys, b.alt, nullptr, nullptr, n, bits, b.sc, s, &in_b)),
         "sort");
  const uint64_t* sorted = in_b ? b.alt : b.keys;
  // runs of equal levels: heads, their ranks, the levels and starts of the runs
  k_heads_u64<<<grid_of(n), 256, 0, s>>>(sorted, nullptr, b.head, n);
  LV_HIP(hipGetLastError(), "heads");
  LV_HIP(scan_i32(b.head, b.seg, n, false, b.sc.scan, s), "scan");
  k_runs_u64<<<grid_of(n), 256, 0, s>>>(sorted, nullptr, b.head, b.seg, lo, 0, b.lev, nullptr,
                                        b.start, n);
  LV_HIP(hipGetLastError(), "runs");
  int32_t last_seg = 0, last_head = 0;
  LV_HIP(hipMemcpyAsync(&last_seg, b.seg + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s),
         "copy");
  LV_HIP(hipMemcpyAsync(&last_head, b.head + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s),
         "copy");
  LV_HIP(hipStreamSynchronize(s), "sync");
  const int32_t m = last_seg + last_head;
  k_run_counts<<<grid_of(m), 256, 0, s>>>(b.start, b.cnt, m, n);
  LV_HIP(hipGetLastError(), "run counts");
  std::vector<int32_t> c32(m);
  lv.resize(m);
  LV_HIP(hipMemcpyAsync(lv.data(), b.lev, sizeof(int64_t) * m, hipMemcpyDeviceToHost, s),
         "copy levels");
  LV_HIP(hipMemcpyAsync(c32.data(), b.cnt, sizeof(int32_t) * m, hipMemcpyDeviceToHost, s),
         "copy counts");
  LV_HIP(hipStreamSynchronize(s), "sync");
  ct.resize(m);
  for (int32_t j = 0; j < m; ++j) ct[j] = c32[j];
  return FQNM_OK;
}

}  // namespace
}  // namespace fqnm

using namespace fqnm;

extern "C" {

fqnm_status fqnm_level_histogram(fqnm_ctx* ctx, int64_t* levels, int64_t* counts, int64_t cap,
                                 int64_t* n_levels) {
  fqnm_status st = check_levels_ctx(ctx);
  if (st) return st;
  if (!n_levels || cap < 0 || (cap > 0 && (!levels || !counts)))
    return fail(FQNM_ERR_ARG, "NULL argument or negative capacity");
  std::vector<int64_t> lv, ct;
  st = levels_of(ctx, lv, ct);
  if (st) return st;
  *n_levels = static_cast<int64_t>(lv.size());
  const int64_t m = std::min<int64_t>(cap, static_cast<int64_t>(lv.size()));
  std::copy(lv.begin(), lv.begin() + m, levels);
  std::copy(ct.begin(), ct.begin() + m, counts);
  return FQNM_OK;
}

fqnm_status fqnm_entropy(fqnm_ctx* ctx, double* S, double* n_eff) {
  fqnm_status st = check_levels_ctx(ctx);
  if (st) return st;
  if (!S) return fail(FQNM_ERR_ARG, "S is NULL");
  std::vector<int64_t> lv, ct;
  st = levels_of(ctx, lv, ct);
  if (st) return st;
  const double n = static_cast<double>(ctx->prob.n);
  double s = 0.0;
  for (size_t k = 0; k < ct.size(); ++k) {  // increasing level order
    const double pk = static_cast<double>(ct[k]) / n;
    s -= pk * std::log(pk);
  }
  *S = s;
  if (n_eff) *n_eff = std::exp(s);
  return FQNM_OK;
}

fqnm_status fqnm_step_transitions(fqnm_ctx* ctx, int64_t* from, int64_t* to, int64_t* count,
                                  int64_t cap, int64_t* n_pairs, double* row_defect) {
  fqnm_status st = check_levels_ctx(ctx);
  if (st) return st;
  if (!n_pairs || cap < 0 || (cap > 0 && (!from || !to || !count)))
    return fail(FQNM_ERR_ARG, "NULL argument or negative capacity");
  const int64_t n = ctx->prob.n;
  hipStream_t s = ctx->stream;
  const bool i32 = ctx->prob.itype == FQNM_I32;

  int64_t lo0 = 0, hi0 = 0, lo1 = 0, hi1 = 0;
  st = ctx_minmax(ctx, 0, &lo0, &hi0);
  if (st) return st;

  struct Bufs {
    int64_t* k0;
    uint64_t *A, *B, *C, *D, *skey, *skey2;
    int64_t *rk, *rk2;
    double *v, *d, *part, *rho;
    int32_t *head, *seg, *cnt, *P, *idx, *idx2, *start;
    SortScratch sc;
  } b{};
  auto layout = [&](char* base, Bufs* o) {
    Carver c{base};
    o->k0 = c.take<int64_t>(n);
    o->A = c.take<uint64_t>(n);
    o->B = c.take<uint64_t>(n);
    o->C = c.take<uint64_t>(n);
    o->D = c.take<uint64_t>(n);
    o->skey = c.take<uint64_t>(n);
    o->skey2 = c.take<uint64_t>(n);
    o->rk = c.take<int64_t>(n);
    o->rk2 = c.take<int64_t>(n);
    o->v = c.take<double>(n);
    o->d = c.take<double>(n);
    o->part = c.take<double>(256);
    o->rho = c.take<double>(1);
    o->head = c.take<int32_t>(n);
    o->seg = c.take<int32_t>(n);
    o->cnt = c.take<int32_t>(n);
    o->P = c.take<int32_t>(n);
    o->idx = c.take<int32_t>(n);
    o->idx2 = c.take<int32_t>(n);
    o->start = c.take<int32_t>(n);
    take_sort_scratch(c, n, &o->sc);
    return c.off;
  };
  char* base = nullptr;
  st = workspace(ctx, layout(nullptr, &b), &base);
  if (st) return st;
  layout(base, &b);

  if (i32)
    k_widen<int32_t><<<grid_of(n), 256, 0, s>>>(static_cast<const int32_t*>(ctx->buf[ctx->cur]),
                                                b.k0, n);
  else
    k_widen<int64_t><<<grid_of(n), 256, 0, s>>>(static_cast<const int64_t*>(ctx->buf[ctx->cur]),
                                                b.k0, n);
  LV_HIP(hipGetLastError(), "widen");
  st = fqnm_step(ctx, 1);
  if (st) return st;
  st = ctx_minmax(ctx, 0, &lo1, &hi1);
  if (st) return st;
  const void* q1 = ctx->buf[ctx->cur];

  const int b0 = bit_length(static_cast<uint64_t>(hi0 - lo0));
  const int b1 = bit_length(static_cast<uint64_t>(hi1 - lo1));
  bool in_b = false;
  const uint64_t *sk = nullptr, *sk2 = nullptr;  // sorted (k, k') offsets, or packed pairs
  int64_t base0 = lo0;
  if (b0 + b1 <= 64) {
    // one sort of packed (k, k') keys
    if (i32)
      k_pair_keys<int32_t><<<grid_of(n), 256, 0, s>>>(b.k0, static_cast<const int32_t*>(q1), lo0,
                                                      lo1, b1, b.A, n);
    else
      k_pair_keys<int64_t><<<grid_of(n), 256, 0, s>>>(b.k0, static_cast<const int64_t*>(q1), lo0,
                                                      lo1, b1, b.A, n);
    LV_HIP(hipGetLastError(), "pair keys");
    LV_HIP((radix_sort<int32_t, false>(b.A, b.B, nullptr, nullptr, n, b0 + b1, b.sc, s, &in_b)),
           "sort pairs");
    sk = in_b ? b.B : b.A;
    base0 = 0;  // unpacked below
  } else {
    // wide level ranges: a stable sort by k' carrying k, then by k carrying k'
    if (i32)
      k_offset_keys<int32_t><<<grid_of(n), 256, 0, s>>>(static_cast<const int32_t*>(q1), lo1,
                                                        b.A, n);
    else
      k_offset_keys<int64_t><<<grid_of(n), 256, 0, s>>>(static_cast<const int64_t*>(q1), lo1,
                                                        b.A, n);
    k_offset_keys<int64_t><<<grid_of(n), 256, 0, s>>>(b.k0, lo0, b.C, n);
    LV_HIP(hipGetLastError(), "offset keys");
    LV_HIP((radix_sort<uint64_t, true>(b.A, b.B, b.C, b.D, n, b1, b.sc, s, &in_b)), "sort by k'");
    uint64_t* kp = in_b ? b.B : b.A;  // k' offsets, sorted
    uint64_t* kk = in_b ? b.D : b.C;  // k offsets in that order
    uint64_t* kp_alt = in_b ? b.A : b.B;
    uint64_t* kk_alt = in_b ? b.C : b.D;
    LV_HIP((radix_sort<uint64_t, true>(kk, kk_alt, kp, kp_alt, n, b0, b.sc, s, &in_b)),
           "sort by k");
    sk = in_b ? kk_alt : kk;
    sk2 = in_b ? kp_alt : kp;
  }
  // runs of equal pairs: heads, their ranks, the pairs and starts of the runs
  k_heads_u64<<<grid_of(n), 256, 0, s>>>(sk, sk2, b.head, n);
  LV_HIP(hipGetLastError(), "heads");
  LV_HIP(scan_i32(b.head, b.seg, n, false, b.sc.scan, s), "scan heads");
  k_runs_u64<<<grid_of(n), 256, 0, s>>>(sk, sk2, b.head, b.seg, base0, lo1, b.rk, b.rk2, b.start,
                                        n);
  LV_HIP(hipGetLastError(), "runs");
  int32_t last_seg = 0, last_head = 0;
  LV_HIP(hipMemcpyAsync(&last_seg, b.seg + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s),
         "copy");
  LV_HIP(hipMemcpyAsync(&last_head, b.head + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s),
         "copy");
  LV_HIP(hipStreamSynchronize(s), "sync");
  const int32_t m = last_seg + last_head;
  k_run_counts<<<grid_of(m), 256, 0, s>>>(b.start, b.cnt, m, n);
  LV_HIP(hipGetLastError(), "run counts");
  if (!sk2) {
    // the runs' packed keys, back to (k, k')
    k_unpack_runs<<<grid_of(m), 256, 0, s>>>(b.rk, lo0, lo1, b1, b.rk2, m);
    LV_HIP(hipGetLastError(), "unpack");
  }

  // row sums of M and their largest deviation from 1
  LV_HIP(scan_i32(b.cnt, b.P, m, true, b.sc.scan, s), "scan counts");
  k_row_terms<<<grid_of(m), 256, 0, s>>>(b.rk, b.cnt, b.P, b.v, b.idx, m);
  LV_HIP(hipGetLastError(), "row terms");
  // the runs by k' (stable: each row keeps increasing k)
  k_offset_keys<int64_t><<<grid_of(m), 256, 0, s>>>(b.rk2, lo1, b.skey, m);
  LV_HIP(hipGetLastError(), "row keys");
  LV_HIP((radix_sort<int32_t, true>(b.skey, b.skey2, b.idx, b.idx2, m, b1, b.sc, s, &in_b)),
         "sort rows");
  const uint64_t* rows = in_b ? b.skey2 : b.skey;
  const int32_t* ridx = in_b ? b.idx2 : b.idx;
  k_row_defects<<<grid_of(m), 256, 0, s>>>(rows, ridx, b.v, b.d, m);
  LV_HIP(hipGetLastError(), "row defects");
  const unsigned g = std::min<unsigned>(256u, grid_of(m));
  k_max_partial<<<g, 256, 0, s>>>(b.d, m, b.part);
  k_max_partial<<<1, 256, 0, s>>>(b.part, g, b.rho);
  LV_HIP(hipGetLastError(), "max");

  const int64_t w = std::min<int64_t>(cap, m);
  std::vector<int32_t> c32(w);
  double rho = 0.0;
  if (w > 0) {
    LV_HIP(hipMemcpyAsync(from, b.rk, sizeof(int64_t) * w, hipMemcpyDeviceToHost, s), "copy");
    LV_HIP(hipMemcpyAsync(to, b.rk2, sizeof(int64_t) * w, hipMemcpyDeviceToHost, s), "copy");
    LV_HIP(hipMemcpyAsync(c32.data(), b.cnt, sizeof(int32_t) * w, hipMemcpyDeviceToHost, s),
           "copy");
  }
  LV_HIP(hipMemcpyAsync(&rho, b.rho, sizeof(double), hipMemcpyDeviceToHost, s), "copy");
  LV_HIP(hipStreamSynchronize(s), "sync");
  for (int64_t r = 0; r < w; ++r) count[r] = c32[r];
  *n_pairs = m;
  if (row_defect) *row_defect = rho;
  return FQNM_OK;
}

}  // extern "C"
