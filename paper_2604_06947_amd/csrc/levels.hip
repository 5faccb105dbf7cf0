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
// else two stable 64-bit passes sort by k' then by k.  Run-length encoding
// gives the occupied levels / nonzero transitions.  Row sums of M are formed
// on the device, each by one thread adding its row's terms in increasing k,
// so the value is the same double a sequential sum in that order gives.  The
// entropy sum (one log per occupied level) runs on the host, in increasing
// level order.  A workspace is kept per context and grown on demand.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

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

__global__ void k_unpack_pairs(const uint64_t* __restrict__ key, int64_t lo0, int64_t lo1, int b1,
                               int64_t* __restrict__ rk, int64_t* __restrict__ rk2, int64_t m) {
  const uint64_t mask = b1 == 0 ? 0 : (~uint64_t(0) >> (64 - b1));
  GRID_STRIDE(r, m) {
    rk[r] = static_cast<int64_t>(key[r] >> b1) + lo0;
    rk2[r] = static_cast<int64_t>(key[r] & mask) + lo1;
  }
}

// head[i] = 1 where a new (k, k') run starts in the pair sequence sorted by (k, k')
__global__ void k_pair_heads(const int64_t* __restrict__ k, const int64_t* __restrict__ k2,
                             int32_t* __restrict__ head, int64_t n) {
  GRID_STRIDE(i, n) head[i] = (i == 0 || k[i] != k[i - 1] || k2[i] != k2[i - 1]) ? 1 : 0;
}

// run seg[i] starts at every head position i
__global__ void k_pair_runs(const int64_t* __restrict__ k, const int64_t* __restrict__ k2,
                            const int32_t* __restrict__ head, const int32_t* __restrict__ seg,
                            int64_t* __restrict__ rk, int64_t* __restrict__ rk2,
                            int32_t* __restrict__ rstart, int64_t n) {
  GRID_STRIDE(i, n) {
    if (head[i]) {
      const int32_t r = seg[i];
      rk[r] = k[i];
      rk2[r] = k2[i];
      rstart[r] = static_cast<int32_t>(i);
    }
  }
}

__global__ void k_run_counts(const int32_t* __restrict__ rstart, int32_t* __restrict__ cnt,
                             int64_t m, int64_t n) {
  GRID_STRIDE(r, m) cnt[r] = static_cast<int32_t>((r + 1 < m ? rstart[r + 1] : n) - rstart[r]);
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
__global__ void k_row_defects(const int64_t* __restrict__ skey, const int32_t* __restrict__ idx,
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

// A library call's temporary storage must fit the carved block: query the
// exact call first.
#define LV_FITS(query, have)                                                        \
  do {                                                                              \
    size_t need_ = 0;                                                               \
    hipError_t e_ = (query);                                                        \
    if (e_ != hipSuccess) return hip_fail(e_, "temporary size");                    \
    if (need_ > (have)) return fail(FQNM_ERR_DEVICE, "temporary storage too small"); \
  } while (0)

fqnm_status check_levels_ctx(fqnm_ctx* ctx) {
  if (!ctx) return fail(FQNM_ERR_ARG, "ctx is NULL");
  if (ctx->poisoned) return fail(FQNM_ERR_DEVICE, "context is poisoned");
  if (ctx->euler || ctx->classical)
    return fail(FQNM_ERR_UNSUPPORTED, "level statistics are defined for scalar integer states");
  if (ctx->prob.n > INT32_MAX) return fail(FQNM_ERR_UNSUPPORTED, "state too large");
  return FQNM_OK;
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
  const int bits = bit_length(static_cast<uint64_t>(hi - lo));
  const int ni = static_cast<int>(n);
  size_t tb1 = 0, tb2 = 0;
  LV_HIP(hipcub::DeviceRadixSort::SortKeys(nullptr, tb1, (const uint64_t*)nullptr,
                                           (uint64_t*)nullptr, ni, 0, bits, s), "sort size");
  LV_HIP(hipcub::DeviceRunLengthEncode::Encode(nullptr, tb2, (const uint64_t*)nullptr,
                                               (uint64_t*)nullptr, (int32_t*)nullptr,
                                               (int32_t*)nullptr, ni, s), "encode size");
  auto layout = [&](char* base, uint64_t** keys, uint64_t** sorted, uint64_t** uniq,
                    int32_t** counts, int32_t** nruns, void** tmp) {
    Carver c{base};
    *keys = c.take<uint64_t>(n);
    *sorted = c.take<uint64_t>(n);
    *uniq = c.take<uint64_t>(n);
    *counts = c.take<int32_t>(n);
    *nruns = c.take<int32_t>(1);
    *tmp = c.take<char>(std::max(tb1, tb2));
    return c.off;
  };
  uint64_t *keys, *sorted, *uniq;
  int32_t *counts, *nruns;
  void* tmp;
  char* base = nullptr;
  st = workspace(ctx, layout(nullptr, &keys, &sorted, &uniq, &counts, &nruns, &tmp), &base);
  if (st) return st;
  layout(base, &keys, &sorted, &uniq, &counts, &nruns, &tmp);
  if (ctx->prob.itype == FQNM_I32)
    k_offset_keys<int32_t><<<grid_of(n), 256, 0, s>>>(
        static_cast<const int32_t*>(ctx->buf[ctx->cur]), lo, keys, n);
  else
    k_offset_keys<int64_t><<<grid_of(n), 256, 0, s>>>(
        static_cast<const int64_t*>(ctx->buf[ctx->cur]), lo, keys, n);
  LV_HIP(hipGetLastError(), "offset keys");
  LV_HIP(hipcub::DeviceRadixSort::SortKeys(tmp, tb1, keys, sorted, ni, 0, bits, s), "sort");
  LV_HIP(hipcub::DeviceRunLengthEncode::Encode(tmp, tb2, sorted, uniq, counts, nruns, ni, s),
         "encode");
  int32_t m = 0;
  LV_HIP(hipMemcpyAsync(&m, nruns, sizeof m, hipMemcpyDeviceToHost, s), "copy run count");
  LV_HIP(hipStreamSynchronize(s), "sync");
  std::vector<uint64_t> u(m);
  std::vector<int32_t> c32(m);
  LV_HIP(hipMemcpyAsync(u.data(), uniq, sizeof(uint64_t) * m, hipMemcpyDeviceToHost, s),
         "copy levels");
  LV_HIP(hipMemcpyAsync(c32.data(), counts, sizeof(int32_t) * m, hipMemcpyDeviceToHost, s),
         "copy counts");
  LV_HIP(hipStreamSynchronize(s), "sync");
  lv.resize(m);
  ct.resize(m);
  for (int32_t j = 0; j < m; ++j) {
    lv[j] = static_cast<int64_t>(u[j]) + lo;
    ct[j] = c32[j];
  }
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
  const int ni = static_cast<int>(n);
  hipStream_t s = ctx->stream;
  const bool i32 = ctx->prob.itype == FQNM_I32;

  int64_t lo0 = 0, hi0 = 0, lo1 = 0, hi1 = 0;
  st = ctx_minmax(ctx, 0, &lo0, &hi0);
  if (st) return st;

  // temporary storage: the largest over the library calls below at full size
  size_t tb = 0, t = 0;
  LV_HIP(hipcub::DeviceRadixSort::SortKeys(nullptr, t, (const uint64_t*)nullptr,
                                           (uint64_t*)nullptr, ni, 0, 64, s), "size");
  tb = std::max(tb, t);
  LV_HIP(hipcub::DeviceRunLengthEncode::Encode(nullptr, t, (const uint64_t*)nullptr,
                                               (uint64_t*)nullptr, (int32_t*)nullptr,
                                               (int32_t*)nullptr, ni, s), "size");
  tb = std::max(tb, t);
  LV_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, t, (const int64_t*)nullptr,
                                            (int64_t*)nullptr, (const int64_t*)nullptr,
                                            (int64_t*)nullptr, ni, 0, 64, s), "size");
  tb = std::max(tb, t);
  LV_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, t, (const int64_t*)nullptr,
                                            (int64_t*)nullptr, (const int32_t*)nullptr,
                                            (int32_t*)nullptr, ni, 0, 64, s), "size");
  tb = std::max(tb, t);
  LV_HIP(hipcub::DeviceScan::InclusiveSum(nullptr, t, (const int32_t*)nullptr, (int32_t*)nullptr,
                                          ni, s), "size");
  tb = std::max(tb, t);
  LV_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, t, (const int32_t*)nullptr, (int32_t*)nullptr,
                                          ni, s), "size");
  tb = std::max(tb, t);
  LV_HIP(hipcub::DeviceReduce::Max(nullptr, t, (const double*)nullptr, (double*)nullptr, ni, s),
         "size");
  tb = std::max(tb, t);

  struct Bufs {
    int64_t *k0, *A, *B, *C, *D, *rk, *rk2, *skey;
    double *v, *d, *rho;
    int32_t *head, *seg, *cnt, *P, *idx, *idx2, *nruns;
    void* tmp;
  } b{};
  auto layout = [&](char* base, Bufs* o) {
    Carver c{base};
    o->k0 = c.take<int64_t>(n);
    o->A = c.take<int64_t>(n);
    o->B = c.take<int64_t>(n);
    o->C = c.take<int64_t>(n);
    o->D = c.take<int64_t>(n);
    o->rk = c.take<int64_t>(n);
    o->rk2 = c.take<int64_t>(n);
    o->skey = c.take<int64_t>(n);
    o->v = c.take<double>(n);
    o->d = c.take<double>(n);
    o->rho = c.take<double>(1);
    o->head = c.take<int32_t>(n);
    o->seg = c.take<int32_t>(n);
    o->cnt = c.take<int32_t>(n);
    o->P = c.take<int32_t>(n);
    o->idx = c.take<int32_t>(n);
    o->idx2 = c.take<int32_t>(n);
    o->nruns = c.take<int32_t>(1);
    o->tmp = c.take<char>(tb);
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
  int32_t m = 0;
  if (b0 + b1 <= 64) {
    // one sort of packed (k, k') keys, then run-length encoding
    uint64_t* keys = reinterpret_cast<uint64_t*>(b.A);
    uint64_t* sorted = reinterpret_cast<uint64_t*>(b.B);
    uint64_t* uniq = reinterpret_cast<uint64_t*>(b.C);
    if (i32)
      k_pair_keys<int32_t><<<grid_of(n), 256, 0, s>>>(b.k0, static_cast<const int32_t*>(q1), lo0,
                                                      lo1, b1, keys, n);
    else
      k_pair_keys<int64_t><<<grid_of(n), 256, 0, s>>>(b.k0, static_cast<const int64_t*>(q1), lo0,
                                                      lo1, b1, keys, n);
    LV_HIP(hipGetLastError(), "pair keys");
    const int bits = b0 + b1;
    if (bits > 0) {
      LV_FITS(hipcub::DeviceRadixSort::SortKeys(nullptr, need_, keys, sorted, ni, 0, bits, s), tb);
      LV_HIP(hipcub::DeviceRadixSort::SortKeys(b.tmp, tb, keys, sorted, ni, 0, bits, s), "sort");
    } else {
      LV_HIP(hipMemcpyAsync(sorted, keys, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s),
             "copy");
    }
    LV_HIP(hipcub::DeviceRunLengthEncode::Encode(b.tmp, tb, sorted, uniq, b.cnt, b.nruns, ni, s),
           "encode");
    LV_HIP(hipMemcpyAsync(&m, b.nruns, sizeof m, hipMemcpyDeviceToHost, s), "copy run count");
    LV_HIP(hipStreamSynchronize(s), "sync");
    k_unpack_pairs<<<grid_of(m), 256, 0, s>>>(uniq, lo0, lo1, b1, b.rk, b.rk2, m);
    LV_HIP(hipGetLastError(), "unpack");
  } else {
    // wide level ranges: stable sort by k' carrying k, then by k carrying k'
    if (i32)
      k_widen<int32_t><<<grid_of(n), 256, 0, s>>>(static_cast<const int32_t*>(q1), b.A, n);
    else
      k_widen<int64_t><<<grid_of(n), 256, 0, s>>>(static_cast<const int64_t*>(q1), b.A, n);
    LV_HIP(hipGetLastError(), "widen");
    LV_HIP(hipcub::DeviceRadixSort::SortPairs(b.tmp, tb, b.A, b.B, b.k0, b.C, ni, 0, 64, s),
           "sort by k'");
    LV_HIP(hipcub::DeviceRadixSort::SortPairs(b.tmp, tb, b.C, b.D, b.B, b.A, ni, 0, 64, s),
           "sort by k");
    k_pair_heads<<<grid_of(n), 256, 0, s>>>(b.D, b.A, b.head, n);
    LV_HIP(hipGetLastError(), "heads");
    LV_HIP(hipcub::DeviceScan::ExclusiveSum(b.tmp, tb, b.head, b.seg, ni, s), "scan");
    k_pair_runs<<<grid_of(n), 256, 0, s>>>(b.D, b.A, b.head, b.seg, b.rk, b.rk2, b.idx, n);
    LV_HIP(hipGetLastError(), "runs");
    int32_t last_seg = 0, last_head = 0;
    LV_HIP(hipMemcpyAsync(&last_seg, b.seg + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s),
           "copy");
    LV_HIP(hipMemcpyAsync(&last_head, b.head + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost,
                          s), "copy");
    LV_HIP(hipStreamSynchronize(s), "sync");
    m = last_seg + last_head;
    k_run_counts<<<grid_of(m), 256, 0, s>>>(b.idx, b.cnt, m, n);
    LV_HIP(hipGetLastError(), "run counts");
  }

  // row sums of M and their largest deviation from 1
  LV_FITS(hipcub::DeviceScan::InclusiveSum(nullptr, need_, b.cnt, b.P, m, s), tb);
  LV_HIP(hipcub::DeviceScan::InclusiveSum(b.tmp, tb, b.cnt, b.P, m, s), "scan counts");
  k_row_terms<<<grid_of(m), 256, 0, s>>>(b.rk, b.cnt, b.P, b.v, b.idx, m);
  LV_HIP(hipGetLastError(), "row terms");
  LV_FITS(hipcub::DeviceRadixSort::SortPairs(nullptr, need_, b.rk2, b.skey, b.idx, b.idx2, m, 0,
                                             64, s), tb);
  LV_HIP(hipcub::DeviceRadixSort::SortPairs(b.tmp, tb, b.rk2, b.skey, b.idx, b.idx2, m, 0, 64, s),
         "sort rows");
  k_row_defects<<<grid_of(m), 256, 0, s>>>(b.skey, b.idx2, b.v, b.d, m);
  LV_HIP(hipGetLastError(), "row defects");
  LV_FITS(hipcub::DeviceReduce::Max(nullptr, need_, b.d, b.rho, m, s), tb);
  LV_HIP(hipcub::DeviceReduce::Max(b.tmp, tb, b.d, b.rho, m, s), "max");

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
