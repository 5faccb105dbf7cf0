// nd.hip -- d-dimensional grids by directional composition (Thm dimension_extension).
//
// One step of eq:nd_transfer_rule: every cell subtracts, direction by
// direction, the difference of the one-dimensional transfers across its two
// faces orthogonal to that direction (eq:nd_flux_definition), all taken from
// the state before the step.  Axis 0 is contiguous in memory.
//
// k_nd_march: a wavefront owns a strip of 64*V consecutive cells of axis 0
// (V per lane) and marches along the last axis over `rows` positions.  Each
// state row is loaded once (plus one halo row per block of positions), its
// maps are evaluated once, and the flux of the face behind is carried in
// registers.  The loads of the next two positions are always in flight
// while a row is computed (two stage buffers used in turn).
// Neighbours along axis 0 come from the adjacent lanes by cross-lane moves;
// in 3-D the two neighbouring rows of the middle axis are read at each
// position (they are other wavefronts' rows, usually found in L2).  Periodic
// ends wrap; outflow ends read the cell itself as its ghost, per direction,
// and the counts crossing outflow faces are added to the device ledger.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "nd_common.h"

namespace fqnm {
namespace {

// Raw loads of one marching position r: the lane's V cells, the two cells
// beside the strip (lanes 0 and 63 only) and, in 3-D, the neighbouring rows
// of the middle axis.
template <typename IT, int V, int DIM>
struct Stage {
  IT q[V];
  IT gl, gr;
  IT ql[V], qr[V];
};

// A position after its own work: the state, the axis-0 (and axis-1) flux
// divergence, phi+ along the marching axis, and the counts crossing outflow
// faces of axis 0 (and 1) in this row.
template <typename IT, int V>
struct Ready {
  IT q[V];
  IT d[V];
  IT ppm[V];
  long long led;
};

template <typename IT, int POL, int V, int DIM>
struct Marcher {
  const IT* __restrict__ src;
  const NdParams& P;
  int64_t nx, ny, nm, SM, base, x0, y;
  int32_t klast;       // index k of the row's last cell if this lane holds it, else -1
  int32_t nvalid;      // cells of this lane inside the row (0..V)
  int32_t xl, xr;      // offsets of the cells beside the strip within a row
  int32_t xo[V];       // offsets of the lane's cells within a row (ghost rules applied)
  int64_t yl, yr;      // 3-D: offsets of the neighbouring rows of the middle axis
  int lane;
  bool vec_row;
  bool same_m;  // the marching axis has axis 0's map constants: its maps are axis 0's
  bool same_y;  // 3-D: the same for the middle axis

  __device__ __forceinline__ void load_row(const IT* __restrict__ row, IT (&q)[V]) const {
    if (vec_row) {
      nd_load<IT, V>(row + x0, q);
    } else {
#pragma unroll
      for (int k = 0; k < V; ++k) q[k] = row[xo[k]];
    }
  }

  // marching position r in [-1, nm + 1] to a row index (ghost rules applied)
  __device__ __forceinline__ int64_t march_row(int64_t r) const {
    if (r >= 0 && r < nm) return r;
    if (P.ax[DIM - 1].bc != FQNM_BC_PERIODIC) return r < 0 ? 0 : nm - 1;
    r = r < 0 ? r + nm : r - nm;
    return r >= nm ? r - nm : r;
  }

  // issue the loads of marching position r
  __device__ __forceinline__ void load(int64_t r, Stage<IT, V, DIM>& S) const {
    const int64_t rs = march_row(r) * SM;
    const IT* row = src + base + rs;
    load_row(row, S.q);
    S.gl = IT(0);
    S.gr = IT(0);
    if (lane == 0) S.gl = row[xl];
    if (lane == 63) S.gr = row[xr];
    if constexpr (DIM == 3) {
      load_row(src + rs + yl, S.ql);
      load_row(src + rs + yr, S.qr);
    }
  }

  // the position's own work; pmm receives phi- along the marching axis
  __device__ __forceinline__ void process(const Stage<IT, V, DIM>& S, Ready<IT, V>& R,
                                          IT (&pmm)[V]) const {
    const NdAxis& AX = P.ax[0];
    IT Fx[V], Fl;
    if constexpr (NdSplit<POL>::value) {
      IT ppx[V], pmx[V];
#pragma unroll
      for (int k = 0; k < V; ++k) axis_maps<IT, POL>(AX, S.q[k], ppx[k], pmx[k]);
      if (same_m) {  // uniform
#pragma unroll
        for (int k = 0; k < V; ++k) {
          R.ppm[k] = ppx[k];
          pmm[k] = pmx[k];
        }
      } else {
#pragma unroll
        for (int k = 0; k < V; ++k) axis_maps<IT, POL>(P.ax[DIM - 1], S.q[k], R.ppm[k], pmm[k]);
      }
      IT gp, gm, hp, hm;
      axis_maps<IT, POL>(AX, S.gl, gp, gm);
      axis_maps<IT, POL>(AX, S.gr, hp, hm);
      IT pmn = lane_from_next<IT>(pmx[0]);
      if (lane == 63) pmn = hm;
#pragma unroll
      for (int k = 0; k < V; ++k) Fx[k] = ppx[k] + (k + 1 < V ? pmx[k + 1] : pmn);
      Fl = lane_from_prev<IT>(Fx[V - 1]);
      if (lane == 0) Fl = gp + pmx[0];
    } else {
      IT qn = lane_from_next<IT>(S.q[0]);
      if (lane == 63) qn = S.gr;
#pragma unroll
      for (int k = 0; k < V; ++k)
        Fx[k] = transfer<IT, POL>(AX.x, S.q[k], k + 1 < V ? S.q[k + 1] : qn);
      Fl = lane_from_prev<IT>(Fx[V - 1]);
      if (lane == 0) Fl = transfer<IT, POL>(AX.x, S.gl, S.q[0]);
    }
    long long led = 0;
#pragma unroll
    for (int k = 0; k < V; ++k) {
      R.q[k] = S.q[k];
      R.d[k] = wsub<IT>(Fx[k], k == 0 ? Fl : Fx[k - 1]);
    }
    if (AX.bc == FQNM_BC_OUTFLOW) {  // uniform
      if (x0 == 0) led += static_cast<long long>(Fl);
#pragma unroll
      for (int k = 0; k < V; ++k)
        if (k == klast) led -= static_cast<long long>(Fx[k]);
    }
    if constexpr (DIM == 3) {
      const NdAxis& AY = P.ax[1];
#pragma unroll
      for (int k = 0; k < V; ++k) {
        IT lo, hi;
        if constexpr (NdSplit<POL>::value) {
          IT pl, ml, pr, mr, pq, mq;
          axis_maps<IT, POL>(AY, S.ql[k], pl, ml);
          axis_maps<IT, POL>(AY, S.qr[k], pr, mr);
          if (same_y) {  // uniform
            axis_maps<IT, POL>(AX, S.q[k], pq, mq);  // shares the axis-0 evaluation above
          } else {
            axis_maps<IT, POL>(AY, S.q[k], pq, mq);
          }
          lo = pl + mq;
          hi = pq + mr;
        } else {
          lo = transfer<IT, POL>(AY.x, S.ql[k], S.q[k]);
          hi = transfer<IT, POL>(AY.x, S.q[k], S.qr[k]);
        }
        R.d[k] = wsub<IT>(R.d[k], wsub<IT>(lo, hi));  // d + (hi - lo), wrapping
        if (AY.bc == FQNM_BC_OUTFLOW && (y == 0 || y == ny - 1) && k < nvalid) {  // uniform bc, y
          if (y == 0) led += static_cast<long long>(lo);
          if (y == ny - 1) led -= static_cast<long long>(hi);
        }
      }
    }
    if constexpr (!NdSplit<POL>::value) {
#pragma unroll
      for (int k = 0; k < V; ++k) {
        R.ppm[k] = IT(0);
        pmm[k] = IT(0);
      }
    }
    R.led = led;
  }
};

template <typename IT, int POL, int V, int DIM>
__global__ __launch_bounds__(256) void k_nd_march(const IT* __restrict__ src, IT* __restrict__ dst,
                                                  NdParams P, int rows, int64_t nstrips,
                                                  int64_t nwaves, int vec_ok,
                                                  long long* __restrict__ ledger) {
  // the wavefront index is uniform: keep it (and all row arithmetic) scalar
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int64_t w = xcd_tile(blockIdx.x, gridDim.x) * 4 + wave;
  if (w >= nwaves) return;
  const NdAxis& AX = P.ax[0];
  const NdAxis& AM = P.ax[DIM - 1];
  Marcher<IT, POL, V, DIM> M{src, P};
  M.lane = lane;
  M.nx = AX.n;
  M.nm = AM.n;
  M.ny = DIM == 3 ? P.ax[1].n : 1;
  M.SM = DIM == 3 ? M.nx * M.ny : M.nx;  // stride of the marching axis
  const int64_t strip = w % nstrips;
  int64_t rest = w / nstrips;
  M.y = 0;
  if constexpr (DIM == 3) {
    M.y = rest % M.ny;
    rest /= M.ny;
  }
  const int64_t j0 = rest * rows;
  const int64_t jend = j0 + rows < M.nm ? j0 + rows : M.nm;
  const int64_t xs = strip * 64 * V;
  M.x0 = xs + static_cast<int64_t>(lane) * V;
  M.base = M.y * M.nx;  // offset of (x = 0, y, r = 0)
  M.vec_row = vec_ok && M.x0 + V <= M.nx;
  M.xl = static_cast<int32_t>(nd_ghost(xs - 1, M.nx, AX.bc));  // beside the strip
  M.xr = static_cast<int32_t>(nd_ghost(xs + 64 * V, M.nx, AX.bc));
#pragma unroll
  for (int k = 0; k < V; ++k) M.xo[k] = static_cast<int32_t>(nd_ghost(M.x0 + k, M.nx, AX.bc));
  {
    const int64_t left = M.nx - M.x0;
    M.nvalid = static_cast<int32_t>(left < 0 ? 0 : (left > V ? V : left));
    M.klast = left >= 1 && left <= V ? static_cast<int32_t>(left - 1) : -1;
  }
  M.same_m = nd_same_axis(AX, AM);
  M.same_y = DIM == 3 && nd_same_axis(AX, P.ax[1]);
  M.yl = M.yr = 0;
  if constexpr (DIM == 3) {
    M.yl = nd_ghost(M.y - 1, M.ny, P.ax[1].bc) * M.nx;
    M.yr = nd_ghost(M.y + 1, M.ny, P.ax[1].bc) * M.nx;
  }

  // prologue: the row behind the block (only its marching-axis map or state),
  // the first row and the one after it; then the loads of the next two rows
  Stage<IT, V, DIM> S0, S1;
  Ready<IT, V> rb, rc;
  IT pmm_b[V], pmm_c[V], FMlo[V];
  IT q_a[V];
  M.load_row(src + M.base + M.march_row(j0 - 1) * M.SM, q_a);
  M.load(j0, S0);
  M.load(j0 + 1, S1);
  M.process(S0, rb, pmm_b);
#pragma unroll
  for (int k = 0; k < V; ++k) {
    if constexpr (NdSplit<POL>::value) {
      IT pa, ma;
      axis_maps<IT, POL>(AM, q_a[k], pa, ma);
      FMlo[k] = pa + pmm_b[k];
    } else {
      FMlo[k] = transfer<IT, POL>(AM.x, q_a[k], rb.q[k]);
    }
  }
  M.process(S1, rc, pmm_c);
  if (j0 + 2 <= jend) M.load(j0 + 2, S0);
  if (j0 + 3 <= jend) M.load(j0 + 3, S1);

  // Row j leaves with the position j + 2 processed from the buffer that was
  // loaded two rows earlier; the buffer is then refilled with position j + 4,
  // so two positions are always in flight.  Positions up to jend are needed
  // (jend for the flux of the last row's upper face).
  long long led = 0;
  // cur = row j, nxt = row j + 1 (with its phi- along the marching axis); after
  // row j is finished, cur's registers take position j + 2, so the two buffers
  // trade roles every row instead of being copied
  auto row = [&](int64_t j, Stage<IT, V, DIM>& S, Ready<IT, V>& cur, Ready<IT, V>& nxt,
                 IT (&pmm_nxt)[V], IT (&pmm_cur)[V]) {
    const int64_t off = M.base + j * M.SM;
    IT out[V];
#pragma unroll
    for (int k = 0; k < V; ++k) {
      IT FMhi;
      if constexpr (NdSplit<POL>::value) FMhi = cur.ppm[k] + pmm_nxt[k];
      else FMhi = transfer<IT, POL>(AM.x, cur.q[k], nxt.q[k]);
      out[k] = wsub<IT>(wsub<IT>(cur.q[k], cur.d[k]), wsub<IT>(FMhi, FMlo[k]));
      if (AM.bc == FQNM_BC_OUTFLOW && (j == 0 || j == M.nm - 1) && k < M.nvalid) {  // uniform
        if (j == 0) led += static_cast<long long>(FMlo[k]);
        if (j == M.nm - 1) led -= static_cast<long long>(FMhi);
      }
      FMlo[k] = FMhi;
    }
    led += cur.led;
    if (j + 2 <= jend) {  // uniform
      M.process(S, cur, pmm_cur);
      if (j + 4 <= jend) M.load(j + 4, S);
    }
    if (M.vec_row) {
      nd_store<IT, V>(dst + off + M.x0, out);
    } else {
#pragma unroll
      for (int k = 0; k < V; ++k)
        if (k < M.nvalid) dst[off + M.x0 + k] = out[k];
    }
  };
  for (int64_t j = j0; j < jend; j += 2) {
    row(j, S0, rb, rc, pmm_c, pmm_b);
    if (j + 1 < jend) row(j + 1, S1, rc, rb, pmm_b, pmm_c);
  }
  if (led != 0)
    atomicAdd(reinterpret_cast<unsigned long long*>(ledger), static_cast<unsigned long long>(led));
}

template <typename IT, int POL, int V>
hipError_t nd_launch(const void* src, void* dst, const NdParams& P, int rows, long long* led,
                     hipStream_t s) {
  const int64_t nx = P.ax[0].n;
  const int64_t nstrips = (nx + 64 * V - 1) / (64 * V);
  const int64_t nm = P.ax[P.dim - 1].n;
  const int64_t nrb = (nm + rows - 1) / rows;
  const int64_t ny = P.dim == 3 ? P.ax[1].n : 1;
  const int64_t nwaves = nstrips * ny * nrb;
  const int64_t blocks = (nwaves + 3) / 4;
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  const int vec_ok = (nx * static_cast<int64_t>(sizeof(IT))) % NdVec<IT, V>::BYTES == 0;
  const IT* a = static_cast<const IT*>(src);
  IT* b = static_cast<IT*>(dst);
  if (P.dim == 2)
    k_nd_march<IT, POL, V, 2><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(a, b, P, rows, nstrips,
                                                                           nwaves, vec_ok, led);
  else
    k_nd_march<IT, POL, V, 3><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(a, b, P, rows, nstrips,
                                                                           nwaves, vec_ok, led);
  return hipGetLastError();
}

template <typename IT, int POL>
hipError_t nd_by_vec(int vec, const void* src, void* dst, const NdParams& P, int rows,
                     long long* led, hipStream_t s) {
  if constexpr (sizeof(IT) == 4) {
    switch (vec) {
      case 2: return nd_launch<IT, POL, 2>(src, dst, P, rows, led, s);
      case 4: return nd_launch<IT, POL, 4>(src, dst, P, rows, led, s);
      case 8: return nd_launch<IT, POL, 8>(src, dst, P, rows, led, s);
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (vec) {
      case 2: return nd_launch<IT, POL, 2>(src, dst, P, rows, led, s);
      case 4: return nd_launch<IT, POL, 4>(src, dst, P, rows, led, s);
      default: return hipErrorInvalidValue;
    }
  }
}

template <typename IT>
hipError_t nd_by_pol(int pol, int vec, const void* src, void* dst, const NdParams& P, int rows,
                     long long* led, hipStream_t s) {
  switch (pol) {
    case P_UPWIND_POS: return nd_by_vec<IT, P_UPWIND_POS>(vec, src, dst, P, rows, led, s);
    case P_EO: return nd_by_vec<IT, P_EO>(vec, src, dst, P, rows, led, s);
    case P_GODUNOV: return nd_by_vec<IT, P_GODUNOV>(vec, src, dst, P, rows, led, s);
    case P_MURMAN_ROE: return nd_by_vec<IT, P_MURMAN_ROE>(vec, src, dst, P, rows, led, s);
    case P_LF_LINEAR: return nd_by_vec<IT, P_LF_LINEAR>(vec, src, dst, P, rows, led, s);
    case P_LF_BURGERS: return nd_by_vec<IT, P_LF_BURGERS>(vec, src, dst, P, rows, led, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool nd_variant_available(int itype, int pol, int vec) {
  if (pol != P_UPWIND_POS && pol != P_EO && pol != P_GODUNOV && pol != P_MURMAN_ROE &&
      pol != P_LF_LINEAR && pol != P_LF_BURGERS)
    return false;
  return itype == FQNM_I32 ? (vec == 2 || vec == 4 || vec == 8) : (vec == 2 || vec == 4);
}

hipError_t launch_nd(int itype, int pol, int vec, int rows, const void* src, void* dst,
                     const NdParams& P, long long* d_ledger, hipStream_t s) {
  if (!nd_variant_available(itype, pol, vec) || rows < 1 || (P.dim != 2 && P.dim != 3))
    return hipErrorInvalidValue;
  if (itype == FQNM_I32) return nd_by_pol<int32_t>(pol, vec, src, dst, P, rows, d_ledger, s);
  return nd_by_pol<int64_t>(pol, vec, src, dst, P, rows, d_ledger, s);
}

}  // namespace fqnm
