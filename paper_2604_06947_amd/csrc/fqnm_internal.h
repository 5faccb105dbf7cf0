// fqnm_internal.h -- host-side declarations shared by the library's translation
// units (kernel launchers and the runtime).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/fqnm.h"
#include "fqnm_device.h"

namespace fqnm {

enum : int {
  K_STREAM = 0,
  K_TBLOCK = 1,
  K_TBLOCK_IL = 2,
  K_TBLOCK_B2 = 3,  // workgroup tiles of 2, 4 or 8 wavefronts
  K_TBLOCK_B4 = 4,
  K_TBLOCK_B8 = 5,
  K_ND_MARCH = 6,  // d-D grids: strips along axis 0 marching along the last axis
  K_TBLOCK_WG4 = 7,  // workgroup tiles of 4 or 8 wavefronts with overlapping windows
  K_TBLOCK_WG8 = 8,  // (int32 tables, periodic grids)
  K_ND_TB = 9,       // 2-D grids: several steps per pass
  K_TBLOCK_PERSIST = 10  // every pass of a temporally blocked plan in one cooperative launch
};

// Per-block partial results of the reduction kernel (one record per block).
struct ReducePartial {
  uint64_t sum_lo;
  int64_t sum_hi;
  int64_t qmin;
  int64_t qmax;
  uint64_t tv_lo;
  int64_t tv_hi;
};

// Single-grid scalar stepper: one launch advancing `ksteps` steps from src to
// dst.  kernel = K_STREAM requires ksteps == 1.  Returns hipSuccess or the
// launch error; hipErrorInvalidValue for an unavailable (itype, pol, vec).
hipError_t launch_scalar(int itype, int pol, int kernel, int vec, const void* src, void* dst,
                         int64_t n, int bc, int ksteps, int khalo, const XParams& P,
                         long long* d_ledger, hipStream_t s);
bool scalar_variant_available(int itype, int pol, int kernel, int vec);
int scalar_halo(int kernel, int vec, int ksteps);  // halo width of the temporal-blocking kernels
int scalar_tile_positions(int kernel, int vec);     // cells loaded per tile

// Workgroup tiles with overlapping wavefront windows (K_TBLOCK_WG4/8): int32
// LUT policy, periodic grids, vec 2 or 4, ksteps up to 64*vec - 16.
bool tblock_wg_valid(int nw, int vec, int ksteps);
hipError_t launch_tblock_wg(int nw, int vec, const int32_t* src, int32_t* dst, int64_t n,
                            int ksteps, const XParams& P, hipStream_t s);

// Tiled work items of several grids, one step block per launch (K2 on each
// item's tile).  A grid: its two buffers, size, boundary, halo, constants and
// ledger.  A launch lists, per grid it covers, the steps of this block
// (<= the grid's halo), which buffer it reads (buf0, or buf1 when `parity`
// is set; it writes the other) and the index of the grid's first item
// (entries in increasing `first`, the grid's tiles following it).
struct TileGrid {
  const void* buf0;
  const void* buf1;
  int64_t n;
  int32_t bc;
  int32_t khalo;
  long long* ledger;
  XParams P;
};
struct BlockGrid {
  int64_t first;
  int32_t grid;
  int32_t ksteps;
  int32_t parity;
  int32_t pad_;
};
bool items_variant_available(int itype, int pol, int vec);
// Device copy of `bytes` (a multiple of 4) by a kernel (no copy or memset
// nodes in captured graphs).
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s);
hipError_t launch_tile_items(int itype, int pol, int vec, const BlockGrid* entries,
                             int32_t nentries, int64_t nitems, const TileGrid* grids,
                             hipStream_t s);

// Persistent temporal blocking (K_TBLOCK_PERSIST): int32 states on periodic
// grids, table or direct split policies, vec 4 or 8.  persist_geometry gives
// the halo and the tile count of a plan (false if the grid cannot be tiled
// with at least khalo cells per tile); persist_fits whether the cooperative
// grid can be resident at once; the exchange buffer holds
// 2 * 2 * ntiles * khalo 64-bit words, zero or holding tags below tag0 + 1;
// one launch advances nsteps steps, tags tag0 + 1 .. tag0 + passes - 1.
bool persist_available(int itype, int pol, int vec, int bc);
bool persist_geometry(int64_t n, int vec, int depth, int* khalo, int64_t* ntiles);
hipError_t persist_fits(int pol, int vec, int64_t ntiles, bool* fits);
hipError_t launch_persist(int pol, int vec, const int32_t* src, int32_t* dst, int64_t n,
                          int nsteps, int depth, const XParams& P, uint64_t* exch, uint32_t tag0,
                          int* err, int spin, hipStream_t s);

// FP64 split finite-volume twin (state u in doubles).
bool classical_variant_available(int pol, int kernel, int vec);
hipError_t launch_classical(int pol, int kernel, int vec, const double* src, double* dst,
                            int64_t n, int bc, int ksteps, int khalo, const XParams& P,
                            hipStream_t s);

// d-dimensional grid (d = 2 or 3), axis 0 contiguous.  Each axis carries its
// own one-dimensional rule; all axes share the flux kind, storage type and delta.
struct NdAxis {
  XParams x;       // the axis's map constants (c, h, a, alpha, delta, lambda)
  double cp, cm;   // UPWIND: max(c, 0) and min(c, 0)
  int64_t n;       // cells along the axis
  int32_t bc;
  int32_t pad_;
};
struct NdParams {
  NdAxis ax[3];
  int32_t dim;
  int32_t pad_;
};
bool nd_variant_available(int itype, int pol, int vec);
// One step of eq:nd_transfer_rule from src to dst; `rows` cells of the last
// axis per wavefront.  pol is the direct policy (P_UPWIND_POS stands for
// UPWIND of either sign).
hipError_t launch_nd(int itype, int pol, int vec, int rows, const void* src, void* dst,
                     const NdParams& P, long long* d_ledger, hipStream_t s);
// Temporal blocking on 2-D grids (K_ND_TB): `depth` steps of
// eq:nd_transfer_rule per launch, depth in {1, 2, 4, 8}; vec 2 or 4 (int64: 2)
// and a first axis whose length is a multiple of vec.  nd_tb_step_depth gives the largest
// available depth not above max_depth.
bool nd_tb_valid(int itype, int pol, int vec, const NdParams& P);
int nd_tb_step_depth(int max_depth);
hipError_t launch_nd_tb(int itype, int pol, int vec, int depth, int rows, const void* src,
                        void* dst, const NdParams& P, long long* d_ledger, hipStream_t s);

hipError_t launch_lut_build(int itype, int pol, const XParams& P, void* lut, int64_t lo,
                            int64_t count, int* violation, hipStream_t s);
hipError_t launch_quantise(int itype, const double* u, void* q, int64_t n, double delta,
                           int* d_err, hipStream_t s);
hipError_t launch_reconstruct(int itype, const void* q, double* u, int64_t n, double delta,
                              hipStream_t s);
// Reduction over a state of n integers; writes reduce_blocks(n) partials.
int64_t reduce_blocks(int64_t n);
hipError_t launch_reduce(int itype, const void* q, int64_t n, int periodic, ReducePartial* out,
                         hipStream_t s);
// The same with cpb cells per block (ceil(n / cpb) partials), and the
// combination of count partials into one record out[0].
int64_t reduce_min_cells_per_block();
hipError_t launch_reduce_cpb(int itype, const void* q, int64_t n, int periodic, int64_t cpb,
                             ReducePartial* out, hipStream_t s);
hipError_t launch_reduce_final(const ReducePartial* in, int count, ReducePartial* out,
                               hipStream_t s);

// Euler (3 x 8-byte components, structure of arrays): one step per launch.
struct EulerParams {
  double delta;
  double lambda;
  double g1;  // gamma - 1
  int fix;    // entropy fix on the acoustic waves
  int dens;   // density-only: components 1, 2 hold FP64 m and E (bit patterns)
  int* err;   // set to 1 when a cell's density or pressure is not positive
              // (or not a number) at the start of a step; sticky, may be null
};
// nsteps (1 .. euler_steps_per_launch()) steps in one launch.
hipError_t launch_euler_step(const int64_t* src, int64_t* dst, int64_t n, int bc,
                             const EulerParams& E, int nsteps, long long* d_ledger, hipStream_t s);
int euler_steps_per_launch();

// Many Euler problems advanced together, one step per launch.
struct EulerReq {
  int64_t* buf0;
  int64_t* buf1;
  int64_t n;
  int32_t bc;
  int32_t steps;   // steps this request takes in the current tick
  int32_t parity;  // buffer holding its state at the start of the tick
  int32_t pad_;
  long long* ledger;
  EulerParams E;
};
struct EulerTile {
  int32_t req;
  int32_t pad_;
  int64_t start;   // first cell of the tile
};
int64_t euler_tiles(int64_t n);
int64_t euler_tile_cells();
// Steps s .. s + euler_steps_per_launch() - 1 of the current tick (s a
// multiple of euler_steps_per_launch()), for every request that has them.
hipError_t launch_euler_multi(const EulerTile* d_tiles, int64_t ntiles, const EulerReq* d_reqs,
                              int s, hipStream_t st);

// Register-resident scalar instances (int32 cells), run by the persistent
// batch kernel: each instance advances `steps` steps in place.
struct ResidentInst {
  int64_t off;     // first cell in the state array
  int32_t n;
  int32_t steps;
  int32_t pol;
  int32_t vec;
  int32_t bc;
  int32_t cls;     // which persistent kernel runs it (resident_layout)
  double c;
  double h;
};
bool resident_eligible(const fqnm_problem& p, int pol, int64_t steps);
// cells per lane and kernel class of a resident instance of n cells
void resident_layout(int64_t n, int pol, int32_t* vec, int32_t* cls);
// The same under a batch layout (fqnm_batch_config; zero fields: default).
void resident_layout_cfg(int64_t n, int pol, const fqnm_batch_config& cfg, int32_t* vec,
                         int32_t* cls);
bool batch_config_valid(const fqnm_batch_config& c);
// Launch state of the persistent batch kernels (one per register-footprint
// class): the classes other than the widest nonempty one run on the side
// streams, forked from the caller's stream by `fork` and joined back by
// `join`; d_counters holds the kernels' work counters.
constexpr int RCLASSES = 3;
struct ResidentLauncher {
  hipStream_t side[RCLASSES - 1] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[RCLASSES - 1] = {};
  int32_t* d_counters = nullptr;
};
fqnm_status resident_launcher_init(ResidentLauncher* L);
void resident_launcher_free(ResidentLauncher* L);
// instances of each class among insts[0..count)
void resident_class_counts(const ResidentInst* insts, int32_t count, int32_t* per_class);
hipError_t launch_resident(const ResidentInst* d_insts, const int32_t* d_order, int32_t count,
                           const int32_t* per_class, const ResidentLauncher& L, int32_t* d_state,
                           hipStream_t s);

// Thread-local error message of the public ABI.
void set_error(const std::string& msg);

}  // namespace fqnm
