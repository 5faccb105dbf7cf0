"""Launch plans (kernel, cells per lane, steps per pass) used by the benchmark
for its timed workloads, chosen from autotuner sweeps on MI355X.  The parity
tests run the same plans at full size."""
from .fqnm import KERNEL_STREAM, KERNEL_TBLOCK

# Burgers, 2^20 int32 cells, Engquist-Osher LUT, 10000 steps
BENCH_PLAN_W2 = (KERNEL_TBLOCK, 4, 40)
# near-Nyquist advection, 2^24 int64 cells, 2000 steps
BENCH_PLAN_W3 = (KERNEL_TBLOCK, 8, 24)
# the one-step-per-pass streaming plan reported beside it
STREAM_PLAN_W3 = (KERNEL_STREAM, 4, 1)

# HBM traffic per launch of the timed kernels, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs scaled by a plain device copy of known size (see profiles/).
# Valid only for the kernel sources they were measured on: the benchmark
# reports null when the hash of those sources differs.
KERNEL_SOURCES = ("csrc/scalar.hip", "csrc/fqnm_device.h")
MEASURED_SOURCES_SHA = "cce23d36ccc8e6ea"
TRAFFIC_BYTES_PER_LAUNCH = {
    "w2": 11415 * 1024,  # k_tblock<int, P_LUT, 4>, 40 steps per launch
    "w6": 153359 * 1024,  # k_nd_tb<int, P_EO, 2, 4, true>, 24 rows per wavefront, 4 steps
}
ND_KERNEL_SOURCES = ("csrc/nd_tb.hip", "csrc/nd_common.h", "csrc/fqnm_device.h")
ND_MEASURED_SOURCES_SHA = "beac81b3b4612721"

# the FP64 finite-volume twin of the Burgers workload, same tiling machinery
TWIN_PLAN_W2 = (KERNEL_TBLOCK, 4, 24)

# W6 (2-D Burgers, 4096 x 4096 int32): marching with temporal blocking --
# kernel, cells per lane, steps per pass, rows per wavefront; and the
# one-step-per-pass marching kernel (cells per lane, rows) timed beside it
KERNEL_ND_MARCH, KERNEL_ND_TB = 6, 9
ND_PLAN_W6 = (KERNEL_ND_TB, 2, 4, 24)
ND_MARCH_PLAN_W6 = (8, 12)
