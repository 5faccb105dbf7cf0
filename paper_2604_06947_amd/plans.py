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

# Counter results of the timed kernels (rocprofv3 runs recorded under
# profiles/), per launch of the benchmark's plan: HBM traffic (FETCH_SIZE and
# WRITE_SIZE scaled by a plain device copy of known size), VALU
# wavefront-instructions (SQ_INSTS_VALU) and the share of LDS-active cycles
# lost to bank conflicts.  Valid only for the kernel sources they were
# measured on: the benchmark reports null when the hash of those sources
# (first 16 hex digits of SHA-256 over the files in order) differs.
KERNEL_SOURCES = ("csrc/scalar.hip", "csrc/fqnm_device.h")
ND_KERNEL_SOURCES = ("csrc/nd_tb.hip", "csrc/nd_common.h", "csrc/fqnm_device.h")
EULER_KERNEL_SOURCES = ("csrc/euler.hip", "csrc/fqnm_device.h")
COUNTERS = {
    "w2": {"sources": KERNEL_SOURCES, "sources_sha": None, "traffic_bytes": None,
           "valu_insts": None, "lds_bank_conflict_frac": None},
    "w3_stream": {"sources": KERNEL_SOURCES, "sources_sha": None, "traffic_bytes": None,
                  "valu_insts": None, "lds_bank_conflict_frac": None},
    "w6": {"sources": ND_KERNEL_SOURCES, "sources_sha": None, "traffic_bytes": None,
           "valu_insts": None, "lds_bank_conflict_frac": None},
    "euler_multi": {"sources": EULER_KERNEL_SOURCES, "sources_sha": None, "traffic_bytes": None,
                    "valu_insts": None, "lds_bank_conflict_frac": None},
}

# the FP64 finite-volume twin of the Burgers workload, same tiling machinery
TWIN_PLAN_W2 = (KERNEL_TBLOCK, 4, 24)

# W6 (2-D Burgers, 4096 x 4096 int32): marching with temporal blocking --
# kernel, cells per lane, steps per pass, rows per wavefront; and the
# one-step-per-pass marching kernel (cells per lane, rows) timed beside it
KERNEL_ND_MARCH, KERNEL_ND_TB = 6, 9
ND_PLAN_W6 = (KERNEL_ND_TB, 2, 4, 24)
ND_MARCH_PLAN_W6 = (8, 12)
