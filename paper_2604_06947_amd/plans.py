"""Launch plans (kernel, cells per lane, steps per pass) used by the benchmark
for its timed workloads, chosen from autotuner sweeps on MI355X.  The parity
tests run the same plans at full size."""
from .fqnm import KERNEL_STREAM, KERNEL_TBLOCK

# Burgers, 2^20 int32 cells, Engquist-Osher LUT, 10000 steps
BENCH_PLAN_W2 = (KERNEL_TBLOCK, 4, 52)
# near-Nyquist advection, 2^24 int64 cells, 2000 steps
BENCH_PLAN_W3 = (KERNEL_TBLOCK, 16, 48)
# the one-step-per-pass streaming plan reported beside it
STREAM_PLAN_W3 = (KERNEL_STREAM, 4, 1)

# Counter results of the timed kernels (rocprofv3 runs recorded under
# profiles/), as means per launch over the launches of one solve of the
# benchmark's plan: HBM traffic (FETCH_SIZE and WRITE_SIZE, each scaled by
# what the counter reads for a plain device copy of known size: FETCH x
# 1.99982, WRITE x 1.0), VALU wavefront-instructions (SQ_INSTS_VALU), the
# share of LDS-active cycles lost to bank conflicts and, for the FP64 Euler
# kernels, FP64 VALU wavefront-instructions.  Valid only for the kernel
# sources they were measured on: the benchmark reports null when the hash of
# those sources (first 16 hex digits of SHA-256 over the files in order)
# differs.
KERNEL_SOURCES = ("csrc/scalar.hip", "csrc/fqnm_device.h")
ND_KERNEL_SOURCES = ("csrc/nd_tb.hip", "csrc/nd_common.h", "csrc/fqnm_device.h")
EULER_KERNEL_SOURCES = ("csrc/euler.hip", "csrc/fqnm_device.h")
COUNTERS = {
    # k_tblock<int, P_LUT, 4>, 52 steps per launch: 192 launches of 52 steps and
    # one of 16 per 10000-step solve
    "w2": {"sources": KERNEL_SOURCES, "sources_sha": "301355d6fae1597f",
           "traffic_bytes": 11704636, "valu_insts": 4624531,
           "lds_bank_conflict_frac": 0.6126},
    # k_stream<long, P_UPWIND_POS, 4>, one step per launch
    "w3_stream": {"sources": KERNEL_SOURCES, "sources_sha": "301355d6fae1597f",
                  "traffic_bytes": 268469345, "valu_insts": 4259912,
                  "lds_bank_conflict_frac": None},
    # k_tblock<long, P_UPWIND_POS, 16>, 48 steps per launch: 41 launches of
    # 48 steps and one of 32 per 2000-step solve
    "w3_tblock": {"sources": KERNEL_SOURCES, "sources_sha": "301355d6fae1597f",
                  "traffic_bytes": 268575323, "valu_insts": 60318516,
                  "lds_bank_conflict_frac": None},
    # k_nd_tb<int, P_EO, 2, 4>, 4 steps per launch, 24 rows per wavefront
    "w6": {"sources": ND_KERNEL_SOURCES, "sources_sha": "0f0e3440c669dd13",
           "traffic_bytes": 157065418, "valu_insts": 18522603,
           "lds_bank_conflict_frac": None},
    # k_euler_step, componentwise Sod at 2^20 cells, 8 steps per launch; FP64
    # wavefront-instructions (ADD + MUL + FMA + TRANS) and FLOPs per lane
    # (an FMA counts two)
    "euler_step": {"sources": EULER_KERNEL_SOURCES, "sources_sha": "bcab913dbf5b785a",
                   "traffic_bytes": None, "valu_insts": 43893037,
                   "lds_bank_conflict_frac": None,
                   "f64_insts": 27985480, "f64_flops": 40151560},
    # k_euler_multi over served Sod requests (100 requests, 2^10..2^16
    # cells, one closed loop): wavefront-instructions per cell-update (its
    # launches differ in size, so per-launch means say little)
    "euler_multi": {"sources": EULER_KERNEL_SOURCES, "sources_sha": "bcab913dbf5b785a",
                    "valu_insts_per_cell_update": 5.3061,
                    "f64_insts_per_cell_update": 3.3631,
                    "f64_flops_per_cell_update": 4.8188},
}

# the FP64 finite-volume twin of the Burgers workload, same tiling machinery
TWIN_PLAN_W2 = (KERNEL_TBLOCK, 4, 24)

# W6 (2-D Burgers, 4096 x 4096 int32): marching with temporal blocking --
# kernel, cells per lane, steps per pass, rows per wavefront; and the
# one-step-per-pass marching kernel (cells per lane, rows) timed beside it
KERNEL_ND_MARCH, KERNEL_ND_TB = 6, 9
ND_PLAN_W6 = (KERNEL_ND_TB, 2, 4, 24)
ND_MARCH_PLAN_W6 = (8, 12)
