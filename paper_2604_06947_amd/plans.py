"""Launch plans (kernel, cells per lane, steps per pass) used by the benchmark
for its timed workloads, chosen from autotuner sweeps on MI355X.  The parity
tests run the same plans at full size."""
from .fqnm import KERNEL_STREAM, KERNEL_TBLOCK

# Burgers, 2^20 int32 cells, Engquist-Osher LUT, 10000 steps
BENCH_PLAN_W2 = (KERNEL_TBLOCK, 16, 32)
# near-Nyquist advection, 2^24 int64 cells, 2000 steps
BENCH_PLAN_W3 = (KERNEL_TBLOCK, 8, 16)
# the one-step-per-pass streaming plan reported beside it
STREAM_PLAN_W3 = (KERNEL_STREAM, 4, 1)
