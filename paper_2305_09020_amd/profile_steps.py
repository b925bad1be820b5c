"""Steady-state steps for the profiler: build a benchmark workload's context exactly as
bench.py does (graph replays, autotuned kernels), run the warm-up steps, then the measured
steps between two marker kernels (torch's device sleep, a kernel named spin_kernel) so
that a rocprofv3 kernel trace or counter collection of this process can be cut to the
steps alone (the autotuner, the initial potential and the warm-up fall outside).

Usage (from the repository root):
  python -m paper_2305_09020_amd.profile_steps --workload c2 --path refined --steps 50
"""
import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--path", choices=["refined", "fp64"], default="refined")
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    a = ap.parse_args()
    sys.path.insert(0, ROOT)
    import torch
    import bench
    import paper_2305_09020_amd as pfd
    prec = pfd.REFINED_FP32 if a.path == "refined" else pfd.PLAIN_FP64
    run = bench.build_workload(a.workload, prec)
    run.step(a.warmup)
    torch.cuda.synchronize()
    st = run.stream
    with torch.cuda.stream(st):
        torch.cuda._sleep(1000)   # marker: the measured steps follow
    run.step_async(a.steps)
    with torch.cuda.stream(st):
        torch.cuda._sleep(1000)   # marker: the measured steps ended
    torch.cuda.synchronize()
    print("profiled %d steps of %s (%s path)" % (a.steps, a.workload, a.path), flush=True)


if __name__ == "__main__":
    main()
