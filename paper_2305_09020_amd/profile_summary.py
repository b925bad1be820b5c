"""Condense rocprofv3 output of bench.py runs into the short text summaries kept under
profiles/ (kernel-time table per workload; HBM bytes per launch per kernel class from the
FETCH_SIZE / WRITE_SIZE counters, scaled by what the counters read for a plain device copy).

Usage: python -m paper_2305_09020_amd.profile_summary <rocprof output dir> <profiles dir>
where the output dir holds stats_<wl>/, {FETCH,WRITE}_SIZE_<wl>_<path>/ and
{FETCH,WRITE}_SIZE_copy/ as written by the commands listed in each summary."""
import collections
import csv
import os
import sys

CLASSES = [("gemm64", lambda n: ("k_gemm" in n or "k_fdm" in n) and ("<double" in n or "IdE" in n)),
           # FP32 matrix-core passes: the GEMMs and fused middle passes in float, and the
           # refined path's first / last pass kernels (k_srp, k_p4), which compute in FP32
           ("gemm32", lambda n: (("k_gemm" in n or "k_fdm" in n) and ("<float" in n or "IfE" in n))
            or "k_p4" in n or "k_srp" in n),
           ("residual", lambda n: "k_residual" in n or "k_res_p1" in n),
           ("zfft", lambda n: "k_zfft" in n),
           ("element", lambda n: "_elem" in n),
           ("nodal", lambda n: "_rhs" in n or "k_E_nodal" in n or "k_Phi_hat3" in n or "k_phi_bnd3" in n)]

WORKLOADS = {"c2": ("2D benchmark workload: 20x20 elements, K = 8, 4 instances (161 x 161 x 4 nodes)", 200, 10),
             "c3": ("3D workload: 16x16 elements, K = 8, 128 Fourier planes (129 x 129 x 128 nodes)", 10, 3)}


def _sha():
    import hashlib
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "pfd_kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()


def cls_of(name):
    for c, f in CLASSES:
        if f(name):
            return c
    return "other"


def counters(path):
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(os.path.join(path, "run_counter_collection.csv"))):
        agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return agg


def main(src, dst):
    cf = counters(os.path.join(src, "FETCH_SIZE_copy"))["__amd_rocclr_copyBuffer"]
    cw = counters(os.path.join(src, "WRITE_SIZE_copy"))["__amd_rocclr_copyBuffer"]
    copy_kib = 256 * 1024
    fs, ws = copy_kib / (sum(cf) / len(cf)), copy_kib / (sum(cw) / len(cw))
    for wl, (desc, steps, psteps) in WORKLOADS.items():
        lines = ["# Kernel time, %s; FP32-refined then plain-FP64 context in one process" % desc,
                 "# command (from /tmp, TMPDIR=/tmp):",
                 "#   rocprofv3 --kernel-trace --stats --output-format csv -d <out>/stats_%s -o run -- "
                 "python3 bench.py --workload %s --steps %d --warmup 2 --no-cpu-baseline" % (wl, wl, steps),
                 "# includes each context's create (autotuner), initial-potential fixed point and the bench's",
                 "# instrumented and replay runs; kernel durations are the profiler's",
                 "#", "# %-64s %7s %12s %10s %6s %s" % ("kernel", "calls", "total_us", "avg_us", "pct", "class")]
        tot = collections.defaultdict(lambda: [0.0, 0])
        rows = list(csv.DictReader(open(os.path.join(src, "stats_%s" % wl, "run_kernel_stats.csv"))))
        # the autotuner's stream holds (k_hold: a timed wait before each timing run) are no work
        holds = [r for r in rows if "k_hold" in r["Name"]]
        rows = [r for r in rows if "k_hold" not in r["Name"]]
        grand = sum(float(r["TotalDurationNs"]) for r in rows)
        if holds:
            lines.insert(5, "# (the autotuner's stream holds, k_hold: %d launches, %.1f us, are left out)"
                         % (sum(int(r["Calls"]) for r in holds), sum(float(r["TotalDurationNs"]) for r in holds) / 1e3))
        for r in rows:
            n = r["Name"]
            c = cls_of(n)
            tot[c][0] += float(r["TotalDurationNs"])
            tot[c][1] += int(r["Calls"])
            pct = 100.0 * float(r["TotalDurationNs"]) / grand
            if pct >= 0.3:
                lines.append("  %-64s %7s %12.1f %10.2f %6.2f %s" % (n.split("(")[0][:64], r["Calls"],
                             float(r["TotalDurationNs"]) / 1e3, float(r["AverageNs"]) / 1e3, pct, c))
        lines.append("#")
        for c, (t, n) in sorted(tot.items(), key=lambda kv: -kv[1][0]):
            lines.append("# class %-9s %8.1f us total, average launch %8.2f us over %d launches" % (c, t / 1e3, t / n / 1e3, n))
        open(os.path.join(dst, "kernel_stats_%s.txt" % wl), "w").write("\n".join(lines) + "\n")
        # HBM traffic per launch per class
        out = ["# HBM traffic per launch by kernel class, %s" % desc,
               "# commands (from /tmp, TMPDIR=/tmp), one counter per run, <path> = refined | fp64:",
               "#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out>/FETCH_SIZE_%s_<path> -o run -- "
               "python3 bench.py --workload %s --steps %d --warmup 1 --no-cpu-baseline --only <path>" % (wl, wl, psteps),
               "#   rocprofv3 --pmc WRITE_SIZE ... (same, -d <out>/WRITE_SIZE_%s_<path>)" % wl,
               "#   rocprofv3 --pmc FETCH_SIZE|WRITE_SIZE --output-format csv -d <out>/<CTR>_copy -o run -- "
               "python3 bench.py --calibrate-copy",
               "# copy calibration: a 256 MiB device copy reads FETCH_SIZE %.0f KiB and WRITE_SIZE %.0f KiB,"
               % (sum(cf) / len(cf), sum(cw) / len(cw)),
               "# so FETCH_SIZE x %.3f and WRITE_SIZE x %.3f give bytes moved" % (fs, ws),
               "# (averages over every dispatch of the class in the run, autotuned kernels as chosen there;",
               "#  L2 write-backs are counted when they happen, so WRITE_SIZE of one class can land on another)",
               "# kernel source sha256 (pfd_kernels.hip): %s" % _sha(),
               "#", "# %-8s %-9s %10s %14s %14s %16s" % ("path", "class", "launches", "fetch_KiB", "write_KiB",
                                                        "hbm_bytes/launch")]
        for path in ("refined", "fp64"):
            F = counters(os.path.join(src, "FETCH_SIZE_%s_%s" % (wl, path)))
            W = counters(os.path.join(src, "WRITE_SIZE_%s_%s" % (wl, path)))
            agg = collections.defaultdict(lambda: [0.0, 0.0, 0])
            for k, v in F.items():
                c = cls_of(k)
                agg[c][0] += sum(v)
                agg[c][2] += len(v)
            for k, v in W.items():
                agg[cls_of(k)][1] += sum(v)
            for c, (f, w, n) in sorted(agg.items()):
                if n == 0 or c == "other":
                    continue
                out.append("  %-8s %-9s %10d %14.1f %14.1f %16.0f" % (path, c, n, f / n, w / n,
                                                                    1024 * (f / n * fs + w / n * ws)))
        open(os.path.join(dst, "hbm_traffic_%s.txt" % wl), "w").write("\n".join(out) + "\n")


if __name__ == "__main__":
    main(sys.argv[1], sys.argv[2])
