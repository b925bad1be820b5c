"""Condense rocprofv3 output of steady-state steps (paper_2305_09020_amd.profile_steps) into
the short text summaries kept under profiles/:

  kernel_stats_<wl>.txt   per kernel and per kernel class: launches and device time per
                          step, average launch, share of the step's kernel time;
  hbm_traffic_<wl>.txt    HBM bytes per step and per launch of each class from the FETCH_SIZE
                          and WRITE_SIZE counters (KiB per dispatch), each scaled by what the
                          same counter reads for a plain device copy of known size.

Only the dispatches between the two marker kernels (spin_kernel) that profile_steps launches
around its measured steps are counted: the autotuner, the initial potential and the warm-up
steps fall outside.

Usage: python -m paper_2305_09020_amd.profile_summary <rocprof output dir> <profiles dir>
where the output dir holds trace_<wl>_<path>/, fetch_<wl>_<path>/, write_<wl>_<path>/,
fetch_copy/ and write_copy/ as written by the commands each summary lists."""
import collections
import csv
import glob
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))

CLASSES = [("gemm64", lambda n: ("k_gemm" in n or "k_fdm" in n) and ("<double" in n or "IdE" in n)),
           # FP32 matrix-core passes: the GEMMs and fused middle passes in float, and the
           # refined path's first / last pass kernels (k_srp, k_p4), which compute in FP32
           ("gemm32", lambda n: (("k_gemm" in n or "k_fdm" in n) and ("<float" in n or "IfE" in n))
            or "k_p4" in n or "k_srp" in n),
           ("residual", lambda n: "k_residual" in n or "k_res_p1" in n),
           ("zfft", lambda n: "k_zfft" in n),
           ("element", lambda n: "_elem" in n),
           ("nodal", lambda n: "_rhs" in n or "k_E_nodal" in n or "k_Phi_hat3" in n or "k_phi_bnd3" in n)]

# workload: (description, measured steps of the trace, measured steps of the counter passes)
WORKLOADS = {"c2": ("2D benchmark workload: 20x20 elements, K = 8, 4 instances (161 x 161 x 4 nodes)", 50, 5),
             "c3": ("3D workload: 16x16 elements, K = 8, 128 Fourier planes (129 x 129 x 128 nodes)", 10, 2),
             "c4": ("batched workload: 64 uneven 2D instances (n x n elements, n 8..24, order 4..10) as "
                    "multi-instance launches", 20, 2)}
PATHS = ("refined", "fp64")


def sources_sha():
    h = hashlib.sha256()
    cs = os.path.join(HERE, "csrc")
    for f in sorted(os.listdir(cs)):
        if f.endswith((".hip", ".cpp", ".h")):
            h.update(open(os.path.join(cs, f), "rb").read())
    return h.hexdigest()


def cls_of(name):
    for c, f in CLASSES:
        if f(name):
            return c
    return "other"


def short(name):
    """Kernel name without its parameter list; a kernel of the launch layer (k_single /
    k_multi<body, argument types...>) is named by its body, multi-instance launches marked."""
    n = name.split("(")[0]
    for w in ("k_single_w<", "k_single<", "k_multi_w<", "k_multi<"):
        i = n.find(w)
        if i < 0:
            continue
        inner, d, j = n[i + len(w):], 0, 0
        for j, ch in enumerate(inner):
            if ch == "<":
                d += 1
            elif ch == ">":
                if d == 0:
                    break
                d -= 1
            elif ch == "," and d == 0:
                break
        return inner[:j].replace("pfd::", "").strip() + (" [multi]" if "multi" in w else "")
    return n


def _rows(d, fname):
    files = glob.glob(os.path.join(d, "**", fname), recursive=True)
    if not files:
        raise FileNotFoundError(os.path.join(d, fname))
    return list(csv.DictReader(open(files[0])))


def window(rows):
    """The rows strictly between the two marker kernels, in dispatch order."""
    rows = sorted(rows, key=lambda r: int(r["Dispatch_Id"]))
    marks = [i for i, r in enumerate(rows) if "spin_kernel" in r["Kernel_Name"]]
    if len(marks) < 2:
        raise ValueError("marker kernels not found")
    return rows[marks[-2] + 1:marks[-1]]


def trace_stats(d, steps):
    per = collections.defaultdict(lambda: [0, 0.0])
    for r in window(_rows(d, "run_kernel_trace.csv")):
        a = per[short(r["Kernel_Name"])]
        a[0] += 1
        a[1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
    return {k: (v[0] / steps, v[1] / steps) for k, v in per.items()}   # launches, us per step


def counter_kib(d):
    per = collections.defaultdict(list)
    for r in window(_rows(d, "run_counter_collection.csv")):
        per[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return per


def copy_scale(d):
    vals = [float(r["Counter_Value"]) for r in _rows(d, "run_counter_collection.csv")
            if "copyBuffer" in r["Kernel_Name"]]
    big = max(vals)   # the 256 MiB copies (small runtime copies read far less)
    return 256 * 1024 / big


def command(wl, path, what, steps):
    prog = "python3 -m paper_2305_09020_amd.profile_steps --workload %s --path %s --steps %d" % (wl, path, steps)
    if what == "trace":
        return "rocprofv3 --kernel-trace --output-format csv -d <out>/trace_%s_%s -o run -- %s" % (wl, path, prog)
    return ("timeout -s KILL 300 rocprofv3 --pmc %s_SIZE --output-format csv -d <out>/%s_%s_%s -o run -- %s"
            % (what.upper(), what, wl, path, prog))


def main(src, dst):
    fs = copy_scale(os.path.join(src, "fetch_copy"))
    ws = copy_scale(os.path.join(src, "write_copy"))
    sha = sources_sha()
    for wl, (desc, steps, csteps) in WORKLOADS.items():
        if not any(os.path.isdir(os.path.join(src, "trace_%s_%s" % (wl, p))) for p in PATHS):
            continue   # no trace of this workload in src: its summaries stay as they are
        lines = ["# Kernel time per step of the steady-state steps, %s" % desc,
                 "# commands (from /tmp, TMPDIR=/tmp; repository root as working directory of python3):"]
        for p in PATHS:
            lines.append("#   " + command(wl, p, "trace", steps))
        lines += ["# only the dispatches between profile_steps' two marker kernels are counted (no set-up,",
                  "# autotuning, initial potential or warm-up); durations are the profiler's",
                  "# library sources sha256 %s" % sha]
        tlines = ["# HBM bytes of the steady-state steps, %s" % desc,
                  "# FETCH_SIZE and WRITE_SIZE (KiB per dispatch, own runs), scaled by a plain 256 MiB device",
                  "# copy: FETCH x %.3f, WRITE x %.3f; commands:" % (fs, ws)]
        for p in PATHS:
            for what in ("fetch", "write"):
                tlines.append("#   " + command(wl, p, what, csteps))
        tlines += ["#   timeout -s KILL 300 rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out>/fetch_copy -o "
                   "run -- python3 bench.py --calibrate-copy   (and WRITE_SIZE -> <out>/write_copy)",
                   "# library sources sha256 %s" % sha,
                   "# step <path> <bytes per step> | class <path> <class> <bytes per launch>"]
        for p in PATHS:
            tdir = os.path.join(src, "trace_%s_%s" % (wl, p))
            if not os.path.isdir(tdir):
                continue
            st = trace_stats(tdir, steps)
            tot_us = sum(v[1] for v in st.values())
            lines += ["#", "## %s path: %.1f us of kernel time per step, %.1f launches per step"
                      % (p, tot_us, sum(v[0] for v in st.values())),
                      "# %-60s %9s %10s %9s %6s %s" % ("kernel", "per_step", "us/step", "avg_us", "pct", "class")]
            cls = collections.defaultdict(lambda: [0.0, 0.0])
            for k, (n, us) in sorted(st.items(), key=lambda kv: -kv[1][1]):
                lines.append("  %-60s %9.2f %10.2f %9.2f %6.2f %s" % (k[:60], n, us, us / n, 100 * us / tot_us, cls_of(k)))
                cls[cls_of(k)][0] += n
                cls[cls_of(k)][1] += us
            lines.append("# class totals per step: launches, us, avg us per launch, pct")
            for c, (n, us) in sorted(cls.items(), key=lambda kv: -kv[1][1]):
                lines.append("  class %-10s %8.2f %10.2f %9.2f %6.2f" % (c, n, us, us / n, 100 * us / tot_us))
            fdir, wdir = os.path.join(src, "fetch_%s_%s" % (wl, p)), os.path.join(src, "write_%s_%s" % (wl, p))
            if os.path.isdir(fdir) and os.path.isdir(wdir):
                fk, wk = counter_kib(fdir), counter_kib(wdir)
                byc = collections.defaultdict(lambda: [0.0, 0])
                step_bytes = 0.0
                for k in fk:
                    b = 1024.0 * (fs * sum(fk[k]) + ws * sum(wk.get(k, [])))
                    step_bytes += b / csteps
                    byc[cls_of(k)][0] += b
                    byc[cls_of(k)][1] += len(fk[k])
                tlines.append("step %s %.0f" % (p, step_bytes))
                for c, (b, n) in sorted(byc.items()):
                    tlines.append("class %s %s %.0f" % (p, c, b / n))
        open(os.path.join(dst, "kernel_stats_%s.txt" % wl), "w").write("\n".join(lines) + "\n")
        if len(tlines) > 12:
            open(os.path.join(dst, "hbm_traffic_%s.txt" % wl), "w").write("\n".join(tlines) + "\n")


if __name__ == "__main__":
    main(sys.argv[1], sys.argv[2])
