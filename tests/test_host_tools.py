"""Host-side logic around the library: the bench refuses more than one GPU, and the profile
summaries put each kernel in the class the bench's roofline uses (CPU only)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_bench_refuses_more_than_one_gpu():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""   # no bench line


def test_profile_summary_classes():
    from paper_2305_09020_amd.profile_summary import cls_of
    cases = {
        "void pfd::k_fdm_mid<float, 1, 2>(int, int)": "gemm32",
        "void pfd::k_fdm_mid<double, 1, 1>(int, int)": "gemm64",
        "void pfd::k_gemm_sr<double, double, 2, 3, 1>(double const*)": "gemm64",
        "void pfd::k_gemm_sr<float, double, 0, 3, 1>(double const*)": "gemm32",
        "void pfd::k_p4<2, 1, 4>(float const*)": "gemm32",
        "void pfd::k_srp<double, 0>(double const*)": "gemm32",   # FP64 input, FP32 matrix cores
        "void pfd::k_res_p1<8, 3>(int)": "residual",
        "void pfd::k_residual_lds<8>(int)": "residual",
        "void pfd::k_zfft<7, false>(pfd::ZBatch)": "zfft",
        "void pfd::k_mom_elem<true>(pfd::Geo)": "element",
        "pfd::k_spec_rhs(pfd::Geo)": "nodal",
        "pfd::k_E_nodal(pfd::Geo)": "nodal",
        "pfd::k_hold(long long)": "other",
        "pfd::k_check_finite(long)": "other",
    }
    for name, cls in cases.items():
        assert cls_of(name) == cls, (name, cls_of(name), cls)


def test_profile_summary_names_launch_layer_kernels():
    """Kernels of the launch layer (single- and multi-instance forms of a body, with or without
    the waves-per-EU request) are named by their body, multi-instance launches marked, and
    land in the body's class."""
    from paper_2305_09020_amd.profile_summary import short, cls_of
    cases = {
        "void pfd::k_single<pfd::k_gemm_sr<float, double, 0, 3, 1>, double const*, float const*, int>"
        "(double const*, float const*, int)": ("k_gemm_sr<float, double, 0, 3, 1>", "gemm32"),
        "void pfd::k_multi<pfd::k_residual<0>, int, int>(unsigned int, unsigned int const*, "
        "pfd::MEnt const*, pfd::Tup<int, int> const*)": ("k_residual<0> [multi]", "residual"),
        "void pfd::k_single_w<pfd::k_fdm_mid<double, 1, 1>, int>(int)": ("k_fdm_mid<double, 1, 1>", "gemm64"),
        "void pfd::k_multi_w<pfd::k_res_p1<8, 3>, int>(unsigned int)": ("k_res_p1<8, 3> [multi]", "residual"),
        "void pfd::k_single<pfd::k_V_rhs, pfd::Geo, pfd::Par>(pfd::Geo, pfd::Par)": ("k_V_rhs", "nodal"),
        "void pfd::k_multi<pfd::k_mom_elem<false>, pfd::Geo>(unsigned int)": ("k_mom_elem<false> [multi]",
                                                                             "element"),
        "pfd::k_hold(long long)": ("pfd::k_hold", "other"),
    }
    for name, (sname, cls) in cases.items():
        assert short(name) == sname, (name, short(name))
        assert cls_of(short(name)) == cls, (name, cls_of(short(name)), cls)


def test_bench_matrix_core_figure():
    """The fast-diagonalisation flop count behind the bench's matrix-core figure: 4 Ny Nx
    (Nx + Ny) per plane and correction, one correction per plane and family on the FP64 path
    (the velocity family counts its two components in 2D), the refined path's corrections from
    the refinement record, the FP64 rung's planes at one correction."""
    import types
    import bench
    Nx, Ny, planes = 33, 17, 4
    per = 4.0 * Ny * Nx * (Nx + Ny)

    class Ctx:
        planes_are_z = False

        def residual_variant(self):
            return (1, [0.0, 0.0, 0.0])
    c = Ctx()
    c.Nx, c.Ny, c.planes = Nx, Ny, planes
    run = types.SimpleNamespace(ctx=c, batch=None, equilibrium=False)
    classes = {"gemm32": {"avg_launch_us": 10.0, "launches_per_step": 10},
               "gemm64": {"avg_launch_us": 5.0, "launches_per_step": 4}}
    out = bench.fdm_mfma(run, classes, None, {"fp32": 100.0, "fp64": 50.0})
    assert abs(out["gemm64"]["flops_per_step"] - 6 * planes * per) < 1e-6
    assert abs(out["gemm64"]["achieved_TFLOPs"] - round(6 * planes * per / 20e-6 / 1e12, 3)) < 1e-9
    assert "gemm32" not in out
    ref = {f: {"fp64_planes": planes if f == "P" else 0, "last_corrections": 2} for f in bench.FAMILIES}
    out = bench.fdm_mfma(run, classes, ref, None)
    assert abs(out["gemm32"]["flops_per_step"] - 2 * per * planes * (1 + 1 + 1 + 2)) < 1e-6
    assert abs(out["gemm64"]["flops_per_step"] - planes * per) < 1e-6
    assert bench.fdm_mfma(types.SimpleNamespace(ctx=c, batch=object(), equilibrium=False), classes, ref,
                          None) is None
