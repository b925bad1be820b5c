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
