"""The allocation-free solve entry point (pfd_solve_static) against pfd_solve, through the
C-ABI: two calls in a row on every solve family, the second on a smaller problem, each equal
to pfd_solve's result on the same inputs (the same kernels in the same order)."""
import numpy as np
import pytest

from oracle.sem import Mesh2D, BOTTOM, TOP, LEFT, RIGHT
from oracle.scheme import BCs, WALL, OPEN
from cases import c1_params
from gpu_cases import gpu_context

pytestmark = pytest.mark.gpu


def _case(n, K, nbatch, nz=0, electrodes=()):
    xb = np.linspace(0.0, 1.0, n + 1)
    periodic = bool(electrodes)
    m = Mesh2D(xb, xb, K, periodic_x=periodic)
    if electrodes:
        bc = BCs(side={BOTTOM: WALL, TOP: OPEN}, electrodes=list(electrodes))
    else:
        bc = BCs(side={BOTTOM: WALL, TOP: WALL, LEFT: WALL, RIGHT: WALL}, pot_sides=(BOTTOM, TOP))
    return m, bc


@pytest.mark.parametrize("precision", [0, 1])
def test_static_solve_equals_solve(precision):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    par = c1_params()
    rng = np.random.default_rng(11)
    cases = [(_case(20, 8, 4), dict(nbatch=4)),                       # 103,684 nodes
             (_case(3, 6, 1, electrodes=[(1.0 / 3.0, 2.0 / 3.0)]), dict(nz=8, lz=1.5))]   # smaller
    for (m, bc), kw in cases:
        ctx = gpu_context(m, par, bc, precision=precision, **kw)
        planes = kw.get("nbatch", kw.get("nz", 1))
        for fam in range(5):
            b = torch.tensor(rng.standard_normal((planes, m.Ny, m.Nx)), device="cuda")
            x0 = torch.tensor(rng.standard_normal((planes, m.Ny, m.Nx)), device="cuda")
            xa, xb = x0.clone(), x0.clone()
            ctx.solve(fam, b, xa)
            ctx.solve_static(fam, b, xb)
            torch.cuda.synchronize()
            d = (xa - xb).abs().max().item()
            assert d == 0.0, (m.Nx, fam, d)
            assert torch.isfinite(xb).all()
