"""Edge sizes of the step against the oracle: the smallest and largest element orders the
library takes (K = 2 and 15), meshes of one element along x or along y, and the smallest and
largest Fourier plane counts (Nz = 2: no complex mode; Nz = 512, above the FFT kernels' range,
so the z transform is the DFT GEMM).  Every field after each of three steps, both
precisions."""
import math

import numpy as np
import pytest

from oracle.sem import Mesh2D, BOTTOM, TOP, LEFT, RIGHT
from oracle.scheme import Params, BCs, WALL
from cases import c1_params
from test_gpu_parity import run_pair, check_parity
from test_gpu_3d import run3d, check

pytestmark = pytest.mark.gpu


def _par(eta):
    return Params(**{**c1_params().__dict__, "eta": eta, "lam": 3 * eta / (2 * math.sqrt(2)),
                     "theta_s_deg": 70.0})


@pytest.mark.parametrize("nx,ny,K", [(6, 5, 2), (1, 2, 15), (3, 1, 12)])
@pytest.mark.parametrize("precision,tol", [(0, 1e-9), (1, 1e-8)])
def test_2d_edge_orders_and_single_elements(nx, ny, K, precision, tol):
    m = Mesh2D(np.linspace(0.0, 1.0, nx + 1), np.linspace(0.0, 1.0, ny + 1), K)
    bc = BCs(side={BOTTOM: WALL, TOP: WALL, LEFT: WALL, RIGHT: WALL}, pot_sides=(BOTTOM, TOP))
    par = _par(0.15)
    X, Y = m.X.ravel(), m.Y.ravel()
    phi0 = np.tanh((np.hypot(X - 0.5, Y - 0.4) - 0.3) / (math.sqrt(2) * par.eta))
    u0 = (0.05 * np.sin(np.pi * X) * np.sin(np.pi * Y), 0.03 * np.sin(2 * np.pi * X) * np.sin(np.pi * Y))
    vd = np.where(np.isclose(Y, 1.0), 1.0, 0.0)
    out, _ = run_pair(m, par, bc, phi0, u0, dict(Vd=vd), 3, precision=precision)
    check_parity(out, tol)


@pytest.mark.parametrize("Nz,K", [(2, 5), (512, 5)])
@pytest.mark.parametrize("precision,tol", [(0, 1e-9), (1, 1e-8)])
def test_3d_edge_plane_counts(Nz, K, precision, tol):
    Lz = 1.0
    m = Mesh2D(np.linspace(0.0, 1.0, 3), np.linspace(0.0, 1.0, 3), K, periodic_x=True)
    bc = BCs(side={BOTTOM: WALL, TOP: WALL}, pot_sides=(BOTTOM, TOP))
    par = _par(0.2)
    z = np.arange(Nz) * Lz / Nz
    X = np.broadcast_to(m.X.ravel()[None, :], (Nz, m.Ng))
    Y = np.broadcast_to(m.Y.ravel()[None, :], (Nz, m.Ng))
    Z = np.broadcast_to(z[:, None], (Nz, m.Ng))
    d = np.sqrt((X - 0.5) ** 2 + (Y - 0.3) ** 2 + 0.5 * (Z - 0.5) ** 2)
    phi0 = np.tanh((d - 0.3) / (math.sqrt(2) * par.eta))
    # velocity with content up to the Nyquist plane (cos(pi Nz z / Lz) alternates in sign)
    u0 = tuple(0.05 * np.sin(np.pi * X) * np.sin(np.pi * Y) * np.cos(2 * np.pi * (Z / Lz + 0.1 * i))
               + 0.01 * np.sin(np.pi * Y) * np.cos(np.pi * Nz * Z / Lz) for i in range(3))
    vd = np.where(np.isclose(Y, 1.0), 1.0, 0.0)
    out, _ = run3d(m, bc, par, Nz, Lz, phi0, u0, dict(Vd=vd), 3, precision=precision)
    check(out, tol)
