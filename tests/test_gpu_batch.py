"""Batches of uneven instances stepped through one hipGraph per step, in both forms (multi-
instance launches and per-instance graph branches): every instance matches the same context
stepped on its own (same kernels) bit for bit, and the oracle."""
import math

import numpy as np
import pytest

from oracle.sem import Mesh2D, BOTTOM, TOP, LEFT, RIGHT
from oracle.scheme import Scheme, Params, BCs, WALL, OPEN
from gpu_cases import gpu_context, rel_err, params_dict
from synth import drop_field, c4_param_dict

pytestmark = pytest.mark.gpu

FIELDS = ("phi", "psi", "V", "P", "ux", "uy", "Ex", "Ey")


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _pin(b, a):
    """Same kernels on b as the autotuner chose for a."""
    b.set_tuning(a.tuning())


def _instance(n, K, vtop, eps_ratio, precision, nz=0, tune_from=None, tuning=None):
    par = Params(**{k if k != "lam" else "lam": v for k, v in c4_param_dict(eps_ratio).items()})
    xb = np.linspace(0.0, 1.0, n + 1)
    if nz:
        m = Mesh2D(xb, xb, K, periodic_x=True)
        bc = BCs(side={BOTTOM: WALL, TOP: OPEN}, pot_sides=(BOTTOM, TOP))
    else:
        m = Mesh2D(xb, xb, K)
        bc = BCs(side={BOTTOM: WALL, TOP: WALL, LEFT: WALL, RIGHT: WALL}, pot_sides=(BOTTOM, TOP))
    ctx = gpu_context(m, par, bc, precision=precision, nz=nz, lz=1.0 if nz else 0.0)
    if tune_from is not None:   # before the initial potential, which the kernels also compute
        _pin(ctx, tune_from)
    if tuning is not None:
        ctx.set_tuning(tuning)
    planes = max(nz, 1)
    phi = drop_field(m.X.ravel(), m.Y.ravel(), (0.5, 0.5), 0.25, par.eta)
    phi = np.broadcast_to(phi, (planes, m.Ng)).copy()
    vd = np.where(np.isclose(m.Y.ravel(), 1.0), vtop, 0.0)
    vd = np.broadcast_to(vd, (planes, m.Ng)).copy()
    shape = (planes, m.Ny, m.Nx)
    ctx.set_field("phi", phi.reshape(shape))
    ctx.set_sources({"Vd": vd.reshape(shape)})
    ctx.init_potential(tol=1e-12, max_iter=5000)
    return ctx, (m, par, bc, phi, vd)


SPECS = [(2, 5, 1.0, 4.0, 0), (3, 4, 0.5, 20.0, 0), (2, 7, 2.0, 1.5, 0), (2, 5, 1.5, 10.0, 8)]


MODES = [1, 0]   # BATCH_MULTI, BATCH_BRANCHES


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("precision", [0, 1])
def test_batch_graph_equals_separate_steps(precision, mode):
    """Four uneven instances (three 2D meshes of different order, one 3D) in one batch:
    after each of 6 batch steps (the refined path's first two run eagerly, then both
    time-level parities are captured and replayed) every field equals the same instance
    stepped alone."""
    _torch()
    import paper_2305_09020_amd as pfd
    batch_ctx = [_instance(*s[:4], precision, nz=s[4])[0] for s in SPECS]
    solo_ctx = [_instance(*s[:4], precision, nz=s[4], tune_from=a)[0]   # same kernels on both sides
                for s, a in zip(SPECS, batch_ctx)]
    batch = pfd.Batch(batch_ctx, nlanes=3, mode=mode)
    for n in range(6):
        batch.step(1)
        for c in solo_ctx:
            c.step(1)
        for i, (a, b) in enumerate(zip(batch_ctx, solo_ctx)):
            for k in FIELDS:
                fa, fb = a.get_field(k), b.get_field(k)
                assert np.array_equal(fa, fb), (n, i, k, np.max(np.abs(fa - fb)))
    batch.close()


def test_batch_instance_matches_oracle():
    """A 2D instance stepped inside a batch with two others (multi-instance launches) follows
    the oracle (refined path, 1e-8 per field)."""
    _torch()
    import paper_2305_09020_amd as pfd
    ctxs, infos = zip(*[_instance(*s[:4], 1) for s in SPECS[:3]])
    batch = pfd.Batch(list(ctxs))
    m, par, bc, phi, vd = infos[1]
    sch = Scheme(m, par, bc)
    sch.set_state(phi[0])
    sch.init_potential(dict(Vd=vd[0]))
    for n in range(5):
        o = sch.step(dict(Vd=vd[0]))
        batch.step(1)
        for k in FIELDS:
            ref = o[k][0] if np.ndim(o[k]) > 1 else o[k]
            got = ctxs[1].get_field(k).ravel()
            scale = max(np.linalg.norm(ref), 1e-12 * np.linalg.norm(o["phi"]))
            assert np.linalg.norm(got - np.ravel(ref)) / scale < 1e-8, (n, k)
    batch.close()


@pytest.mark.parametrize("mode", MODES)
def test_batch_recaptures_after_member_changes(mode):
    """A member's parameters changed between batch steps (pfd_update_params): the batch's
    graphs are recaptured (the member's graph generation changed), so the member keeps
    matching the same instance stepped alone with the same change."""
    _torch()
    import paper_2305_09020_amd as pfd
    precision = 1
    batch_ctx = [_instance(*s[:4], precision, nz=s[4])[0] for s in SPECS[:3]]
    solo_ctx = [_instance(*s[:4], precision, nz=s[4], tune_from=a)[0] for s, a in zip(SPECS[:3], batch_ctx)]
    batch = pfd.Batch(batch_ctx, nlanes=2, mode=mode)
    new = c4_param_dict(30.0)        # permittivity ratio 20 -> 30 on instance 1
    new["theta_s_deg"] = 80.0
    for n in range(6):
        if n == 3:
            batch_ctx[1].update_params(new)
            solo_ctx[1].update_params(new)
        batch.step(1)
        for c in solo_ctx:
            c.step(1)
        for i, (a, b) in enumerate(zip(batch_ctx, solo_ctx)):
            for k in FIELDS:
                fa, fb = a.get_field(k), b.get_field(k)
                assert np.array_equal(fa, fb), (n, i, k, np.max(np.abs(fa - fb)))
    # and the change took effect: instance 1 differs from a twin that kept the old parameters
    twin = _instance(*SPECS[1][:4], precision, tune_from=batch_ctx[1])[0]
    twin.step(6)
    assert not np.array_equal(twin.get_field("phi"), batch_ctx[1].get_field("phi"))
    batch.close()


# the generic GEMM tile for every call site, the four-pass solver, the LDS residual, no
# LDS-resident passes: kernels whose work-group shape does not depend on the mesh
FIXED_TUNING = [0] * 10 + [0, 1, 1, 0, 0]


@pytest.mark.parametrize("precision", [0, 1])
def test_multi_instance_launches_do_not_grow_with_instances(precision):
    """Multi-instance form: a batch of 8 instances of one order on meshes of 2..5 elements per
    side, all on one kernel configuration whose work-group shapes do not depend on the mesh,
    takes as many launches per step as a batch of 2 of them, and every member still equals
    the same instance stepped alone."""
    _torch()
    import paper_2305_09020_amd as pfd
    specs = [(2 + i % 4, 6, 0.25 * i, 2.0 + 3 * i, 0) for i in range(8)]
    counts = []
    for sub in (specs[:2], specs):
        batch_ctx = [_instance(*s[:4], precision, tuning=FIXED_TUNING)[0] for s in sub]
        solo_ctx = [_instance(*s[:4], precision, tuning=FIXED_TUNING)[0] for s in sub]
        batch = pfd.Batch(batch_ctx)
        for n in range(4):
            batch.step(1)
            for c in solo_ctx:
                c.step(1)
        for i, (a, b) in enumerate(zip(batch_ctx, solo_ctx)):
            for k in FIELDS:
                assert np.array_equal(a.get_field(k), b.get_field(k)), (len(sub), i, k)
        counts.append(batch.launches())
        batch.close()
    assert counts[0] > 0 and counts[0] == counts[1], counts


@pytest.mark.parametrize("mode", MODES)
def test_batch_equilibrium_steps_equal_separate_steps(mode):
    """Steps of the equilibrium system (Sec. 2.4) in a batch of three uneven 2D instances on the
    refined path: every field equals the same instance stepped alone, after each of 6 steps."""
    _torch()
    import paper_2305_09020_amd as pfd
    batch_ctx = [_instance(*s[:4], 1)[0] for s in SPECS[:3]]
    solo_ctx = [_instance(*s[:4], 1, tune_from=a)[0] for s, a in zip(SPECS[:3], batch_ctx)]
    batch = pfd.Batch(batch_ctx, mode=mode)
    for n in range(6):
        batch.step(1, equilibrium=True)
        for c in solo_ctx:
            c.step(1, True)
        for i, (a, b) in enumerate(zip(batch_ctx, solo_ctx)):
            for k in ("phi", "psi", "V"):
                assert np.array_equal(a.get_field(k), b.get_field(k)), (n, i, k)
    batch.close()


def test_batch_mode_validation():
    """pfd_batch_set_mode takes only the two forms; the multi-instance launch count is -1 until
    a multi-instance graph has been captured (refined: from the third step on)."""
    _torch()
    import paper_2305_09020_amd as pfd
    ctx = _instance(*SPECS[0][:4], 1)[0]
    batch = pfd.Batch([ctx], mode=pfd.BATCH_BRANCHES)
    batch.step(3)
    assert batch.launches() == -1
    with pytest.raises(pfd.PfdError):
        batch.set_mode(2)
    batch.set_mode(pfd.BATCH_MULTI)
    batch.step(2)
    assert batch.launches() > 0
    batch.close()


def _electrode_instance(n, K, volt, precision, tune_from=None):
    """x-periodic box, open top, one electrode segment [0.25, 0.5] on the bottom wall at volt
    (the potential solve takes the gap-node correction), a drop sitting on the bottom."""
    par = Params(**{**c4_param_dict(8.0), "theta_s_deg": 75.0})
    xb = np.linspace(0.0, 1.0, n + 1)
    m = Mesh2D(xb, xb, K, periodic_x=True)
    bc = BCs(side={BOTTOM: WALL, TOP: OPEN}, electrodes=[(0.25, 0.5)])
    ctx = gpu_context(m, par, bc, precision=precision)
    if tune_from is not None:
        _pin(ctx, tune_from)
    X, Y = m.X.ravel(), m.Y.ravel()
    phi = drop_field(X, Y, (0.5, 0.0), 0.3, par.eta)
    vd = np.where(np.isclose(Y, 0.0) & (X >= 0.25 - 1e-12) & (X <= 0.5 + 1e-12), volt, 0.0)
    shape = (1, m.Ny, m.Nx)
    ctx.set_field("phi", phi.reshape(shape))
    ctx.set_sources({"Vd": vd.reshape(shape)})
    ctx.init_potential(tol=1e-12, max_iter=5000)
    return ctx


@pytest.mark.parametrize("mode", MODES)
def test_batch_with_electrode_instances(mode):
    """Two electrode instances (gap-node potential solve; n = 4 and 8 elements per side) and
    a closed box in one batch, refined path: every field equals the same instance stepped
    alone after each of 6 steps."""
    _torch()
    import paper_2305_09020_amd as pfd
    batch_ctx = [_electrode_instance(4, 6, 1.0, 1), _electrode_instance(8, 5, 0.5, 1),
                 _instance(*SPECS[1][:4], 1)[0]]
    solo_ctx = [_electrode_instance(4, 6, 1.0, 1, tune_from=batch_ctx[0]),
                _electrode_instance(8, 5, 0.5, 1, tune_from=batch_ctx[1]),
                _instance(*SPECS[1][:4], 1, tune_from=batch_ctx[2])[0]]
    batch = pfd.Batch(batch_ctx, mode=mode)
    for n in range(6):
        batch.step(1)
        for c in solo_ctx:
            c.step(1)
        for i, (a, b) in enumerate(zip(batch_ctx, solo_ctx)):
            for k in FIELDS:
                fa, fb = a.get_field(k), b.get_field(k)
                assert np.array_equal(fa, fb), (n, i, k, np.max(np.abs(fa - fb)))
    batch.close()


@pytest.mark.parametrize("mode", MODES)
def test_batch_of_3d_instances_with_different_plane_counts(mode):
    """Two 3D instances of different Fourier plane counts (8 and 16: different z-transform
    kernels) and one 2D instance in one batch, refined path: every field equals the same
    instance stepped alone after each of 6 steps."""
    _torch()
    import paper_2305_09020_amd as pfd
    specs = [(2, 5, 1.5, 10.0, 8), (2, 4, 0.5, 3.0, 16), (3, 4, 0.5, 20.0, 0)]
    batch_ctx = [_instance(*s[:4], 1, nz=s[4])[0] for s in specs]
    solo_ctx = [_instance(*s[:4], 1, nz=s[4], tune_from=a)[0] for s, a in zip(specs, batch_ctx)]
    batch = pfd.Batch(batch_ctx, mode=mode)
    for n in range(6):
        batch.step(1)
        for c in solo_ctx:
            c.step(1)
        for i, (a, b) in enumerate(zip(batch_ctx, solo_ctx)):
            for k in FIELDS:
                fa, fb = a.get_field(k), b.get_field(k)
                assert np.array_equal(fa, fb), (n, i, k, np.max(np.abs(fa - fb)))
    batch.close()
