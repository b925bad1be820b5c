"""Python binding of the pfd C-ABI library (libpfd.so, HIP for gfx950).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch provides the device workspace and the stream.  Importing this
module loads the in-tree libpfd.so and raises if it is missing; build it with
``python -m paper_2305_09020_amd.build`` (or ``__graft_entry__.build()``).
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libpfd.so")

if not os.path.exists(LIBPATH):
    raise ImportError("libpfd.so is not built (run paper_2305_09020_amd/build.py)")
# torch ships its own HIP runtime: loading it before the library makes the library's HIP
# dependency resolve to that same runtime (one per process).  Loaded the other way round, the
# process held two runtimes and the library's found no device.
import torch  # noqa: E402,F401
_lib = ctypes.CDLL(LIBPATH)

# ---- enums (mirror include/pfd.h) -------------------------------------------------
OK, EINVAL, ENOMEM, EHIP, ENONFINITE, ENOCONV, ESTATE, ENOTIMPL = range(8)
UX, UY, UZ, P, PHI, PSI, V, EX, EY, EZ = range(10)
FIELDS = dict(ux=UX, uy=UY, uz=UZ, P=P, phi=PHI, psi=PSI, V=V, Ex=EX, Ey=EY, Ez=EZ)
SOURCES = dict(g=0, fx=1, fy=2, fz=3, fV=4, g1=5, g2=6, g3=7, f1x=8, f1y=9, f1z=10, f2=11,
               wx=12, wy=13, wz=14, Vd=15)
PLAIN_FP64, REFINED_FP32, REFINED_BF16 = 0, 1, 2
WALL, OPEN, PERIODIC = 0, 1, 2
BOTTOM, TOP, LEFT, RIGHT = 0, 1, 2, 3
FAM_V, FAM_PSI, FAM_PHI, FAM_P, FAM_U = range(5)
PROF_CLASSES = ("gemm64", "gemm32", "residual", "element", "nodal", "other", "zfft")

_dp = ctypes.POINTER(ctypes.c_double)


class Mesh(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("K", ctypes.c_int),
                ("xb", _dp), ("yb", _dp), ("periodic_x", ctypes.c_int), ("nz", ctypes.c_int),
                ("lz", ctypes.c_double), ("nbatch", ctypes.c_int)]


class Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("rho1", "rho2", "mu1", "mu2", "eps1", "eps2", "lam", "eta", "gamma1",
                 "theta_s_deg", "dt")] + [("bdf_order", ctypes.c_int), ("S", ctypes.c_double),
                                          ("nu_m", ctypes.c_double)]


class BCs(ctypes.Structure):
    _fields_ = [("side_type", ctypes.c_int * 4), ("pot_dirichlet", ctypes.c_int * 4),
                ("n_electrodes", ctypes.c_int), ("electrode_x0", _dp), ("electrode_x1", _dp)]


class Problem(ctypes.Structure):
    _fields_ = [("mesh", Mesh), ("par", Params), ("bc", BCs), ("precision", ctypes.c_int),
                ("refine_max", ctypes.c_int), ("refine_tol", ctypes.c_double)]


class Diag(ctypes.Structure):
    _fields_ = [("derived", ctypes.c_double * 10), ("last_residual", ctypes.c_double),
                ("nonfinite", ctypes.c_int), ("unconverged", ctypes.c_int), ("steps", ctypes.c_long)]


class RefineStats(ctypes.Structure):
    _fields_ = [("n_fp64_planes", ctypes.c_int), ("last_corrections", ctypes.c_int),
                ("max_corrections", ctypes.c_int), ("failures", ctypes.c_long),
                ("last_eta", ctypes.c_double), ("kappa_min", ctypes.c_double),
                ("kappa_max", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double), ("kinetic", ctypes.c_double), ("mixing", ctypes.c_double),
                ("electric", ctypes.c_double), ("wall", ctypes.c_double), ("total", ctypes.c_double),
                ("phi_max_abs", ctypes.c_double), ("nonfinite", ctypes.c_int)]


class WsArch(ctypes.Structure):
    _fields_ = [("hidden1", ctypes.c_int), ("hidden2", ctypes.c_int), ("channels", ctypes.c_int),
                ("nz", ctypes.c_int), ("ny", ctypes.c_int), ("nx", ctypes.c_int),
                ("periodic_z", ctypes.c_int), ("periodic_y", ctypes.c_int), ("periodic_x", ctypes.c_int),
                ("seed", ctypes.c_ulonglong)]


_vp = ctypes.c_void_p
_sig = {
    "pfd_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "pfd_last_error": (ctypes.c_char_p, [_vp]),
    "pfd_workspace_query": (ctypes.c_int, [ctypes.POINTER(Problem), ctypes.POINTER(ctypes.c_size_t)]),
    "pfd_create": (ctypes.c_int, [ctypes.POINTER(Problem), _vp, ctypes.c_size_t, _vp,
                                  ctypes.POINTER(_vp)]),
    "pfd_destroy": (None, [_vp]),
    "pfd_get_dims": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_int)]),
    "pfd_get_coords": (ctypes.c_int, [_vp, _dp, _dp, _dp]),
    "pfd_get_diag": (ctypes.c_int, [_vp, ctypes.POINTER(Diag)]),
    "pfd_get_stats": (ctypes.c_int, [_vp, ctypes.POINTER(Stats)]),
    "pfd_get_refine_stats": (ctypes.c_int, [_vp, ctypes.POINTER(RefineStats), ctypes.c_int]),
    "pfd_set_graph": (ctypes.c_int, [_vp, ctypes.c_int]),
    "pfd_batch_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp)]),
    "pfd_batch_step": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int]),
    "pfd_batch_destroy": (None, [_vp]),
    "pfd_batch_last_error": (ctypes.c_char_p, [_vp]),
    "pfd_batch_set_mode": (ctypes.c_int, [_vp, ctypes.c_int]),
    "pfd_batch_launches": (ctypes.c_int, [_vp]),
    "pfd_set_solver_variant": (ctypes.c_int, [_vp, ctypes.c_int]),
    "pfd_update_params": (ctypes.c_int, [_vp, ctypes.POINTER(Params)]),
    "pfd_get_mass_weights": (ctypes.c_int, [_vp, _dp]),
    "pfd_ws_num_weights": (ctypes.c_long, [ctypes.POINTER(WsArch)]),
    "pfd_ws_workspace_query": (ctypes.c_int, [ctypes.POINTER(WsArch), ctypes.POINTER(ctypes.c_size_t)]),
    "pfd_ws_create": (ctypes.c_int, [ctypes.POINTER(WsArch), _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
    "pfd_ws_destroy": (None, [_vp]),
    "pfd_ws_last_error": (ctypes.c_char_p, [_vp]),
    "pfd_ws_get_weights": (ctypes.c_int, [_vp, _vp]),
    "pfd_ws_set_weights": (ctypes.c_int, [_vp, _vp]),
    "pfd_ws_init_output_bias": (ctypes.c_int, [_vp, _vp, ctypes.c_long]),
    "pfd_ws_gradients": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int, _vp, ctypes.POINTER(ctypes.c_double)]),
    "pfd_ws_train_step": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_float,
                                         ctypes.POINTER(ctypes.c_double)]),
    "pfd_ws_train": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_long, ctypes.c_int, ctypes.c_int, ctypes.c_float,
                                    ctypes.c_ulonglong, _vp]),
    "pfd_ws_predict": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, _vp]),
    "pfd_set_gemm_config": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int]),
    "pfd_set_residual_variant": (ctypes.c_int, [_vp, ctypes.c_int]),
    "pfd_get_tuning": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "pfd_set_tuning": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int), ctypes.c_int]),
    "pfd_get_residual_variant": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int),
                                                ctypes.POINTER(ctypes.c_double)]),
    "pfd_get_gemm_config": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]),
    "pfd_get_solver_variant": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int),
                                              ctypes.POINTER(ctypes.c_double)]),
    "pfd_march_to_equilibrium": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_long,
                                                ctypes.POINTER(ctypes.c_long),
                                                ctypes.POINTER(ctypes.c_double)]),
    "pfd_set_field": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int]),
    "pfd_get_field": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int]),
    "pfd_set_source": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_int]),
    "pfd_init_potential": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_int)]),
    "pfd_step": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int]),
    "pfd_step_async": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int]),
    "pfd_solve": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp]),
    "pfd_solve_static": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp]),
    "pfd_apply": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp]),
    "pfd_profile_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "pfd_profile_replay": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]),
    "pfd_profile_read": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_long)]),
}
EXPORTS = tuple(_sig)
for _n, (_res, _args) in _sig.items():
    _f = getattr(_lib, _n)
    _f.restype = _res
    _f.argtypes = _args


class PfdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_lib.pfd_status_string(code).decode(), msg))
        self.code = code


def _check(code, ctx=None):
    if code != OK:
        raise PfdError(code, _lib.pfd_last_error(ctx).decode())


def make_problem(xb, yb, K, params, side_type, pot_dirichlet, periodic_x=False, nbatch=1,
                 nz=0, lz=0.0, precision=PLAIN_FP64, refine_max=0, refine_tol=0.0, electrodes=()):
    """Build the C problem struct.  params: mapping with rho1, rho2, mu1, mu2, eps1, eps2,
    lam, eta, gamma1, theta_s_deg, dt and optional bdf (2), S (0), nu_m (0).  refine_max /
    refine_tol: correction cap and backward-error stop rule of the refined path (0: defaults)."""
    xb = np.ascontiguousarray(xb, dtype=np.float64)
    yb = np.ascontiguousarray(yb, dtype=np.float64)
    pr = Problem()
    pr.mesh = Mesh(len(xb) - 1, len(yb) - 1, K, xb.ctypes.data_as(_dp), yb.ctypes.data_as(_dp),
                   int(periodic_x), int(nz), float(lz), int(nbatch))
    g = params.get
    pr.par = Params(g("rho1"), g("rho2"), g("mu1"), g("mu2"), g("eps1"), g("eps2"), g("lam"),
                    g("eta"), g("gamma1"), g("theta_s_deg"), g("dt"), int(g("bdf", 2)),
                    float(g("S", 0.0)), float(g("nu_m", 0.0)))
    st = (ctypes.c_int * 4)(*side_type)
    pd = (ctypes.c_int * 4)(*pot_dirichlet)
    e0 = np.ascontiguousarray([e[0] for e in electrodes], dtype=np.float64)
    e1 = np.ascontiguousarray([e[1] for e in electrodes], dtype=np.float64)
    pr.bc = BCs(st, pd, len(electrodes), e0.ctypes.data_as(_dp), e1.ctypes.data_as(_dp))
    pr.precision = precision
    pr.refine_max = int(refine_max)
    pr.refine_tol = float(refine_tol)
    pr._keep = (xb, yb, e0, e1)   # keep host arrays alive while pr is used
    return pr


def workspace_bytes(problem):
    n = ctypes.c_size_t(0)
    _check(_lib.pfd_workspace_query(ctypes.byref(problem), ctypes.byref(n)))
    return n.value


class Context:
    """A pfd context on the current torch device and stream.  Device memory is one
    torch uint8 tensor (the workspace) owned by this object."""

    def __init__(self, problem, device="cuda", stream=None):
        import torch
        self.torch = torch
        nbytes = workspace_bytes(problem)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.ws.device)
        h = _vp()
        _check(_lib.pfd_create(ctypes.byref(problem), _vp(base + off), nbytes,
                               _vp(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self._destroy = _lib.pfd_destroy   # kept for interpreter shutdown
        nx, ny, npl = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(_lib.pfd_get_dims(h, ctypes.byref(nx), ctypes.byref(ny), ctypes.byref(npl)), h)
        self.Nx, self.Ny, self.planes = nx.value, ny.value, npl.value
        self.planes_are_z = problem.mesh.nz > 0
        self.shape = (self.planes, self.Ny, self.Nx)

    def close(self):
        if getattr(self, "h", None):
            self._destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    # -- host / device transfers -------------------------------------------------
    def coords(self):
        x = np.zeros(self.Nx)
        y = np.zeros(self.Ny)
        z = np.zeros(self.planes)
        _check(_lib.pfd_get_coords(self.h, x.ctypes.data_as(_dp), y.ctypes.data_as(_dp),
                                   z.ctypes.data_as(_dp)), self.h)
        return x, y, z

    def _arr(self, a):
        """(pointer, on_device, keepalive) for a numpy array or torch tensor of the field shape."""
        t = self.torch
        if isinstance(a, t.Tensor):
            if a.dtype != t.float64 or not a.is_contiguous() or a.numel() != self.planes * self.Ny * self.Nx:
                raise ValueError("need a contiguous float64 tensor of %d values" % (self.planes * self.Ny * self.Nx))
            return _vp(a.data_ptr()), int(a.is_cuda), a
        a = np.ascontiguousarray(a, dtype=np.float64)
        if a.size != self.planes * self.Ny * self.Nx:
            raise ValueError("field has %d values, expected %d" % (a.size, self.planes * self.Ny * self.Nx))
        return _vp(a.ctypes.data), 0, a

    def set_field(self, name, value, level=0):
        p, dev, keep = self._arr(value)
        _check(_lib.pfd_set_field(self.h, FIELDS[name], level, p, dev), self.h)

    def get_field(self, name, level=0, out=None):
        if out is None:
            out = np.zeros(self.shape)
        p, dev, keep = self._arr(out)
        _check(_lib.pfd_get_field(self.h, FIELDS[name], level, p, dev), self.h)
        return out

    def set_source(self, name, value):
        if value is None:
            _check(_lib.pfd_set_source(self.h, SOURCES[name], None, 0), self.h)
            return
        p, dev, keep = self._arr(value)
        _check(_lib.pfd_set_source(self.h, SOURCES[name], p, dev), self.h)

    def set_sources(self, src):
        for k, v in src.items():
            if k in SOURCES:
                self.set_source(k, v)

    # -- the method ------------------------------------------------------------------
    def init_potential(self, tol=1e-13, max_iter=20000):
        it = ctypes.c_int(0)
        _check(_lib.pfd_init_potential(self.h, tol, max_iter, ctypes.byref(it)), self.h)
        return it.value

    def step(self, nsteps=1, equilibrium=False):
        _check(_lib.pfd_step(self.h, int(nsteps), int(bool(equilibrium))), self.h)

    def step_async(self, nsteps=1, equilibrium=False):
        _check(_lib.pfd_step_async(self.h, int(nsteps), int(bool(equilibrium))), self.h)

    def solve(self, fam, b, x):
        """Device tensors b, x (float64, planes*Ny*Nx); x: guess + Dirichlet values in, solution out."""
        _check(_lib.pfd_solve(self.h, fam, _vp(b.data_ptr()), _vp(x.data_ptr())), self.h)

    def solve_static(self, fam, b, x):
        """solve() with the scratch from the library's static device array (no allocation)."""
        _check(_lib.pfd_solve_static(self.h, fam, _vp(b.data_ptr()), _vp(x.data_ptr())), self.h)

    def apply(self, fam, x, y):
        _check(_lib.pfd_apply(self.h, fam, _vp(x.data_ptr()), _vp(y.data_ptr())), self.h)

    def profile_enable(self, on=True):
        _check(_lib.pfd_profile_enable(self.h, int(bool(on))), self.h)

    def profile_read(self):
        """{class: (total_ms, launches)} since profiling was enabled (synchronises)."""
        out = {}
        for k, name in enumerate(PROF_CLASSES):
            ms, n = ctypes.c_double(0), ctypes.c_long(0)
            _check(_lib.pfd_profile_read(self.h, k, ctypes.byref(ms), ctypes.byref(n)), self.h)
            out[name] = (ms.value, n.value)
        return out

    def profile_replay(self, cls, reps=200):
        """Average device microseconds of one launch of class cls (name or index)."""
        k = PROF_CLASSES.index(cls) if isinstance(cls, str) else cls
        us = ctypes.c_double(0)
        _check(_lib.pfd_profile_replay(self.h, k, int(reps), ctypes.byref(us)), self.h)
        return us.value

    def mass_weights(self):
        """Quadrature weights (planes, Ny, Nx): the discrete integral is sum(w * f)."""
        w = np.zeros(self.Ny * self.Nx)
        _check(_lib.pfd_get_mass_weights(self.h, w.ctypes.data_as(_dp)), self.h)
        return np.broadcast_to(w.reshape(1, self.Ny, self.Nx), self.shape).copy()

    def update_params(self, params):
        """Change eps1, eps2 and theta_s_deg (every other parameter must stay as created)."""
        g = params.get
        par = Params(g("rho1"), g("rho2"), g("mu1"), g("mu2"), g("eps1"), g("eps2"), g("lam"),
                     g("eta"), g("gamma1"), g("theta_s_deg"), g("dt"), int(g("bdf", 2)),
                     float(g("S", 0.0)), float(g("nu_m", 0.0)))
        _check(_lib.pfd_update_params(self.h, ctypes.byref(par)), self.h)

    def set_solver_variant(self, variant):
        """0: four GEMM passes, 1: fused strip kernels, 2: fused middle passes (three
        launches), -1: autotune again."""
        _check(_lib.pfd_set_solver_variant(self.h, int(variant)), self.h)

    def tuning(self):
        """The autotuner's choices (opaque list of ints) for set_tuning on another context."""
        cnt = ctypes.c_int(0)
        _check(_lib.pfd_get_tuning(self.h, None, 0, ctypes.byref(cnt)), self.h)
        vals = (ctypes.c_int * cnt.value)()
        _check(_lib.pfd_get_tuning(self.h, vals, cnt.value, ctypes.byref(cnt)), self.h)
        return list(vals)

    def set_tuning(self, vals):
        arr = (ctypes.c_int * len(vals))(*vals)
        _check(_lib.pfd_set_tuning(self.h, arr, len(vals)), self.h)

    def set_residual_variant(self, variant):
        """0: per-node residual kernel, 1: LDS-tiled residual kernel, 2: LDS-tiled residual
        fused with the first fast-diagonalisation pass (refined path), 3: per-node kernel with
        the element order a runtime argument (one kernel for every order)."""
        _check(_lib.pfd_set_residual_variant(self.h, int(variant)), self.h)

    def residual_variant(self):
        """(variant, [us per residual of variants 0 and 1, us per fused residual + first pass])."""
        v = ctypes.c_int(0)
        us = (ctypes.c_double * 3)()
        _check(_lib.pfd_get_residual_variant(self.h, ctypes.byref(v), us), self.h)
        return v.value, [us[0], us[1], us[2]]

    def set_gemm_config(self, site, cfg):
        """Force configuration cfg (0..15; 16 = the FFT at site 4) at call site (0..4, -1 = all)."""
        _check(_lib.pfd_set_gemm_config(self.h, int(site), int(cfg)), self.h)

    def gemm_config(self):
        """(chosen cfg per site [5], autotune us per (site, cfg) [5][17]; 0 = not applicable
        or not tuned; cfg 16 of site 4 is the z FFT)."""
        cfg = (ctypes.c_int * 5)()
        us = (ctypes.c_double * 85)()
        _check(_lib.pfd_get_gemm_config(self.h, cfg, us), self.h)
        return list(cfg), [list(us[17 * s:17 * s + 17]) for s in range(5)]

    def solver_variant(self):
        """(variant, [us per correction of variants 0, 1, 2]) from the autotuner."""
        v = ctypes.c_int(0)
        us = (ctypes.c_double * 3)()
        _check(_lib.pfd_get_solver_variant(self.h, ctypes.byref(v), us), self.h)
        return v.value, [us[0], us[1], us[2]]

    def set_graph(self, on=True):
        """Replay a captured hipGraph per step (identical results, fewer launches)."""
        _check(_lib.pfd_set_graph(self.h, int(bool(on))), self.h)

    def stats(self):
        """List (one per instance) of dicts: mass, kinetic, mixing, electric, wall, total,
        phi_max_abs, nonfinite."""
        n = 1 if self.planes_are_z else self.planes
        arr = (Stats * n)()
        _check(_lib.pfd_get_stats(self.h, arr), self.h)
        return [{k: getattr(a, k) for k, _ in Stats._fields_} for a in arr]

    def march_to_equilibrium(self, tol, max_steps):
        """Equilibrium steps until max|phi^{m+1} - phi^m| <= tol; returns (steps, r_m).
        Raises PfdError (ENOCONV) if max_steps is reached."""
        n = ctypes.c_long(0)
        r = ctypes.c_double(0.0)
        _check(_lib.pfd_march_to_equilibrium(self.h, float(tol), int(max_steps), ctypes.byref(n),
                                             ctypes.byref(r)), self.h)
        return n.value, r.value

    def diag(self):
        d = Diag()
        _check(_lib.pfd_get_diag(self.h, ctypes.byref(d)), self.h)
        return dict(derived=list(d.derived), last_residual=d.last_residual,
                    nonfinite=d.nonfinite, unconverged=d.unconverged, steps=d.steps)

    def refine_stats(self, reset=False):
        """Per solve family (V, psi, phi, P, u): FP64 planes of the precision ladder,
        corrections of the last solve and the most since the last reset, failed solves, the
        last backward error and the condition estimates."""
        arr = (RefineStats * 5)()
        _check(_lib.pfd_get_refine_stats(self.h, arr, int(bool(reset))), self.h)
        return [{k: getattr(a, k) for k, _ in RefineStats._fields_} for a in arr]


BATCH_BRANCHES, BATCH_MULTI = 0, 1


class Batch:
    """Independent contexts (uneven meshes, orders, parameters) created on one stream,
    stepped together, one hipGraph launch per step: multi-instance launches (mode
    BATCH_MULTI, default) or every instance as a parallel branch (BATCH_BRANCHES)."""

    def __init__(self, contexts, nlanes=4, mode=BATCH_MULTI):
        self.contexts = list(contexts)
        arr = (_vp * len(self.contexts))(*[c.h for c in self.contexts])
        h = _vp()
        code = _lib.pfd_batch_create(arr, len(self.contexts), int(nlanes), ctypes.byref(h))
        if code != OK:
            raise PfdError(code, _lib.pfd_batch_last_error(None).decode())
        self.h = h
        self._destroy = _lib.pfd_batch_destroy
        self.set_mode(mode)

    def set_mode(self, mode):
        code = _lib.pfd_batch_set_mode(self.h, int(mode))
        if code != OK:
            raise PfdError(code, "batch mode must be BATCH_BRANCHES or BATCH_MULTI")

    def launches(self):
        """Launches per step of the multi-instance form (-1 before its first capture)."""
        return int(_lib.pfd_batch_launches(self.h))

    def step(self, nsteps=1, equilibrium=False):
        code = _lib.pfd_batch_step(self.h, int(nsteps), int(bool(equilibrium)))
        if code != OK:
            raise PfdError(code, _lib.pfd_batch_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self._destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class WarmStart:
    """The learned warm start (hand-written HIP training and inference kernels): a
    convolutional decoder from three scaled parameters to a field on the grid
    (nz, ny, nx), z slowest; periodic = (z, y, x) flags.  Device memory is one torch uint8
    workspace owned by this object."""

    def __init__(self, grid, periodic=(False, False, False), seed=0, device="cuda", stream=None):
        import torch
        self.torch = torch
        nz, ny, nx = (int(v) for v in grid)
        self.arch = WsArch(64, 128, 16, nz, ny, nx, int(bool(periodic[0])), int(bool(periodic[1])),
                           int(bool(periodic[2])), int(seed))
        self.n_out = nz * ny * nx
        self.nw = _lib.pfd_ws_num_weights(ctypes.byref(self.arch))
        if self.nw <= 0:
            raise PfdError(EINVAL, "invalid warm-start grid %r" % (tuple(grid),))
        n = ctypes.c_size_t(0)
        _check(_lib.pfd_ws_workspace_query(ctypes.byref(self.arch), ctypes.byref(n)))
        self.ws = torch.empty(n.value + 256, dtype=torch.uint8, device=device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.ws.device)
        h = _vp()
        _check(_lib.pfd_ws_create(ctypes.byref(self.arch), _vp(base + off), n.value,
                                  _vp(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self._destroy = _lib.pfd_ws_destroy

    def _chk(self, code):
        if code != OK:
            raise PfdError(code, _lib.pfd_ws_last_error(self.h).decode())

    def get_weights(self):
        w = np.zeros(self.nw, dtype=np.float32)
        self._chk(_lib.pfd_ws_get_weights(self.h, _vp(w.ctypes.data)))
        return w

    def set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        assert w.size == self.nw
        self._chk(_lib.pfd_ws_set_weights(self.h, _vp(w.ctypes.data)))

    def init_output_bias(self, targets):
        self._chk(_lib.pfd_ws_init_output_bias(self.h, _vp(targets.data_ptr()), targets.shape[0]))

    def gradients(self, params, targets, idx):
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        g = np.zeros(self.nw, dtype=np.float32)
        loss = ctypes.c_double(0.0)
        self._chk(_lib.pfd_ws_gradients(self.h, _vp(params.data_ptr()), _vp(targets.data_ptr()),
                                        _vp(idx.ctypes.data), len(idx), _vp(g.ctypes.data), ctypes.byref(loss)))
        return g, loss.value

    def train_step(self, params, targets, idx, lr):
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        loss = ctypes.c_double(0.0)
        self._chk(_lib.pfd_ws_train_step(self.h, _vp(params.data_ptr()), _vp(targets.data_ptr()),
                                         _vp(idx.ctypes.data), len(idx), float(lr), ctypes.byref(loss)))
        return loss.value

    def train(self, params, targets, steps, batch=32, lr=2e-3, seed=0):
        hist = np.zeros(max(int(steps), 1))
        self._chk(_lib.pfd_ws_train(self.h, _vp(params.data_ptr()), _vp(targets.data_ptr()), params.shape[0],
                                    int(steps), int(batch), float(lr), int(seed), _vp(hist.ctypes.data)))
        return hist[:steps]

    def predict(self, p, out, weights=None, mass=0.0):
        """Field for inputs p (3 scaled values) into out (float64 device tensor of nz ny nx);
        with weights (float64 device tensor) shifted to sum(weights * out) = mass."""
        p = np.ascontiguousarray(p, dtype=np.float32)
        self._chk(_lib.pfd_ws_predict(self.h, _vp(p.ctypes.data), _vp(weights.data_ptr()) if weights is not None
                                      else None, float(mass), _vp(out.data_ptr())))
        return out

    def close(self):
        if getattr(self, "h", None):
            self._destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ws_inputs(V, eps_ratio, theta_deg, vmax=2.0, rmin=1.5, rmax=40.0, tmin=60.0, tmax=120.0):
    """Network inputs of the learned warm start: voltage and contact angle mapped linearly,
    the permittivity ratio logarithmically, from their sampling ranges to [-1, 1]."""
    import math
    return np.array([2.0 * V / vmax - 1.0,
                     2.0 * (math.log(eps_ratio) - math.log(rmin)) / (math.log(rmax) - math.log(rmin)) - 1.0,
                     2.0 * (theta_deg - tmin) / (tmax - tmin) - 1.0], dtype=np.float32)
