"""ctypes binding of libpfsh (declared in include/pfsh.h).

Argument marshalling only: shapes and dtypes are checked, device pointers and
the current HIP stream are handed to the C ABI, and every step runs in the
library's HIP kernels.  PyTorch supplies device memory and streams.  If the
library is not built this module raises on first use; there is no fallback.
"""

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpfsh.so")

PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2}
LEGENDRE_RECURRENCE = 0x100   # flag OR-ed into LevelDesc.precision
STATUS = {0: "PFSH_OK", -1: "PFSH_EINVAL", -2: "PFSH_ESHAPE", -3: "PFSH_ENOMEM",
          -4: "PFSH_EHIP", -5: "PFSH_EUNSUPPORTED", -6: "PFSH_ENONFINITE"}


class PfshError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {STATUS.get(code, code)}")


class LevelDesc(ctypes.Structure):
    _fields_ = [("T", ctypes.c_int), ("nlat", ctypes.c_int), ("nlon", ctypes.c_int),
                ("n_nodes", ctypes.c_int), ("max_batch", ctypes.c_int),
                ("radius", ctypes.c_double), ("omega", ctypes.c_double),
                ("phibar", ctypes.c_double), ("nu", ctypes.c_double),
                ("precision", ctypes.c_int)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_SIGS = {
    "pfsh_status_string": ([_I], ctypes.c_char_p),
    "pfsh_level_desc_check": ([ctypes.POINTER(LevelDesc)], _I),
    "pfsh_level_create": ([ctypes.POINTER(LevelDesc), _I, ctypes.POINTER(_P)], _I),
    "pfsh_level_destroy": ([_P], None),
    "pfsh_level_query": ([_P, ctypes.POINTER(_I), ctypes.POINTER(_I), _P, _P, _P, _P, _P, _P], _I),
    "pfsh_level_bytes": ([_P, ctypes.POINTER(ctypes.c_ulonglong), ctypes.POINTER(ctypes.c_ulonglong)], _I),
    "pfsh_sh_synthesis": ([_P, _P, _P, _I, _P], _I),
    "pfsh_sh_analysis": ([_P, _P, _P, _I, _P], _I),
    "pfsh_rhs": ([_P, _P, _P, _P, _I, _P], _I),
    "pfsh_implicit_solve": ([_P, _D, _P, _P, _I, _P], _I),
    "pfsh_sdc_sweep": ([_P, _D, _P, _P, _P, _P, _I, _P], _I),
    "pfsh_residual": ([_P, _D, _P, _P, _P, _P, _P, _I, _P], _I),
    "pfsh_residual_noalloc": ([_P, _D, _P, _P, _P, _P, _P, _I, _P], _I),
    "pfsh_level_set_implicit": ([_P, _I], _I),
    "pfsh_check_finite": ([_P, _I, _P], _I),
    "pfsh_spread": ([_P, _P, _P, _P, _I, _P], _I),
    "pfsh_restrict": ([_P, _P, _P, _P, _I, _P], _I),
    "pfsh_interpolate_add": ([_P, _P, _P, _P, _P, _I, _P], _I),
    "pfsh_fas_tau": ([_P, _P, _D, _P, _P, _P, _P, _P, _I, _P], _I),
    "pfsh_profile_enable": ([_P, _I], _I),
    "pfsh_profile_read": ([_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_D)], _I),
    "pfsh_profile_read_batch": ([_P, _I, _I, ctypes.POINTER(_I), ctypes.POINTER(_D)], _I),
    "pfsh_variant_count": ([_P, _I], _I),
    "pfsh_level_set_variant": ([_P, _I, _I, _I], _I),
    "pfsh_level_get_variant": ([_P, _I, _I, ctypes.POINTER(_I)], _I),
    "pfsh_level_autotune": ([_P, _I, _I, _P, _P], _I),
    "pfsh_level_autotune_ex": ([_P, _I, _I, _I, _P, _P], _I),
    "pfsh_pfasst_create": ([_P, _P, _I, _I, ctypes.POINTER(_P)], _I),
    "pfsh_pfasst_destroy": ([_P], None),
    "pfsh_pfasst_predict": ([_P, _D, _P, _P, _P, _P, _P], _I),
    "pfsh_pfasst_iterate": ([_P, _D, _P, _P, _P, _I, _P], _I),
    "pfsh_pfasst_run": ([_P, _D, _P, _P, _P, _I, _P, _I, _P], _I),
    "pfsh_pfasst_run_tol": ([_P, _D, _P, _P, _P, _I, _P, ctypes.POINTER(_I), _P, _P], _I),
    "pfsh_sdc_run": ([_P, _D, _P, _P, _P, _I, _I, _I, _P], _I),
    "pfsh_mlsdc_run": ([_P, _D, _P, _P, _P, _I, _I, _P], _I),
    "pfsh_pfasst_set_levels": ([_P, _P, _P], _I),
    "pfsh_pfasst_set_graphs": ([_P, _I], _I),
}

_lib = None


def lib():
    """Load libpfsh.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1904_05988_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(code, where):
    if code != 0:
        raise PfshError(code, where)


def _stream(t):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(t, dtype, shape, name):
    if t is None:
        raise ValueError(f"{name} is required")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


C128 = torch.complex128
F64 = torch.float64


class Level:
    """One level of the hierarchy: grid, Legendre tables, SDC matrices, workspace.

    legendre="table" stores the packed P_n^m tables; "recurrence" stores none
    and lets the Legendre kernels evaluate P_n^m by recurrence
    (PFSH_LEGENDRE_RECURRENCE; FP64 and FP32 only)."""

    def __init__(self, T, nlat, nlon, n_nodes, max_batch=1, radius=6.371e6, omega=7.292e-5,
                 phibar=9.81 * 1e4, nu=1e5, precision="fp64", device=0, legendre="table"):
        flag = {"table": 0, "recurrence": LEGENDRE_RECURRENCE}[legendre]
        self.desc = LevelDesc(T, nlat, nlon, n_nodes, max_batch, radius, omega, phibar, nu,
                              PRECISIONS[precision] | flag)
        self.precision = precision
        self.legendre = legendre
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        _check(lib().pfsh_level_create(ctypes.byref(self.desc), device, ctypes.byref(h)),
               "pfsh_level_create")
        self._h = h
        K, nn = ctypes.c_int(), ctypes.c_int()
        import numpy as np
        self.nodes = np.zeros(n_nodes)
        self.Q = np.zeros((n_nodes, n_nodes))
        self.QE = np.zeros((n_nodes, n_nodes))
        self.QI = np.zeros((n_nodes, n_nodes))
        self.mu = np.zeros(nlat)
        self.w = np.zeros(nlat)
        _check(lib().pfsh_level_query(h, ctypes.byref(K), ctypes.byref(nn),
                                      self.nodes.ctypes.data, self.Q.ctypes.data,
                                      self.QE.ctypes.data, self.QI.ctypes.data,
                                      self.mu.ctypes.data, self.w.ctypes.data),
               "pfsh_level_query")
        self.K = K.value
        self.T, self.nlat, self.nlon, self.n_nodes, self.max_batch = T, nlat, nlon, n_nodes, max_batch

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().pfsh_level_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    IMPLICIT = {"combined": 0, "split": 1}

    def set_implicit(self, mode):
        """Implicit step of the level's sweeps: "combined" (one solve with L)
        or "split" (physical linear substep, then diffusion substep)."""
        _check(lib().pfsh_level_set_implicit(self._h, self.IMPLICIT[mode]), "pfsh_level_set_implicit")

    def bytes(self):
        """Device memory of the level: (Legendre tables or their recurrence
        data, workspace) in bytes."""
        t, w = ctypes.c_ulonglong(), ctypes.c_ulonglong()
        _check(lib().pfsh_level_bytes(self._h, ctypes.byref(t), ctypes.byref(w)), "pfsh_level_bytes")
        return t.value, w.value

    # -- diagnostic kernel timing
    KERNELS = {"leg_synth": 0, "ring": 1, "leg_anal": 2, "assemble": 3, "prep": 4,
               "sweep_node": 5}

    def profile(self, on=True):
        _check(lib().pfsh_profile_enable(self._h, int(bool(on))), "pfsh_profile_enable")

    def profile_read(self, kernel, batch=0):
        """(launches, total ms) of a kernel since profile(True); batch > 0 keeps
        only the launches over that many states."""
        n, ms = ctypes.c_int(), ctypes.c_double()
        _check(lib().pfsh_profile_read_batch(self._h, self.KERNELS[kernel], int(batch),
                                             ctypes.byref(n), ctypes.byref(ms)),
               "pfsh_profile_read_batch")
        return n.value, ms.value

    # -- transform-kernel variants and the autotuner
    STAGES = {"synth": 0, "anal": 1, "ring": 2, "fuse": 3}
    TUNED = ("synth", "anal", "ring")
    MAX_VARIANTS = 8

    def variant_count(self, stage):
        n = lib().pfsh_variant_count(self._h, self.STAGES[stage])
        if n < 0:
            _check(n, "pfsh_variant_count")
        return n

    def set_variant(self, stage, batch, variant):
        _check(lib().pfsh_level_set_variant(self._h, self.STAGES[stage], int(batch), int(variant)),
               "pfsh_level_set_variant")

    def get_variant(self, stage, batch):
        v = ctypes.c_int()
        _check(lib().pfsh_level_get_variant(self._h, self.STAGES[stage], int(batch),
                                            ctypes.byref(v)), "pfsh_level_get_variant")
        return v.value

    TUNE_COLD = 1

    def autotune(self, batch, reps=20, cold=False):
        """Time every transform-kernel variant at `batch` on the current stream
        and keep the fastest; cold: each launch timed after the caches are
        rewritten.  Returns {stage: (chosen, [us per variant])}."""
        us = (ctypes.c_float * (3 * self.MAX_VARIANTS))()
        s = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
        _check(lib().pfsh_level_autotune_ex(self._h, int(batch), int(reps),
                                            self.TUNE_COLD if cold else 0, s, us),
               "pfsh_level_autotune_ex")
        out = {}
        for name in self.TUNED:
            st = self.STAGES[name]
            n = self.variant_count(name)
            out[name] = (self.get_variant(name, batch),
                         [us[st * self.MAX_VARIANTS + v] for v in range(n)])
        return out

    # -- allocation helpers (caller-owned device memory)
    def state(self, batch):
        return torch.zeros((batch, 3, self.K), dtype=C128, device=self.device)

    def space_time(self, batch):
        return torch.zeros((batch, self.n_nodes, 3, self.K), dtype=C128, device=self.device)

    # -- transforms
    def sh_synthesis(self, spec, grid=None):
        nf = spec.shape[0]
        _need(spec, C128, (nf, self.K), "spec")
        if grid is None:
            grid = torch.empty((nf, self.nlat, self.nlon), dtype=F64, device=spec.device)
        _need(grid, F64, (nf, self.nlat, self.nlon), "grid")
        _check(lib().pfsh_sh_synthesis(self._h, _ptr(spec), _ptr(grid), nf, _stream(spec)),
               "pfsh_sh_synthesis")
        return grid

    def sh_analysis(self, grid, spec=None):
        nf = grid.shape[0]
        _need(grid, F64, (nf, self.nlat, self.nlon), "grid")
        if spec is None:
            spec = torch.empty((nf, self.K), dtype=C128, device=grid.device)
        _need(spec, C128, (nf, self.K), "spec")
        _check(lib().pfsh_sh_analysis(self._h, _ptr(grid), _ptr(spec), nf, _stream(grid)),
               "pfsh_sh_analysis")
        return spec

    # -- operators
    def rhs(self, state, f_expl=None, f_impl=None, want=("e", "i")):
        B = state.shape[0]
        _need(state, C128, (B, 3, self.K), "state")
        if f_expl is None and "e" in want:
            f_expl = torch.empty_like(state)
        if f_impl is None and "i" in want:
            f_impl = torch.empty_like(state)
        for t, n in ((f_expl, "f_expl"), (f_impl, "f_impl")):
            if t is not None:
                _need(t, C128, (B, 3, self.K), n)
        _check(lib().pfsh_rhs(self._h, _ptr(state), _ptr(f_expl), _ptr(f_impl), B,
                              _stream(state)), "pfsh_rhs")
        return f_expl, f_impl

    def implicit_solve(self, beta, b, x=None):
        B = b.shape[0]
        _need(b, C128, (B, 3, self.K), "b")
        if x is None:
            x = torch.empty_like(b)
        _need(x, C128, (B, 3, self.K), "x")
        _check(lib().pfsh_implicit_solve(self._h, float(beta), _ptr(b), _ptr(x), B, _stream(b)),
               "pfsh_implicit_solve")
        return x

    def _st(self, t, name):
        B = t.shape[0]
        return _need(t, C128, (B, self.n_nodes, 3, self.K), name)

    def sdc_sweep(self, dt, theta, f_expl, f_impl, tau=None):
        B = theta.shape[0]
        for t, n in ((theta, "theta"), (f_expl, "f_expl"), (f_impl, "f_impl")):
            self._st(t, n)
        if tau is not None:
            self._st(tau, "tau")
        _check(lib().pfsh_sdc_sweep(self._h, float(dt), _ptr(theta), _ptr(f_expl), _ptr(f_impl),
                                    _ptr(tau), B, _stream(theta)), "pfsh_sdc_sweep")

    def residual(self, dt, theta, f_expl, f_impl, tau=None, out=None):
        B = theta.shape[0]
        for t, n in ((theta, "theta"), (f_expl, "f_expl"), (f_impl, "f_impl")):
            self._st(t, n)
        if tau is not None:
            self._st(tau, "tau")
        if out is None:
            out = torch.empty((B, 3), dtype=F64, device=theta.device)
        _need(out, F64, (B, 3), "out")
        _check(lib().pfsh_residual(self._h, float(dt), _ptr(theta), _ptr(f_expl), _ptr(f_impl),
                                   _ptr(tau), _ptr(out), B, _stream(theta)), "pfsh_residual")
        return out

    def sdc_run(self, dt, theta, f_expl, f_impl, nsteps, nsweeps):
        """Serial SDC(M+1, nsweeps) over nsteps steps; node 0 of theta holds
        the initial states on entry, the final ones on return."""
        B = theta.shape[0]
        for t, n in ((theta, "theta"), (f_expl, "f_expl"), (f_impl, "f_impl")):
            self._st(t, n)
        _check(lib().pfsh_sdc_run(self._h, float(dt), _ptr(theta), _ptr(f_expl), _ptr(f_impl),
                                  int(nsteps), int(nsweeps), B, _stream(theta)), "pfsh_sdc_run")

    def residual_noalloc(self, dt, theta, f_expl, f_impl, tau=None, out=None):
        """pfsh_residual_noalloc: the residual with its partial maxima in the
        library's static device scratch (no allocation; `out` must be given
        by callers that cannot allocate)."""
        B = theta.shape[0]
        shape = (B, self.n_nodes, 3, self.K)
        for t, n in ((theta, "theta"), (f_expl, "f_expl"), (f_impl, "f_impl")):
            _need(t, C128, shape, n)
        if tau is not None:
            _need(tau, C128, shape, "tau")
        if out is None:
            out = torch.empty((B, 3), dtype=F64, device=theta.device)
        _need(out, F64, (B, 3), "out")
        _check(lib().pfsh_residual_noalloc(self._h, float(dt), _ptr(theta), _ptr(f_expl),
                                           _ptr(f_impl), _ptr(tau), _ptr(out), B, _stream(theta)),
               "pfsh_residual_noalloc")
        return out

    def spread(self, theta=None, f_expl=None, f_impl=None):
        ref = next(t for t in (theta, f_expl, f_impl) if t is not None)
        B = ref.shape[0]
        for t, n in ((theta, "theta"), (f_expl, "f_expl"), (f_impl, "f_impl")):
            if t is not None:
                self._st(t, n)
        _check(lib().pfsh_spread(self._h, _ptr(theta), _ptr(f_expl), _ptr(f_impl), B,
                                 _stream(ref)), "pfsh_spread")


def check_finite(values):
    _need(values, F64, tuple(values.shape), "values")
    return lib().pfsh_check_finite(_ptr(values), values.numel(), _stream(values))


def restrict(fine, coarse, x_f, out=None):
    B = x_f.shape[0]
    _need(x_f, C128, (B, fine.n_nodes, 3, fine.K), "x_f")
    if out is None:
        out = torch.empty((B, coarse.n_nodes, 3, coarse.K), dtype=C128, device=x_f.device)
    _need(out, C128, (B, coarse.n_nodes, 3, coarse.K), "out")
    _check(lib().pfsh_restrict(fine.handle, coarse.handle, _ptr(x_f), _ptr(out), B, _stream(x_f)),
           "pfsh_restrict")
    return out


def interpolate_add(coarse, fine, new_c, old_c, inout_f):
    B = new_c.shape[0]
    _need(new_c, C128, (B, coarse.n_nodes, 3, coarse.K), "new_c")
    if old_c is not None:
        _need(old_c, C128, (B, coarse.n_nodes, 3, coarse.K), "old_c")
    _need(inout_f, C128, (B, fine.n_nodes, 3, fine.K), "inout_f")
    _check(lib().pfsh_interpolate_add(coarse.handle, fine.handle, _ptr(new_c), _ptr(old_c),
                                      _ptr(inout_f), B, _stream(new_c)), "pfsh_interpolate_add")
    return inout_f


def fas_tau(fine, coarse, dt, fe_f, fi_f, fe_c, fi_c, tau=None):
    B = fe_f.shape[0]
    for t, n in ((fe_f, "fe_f"), (fi_f, "fi_f")):
        _need(t, C128, (B, fine.n_nodes, 3, fine.K), n)
    for t, n in ((fe_c, "fe_c"), (fi_c, "fi_c")):
        _need(t, C128, (B, coarse.n_nodes, 3, coarse.K), n)
    if tau is None:
        tau = torch.empty_like(fe_c)
    _need(tau, C128, (B, coarse.n_nodes, 3, coarse.K), "tau")
    _check(lib().pfsh_fas_tau(fine.handle, coarse.handle, float(dt), _ptr(fe_f), _ptr(fi_f),
                              _ptr(fe_c), _ptr(fi_c), _ptr(tau), B, _stream(fe_f)),
           "pfsh_fas_tau")
    return tau


class Pfasst:
    """Two-level PFASST block of n_ts time steps x members on one device."""

    def __init__(self, fine, coarse, n_ts, members=1):
        h = ctypes.c_void_p()
        _check(lib().pfsh_pfasst_create(fine.handle, coarse.handle, n_ts, members,
                                        ctypes.byref(h)), "pfsh_pfasst_create")
        self._h, self.fine, self.coarse = h, fine, coarse
        self.n_ts, self.members, self.B = n_ts, members, n_ts * members

    def close(self):
        if getattr(self, "_h", None):
            lib().pfsh_pfasst_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _fine(self, t, n):
        return _need(t, C128, (self.B, self.fine.n_nodes, 3, self.fine.K), n)

    def run(self, dt, theta_f, fe_f, fi_f, n_iter, fine_alt=None, k_switch=None):
        """n_iter iterations in wavefront order (same arithmetic as n_iter
        iterate() calls, the last one stopping after its fine sweep);
        iterations >= k_switch use fine_alt for the fine level."""
        for t, n in ((theta_f, "theta_f"), (fe_f, "fe_f"), (fi_f, "fi_f")):
            self._fine(t, n)
        ks = n_iter if k_switch is None else int(k_switch)
        _check(lib().pfsh_pfasst_run(self._h, float(dt), _ptr(theta_f), _ptr(fe_f), _ptr(fi_f),
                                     int(n_iter), None if fine_alt is None else fine_alt.handle,
                                     ks, _stream(theta_f)), "pfsh_pfasst_run")

    def set_levels(self, fine, coarse):
        """Continue with levels of the same geometry (e.g. another precision)."""
        _check(lib().pfsh_pfasst_set_levels(self._h, fine.handle, coarse.handle),
               "pfsh_pfasst_set_levels")
        self.fine, self.coarse = fine, coarse

    def set_graphs(self, on=True):
        _check(lib().pfsh_pfasst_set_graphs(self._h, int(bool(on))), "pfsh_pfasst_set_graphs")

    def predict(self, dt, theta0, theta_f, fe_f, fi_f):
        _need(theta0, C128, (self.members, 3, self.fine.K), "theta0")
        for t, n in ((theta_f, "theta_f"), (fe_f, "fe_f"), (fi_f, "fi_f")):
            self._fine(t, n)
        _check(lib().pfsh_pfasst_predict(self._h, float(dt), _ptr(theta0), _ptr(theta_f),
                                         _ptr(fe_f), _ptr(fi_f), _stream(theta0)),
               "pfsh_pfasst_predict")

    def iterate(self, dt, theta_f, fe_f, fi_f, last=False):
        for t, n in ((theta_f, "theta_f"), (fe_f, "fe_f"), (fi_f, "fi_f")):
            self._fine(t, n)
        _check(lib().pfsh_pfasst_iterate(self._h, float(dt), _ptr(theta_f), _ptr(fe_f),
                                         _ptr(fi_f), int(bool(last)), _stream(theta_f)),
               "pfsh_pfasst_iterate")

    def mlsdc_run(self, dt, theta_f, fe_f, fi_f, nsteps, n_iter):
        """MLSDC(Mf+1, Mc+1, n_iter) over nsteps steps (a context with n_ts = 1);
        node 0 of theta_f holds the initial states on entry, the final ones on
        return."""
        for t, n in ((theta_f, "theta_f"), (fe_f, "fe_f"), (fi_f, "fi_f")):
            self._fine(t, n)
        _check(lib().pfsh_mlsdc_run(self._h, float(dt), _ptr(theta_f), _ptr(fe_f), _ptr(fi_f),
                                    int(nsteps), int(n_iter), _stream(theta_f)), "pfsh_mlsdc_run")

    def run_tol(self, dt, theta_f, fe_f, fi_f, max_iter, tol):
        """Iterations until every slice's fine residual is at most tol (three
        per-variable bounds) after a fine sweep, or max_iter; returns (the
        number of iterations, residuals [iterations][B][3] as numpy)."""
        import numpy as np
        for t, n in ((theta_f, "theta_f"), (fe_f, "fe_f"), (fi_f, "fi_f")):
            self._fine(t, n)
        tl = (ctypes.c_double * 3)(*[float(v) for v in tol])
        res = np.zeros((int(max_iter), self.B, 3))
        it = ctypes.c_int()
        code = lib().pfsh_pfasst_run_tol(self._h, float(dt), _ptr(theta_f), _ptr(fe_f), _ptr(fi_f),
                                         int(max_iter), ctypes.cast(tl, ctypes.c_void_p), ctypes.byref(it),
                                         res.ctypes.data_as(ctypes.c_void_p), _stream(theta_f))
        _check(code, "pfsh_pfasst_run_tol")
        return it.value, res[: it.value]
