"""Python binding of libgpweno (GP-WENO FD-Prim for the Euler equations on MI355X).

Argument marshalling only: every step of the scheme runs in the HIP kernels of
``libgpweno.so`` behind the C ABI declared in ``include/gpweno.h``. PyTorch is
used for device memory and streams. There is no CPU fallback: if the library is
not built, or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgpweno.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "gpweno.h")

OK, EINVAL, ENOMEM, EHIP, ENONPHYS, ESTATE = 0, -1, -2, -3, -4, -5
FP64, FP32 = 0, 1
_STATUS = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EHIP: "EHIP", ENONPHYS: "ENONPHYS", ESTATE: "ESTATE"}


class GpwenoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class NonPhysicalState(GpwenoError):
    pass


class _Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_int * 3), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3), ("bc", ctypes.c_int * 6)]


class _Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("cfl", ctypes.c_double), ("fixed_dt", ctypes.c_double),
                ("positivity_fallback", ctypes.c_int), ("stream", ctypes.c_void_p), ("nonzero_mean", ctypes.c_int),
                ("flux_corr_terms", ctypes.c_int)]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def lib():
    """Loads libgpweno.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise GpwenoError(ESTATE, f"{LIB_PATH} is not built; run `python -m paper_1808_04960_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.gpweno_init.argtypes = [ctypes.POINTER(_Grid), ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.POINTER(vp)]
        L.gpweno_init_scheme.argtypes = [ctypes.POINTER(_Grid), ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.POINTER(vp)]
        L.gpweno_set_options.argtypes = [vp, ctypes.POINTER(_Options)]
        L.gpweno_get_options.argtypes = [vp, ctypes.POINTER(_Options)]
        L.gpweno_state_count.argtypes = [vp]
        L.gpweno_state_count.restype = ctypes.c_size_t
        L.gpweno_workspace_bytes.argtypes = [vp]
        L.gpweno_workspace_bytes.restype = ctypes.c_size_t
        L.gpweno_bind.argtypes = [vp, vp, vp]
        L.gpweno_set_time.argtypes = [vp, ctypes.c_double, ctypes.c_long]
        L.gpweno_step.argtypes = [vp, ctypes.c_double, _dp]
        L.gpweno_run.argtypes = [vp, ctypes.c_double, ctypes.c_long, ctypes.POINTER(ctypes.c_long), _dp]
        L.gpweno_get_time.argtypes = [vp, _dp, _dp, ctypes.POINTER(ctypes.c_long)]
        L.gpweno_get_failure.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_long)]
        L.gpweno_get_tables.argtypes = [vp, ctypes.c_int, _dp, _dp, _dp]
        L.gpweno_table_residual.argtypes = [vp, _dp]
        L.gpweno_compute_table_residual.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                                    _dp]
        L.gpweno_debug_poison.argtypes = [vp, ctypes.c_long]
        L.gpweno_step_noalloc.argtypes = [vp, vp, ctypes.c_double]
        L.gpweno_rhs.argtypes = [vp, vp, vp]
        L.gpweno_rhs_dir.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_int]
        L.gpweno_step_kernel.argtypes = [vp, ctypes.c_int]
        L.gpweno_conserved_sums.argtypes = [vp, _dp]
        L.gpweno_compute_tables.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _dp,
                                            _dp, _dp, _dp]
        L.gpweno_compute_ao_tables.argtypes = [ctypes.c_double, ctypes.c_double, _dp, _dp, _dp, _dp, _dp, _dp]
        L.gpweno_set_end.argtypes = [vp, ctypes.c_double, ctypes.c_long]
        L.gpweno_batch_create.argtypes = [ctypes.POINTER(vp)]
        L.gpweno_batch_set.argtypes = [vp, ctypes.POINTER(vp), ctypes.c_int, vp]
        L.gpweno_batch_run.argtypes = [vp, ctypes.c_int, vp]
        L.gpweno_batch_status.argtypes = [vp, _dp, _dp, ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_int), vp]
        L.gpweno_batch_captures.argtypes = [vp]
        L.gpweno_batch_captures.restype = ctypes.c_long
        L.gpweno_batch_destroy.argtypes = [vp]
        L.gpweno_batch_destroy.restype = None
        L.gpweno_batch_last_error.argtypes = [vp]
        L.gpweno_batch_last_error.restype = ctypes.c_char_p
        L.gpweno_last_error.argtypes = [vp]
        L.gpweno_last_error.restype = ctypes.c_char_p
        L.gpweno_destroy.argtypes = [vp]
        L.gpweno_destroy.restype = None
        _lib = L
    return _lib


def declared_symbols():
    """Names of the functions declared in include/gpweno.h."""
    with open(HEADER_PATH) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"\b(gpweno_[a-z_0-9]+)\s*\(", text)))


def _check(code, ctx=None):
    if code != OK:
        msg = lib().gpweno_last_error(ctx).decode()
        if code == ENONPHYS:
            raise NonPhysicalState(code, msg)
        raise GpwenoError(code, msg)


SCHEMES = {"gp-weno": 0, "weno-js": 1, "weno-gp": 2, "gp-ao": 3}   # gpweno_scheme


def _scheme_id(scheme):
    if scheme not in SCHEMES:
        raise GpwenoError(EINVAL, f"unknown scheme {scheme!r}; one of {sorted(SCHEMES)}")
    return SCHEMES[scheme]


def compute_tables(R, ell_over_dx, sigma_over_dx, scheme="gp-weno"):
    """Host-only pre-simulation tables (binary128 arithmetic rounded to float64).
    'P' has shape (4, 4, 4): beta_m = sum_i (P[m, i] . f_m)^2."""
    wp, wm, P = np.zeros((4, 4)), np.zeros((4, 4)), np.zeros((4, 4, 4))
    gp, gm = np.zeros(4), np.zeros(4)
    ptr = lambda a: a.ctypes.data_as(_dp)  # noqa: E731
    _check(lib().gpweno_compute_tables(_scheme_id(scheme), R, ell_over_dx, sigma_over_dx, ptr(wp), ptr(wm),
                                       ptr(gp), ptr(gm), ptr(P)))
    return {"w+": wp, "w-": wm, "gamma+": gp, "gamma-": gm, "P": P}


def compute_table_residual(R, ell_over_dx, sigma_over_dx, scheme="gp-weno"):
    """Host-only: the mirror residual of the tables compute_tables builds (the
    accuracy the binary128 solves reach; see gpweno_table_residual)."""
    r = ctypes.c_double()
    _check(lib().gpweno_compute_table_residual(_scheme_id(scheme), R, ell_over_dx, sigma_over_dx, ctypes.byref(r)))
    return r.value


def compute_ao_tables(ell_over_dx, sigma_over_dx):
    """Host-only extra tables of the adaptive-order GP scheme (binary128 rounded
    to float64): 'w7' (2, 7), 'w5' (2, 5) (rows: x_* = +1/2, -1/2), 'P7', 'P5',
    'P3', and 'c' = (c7, c5, c3)."""
    out = {"w7": np.zeros((2, 7)), "w5": np.zeros((2, 5)), "P7": np.zeros((7, 7)), "P5": np.zeros((5, 5)),
           "P3": np.zeros((3, 3)), "c": np.zeros(3)}
    ptr = lambda a: a.ctypes.data_as(_dp)  # noqa: E731
    _check(lib().gpweno_compute_ao_tables(ell_over_dx, sigma_over_dx, *[ptr(out[k]) for k in
                                                                         ("w7", "w5", "P7", "P5", "P3", "c")]))
    return out


def make_grid(grid):
    """Any object with ndim, n, lo, hi (per axis) and optionally bc ((low, high)
    boundary kinds per axis, gpweno_bc) -> C grid struct."""
    g = _Grid()
    g.ndim = grid.ndim
    for d in range(3):
        g.n[d] = int(grid.n[d]) if d < grid.ndim else 1
        g.lo[d] = float(grid.lo[d]) if d < grid.ndim else 0.0
        g.hi[d] = float(grid.hi[d]) if d < grid.ndim else 1.0
    bc = getattr(grid, "bc", None)
    for d in range(3):
        lo_bc, hi_bc = bc[d] if (bc is not None and d < grid.ndim) else (0, 0)
        g.bc[2 * d] = int(lo_bc)
        g.bc[2 * d + 1] = int(hi_bc)
    return g


class Solver:
    """One GP-WENO problem resident on the GPU.

    ``ell`` and ``sigma`` are physical lengths; ``precision`` is "fp64" or
    "fp32" (float32 sweep arithmetic, float64 state). The state lives in a
    float64 torch tensor of shape ``(nv, *grid.shape)`` owned by this object.
    ``scheme`` is one of ``SCHEMES``: the paper's GP-WENO (default) or one of
    its polynomial-WENO comparison schemes.
    """

    def __init__(self, grid, R, ell, sigma, gamma=1.4, precision="fp64", cfl=0.4, fixed_dt=0.0,
                 positivity_fallback=False, U0=None, device=None, stream=None, scheme="gp-weno", nonzero_mean=False,
                 flux_corr_terms=2):
        import torch

        if not torch.cuda.is_available():
            raise GpwenoError(EHIP, "no GPU available (there is no CPU fallback)")
        self._torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.grid = grid
        self.R = R
        self.nv = 2 + grid.ndim
        self.shape = (self.nv,) + tuple(reversed([grid.n[d] for d in range(grid.ndim)]))
        self._ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
            g = make_grid(grid)
            _check(lib().gpweno_init_scheme(ctypes.byref(g), _scheme_id(scheme), R, ell, sigma, gamma,
                                            ctypes.byref(self._ctx)))
            count = lib().gpweno_state_count(self._ctx)
            assert count == int(np.prod(self.shape))
            self.state = torch.empty(self.shape, dtype=torch.float64, device=self.device)
            self.workspace = torch.empty(lib().gpweno_workspace_bytes(self._ctx), dtype=torch.uint8,
                                         device=self.device)
        self._bound = False
        self.scheme = scheme
        self.nonzero_mean = bool(nonzero_mean)
        self.flux_corr_terms = int(flux_corr_terms)
        self.set_options(precision, cfl, fixed_dt, positivity_fallback)
        if U0 is not None:
            self.set_state(U0)

    # -- configuration -------------------------------------------------------
    def set_options(self, precision="fp64", cfl=0.4, fixed_dt=0.0, positivity_fallback=False, nonzero_mean=None,
                    flux_corr_terms=None):
        """nonzero_mean, flux_corr_terms: None keeps the current choice (see gpweno_options)."""
        if nonzero_mean is not None:
            self.nonzero_mean = bool(nonzero_mean)
        if flux_corr_terms is not None:
            self.flux_corr_terms = int(flux_corr_terms)
        o = _Options()
        o.precision = {"fp64": FP64, "fp32": FP32}[precision]
        o.cfl = cfl
        o.fixed_dt = fixed_dt
        o.positivity_fallback = 1 if positivity_fallback else 0
        o.stream = self.stream.cuda_stream
        o.nonzero_mean = 1 if self.nonzero_mean else 0
        o.flux_corr_terms = self.flux_corr_terms
        _check(lib().gpweno_set_options(self._ctx, ctypes.byref(o)), self._ctx)
        self.precision = precision

    # -- state ---------------------------------------------------------------
    def set_state(self, U, t=0.0, nsteps=0, upload_stream=None):
        """Copies U (numpy or torch, float64, shape (nv, *grid.shape)) into the device state.
        upload_stream: copy from pinned host memory on that stream and make this
        solver's stream wait for it, without the host waiting for work already
        enqueued on the solver's stream (the serving loop admits problems so)."""
        torch = self._torch
        src = torch.as_tensor(np.ascontiguousarray(U) if isinstance(U, np.ndarray) else U, dtype=torch.float64)
        if tuple(src.shape) != self.shape:
            raise GpwenoError(EINVAL, f"state shape {tuple(src.shape)} != {self.shape}")
        if upload_stream is not None:
            staged = src.pin_memory() if src.device.type == "cpu" else src
            with torch.cuda.stream(upload_stream):
                self.state.copy_(staged, non_blocking=True)
            self.stream.wait_stream(upload_stream)
        else:
            torch.cuda.current_stream(self.device).synchronize()
            with torch.cuda.stream(self.stream):
                self.state.copy_(src)
        if not self._bound:
            _check(lib().gpweno_bind(self._ctx, ctypes.c_void_p(self.state.data_ptr()),
                                     ctypes.c_void_p(self.workspace.data_ptr())), self._ctx)
            self._bound = True
        _check(lib().gpweno_set_time(self._ctx, t, nsteps), self._ctx)

    def get_state(self):
        """Blocking copy of the state to a numpy array."""
        with self._torch.cuda.stream(self.stream):
            host = self.state.to("cpu", non_blocking=False)
        self.stream.synchronize()
        return host.numpy()

    # -- time stepping ---------------------------------------------------------
    def step(self, t_final, wait=False):
        """One step toward t_final. wait=False enqueues it and returns None;
        wait=True blocks and returns the dt the step took (0 if it did not run)."""
        if not wait:
            _check(lib().gpweno_step(self._ctx, t_final, None), self._ctx)
            return None
        dt = ctypes.c_double()
        _check(lib().gpweno_step(self._ctx, t_final, ctypes.byref(dt)), self._ctx)
        return dt.value

    def step_noalloc(self, t_final, state=None):
        """One step (enqueued) of `state` (a float64 device tensor of this
        problem's shape; default: this solver's own state) through the entry
        point that allocates nothing: stage states and accumulator in the
        library's fixed device scratch instead of this solver's workspace."""
        st = self.state if state is None else state
        if tuple(st.shape) != self.shape or st.dtype != self._torch.float64 or not st.is_contiguous():
            raise GpwenoError(EINVAL, "state must be a contiguous float64 tensor of the problem's shape")
        _check(lib().gpweno_step_noalloc(self._ctx, ctypes.c_void_p(st.data_ptr()), t_final), self._ctx)

    def set_end(self, t_final, step_limit=-1):
        """End time and absolute step limit honoured by batched execution (enqueued)."""
        _check(lib().gpweno_set_end(self._ctx, t_final, step_limit), self._ctx)

    def step_kernel(self, k):
        """Enqueue the k-th of the 3*ndim launches of a step (instrumentation)."""
        _check(lib().gpweno_step_kernel(self._ctx, k), self._ctx)

    def run(self, t_final, max_steps=-1):
        """Blocking: advance to t_final (or max_steps more steps). Returns (nsteps, t)."""
        n = ctypes.c_long()
        t = ctypes.c_double()
        _check(lib().gpweno_run(self._ctx, t_final, max_steps, ctypes.byref(n), ctypes.byref(t)), self._ctx)
        return n.value, t.value

    def time(self):
        t, dt = ctypes.c_double(), ctypes.c_double()
        n = ctypes.c_long()
        _check(lib().gpweno_get_time(self._ctx, ctypes.byref(t), ctypes.byref(dt), ctypes.byref(n)), self._ctx)
        return t.value, dt.value, n.value

    def failure(self):
        """Blocking: (failed, smallest flagged cell index or -1)."""
        f, cell = ctypes.c_int(), ctypes.c_long()
        _check(lib().gpweno_get_failure(self._ctx, ctypes.byref(f), ctypes.byref(cell)), self._ctx)
        return bool(f.value), cell.value

    def tables(self, dir=0):
        """The tables this context uses along axis dir: 'w' (2, n, n) with rows
        x_* = +1/2 and -1/2, 'gamma' (2, n), 'P' (n, n) (None for WENO-JS), where
        n = R + 1 (3 for GP-AO's sub-stencils)."""
        n = 3 if self.scheme == "gp-ao" else self.R + 1
        w, g, P = np.zeros((2, n, n)), np.zeros((2, n)), np.zeros((n, n))
        ptr = lambda a: a.ctypes.data_as(_dp)  # noqa: E731
        js = self.scheme == "weno-js"
        _check(lib().gpweno_get_tables(self._ctx, dir, ptr(w), ptr(g), None if js else ptr(P)), self._ctx)
        return {"w": w, "gamma": g, "P": None if js else P}

    def table_residual(self):
        r = ctypes.c_double()
        _check(lib().gpweno_table_residual(self._ctx, ctypes.byref(r)), self._ctx)
        return r.value

    def debug_poison(self, cell):
        """Test hook: make cell `cell` of the state non-physical (enqueued)."""
        _check(lib().gpweno_debug_poison(self._ctx, int(cell)), self._ctx)

    def synchronize(self):
        self.stream.synchronize()

    # -- diagnostics -----------------------------------------------------------
    def rhs(self, U):
        """Right-hand side of the semi-discrete scheme for an arbitrary state (numpy in, numpy out)."""
        torch = self._torch
        src = torch.as_tensor(np.ascontiguousarray(U), dtype=torch.float64).to(self.device)
        out = torch.empty_like(src)
        torch.cuda.current_stream(self.device).synchronize()
        _check(lib().gpweno_rhs(self._ctx, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(out.data_ptr())),
               self._ctx)
        self.stream.synchronize()
        return out.cpu().numpy()

    def rhs_dir_device(self, dir, U_dev, L_dev, accumulate=False):
        """Enqueue one direction's sweep on device tensors (no synchronisation)."""
        _check(lib().gpweno_rhs_dir(self._ctx, dir, ctypes.c_void_p(U_dev.data_ptr()),
                                    ctypes.c_void_p(L_dev.data_ptr()), 1 if accumulate else 0), self._ctx)

    def conserved_sums(self):
        out = np.zeros(8)
        _check(lib().gpweno_conserved_sums(self._ctx, out.ctypes.data_as(_dp)), self._ctx)
        return out[: self.nv]

    def close(self):
        if self._ctx:
            lib().gpweno_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _bcheck(code, b=None):
    if code != OK:
        raise GpwenoError(code, lib().gpweno_batch_last_error(b).decode())


class Batch:
    """Advances many independent Solvers together (one batched launch per sweep
    and group of problems of one kind: ndim, R, precision, scheme, correction
    terms, boundary kinds and tables). All member solvers and the batch must use
    the same stream."""

    def __init__(self, stream):
        self._b = ctypes.c_void_p()
        self.stream = stream
        _bcheck(lib().gpweno_batch_create(ctypes.byref(self._b)))
        self.members = []

    def set(self, solvers):
        arr = (ctypes.c_void_p * max(1, len(solvers)))(*[sv._ctx.value for sv in solvers])
        _bcheck(lib().gpweno_batch_set(self._b, arr, len(solvers), ctypes.c_void_p(self.stream.cuda_stream)), self._b)
        self.members = list(solvers)

    def run(self, nsteps):
        _bcheck(lib().gpweno_batch_run(self._b, nsteps, ctypes.c_void_p(self.stream.cuda_stream)), self._b)

    def status(self):
        """Blocking: (t, dt, nsteps, err) arrays in member order."""
        n = len(self.members)
        t, dt = np.zeros(max(n, 1)), np.zeros(max(n, 1))
        ns = (ctypes.c_long * max(n, 1))()
        er = (ctypes.c_int * max(n, 1))()
        _bcheck(lib().gpweno_batch_status(self._b, t.ctypes.data_as(_dp), dt.ctypes.data_as(_dp), ns, er,
                                          ctypes.c_void_p(self.stream.cuda_stream)), self._b)
        return t[:n], dt[:n], np.array(ns[:n], dtype=np.int64), np.array(er[:n], dtype=np.int32)

    def captures(self):
        """Times the batch has captured its step graphs (one per kind, together)."""
        return lib().gpweno_batch_captures(self._b)

    def close(self):
        if self._b:
            lib().gpweno_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
