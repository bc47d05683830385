"""CPU oracle for the GP-WENO FD-Prim scheme.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this package;
the product library never does, and the two share no code.

Pieces:
  * :mod:`oracle.tables` -- pre-simulation GP tables in 60-digit arithmetic (mpmath);
  * ``gpweno_oracle.c``  -- the scheme in plain float64 C (built into ``liboracle.so``);
  * this module          -- ctypes loader and a small ``OracleSolver`` wrapper.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .tables import SCHEMES, gp_ao_tables, gp_tables, scheme_tables  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gpweno_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c11"]


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` next to its source with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Cfg(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("n", ctypes.c_int * 3),
        ("dx", ctypes.c_double * 3),
        ("R", ctypes.c_int),
        ("gamma", ctypes.c_double),
        ("positivity_fallback", ctypes.c_int),
        ("wp", ctypes.c_double * 48),
        ("wm", ctypes.c_double * 48),
        ("gp", ctypes.c_double * 12),
        ("gm", ctypes.c_double * 12),
        ("P", ctypes.c_double * 48),
        ("beta_form", ctypes.c_int),
        ("B", ctypes.c_double * 192),
        ("bc", ctypes.c_int * 6),
        ("nonzero_mean", ctypes.c_int),
        ("ao", ctypes.c_int),
        ("ao_w7", ctypes.c_double * 42),
        ("ao_w5", ctypes.c_double * 30),
        ("ao_w3", ctypes.c_double * 54),
        ("ao_P7", ctypes.c_double * 147),
        ("ao_P5", ctypes.c_double * 75),
        ("ao_P3", ctypes.c_double * 27),
        ("ao_c", ctypes.c_double * 9),
        ("ao_gam", ctypes.c_double * 4),
        ("flux_corr_terms", ctypes.c_int),
    ]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        L.oracle_cfg_size.restype = ctypes.c_size_t
        assert L.oracle_cfg_size() == ctypes.sizeof(Cfg), "oracle_cfg layout mismatch"
        L.oracle_rhs.restype = ctypes.c_long
        L.oracle_rhs.argtypes = [ctypes.POINTER(Cfg), _dp, _dp]
        L.oracle_max_speed.restype = ctypes.c_double
        L.oracle_max_speed.argtypes = [ctypes.POINTER(Cfg), _dp]
        L.oracle_dt.restype = ctypes.c_double
        L.oracle_dt.argtypes = [ctypes.POINTER(Cfg), _dp, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.oracle_step_dt.restype = ctypes.c_long
        L.oracle_step_dt.argtypes = [ctypes.POINTER(Cfg), _dp, ctypes.c_double]
        L.oracle_run.restype = ctypes.c_long
        L.oracle_run.argtypes = [ctypes.POINTER(Cfg), _dp, ctypes.c_double, ctypes.c_double, ctypes.c_long,
                                 _dp, ctypes.POINTER(ctypes.c_long)]
        L.oracle_run_fixed.restype = ctypes.c_long
        L.oracle_run_fixed.argtypes = [ctypes.POINTER(Cfg), _dp, ctypes.c_double, ctypes.c_long]
        L.oracle_gp_weno.restype = None
        L.oracle_gp_weno.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_int, _dp, _dp, _dp,
                                     _dp, _dp]
        L.oracle_gp_ao.restype = None
        L.oracle_gp_ao.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.oracle_ao_hybrid.restype = ctypes.c_double
        L.oracle_ao_hybrid.argtypes = [ctypes.c_double, ctypes.c_double, _dp, _dp, _dp]
        L.oracle_ao_recursive.restype = ctypes.c_double
        L.oracle_ao_recursive.argtypes = [ctypes.c_double] * 5
        L.oracle_hllc.restype = None
        L.oracle_hllc.argtypes = [_dp, _dp, ctypes.c_double, _dp]
        L.oracle_flux_hat.restype = ctypes.c_double
        L.oracle_flux_hat.argtypes = [_dp]
        L.oracle_flux_hat7.restype = ctypes.c_double
        L.oracle_flux_hat7.argtypes = [_dp]
        L.oracle_char_vectors.restype = None
        L.oracle_char_vectors.argtypes = [_dp, ctypes.c_double, _dp, _dp]
        L.oracle_rk3_combine.restype = None
        L.oracle_rk3_combine.argtypes = [ctypes.c_int, ctypes.c_size_t, _dp, _dp, _dp, ctypes.c_double, _dp]
        L.oracle_threads.restype = ctypes.c_int
        L.oracle_cons_to_prim.restype = None
        L.oracle_cons_to_prim.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp]
        _lib = L
    return _lib


def threads() -> int:
    """OpenMP threads used by the oracle's pencil loops."""
    return lib().oracle_threads()


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


# ----------------------------------------------------------------------------
# Thin wrappers over the per-step building blocks (used by the pin tests).
# ----------------------------------------------------------------------------
def gp_weno(f, tab, nonzero_mean=False):
    """WENO interpolation of one variable; ``f`` has 2R+1 entries. ``tab`` is a
    table dict (``gp_tables`` or ``scheme_tables``); a 'B' beta form selects the
    polynomial smoothness indicator. Returns (q+, q-, beta, omega+, omega-)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    R = (len(f) - 1) // 2
    qp = ctypes.c_double()
    qm = ctypes.c_double()
    beta = np.zeros(4)
    omp = np.zeros(4)
    omm = np.zeros(4)
    arrs = [np.ascontiguousarray(tab[k], dtype=np.float64) for k in ("w+", "w-", "gamma+", "gamma-", "P")]
    B = None
    if tab.get("beta_form") == "B":
        B = np.ascontiguousarray(tab["B"], dtype=np.float64)
    lib().oracle_gp_weno(R, _ptr(f), *[_ptr(a) for a in arrs], _ptr(B) if B is not None else None,
                         1 if nonzero_mean else 0, ctypes.byref(qp), ctypes.byref(qm), _ptr(beta), _ptr(omp),
                         _ptr(omm))
    return qp.value, qm.value, beta[: R + 1], omp[: R + 1], omm[: R + 1]


def gp_ao(f, tab, side):
    """GP-AO interpolation of one variable (App. A): f has 7 entries (GP-AO(3,2,3))
    or 5 (GP-AO(2,3)); side 0 is x_* = +1/2, side 1 is x_* = -1/2. ``tab`` is
    ``gp_ao_tables``. Returns (q, beta) with beta = (beta^7, beta^5, beta_1..3)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    R = (len(f) - 1) // 2
    key = "+" if side == 0 else "-"
    arrs = [np.ascontiguousarray(tab[k], dtype=np.float64) for k in
            ("w7" + key, "w5" + key, "w3" + key, "P7", "P5", "P3")]
    cN = np.array([tab["c7"], tab["c5"], tab["c3"]])
    gam = np.array(list(tab["gamma"]) + [tab["gamma_hi"]])
    q = ctypes.c_double()
    beta = np.zeros(5)
    lib().oracle_gp_ao(R, _ptr(f), *[_ptr(a) for a in arrs], _ptr(cN), _ptr(gam), ctypes.byref(q), _ptr(beta))
    return q.value, beta


def ao_hybrid(qR, bR, qm, bm, gam, g_hi):
    """Eq. (GP-AO) with its weights (Eq. (nonlin-AO)) from given indicators."""
    qm, bm = np.ascontiguousarray(qm, dtype=np.float64), np.ascontiguousarray(bm, dtype=np.float64)
    g = np.array(list(gam) + [g_hi], dtype=np.float64)
    return lib().oracle_ao_hybrid(qR, bR, _ptr(qm), _ptr(bm), _ptr(g))


def ao_recursive(ao_hi, b_hi, ao_lo, b_lo, g_hi):
    """Eq. (AO-recursive) with the weights of Eq. (recursive-weights)."""
    return lib().oracle_ao_recursive(ao_hi, b_hi, ao_lo, b_lo, g_hi)


def hllc(qL, qR, gamma):
    """HLLC flux in the rotated frame; q = (rho, u_n, u_t1, u_t2, p)."""
    qL = np.ascontiguousarray(qL, dtype=np.float64)
    qR = np.ascontiguousarray(qR, dtype=np.float64)
    F = np.zeros(5)
    lib().oracle_hllc(_ptr(qL), _ptr(qR), gamma, _ptr(F))
    return F


def flux_hat(F):
    """Corrected flux from 5 face fluxes (alpha, beta) or 7 (with the sixth
    difference), centred on the face."""
    F = np.ascontiguousarray(F, dtype=np.float64)
    if F.size == 7:
        return lib().oracle_flux_hat7(_ptr(F))
    assert F.size == 5
    return lib().oracle_flux_hat(_ptr(F))


def char_vectors(q, gamma):
    q = np.ascontiguousarray(q, dtype=np.float64)
    L = np.zeros((5, 5))
    Rm = np.zeros((5, 5))
    lib().oracle_char_vectors(_ptr(q), gamma, _ptr(L), _ptr(Rm))
    return L, Rm  # rows l_k, and Rm[k] = r_k


def rk3_combine(stage, Un, Uin, L, dt):
    Un, Uin, L = (np.ascontiguousarray(a, dtype=np.float64) for a in (Un, Uin, L))
    out = np.empty_like(Un)
    lib().oracle_rk3_combine(stage, Un.size, _ptr(Un), _ptr(Uin), _ptr(L), dt, _ptr(out))
    return out


# ----------------------------------------------------------------------------
# Whole-scheme driver.
# ----------------------------------------------------------------------------
class OracleSolver:
    """FP64 CPU reference solver. ``ell`` and ``sigma`` are physical lengths.
    ``scheme`` is one of ``SCHEMES`` (default: the paper's GP-WENO).
    ``nonzero_mean``: GP indicators of the data minus the centre cell's value."""

    def __init__(self, grid, R, ell, sigma, gamma=1.4, cfl=0.4, positivity_fallback=False, scheme="gp-weno",
                 nonzero_mean=False, flux_corr_terms=2):
        self.grid = grid
        self.R = R
        self.cfl = cfl
        c = Cfg()
        c.ndim = grid.ndim
        for d in range(3):
            c.n[d] = grid.n[d] if d < grid.ndim else 1
            c.dx[d] = grid.dx[d] if d < grid.ndim else 1.0
        c.R = R
        c.gamma = gamma
        c.positivity_fallback = 1 if positivity_fallback else 0
        c.nonzero_mean = 1 if nonzero_mean else 0
        if flux_corr_terms not in (2, 3):
            raise ValueError("flux_corr_terms is 2 or 3")
        c.flux_corr_terms = flux_corr_terms
        bc = getattr(grid, "bc", ((0, 0),) * 3)
        for d in range(3):
            lo_bc, hi_bc = bc[d] if d < grid.ndim else (0, 0)
            if (lo_bc == 0) != (hi_bc == 0):
                raise ValueError("a periodic axis must be periodic on both sides")
            if 2 in (lo_bc, hi_bc) and grid.n[d] < R + 1 + flux_corr_terms:
                raise ValueError("a reflecting side needs at least R + 1 + flux_corr_terms cells on its axis")
            c.bc[2 * d] = lo_bc
            c.bc[2 * d + 1] = hi_bc
        self.tables = []
        if scheme == "gp-ao":
            if R not in (2, 3):
                raise ValueError("GP-AO needs R = 2 (GP-AO(2,3)) or 3 (GP-AO(3,2,3))")
            c.ao = 1
            for d in range(grid.ndim):
                t = gp_ao_tables(ell / grid.dx[d], sigma / grid.dx[d])
                self.tables.append(t)
                for side, key in enumerate("+-"):
                    for j in range(7):
                        c.ao_w7[14 * d + 7 * side + j] = t["w7" + key][j]
                    for j in range(5):
                        c.ao_w5[10 * d + 5 * side + j] = t["w5" + key][j]
                    for m in range(3):
                        for j in range(3):
                            c.ao_w3[18 * d + 9 * side + 3 * m + j] = t["w3" + key][m, j]
                for N, arr in ((7, c.ao_P7), (5, c.ao_P5), (3, c.ao_P3)):
                    for i in range(N):
                        for j in range(N):
                            arr[N * N * d + N * i + j] = t[f"P{N}"][i, j]
                for k, N in enumerate((7, 5, 3)):
                    c.ao_c[3 * d + k] = t[f"c{N}"]
            for m in range(3):
                c.ao_gam[m] = t["gamma"][m]
            c.ao_gam[3] = t["gamma_hi"]
        for d in range(grid.ndim if scheme != "gp-ao" else 0):
            t = scheme_tables(scheme, R, ell / grid.dx[d], sigma / grid.dx[d])
            self.tables.append(t)
            c.beta_form = 1 if t["beta_form"] == "B" else 0
            for idx, v in enumerate(np.asarray(t["B"]).ravel()):
                c.B[64 * d + idx] = v
            for m in range(4):
                c.gp[4 * d + m] = t["gamma+"][m]
                c.gm[4 * d + m] = t["gamma-"][m]
                for j in range(4):
                    c.wp[16 * d + 4 * m + j] = t["w+"][m, j]
                    c.wm[16 * d + 4 * m + j] = t["w-"][m, j]
                    c.P[16 * d + 4 * m + j] = t["P"][m, j]
        self.cfg = c
        self.fallbacks = 0

    def _check(self, U):
        assert U.dtype == np.float64 and U.flags["C_CONTIGUOUS"]
        assert U.size == self.grid.nv * self.grid.ncells

    def rhs(self, U):
        self._check(U)
        L = np.empty_like(U)
        self.fallbacks += lib().oracle_rhs(ctypes.byref(self.cfg), _ptr(U), _ptr(L))
        return L

    def max_speed(self, U):
        self._check(U)
        return lib().oracle_max_speed(ctypes.byref(self.cfg), _ptr(U))

    def dt(self, U, t, t_final):
        return lib().oracle_dt(ctypes.byref(self.cfg), _ptr(U), self.cfl, t, t_final)

    def step(self, U, dt):
        """One SSP-RK3 step of size dt, in place."""
        self._check(U)
        self.fallbacks += lib().oracle_step_dt(ctypes.byref(self.cfg), _ptr(U), dt)
        return U

    def run(self, U, t_final, max_steps=-1, t0=0.0):
        """CFL-limited run to t_final (in place). Returns (t, nsteps)."""
        self._check(U)
        t = ctypes.c_double(t0)
        n = ctypes.c_long(0)
        self.fallbacks += lib().oracle_run(ctypes.byref(self.cfg), _ptr(U), self.cfl, t_final, max_steps,
                                           ctypes.byref(t), ctypes.byref(n))
        return t.value, n.value

    def run_fixed(self, U, dt, nsteps):
        self._check(U)
        self.fallbacks += lib().oracle_run_fixed(ctypes.byref(self.cfg), _ptr(U), dt, nsteps)
        return U
