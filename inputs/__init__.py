"""Seeded synthetic initial data for the compressible Euler problems.

This module is shared by the oracle-based tests and by the GPU path's tests and
benchmark. It holds problem set-up only (grids, initial primitive fields, the
conserved-variable definition of the Euler system, request streams); it contains
none of the GP-WENO scheme's arithmetic.

State layout everywhere: structure-of-arrays ``[nv, nz, ny, nx]`` (x fastest),
float64, with ``nv = 2 + ndim`` conserved fields ``(rho, rho*u[, rho*v[, rho*w]], E)``
(Sec. 2, Eq. (euler)). Point values live at cell centres
``x_i = lo + (i + 1/2) * dx`` (Sec. 2: the scheme evolves pointwise values).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


PERIODIC, OUTFLOW, REFLECT = 0, 1, 2   # boundary kinds, per axis and side


@dataclasses.dataclass(frozen=True)
class Grid:
    """Uniform grid. ``n`` and ``lo``/``hi`` are given per axis (x, y, z).
    ``bc[d] = (low side, high side)`` boundary kinds; periodic by default
    (a periodic axis is periodic on both sides)."""

    ndim: int
    n: tuple
    lo: tuple
    hi: tuple
    bc: tuple = ((PERIODIC, PERIODIC), (PERIODIC, PERIODIC), (PERIODIC, PERIODIC))

    @property
    def nv(self) -> int:
        return 2 + self.ndim

    @property
    def dx(self) -> tuple:
        return tuple((self.hi[d] - self.lo[d]) / self.n[d] for d in range(self.ndim))

    @property
    def ncells(self) -> int:
        return int(np.prod(self.n[: self.ndim]))

    @property
    def shape(self) -> tuple:
        """Array shape of one field, slowest axis first."""
        return tuple(reversed(self.n[: self.ndim]))

    def centres(self, d: int) -> np.ndarray:
        return self.lo[d] + (np.arange(self.n[d]) + 0.5) * self.dx[d]

    def mesh(self):
        """Cell-centre coordinates broadcast to ``shape``; returns (x[, y[, z]])."""
        axes = [self.centres(d) for d in range(self.ndim)]
        grids = np.meshgrid(*reversed(axes), indexing="ij")
        return tuple(reversed(grids))


def _bc(bc, ndim):
    """None: periodic; an int: that kind on every side; else per-axis pairs."""
    if bc is None:
        bc = PERIODIC
    if isinstance(bc, int):
        bc = [(bc, bc)] * ndim
    bc = [tuple(b) for b in bc] + [(PERIODIC, PERIODIC)] * (3 - len(bc))
    return tuple(bc[:3])


def grid1d(n, lo=0.0, hi=1.0, bc=None) -> Grid:
    return Grid(1, (n, 1, 1), (lo, 0.0, 0.0), (hi, 1.0, 1.0), _bc(bc, 1))


def grid2d(nx, ny, lo=(0.0, 0.0), hi=(1.0, 1.0), bc=None) -> Grid:
    return Grid(2, (nx, ny, 1), (lo[0], lo[1], 0.0), (hi[0], hi[1], 1.0), _bc(bc, 2))


def grid3d(nx, ny, nz, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), bc=None) -> Grid:
    return Grid(3, (nx, ny, nz), tuple(lo), tuple(hi), _bc(bc, 3))


def prim_to_cons(grid: Grid, rho, vel, p, gamma):
    """Conserved variables of the Euler system, Sec. 2 Eq. (euler).

    ``vel`` is a sequence of ``ndim`` velocity arrays. Returns ``[nv, *shape]`` float64.
    """
    rho = np.asarray(rho, dtype=np.float64)
    vel = [np.broadcast_to(np.asarray(v, dtype=np.float64), rho.shape) for v in vel]
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), rho.shape)
    kinetic = 0.5 * rho * sum(v * v for v in vel)
    out = np.empty((grid.nv,) + rho.shape, dtype=np.float64)
    out[0] = rho
    for d in range(grid.ndim):
        out[1 + d] = rho * vel[d]
    out[grid.nv - 1] = p / (gamma - 1.0) + kinetic
    return np.ascontiguousarray(out)


def cons_to_prim(grid: Grid, U, gamma):
    """Inverse of :func:`prim_to_cons` (used by tests and reporting only)."""
    rho = U[0]
    vel = [U[1 + d] / rho for d in range(grid.ndim)]
    kinetic = 0.5 * rho * sum(v * v for v in vel)
    p = (gamma - 1.0) * (U[grid.nv - 1] - kinetic)
    return rho, vel, p


# --------------------------------------------------------------------------
# Smooth advection problems (Sec. 6).
# --------------------------------------------------------------------------
def sine_wave_1d(n, gamma=1.4, t=0.0, amp=0.2):
    """rho = 1 + amp*sin(2*pi*(x - t)), u = 1, p = 1 on periodic [0, 1]."""
    g = grid1d(n)
    (x,) = g.mesh()
    rho = 1.0 + amp * np.sin(2.0 * math.pi * (x - t))
    return g, prim_to_cons(g, rho, [np.ones_like(x)], np.ones_like(x), gamma)


def gaussian_1d(n, gamma=5.0 / 3.0, t=0.0):
    """The 1D Gaussian density pulse of Sec. 6.1: rho = 1 + exp(-100 (x-0.5)^2),
    u = 1, p = 1/gamma, periodic [0, 1]; exact solution is the translate."""
    g = grid1d(n)
    (x,) = g.mesh()
    xs = np.mod(x - t, 1.0)
    # periodic images within +-1 so the pulse wraps smoothly
    rho = 1.0 + sum(np.exp(-100.0 * (xs + k - 0.5) ** 2) for k in (-1, 0, 1))
    return g, prim_to_cons(g, rho, [np.ones_like(x)], np.full_like(x, 1.0 / gamma), gamma)


def _vortex_prim(x, y, gamma, strength, u0, v0):
    r2 = x * x + y * y
    f = strength / (2.0 * math.pi) * np.exp(0.5 * (1.0 - r2))
    u = u0 - f * y
    v = v0 + f * x
    T = 1.0 - (gamma - 1.0) * strength**2 / (8.0 * gamma * math.pi**2) * np.exp(1.0 - r2)
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T
    return rho, u, v, p


def isentropic_vortex_2d(n, lo=-5.0, hi=5.0, strength=5.0, gamma=1.4, t=0.0):
    """Isentropic vortex on a periodic square, background (rho,u,v,p) = (1,1,1,1),
    advected diagonally (Sec. 6.2). Vortex centre at the domain centre at t = 0;
    the exact solution at time t is the initial field translated by (t, t)."""
    g = grid2d(n, n, (lo, lo), (hi, hi))
    x, y = g.mesh()
    L = hi - lo
    c = 0.5 * (lo + hi)
    xs = np.mod(x - t - lo, L) + lo - c
    ys = np.mod(y - t - lo, L) + lo - c
    rho, u, v, p = _vortex_prim(xs, ys, gamma, strength, 1.0, 1.0)
    return g, prim_to_cons(g, rho, [u, v], p, gamma)


def kelvin_helmholtz_2d(nx=2048, ny=1024, gamma=1.4, seed=0, amp=0.01):
    """Shear layer on periodic [0,2]x[0,1]: rho=2, u=+0.5 in 0.25<=y<0.75,
    rho=1, u=-0.5 elsewhere, p=2.5, plus seeded uniform velocity noise of
    amplitude ``amp`` drawn once in float64 on the host."""
    g = grid2d(nx, ny, (0.0, 0.0), (2.0, 1.0))
    x, y = g.mesh()
    band = (y >= 0.25) & (y < 0.75)
    rho = np.where(band, 2.0, 1.0)
    u = np.where(band, 0.5, -0.5)
    rng = np.random.default_rng(seed)
    du = amp * (2.0 * rng.random(g.shape) - 1.0)
    dv = amp * (2.0 * rng.random(g.shape) - 1.0)
    return g, prim_to_cons(g, rho, [u + du, dv], np.full_like(x, 2.5), gamma)


def density_wave_3d(n, gamma=1.4, t=0.0, amp=0.2):
    """rho = 1 + amp*sin(2*pi*(x+y+z - 3t)), u=v=w=1, p=1 on periodic [0,1]^3."""
    g = grid3d(n, n, n)
    x, y, z = g.mesh()
    rho = 1.0 + amp * np.sin(2.0 * math.pi * (x + y + z - 3.0 * t))
    one = np.ones_like(x)
    return g, prim_to_cons(g, rho, [one, one, one], one, gamma)


def isentropic_vortex_3d(n, lo=-5.0, hi=5.0, strength=5.0, gamma=1.4):
    """The 2D vortex in (x, y), uniform along z, with w = 0, on a periodic cube."""
    g = grid3d(n, n, n, (lo, lo, lo), (hi, hi, hi))
    x, y, z = g.mesh()
    rho, u, v, p = _vortex_prim(x, y, gamma, strength, 1.0, 1.0)
    return g, prim_to_cons(g, rho, [u, v, np.zeros_like(x)], p, gamma)


def four_quadrant_2d(n, rng, gamma=1.4):
    """Four constant quadrants on periodic [0,1]^2 with rho ~ U[0.1,1.5],
    p ~ U[0.03,1.5], u = v = 0 (random two-dimensional Riemann data)."""
    g = grid2d(n, n)
    x, y = g.mesh()
    rq = rng.uniform(0.1, 1.5, size=4)
    pq = rng.uniform(0.03, 1.5, size=4)
    q = (x >= 0.5).astype(int) + 2 * (y >= 0.5).astype(int)
    rho = rq[q]
    p = pq[q]
    zero = np.zeros_like(x)
    return g, prim_to_cons(g, rho, [zero, zero], p, gamma)


# The paper's 3D explosion (Sec. 7, Eq. (3d-exp)): inside a sphere of radius 0.5
# V = (rho, u, v, w, p) = (1, 0, 0, 0, 1), outside (0.125, 0, 0, 0, 0.1), on
# [-1,1]^3 with outflow boundaries, gamma = 1.4, to t = 0.25.
EXPLOSION_IN = (1.0, 1.0)      # (rho, p)
EXPLOSION_OUT = (0.125, 0.1)


def explosion(ndim, n, gamma=1.4, radius=0.5):
    """The explosion data on [-1,1]^ndim with outflow boundaries: the paper's 3D
    problem for ndim = 3, its plane and line sections for ndim = 2, 1 (ndim = 1
    is a two-sided shock tube with the diaphragms at x = +-0.5)."""
    make = {1: lambda: grid1d(n, -1.0, 1.0, OUTFLOW), 2: lambda: grid2d(n, n, (-1.0, -1.0), (1.0, 1.0), OUTFLOW),
            3: lambda: grid3d(n, n, n, (-1.0,) * 3, (1.0,) * 3, OUTFLOW)}
    g = make[ndim]()
    X = g.mesh()
    r2 = sum(x * x for x in X)
    inside = r2 <= radius * radius
    rho = np.where(inside, EXPLOSION_IN[0], EXPLOSION_OUT[0])
    p = np.where(inside, EXPLOSION_IN[1], EXPLOSION_OUT[1])
    vel = [np.zeros(g.shape) for _ in range(ndim)]
    return g, prim_to_cons(g, rho, vel, p, gamma)


def shock_tube_1d(n, x0=0.5, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1), lo=0.0, hi=1.0, gamma=1.4,
                  bc=OUTFLOW):
    """A 1D Riemann problem: (rho, u, p) = left for x < x0, right beyond. The
    defaults are the two states of the paper's explosion data (Eq. (3d-exp))."""
    g = grid1d(n, lo, hi, bc)
    x = g.centres(0)
    L = x < x0
    rho = np.where(L, left[0], right[0])
    u = np.where(L, left[1], right[1])
    p = np.where(L, left[2], right[2])
    return g, prim_to_cons(g, rho, [u], p, gamma)


def uniform_state(grid: Grid, rho=1.3, vel=(0.7, -0.4, 0.25), p=0.9, gamma=1.4):
    shape = grid.shape
    r = np.full(shape, rho)
    return prim_to_cons(grid, r, [np.full(shape, vel[d]) for d in range(grid.ndim)], np.full(shape, p), gamma)


def random_smooth(grid: Grid, seed=0, gamma=1.4, amp=0.1, modes=3):
    """Positive smooth random state built from a few periodic Fourier modes."""
    rng = np.random.default_rng(seed)
    X = grid.mesh()
    L = [grid.hi[d] - grid.lo[d] for d in range(grid.ndim)]

    def field(base):
        f = np.full(grid.shape, base, dtype=np.float64)
        for _ in range(modes):
            k = rng.integers(1, 4, size=grid.ndim)
            ph = rng.uniform(0, 2 * math.pi)
            arg = sum(2 * math.pi * k[d] * (X[d] - grid.lo[d]) / L[d] for d in range(grid.ndim))
            f += amp * rng.uniform(-1, 1) * np.sin(arg + ph)
        return f

    rho = field(1.0)
    vel = [field(0.3 * (d + 1)) for d in range(grid.ndim)]
    p = field(1.0)
    return prim_to_cons(grid, rho, vel, p, gamma)


def mirror(grid: Grid, U, axis: int):
    """Mirror image x -> -x about the domain centre along ``axis`` (flips the
    normal momentum). Cell i maps to cell n-1-i."""
    arr_axis = grid.ndim - axis  # field axes are (nv, [z,] [y,] x)
    V = np.flip(U, axis=arr_axis).copy()
    V[1 + axis] *= -1.0
    return V


# --------------------------------------------------------------------------
# Serving request stream.
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Request:
    """One independent Euler problem of a serving stream. The initial state is
    built on demand (``state()``) so a long stream costs no memory up front."""

    rid: int
    arrival: float
    n: int
    R: int
    steps: int
    kind: str  # "vortex" or "quadrant"
    grid: Grid
    seed: int
    gamma: float = 1.4

    def cache_state(self):
        """Builds the initial state now (so a timed run does not pay for it)."""
        self.__dict__["_state"] = self.state()

    def state(self):
        if "_state" in self.__dict__:
            return self.__dict__["_state"]
        if self.kind == "vortex":
            return isentropic_vortex_2d(self.n, gamma=self.gamma)[1]
        return four_quadrant_2d(self.n, np.random.default_rng(self.seed), gamma=self.gamma)[1]

    @property
    def cells(self) -> int:
        return self.grid.ncells


def serving_stream(count=200, rate=20.0, seed=0, sizes=(64, 128, 256, 512, 1024),
                   radii=(1, 2, 3), steps=(100, 500)):
    """Poisson arrivals (mean ``rate`` per second) of independent 2D Euler problems:
    grid edge uniform from ``sizes``, R uniform from ``radii``, step count uniform
    integer in ``steps``, initial data half isentropic vortex on [-5,5]^2, half
    four-quadrant Riemann data on [0,1]^2."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(count):
        t += rng.exponential(1.0 / rate)
        n = int(rng.choice(sizes))
        R = int(rng.choice(radii))
        st = int(rng.integers(steps[0], steps[1] + 1))
        kind = "vortex" if rng.random() < 0.5 else "quadrant"
        sub = int(rng.integers(0, 2**62))
        if kind == "vortex":
            g = grid2d(n, n, (-5.0, -5.0), (5.0, 5.0))
        else:
            g = grid2d(n, n)
        out.append(Request(rid, t, n, R, st, kind, g, sub))
    return out
