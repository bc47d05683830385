"""Writes the oracle's full-length reference states of the benchmark-scale
workloads, for the full-length GPU parity tests and the benchmark's accuracy
block. Calls only the CPU oracle (``oracle/``) and the seeded inputs.

  vortex2d_512   2D isentropic vortex, 512^2 on [-5,5]^2, GP-R2, ell = 12 dx,
                 sigma = 3 dx, CFL 0.4, to t = 10 (one period): the whole state.
  wave3d_256     3D density wave, 256^3 on [0,1]^3, GP-R2, CFL 0.4, 50 steps.
                 Its initial data depend only on s = (i + j + k) mod 256 up to
                 the rounding of sin at arguments one period apart, the scheme
                 treats every cell alike and the axes alike (u = v = w), so the
                 oracle's state stays a function of s to that rounding: stored
                 as that function (5 x 256 values, from the cells (i, 0, 0)),
                 with the L1 sum and the maximum of its measured deviation from
                 the whole state (a test that compares with the function bounds
                 its distance to the oracle's state by adding the deviation).
  vortex3d_256   3D isentropic vortex (uniform in z, w = 0), 256^3 on [-5,5]^3,
                 GP-R2, CFL 0.4, 50 steps. The state stays exactly uniform in z:
                 stored as one z-slice (5 x 256^2), after checking every slice
                 equals it bitwise.

Usage: python tests/golden/make_oracle_references.py [name ...]
(about 20 min for vortex2d_512 and 10 min for each 3D case on 8 threads).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import inputs  # noqa: E402
import oracle  # noqa: E402


def path(name):
    return os.path.join(HERE, f"oracle_{name}.npz")


def run(name, grid, U, R, t_final, max_steps):
    dx = grid.dx[0]
    o = oracle.OracleSolver(grid, R, 12 * dx, 3 * dx, cfl=0.4)
    t0 = time.time()
    t, n = o.run(U, t_final, max_steps=max_steps)
    print(f"{name}: {n} steps to t = {t!r} in {time.time() - t0:.0f} s on {oracle.threads()} threads", flush=True)
    return t, n


def vortex2d_512():
    g, U = inputs.isentropic_vortex_2d(512)
    t, n = run("vortex2d_512", g, U, 2, 10.0, -1)
    np.savez_compressed(path("vortex2d_512"), U=U, t=t, nsteps=n, form="full")


def wave3d_256():
    g, U = inputs.density_wave_3d(256)
    t, n = run("wave3d_256", g, U, 2, 1e9, 50)
    N = 256
    # f[:, s] from the cells (i, 0, 0), s = i; then every cell must equal f[(i+j+k) % N]
    f = U[:, 0, 0, :].copy()
    s = (np.arange(N)[:, None, None] + np.arange(N)[None, :, None] + np.arange(N)[None, None, :]) % N
    dev_l1, dev_max, norm_l1 = 0.0, 0.0, 0.0
    for k in range(g.nv):
        d = np.abs(U[k] - f[k][s])
        dev_l1 += float(d.sum())
        dev_max = max(dev_max, float(d.max()))
        norm_l1 += float(np.abs(U[k]).sum())
    print(f"wave3d_256: deviation from the function of s: L1 {dev_l1 / norm_l1:.2e} (relative), "
          f"max {dev_max:.2e}", flush=True)
    if not dev_l1 <= 1e-14 * norm_l1:
        raise SystemExit("wave3d_256: the oracle state is not a function of (i + j + k) mod N")
    np.savez_compressed(path("wave3d_256"), f=f, t=t, nsteps=n, dev_l1=dev_l1, dev_max=dev_max, norm_l1=norm_l1,
                        form="function of (i+j+k) mod n")


def vortex3d_256():
    g, U = inputs.isentropic_vortex_3d(256)
    t, n = run("vortex3d_256", g, U, 2, 1e9, 50)
    sl = U[:, 0].copy()
    for k in range(U.shape[1]):
        if not np.array_equal(U[:, k], sl):
            raise SystemExit("vortex3d_256: the oracle state is not uniform in z")
    np.savez_compressed(path("vortex3d_256"), slice=sl, t=t, nsteps=n, form="uniform in z")


CASES = {"vortex2d_512": vortex2d_512, "wave3d_256": wave3d_256, "vortex3d_256": vortex3d_256}

if __name__ == "__main__":
    for name in sys.argv[1:] or list(CASES):
        CASES[name]()
