"""Writes the oracle's solutions of the paper's one-dimensional Riemann
problems (Sec. 4.2: Sod to t = 0.2, Lax to t = 0.16 on [0,1] x [0,0.5],
h = 1/100, open boundaries) along the centre line, one text file per case:

    python tests/golden/make_riemann_1d.py [case ...]

Calls only the oracle (FP64 NumPy, SSP-RK3 at CFL 0.5 with the oracle's
time-step rule) and the input generator; minutes per case."""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import scheme as osc  # noqa: E402
from oracle import weights as ow  # noqa: E402

# name: (problem, split, jitter)
CASES = {
    "sod_quad": ("sod", "quad", 0.0),
    "sod_quad_irregular": ("sod", "quad", 0.2),
    "sod_tri": ("sod", "tri", 0.0),
    "lax_quad": ("lax", "quad", 0.0),
    "lax_quad_irregular": ("lax", "quad", 0.2),
    "lax_tri": ("lax", "tri", 0.0),
}
# Not stored: Sod and Lax on 20%-jittered triangles, where the scheme as read
# reaches a Gauss-point state with negative pressure next to the open
# boundary (Sod at t = 0.015, Lax at t = 0.011).
BAND = 0.011      # cells whose vertex average lies within this of y = 0.25
CFL = 0.5


def centre_line(mesh):
    cx, cy = wl.cell_centres(mesh)
    return np.flatnonzero(np.abs(cy - 0.25) < BAND)


def run(name):
    problem, split, jitter = CASES[name]
    mesh, W, t_end = wl.riemann_1d(problem, 100, split, jitter)
    T = ow.precompute(mesh)
    ph = osc.Physics("euler")
    t, steps, t0 = 0.0, 0, time.time()
    while t < t_end - 1e-12:
        dt = min(osc.cfl_dt(T, W, ph, CFL), t_end - t)
        W = osc.rk3_step(T, W, ph, dt, t=t)
        t += dt
        steps += 1
    if not np.isfinite(W).all():
        raise RuntimeError(f"{name}: non-finite state")
    idx = centre_line(mesh)
    cx, cy = wl.cell_centres(mesh)
    rho = W[0, idx]
    u = W[1, idx] / rho
    v = W[2, idx] / rho
    p = (wl.GAMMA - 1.0) * (W[3, idx] - 0.5 * rho * (u * u + v * v))
    path = os.path.join(HERE, f"riemann_1d_{name}.txt")
    with open(path, "w") as f:
        f.write(f"# Oracle solution of the {problem} problem (Sec. 4.2) at t = {t_end}: "
                f"workloads.riemann_1d({problem!r}, 100, {split!r}, {jitter}), "
                f"{mesh.n_cells} cells, SSP-RK3 at CFL {CFL}, {steps} steps.\n")
        f.write("# Written by tests/golden/make_riemann_1d.py (oracle only).\n")
        f.write(f"# steps {steps}\n")
        f.write("# columns: cell x y rho u p  (cells whose vertex average is within "
                f"{BAND} of y = 0.25)\n")
        for k, i in enumerate(idx):
            f.write(f"{i} {cx[i]:.17g} {cy[i]:.17g} {rho[k]:.17g} {u[k]:.17g} {p[k]:.17g}\n")
    print(f"{name}: {steps} steps, {len(idx)} cells on the line, {time.time() - t0:.0f} s",
          flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or list(CASES):
        run(name)
