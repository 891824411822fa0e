"""The oracle against numbers the paper prints: its accuracy tests on
regular quadrilateral meshes (Sec. 4.1), the density wave (Table
tab-accuracy1) and the isentropic vortex (Table tab-accuracy3), stored in
tests/golden/paper_accuracy_*.txt.  On uniform squares the mesh is fully
determined, so the scheme as read must give the paper's errors up to what
the paper leaves unstated (how it evaluates the exact solution; here cell
averages): the density wave within 2% at h = 1/8 and 1/16, the vortex, with
the characteristic variables the paper allows for the Euler equations,
within 5% at h = 1/4.  What the paper does not give is fixed by them: eps
= 1e-3 reproduces the density-wave table and eps = 1e-6 misses it by more
than 20%; the vortex table is a characteristic-variable result (the
conserved variables miss it by more than 25%)."""
import os

import numpy as np
import pytest

import workloads as wl
from oracle import weights as ow
from oracle import scheme as osc

HERE = os.path.join(os.path.dirname(__file__), "golden")
GOLD = os.path.join(HERE, "paper_accuracy_regular_quads.txt")
GOLD_VORTEX = os.path.join(HERE, "paper_accuracy_vortex_regular_quads.txt")


def paper_rows(path=GOLD, side=2.0):
    return {round(side / h): (l1, linf) for h, l1, linf in np.loadtxt(path, comments="#")}


def density_wave_errors(n, eps=1e-3):
    """L1 (integral over the domain) and Linf of the density at t = 2 on
    n x n uniform squares of [0,2]^2, dt = 0.3 h, against the exact cell
    averages."""
    mesh = wl.grid_mesh(n, n, 2.0, 2.0, "quad", 0.0, 1, True, name=f"acc{n}")
    W = wl.cell_averages(mesh, wl.density_wave_euler(0.0), 4, q=4)
    T = ow.precompute(mesh, ow.Scheme(eps=eps))
    ph = osc.Physics("euler")
    steps = int(round(2.0 / (0.3 * 2.0 / n)))
    dt = 2.0 / steps
    for _ in range(steps):
        W = osc.rk3_step(T, W, ph, dt)
    ex = wl.cell_averages(mesh, wl.density_wave_euler(2.0), 4, q=4)[0]
    area = wl.signed_areas(mesh.node_xy, mesh.cell_nodes)
    e = np.abs(W[0] - ex)
    return float((area * e).sum()), float(e.max())


@pytest.mark.parametrize("n", [16, 32])
def test_density_wave_errors_match_the_paper_table(n):
    l1, linf = density_wave_errors(n)
    p_l1, p_linf = paper_rows()[n]
    print(n, l1, linf, p_l1, p_linf)
    assert abs(l1 / p_l1 - 1) < 0.02 and abs(linf / p_linf - 1) < 0.02


def test_the_table_fixes_eps_at_the_size_read_here():
    l1, linf = density_wave_errors(16, eps=1e-6)
    p_l1, p_linf = paper_rows()[16]
    assert l1 > 1.15 * p_l1 and linf > 1.15 * p_linf


def vortex_errors(n, variables):
    """As density_wave_errors for the isentropic vortex on n x n uniform
    squares of [0,10]^2."""
    mesh = wl.grid_mesh(n, n, 10.0, 10.0, "quad", 0.0, 1, True, name=f"vortex{n}")
    W = wl.cell_averages(mesh, wl.isentropic_vortex(0.0), 4, q=4)
    T = ow.precompute(mesh, ow.Scheme(variables=variables))
    ph = osc.Physics("euler")
    steps = int(round(2.0 / (0.3 * 10.0 / n)))
    dt = 2.0 / steps
    for _ in range(steps):
        W = osc.rk3_step(T, W, ph, dt)
    ex = wl.cell_averages(mesh, wl.isentropic_vortex(2.0), 4, q=4)[0]
    area = wl.signed_areas(mesh.node_xy, mesh.cell_nodes)
    e = np.abs(W[0] - ex)
    return float((area * e).sum()), float(e.max())


def test_vortex_errors_match_the_paper_table_with_characteristic_variables():
    p_l1, p_linf = paper_rows(GOLD_VORTEX, 10.0)[40]
    l1, linf = vortex_errors(40, "characteristic")
    print(l1, linf, p_l1, p_linf)
    assert abs(l1 / p_l1 - 1) < 0.05 and abs(linf / p_linf - 1) < 0.05
    l1c, linfc = vortex_errors(40, "conserved")
    assert l1c > 1.25 * p_l1 and linfc > 1.25 * p_linf
