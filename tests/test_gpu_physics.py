"""The GPU scheme against the physics rather than the oracle: the rotated
shock tube (the paper's one-dimensional Riemann problem of Sec. 4, turned
by 30 degrees on a mixed mesh) against the exact Riemann solution."""
import math

import numpy as np
import pytest

import workloads as wl
import exact_riemann as er
from gpu_helpers import physics_for

pytestmark = pytest.mark.gpu

LEFT, RIGHT = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)


def _sod_error(n, prec, variables, band):
    """L1 density and velocity errors at t = 0.2 over the cells away from
    the box edges (the transmissive faces where the interface meets the
    boundary are not exact for the turned problem), weighted by area."""
    import torch
    import paper_1712_08317_amd as uw
    mesh = wl.mesh_c3(n=n, jitter=0.15, seed=4, band=band)
    W = wl.initial_state("c3", mesh)
    M = uw.Mesh.from_workload(mesh, device=0)
    M.precompute(uw.make_scheme(variables=uw.UW_CHARACTERISTIC if variables == "characteristic"
                                else uw.UW_CONSERVED))
    Wd = torch.from_numpy(M.to_internal(W)).to("cuda:0")
    t = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    ph = physics_for(uw, "euler", prec)
    steps = 0
    while float(t.cpu()[0]) < 0.2 - 1e-12 and steps < 20 * n:
        for _ in range(50):
            M.rk3_step(ph, Wd, t, cfl=0.5, t_end=0.2)
        steps += 50
        M.check()
    assert abs(float(t.cpu()[0]) - 0.2) < 1e-12
    Wh = M.to_original(Wd.cpu().numpy())
    cx, cy = wl.cell_centres(mesh)
    area = wl.signed_areas(mesh.node_xy, mesh.cell_nodes)
    ca, sa = math.cos(math.pi / 6), math.sin(math.pi / 6)
    xi = (cx - 0.5) * ca + (cy - 0.5) * sa
    eta = -(cx - 0.5) * sa + (cy - 0.5) * ca
    keep = (np.abs(eta) < 0.2) & (np.abs(xi) < 0.45)
    rho_x, u_x, _ = er.sample(LEFT, RIGHT, xi / 0.2)
    rho = Wh[0]
    un = (Wh[1] * ca + Wh[2] * sa) / rho
    a = area[keep]
    err_rho = (a * np.abs(rho - rho_x)[keep]).sum() / a.sum()
    err_u = (a * np.abs(un - u_x)[keep]).sum() / a.sum()
    return err_rho, err_u


@pytest.mark.parametrize("variables,band,sizes", [
    ("conserved", 0.0, (200, 400)),         # all quadrilaterals
    ("characteristic", 0.1, (100, 200)),    # triangles within 0.1 of the interface
])
def test_rotated_shock_tube_converges_to_the_exact_solution(variables, band, sizes):
    """FP32 arithmetic: the L1 errors of density and normal velocity are
    small and shrink on refinement (a solution with a shock and a contact
    converges at less than first order in L1).  On mixed meshes with
    conserved variables, and with characteristic variables from h = 1/400,
    the run leaves the admissible set where the interface meets the open
    bottom boundary (a finding of the scheme as read; the oracle gives the
    same negative Gauss-point pressure from the same state), so the mixed
    mesh is run in characteristic variables at h = 1/100 and 1/200."""
    e1 = _sod_error(sizes[0], "fp32", variables, band)
    e2 = _sod_error(sizes[1], "fp32", variables, band)
    print(variables, band, sizes, e1, e2, flush=True)
    assert e1[0] < 0.03 and e1[1] < 0.06
    assert e2[0] < 0.8 * e1[0] and e2[1] < 0.8 * e1[1]
