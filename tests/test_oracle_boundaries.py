"""Pins of the oracle's boundary faces (the conditions the paper's tests
name: non-reflecting, reflective walls, prescribed states): the wall flux
carries pressure only, a closed box conserves mass and energy exactly and
keeps gas at rest at rest, a face with supersonic inflow on both sides
passes exactly the prescribed state's flux, and a domain filled with the
inflow state is steady."""
import numpy as np
import pytest

import workloads as wl
from oracle import weights as ow
from oracle import scheme as osc

GAMMA = 1.4


def _prim(rho, u, v, p):
    return np.array([rho, rho * u, rho * v, p / (GAMMA - 1) + 0.5 * rho * (u * u + v * v)])


def test_wall_flux_carries_pressure_only():
    rng = np.random.default_rng(1)
    n = 400
    W = _prim(np.exp(rng.uniform(-1, 1, n)), rng.normal(0, 1, n), rng.normal(0, 1, n),
              np.exp(rng.uniform(-1, 1, n)))
    th = rng.uniform(0, 2 * np.pi, n)
    nx, ny = np.cos(th), np.sin(th)
    G = osc.ghost_state(W, np.full(n, osc.BC_REFLECTIVE), nx, ny)
    # the ghost mirrors the normal velocity and keeps the rest
    assert np.allclose(G[0], W[0]) and np.allclose(G[3], W[3])
    assert np.allclose(G[1] * nx + G[2] * ny, -(W[1] * nx + W[2] * ny))
    assert np.allclose(-G[1] * ny + G[2] * nx, -W[1] * ny + W[2] * nx)
    F = osc.hllc_flux(W, G, nx, ny, GAMMA)
    scale = np.abs(F).max()
    assert np.abs(F[0]).max() < 1e-12 * scale                         # no mass through a wall
    assert np.abs(F[3]).max() < 1e-12 * scale                         # no energy
    assert np.abs(-F[1] * ny + F[2] * nx).max() < 1e-12 * scale       # no tangential momentum
    # the normal momentum flux: with Davis speeds S_L = -|u_n| - c and S* = 0,
    # p* = p + rho u_n (u_n + |u_n| + c)
    rho = W[0]
    un = (W[1] * nx + W[2] * ny) / rho
    p = (GAMMA - 1) * (W[3] - 0.5 * (W[1] ** 2 + W[2] ** 2) / rho)
    c = np.sqrt(GAMMA * p / rho)
    pstar = p + rho * un * (un + np.abs(un) + c)
    assert np.abs(F[1] * nx + F[2] * ny - pstar).max() < 1e-12 * scale


def _box(kind, n=12, jitter=0.25, seed=3):
    """Open square of quads and triangles with every boundary face of one kind."""
    split = (np.add.outer(np.arange(n) // 3, np.arange(n) // 3) % 2).astype(bool)
    mesh = wl.grid_mesh(n, n, 1.0, 1.0, split, jitter, seed, False, name=f"box-{kind}")
    mesh.face_bc = np.full((mesh.n_cells, 4), kind, dtype=np.int32)
    return mesh


def _areas(T, n):
    a = np.zeros(n)
    for g in T.groups.values():
        a[g.st.cells] = g.area
    return a


@pytest.mark.parametrize("variables", ["conserved", "characteristic"])
def test_closed_box_conserves_mass_and_energy(variables):
    mesh = _box(wl.BC_REFLECTIVE)
    T = ow.precompute(mesh, ow.Scheme(variables=variables))
    W = wl.seeded_state(mesh, 4, 5)
    L = osc.residual_vectorized(T, W, osc.Physics("euler"))
    area = _areas(T, mesh.n_cells)
    tot = (L * area).sum(axis=1)
    mag = np.abs(L * area).sum(axis=1)
    assert abs(tot[0]) < 1e-12 * mag[0] and abs(tot[3]) < 1e-12 * mag[3]
    # the loop form agrees
    Ll = osc.residual(T, W, osc.Physics("euler"))
    assert np.abs(Ll - L).max() < 1e-12 * np.abs(L).max()
    # with open faces instead, mass does leave or enter
    T2 = ow.precompute(_box(wl.BC_TRANSMISSIVE), ow.Scheme(variables=variables))
    L2 = osc.residual_vectorized(T2, W, osc.Physics("euler"))
    assert abs((L2 * area).sum(axis=1)[0]) > 1e-6 * np.abs(L2 * area).sum(axis=1)[0]


def test_gas_at_rest_in_a_closed_box_stays_at_rest():
    mesh = _box(wl.BC_REFLECTIVE)
    T = ow.precompute(mesh)
    W = np.tile(_prim(1.3, 0.0, 0.0, 2.0)[:, None], (1, mesh.n_cells))
    L = osc.residual_vectorized(T, W, osc.Physics("euler"))
    assert np.abs(L).max() < 1e-11


def test_inflow_state_filling_the_domain_is_steady_and_supersonic_inflow_is_exact():
    W_in = _prim(1.0, 3.0, 0.5, 1.0)           # Mach about 2.7
    mesh = _box(wl.BC_INFLOW)
    mesh.inflow = W_in[None, :]
    T = ow.precompute(mesh)
    W = np.tile(W_in[:, None], (1, mesh.n_cells))
    L = osc.residual_vectorized(T, W, osc.Physics("euler"))
    assert np.abs(L).max() < 1e-10
    # a face through which the flow enters supersonically on both sides (every
    # wave speed points inward) passes exactly the prescribed state's flux
    rng = np.random.default_rng(2)
    inside = _prim(np.exp(rng.uniform(-0.5, 0.5, 50)), rng.uniform(2.5, 4.0, 50),
                   rng.normal(0, 0.3, 50), np.exp(rng.uniform(-1.0, 0.0, 50)))
    nx, ny = -np.ones(50), np.zeros(50)      # outward normal of a left boundary face
    G = osc.ghost_state(inside, np.full(50, wl.BC_INFLOW), nx, ny, mesh.inflow)
    F = osc.hllc_flux(inside, G, nx, ny, GAMMA)
    Fin = osc.physical_flux(np.repeat(W_in[:, None], 50, 1), nx, ny, GAMMA)
    assert np.abs(F - Fin).max() < 1e-12 * np.abs(Fin).max()


def test_mixed_kinds_on_one_mesh():
    """Walls top and bottom, inflow left, open right: the per-face kinds are
    read per face (a state with no normal velocity on the walls and the
    inflow state everywhere is steady)."""
    n = 10
    mesh = wl.grid_mesh(2 * n, n, 2.0, 1.0, "tri", 0.2, 9, False, name="channel")
    cn = mesh.cell_nodes
    kinds = np.zeros((mesh.n_cells, 4), np.int32)
    xy = mesh.node_xy
    for c in range(mesh.n_cells):
        nf = 3 if cn[c, 3] < 0 else 4
        for k in range(nf):
            a, b = xy[cn[c, k]], xy[cn[c, (k + 1) % nf]]
            if abs(a[1] - b[1]) < 1e-12 and a[1] in (0.0, 1.0):
                kinds[c, k] = wl.BC_REFLECTIVE
            elif abs(a[0] - b[0]) < 1e-12 and a[0] == 0.0:
                kinds[c, k] = wl.BC_INFLOW
            else:
                kinds[c, k] = wl.BC_TRANSMISSIVE
    mesh.face_bc = kinds
    W_in = _prim(1.0, 2.0, 0.0, 1.0)
    mesh.inflow = W_in[None, :]
    T = ow.precompute(mesh)
    W = np.tile(W_in[:, None], (1, mesh.n_cells))
    assert np.abs(osc.residual_vectorized(T, W, osc.Physics("euler"))).max() < 1e-10
    # with vertical velocity the walls act: not steady any more
    W2 = np.tile(_prim(1.0, 2.0, 0.5, 1.0)[:, None], (1, mesh.n_cells))
    assert np.abs(osc.residual_vectorized(T, W2, osc.Physics("euler"))).max() > 1e-3
