"""Pins of the oracle's characteristic-variable reconstruction (Sec. 4,
Euler systems): the eigen-decomposition against the flux Jacobian obtained
by complex-step differentiation, Roe's defining property of the mean state,
and the reductions of the characteristic WENO to the linear scheme and to
exact reproduction."""
import numpy as np
import pytest

import workloads as wl
from oracle import weights as ow
from oracle import scheme as osc

GAMMA = 1.4


def _states(rng, n):
    rho = np.exp(rng.uniform(-2, 2, n))
    u, v = rng.normal(0, 2, n), rng.normal(0, 2, n)
    p = np.exp(rng.uniform(-2, 2, n))
    E = p / (GAMMA - 1) + 0.5 * rho * (u * u + v * v)
    return np.stack([rho, rho * u, rho * v, E])


def _normals(rng, n):
    th = rng.uniform(0, 2 * np.pi, n)
    return np.cos(th), np.sin(th)


def _flux(W, nx, ny):
    return osc.physical_flux(W, nx, ny, GAMMA)


def test_eigenvectors_invert_each_other():
    rng = np.random.default_rng(1)
    W = _states(rng, 500)
    nx, ny = _normals(rng, 500)
    u, v, H, c = osc.roe_average(W, W, GAMMA)
    R, Li, _ = osc.eigenvectors(u, v, H, c, nx, ny, GAMMA)
    eye = np.einsum("mij,mjk->mik", Li, R)
    assert np.abs(eye - np.eye(4)).max() < 1e-11


def test_decomposition_is_the_flux_jacobian():
    """R diag(lambda) R^-1 = n_x dF/dW + n_y dG/dW, the Jacobian taken by
    complex-step differentiation of the flux (exact to rounding)."""
    rng = np.random.default_rng(2)
    n = 300
    W = _states(rng, n)
    nx, ny = _normals(rng, n)
    h = 1e-30
    J = np.zeros((n, 4, 4))
    for k in range(4):
        Wc = W.astype(complex)
        Wc[k] += 1j * h
        J[:, :, k] = np.imag(_flux(Wc, nx, ny)).T / h
    u, v, H, c = osc.roe_average(W, W, GAMMA)
    R, Li, lam = osc.eigenvectors(u, v, H, c, nx, ny, GAMMA)
    A = np.einsum("mij,mj,mjk->mik", R, lam, Li)
    scale = np.abs(J).max(axis=(1, 2), keepdims=True)
    assert (np.abs(A - J) / scale).max() < 1e-12


def test_roe_mean_matrix_property():
    """The Roe mean matrix maps the jump of the states onto the jump of the
    normal fluxes exactly."""
    rng = np.random.default_rng(3)
    n = 500
    WL, WR = _states(rng, n), _states(rng, n)
    nx, ny = _normals(rng, n)
    u, v, H, c = osc.roe_average(WL, WR, GAMMA)
    R, Li, lam = osc.eigenvectors(u, v, H, c, nx, ny, GAMMA)
    A = np.einsum("mij,mj,mjk->mik", R, lam, Li)
    lhs = np.einsum("mij,jm->im", A, WR - WL)
    rhs = _flux(WR, nx, ny) - _flux(WL, nx, ny)
    assert np.abs(lhs - rhs).max() < 1e-10 * np.abs(rhs).max()


def _tables(mesh, **kw):
    return ow.precompute(mesh, ow.Scheme(variables="characteristic", **kw))


@pytest.mark.parametrize("kind", ["quad", "tri"])
def test_large_eps_reduces_to_the_linear_scheme(kind):
    mesh = wl.grid_mesh(10, 10, 2.0, 2.0, kind, 0.25, 41, True)
    W = wl.seeded_state(mesh, 4, 42)
    ph = osc.Physics("euler")
    lin = osc.residual_vectorized(ow.precompute(mesh, ow.Scheme(mode="linear")), W, ph)
    ch = osc.residual_vectorized(_tables(mesh, eps=1e30), W, ph)
    assert np.allclose(ch, lin, rtol=1e-9, atol=1e-9 * np.abs(lin).max())


def test_uniform_and_linear_states_are_reproduced():
    mesh = wl.mesh_c5(n=16, block=4, jitter=0.3, seed=43)
    T = _tables(mesh)
    W = np.tile(np.array([[1.3], [0.4], [-0.2], [3.1]]), (1, mesh.n_cells))
    for r in osc.reconstruct_face_states(T, W).values():
        assert np.array_equal(r, np.repeat(W[:, :1], r.shape[1], 1))
    # linear data on an open mixed mesh, away from its boundary: every
    # candidate is exact, so the reconstruction equals the linear scheme's
    # (which reproduces quadratics)
    split = (np.add.outer(np.arange(16) // 4, np.arange(16) // 4) % 2).astype(bool)
    om = wl.grid_mesh(16, 16, 2.0, 2.0, split, 0.3, 47, False)
    lin = wl.cell_averages(om, lambda X, Y: np.stack(
        [1 + 0.1 * X + 0.05 * Y, 0.2 + 0.03 * X, -0.1 + 0.02 * Y, 3.0 + 0.1 * X - 0.1 * Y]), 4)
    a = osc.reconstruct_face_states(_tables(om), lin)
    b = osc.reconstruct_face_states(ow.precompute(om, ow.Scheme(mode="linear")), lin)
    cn = om.cell_nodes
    xy = (np.where((cn >= 0)[:, :, None], om.node_xy[np.maximum(cn, 0)], 0.0).sum(1)
          / np.where(cn[:, 3] < 0, 3, 4)[:, None])
    inner = np.flatnonzero((xy.min(1) > 3 * om.h) & (xy.max(1) < 2 - 3 * om.h))
    assert inner.size > 50
    for c in inner:
        assert np.abs(a[c] - b[c]).max() < 1e-12


def test_entropy_wave_is_reconstructed_as_one_field():
    """A density wave at constant velocity and pressure varies along the
    entropy eigenvector only, so its characteristic reconstruction is the
    scalar WENO reconstruction of the density carried along that vector:
    velocity and pressure stay exactly uniform at every Gauss point.  The
    conserved-variable reconstruction weights each component separately and
    does not keep them uniform."""
    mesh = wl.mesh_c5(n=16, block=4, jitter=0.3, seed=46)
    rho = wl.initial_state("c2q", mesh)[0]     # 1 + 0.2 sin(pi(x+y))
    u, v, p0 = 0.5, -2.0, 1.0                  # unequal components: distinct indicators
    W = np.stack([rho, u * rho, v * rho, p0 / (GAMMA - 1) + 0.5 * (u * u + v * v) * rho])
    ch = osc.reconstruct_face_states(_tables(mesh), W)
    co = osc.reconstruct_face_states(ow.precompute(mesh), W)
    worst_ch = worst_co = 0.0
    for c in ch:
        for R, which in ((ch[c], "ch"), (co[c], "co")):
            rho, mu, mv, E = R
            p = (GAMMA - 1) * (E - 0.5 * (mu * mu + mv * mv) / rho)
            dev = max(np.abs(mu / rho - u).max(), np.abs(mv / rho - v).max(),
                      np.abs(p - p0).max())
            if which == "ch":
                worst_ch = max(worst_ch, dev)
            else:
                worst_co = max(worst_co, dev)
        # the density itself is the scalar reconstruction (component 0 of
        # the conserved path sees the same increments and indicators)
        assert np.abs(ch[c][0] - co[c][0]).max() < 1e-12
    assert worst_ch < 1e-12
    assert worst_co > 1e-8
