"""Pins of the oracle's per-stage operator (paper Sec. 2, 3.4, 4)."""
import numpy as np
import pytest

import workloads as wl
from oracle import weights as ow
from oracle import scheme as osc

EULER = osc.Physics("euler")
ADV = osc.Physics("advection", 1.0, 1.0)


@pytest.fixture(scope="module")
def tri_tables():
    mesh = wl.grid_mesh(10, 10, 2.0, 2.0, "tri", 0.3, 41, True)
    return mesh, ow.precompute(mesh)


@pytest.fixture(scope="module")
def mixed_tables():
    mesh = wl.mesh_c5(n=12, block=3, jitter=0.3, seed=42)
    return mesh, ow.precompute(mesh)


def test_large_eps_equals_linear_mode(tri_tables):
    mesh, _ = tri_tables
    W = wl.seeded_state(mesh, 4, 1)
    Tw = ow.precompute(mesh, ow.Scheme(eps=1e30))
    Tl = ow.precompute(mesh, ow.Scheme(mode="linear"))
    Rw = osc.reconstruct_face_states(Tw, W)
    Rl = osc.reconstruct_face_states(Tl, W)
    for c in Rw:
        # equal up to the consistency residual of B gamma = eta
        np.testing.assert_allclose(Rw[c], Rl[c], rtol=1e-10, atol=1e-12)


def test_uniform_state_is_reconstructed_exactly(mixed_tables):
    mesh, T = mixed_tables
    W = np.tile(np.array([[1.3], [0.2], [-0.7], [4.1]]), (1, mesh.n_cells))
    R = osc.reconstruct_face_states(T, W)
    for c, r in R.items():
        assert (r == W[:, :1]).all()
    L = osc.residual_vectorized(T, W, EULER)
    assert np.abs(L).max() < 1e-12


def test_linear_data_is_reconstructed_exactly(mixed_tables):
    """Every candidate reproduces linear functions, so R(x_G) is exact for
    any nonlinear weights (the split sum sigma^+ - sigma^- = sum gamma = 1)."""
    mesh, T = mixed_tables
    # a linear field is not periodic: use one interior cell away from the seam
    lin = lambda x, y: 0.3 + 1.7 * x - 0.9 * y  # noqa: E731
    Wavg = wl.cell_averages(mesh, lambda x, y: lin(x, y)[None], 1, q=3)
    cells = [i for i in range(mesh.n_cells)
             if 0.6 < mesh.node_xy[mesh.cell_nodes[i, 0], 0] < 1.4
             and 0.6 < mesh.node_xy[mesh.cell_nodes[i, 0], 1] < 1.4][:20]
    R = osc.reconstruct_face_states(T, Wavg, cells)
    for c in cells:
        P = mesh.node_xy[[v for v in mesh.cell_nodes[c] if v >= 0]]
        n = len(P)
        for k in range(n):
            a, b = P[k], P[(k + 1) % n]
            ga, gb = (3 + 3 ** .5) / 6, (3 - 3 ** .5) / 6
            for q, (wa, wb) in enumerate(((ga, gb), (gb, ga))):
                x = wa * a + wb * b
                assert abs(R[c][0, 2 * k + q] - lin(*x)) < 1e-9


def test_hllc_consistency_and_upwinding():
    rng = np.random.Generator(np.random.PCG64(9))
    for _ in range(50):
        rho, p = rng.uniform(0.2, 2, 2)
        u, v = rng.uniform(-2, 2, 2)
        W = wl.primitive_to_conserved(rho, u, v, p)
        th = rng.uniform(0, 2 * np.pi)
        nx, ny = np.cos(th), np.sin(th)
        np.testing.assert_allclose(osc.hllc_flux(W, W, nx, ny, 1.4),
                                   osc.physical_flux(W, nx, ny, 1.4), rtol=1e-13, atol=1e-13)
    # supersonic to the right: pure upwind (left) flux
    WL = wl.primitive_to_conserved(1.0, 3.0, 0.2, 1.0)
    WR = wl.primitive_to_conserved(0.5, 2.5, -0.1, 0.7)
    np.testing.assert_allclose(osc.hllc_flux(WL, WR, 1.0, 0.0, 1.4), osc.physical_flux(WL, 1.0, 0.0, 1.4))
    WL = wl.primitive_to_conserved(1.0, -3.0, 0.2, 1.0)
    WR = wl.primitive_to_conserved(0.5, -3.5, -0.1, 0.7)
    np.testing.assert_allclose(osc.hllc_flux(WL, WR, 1.0, 0.0, 1.4), osc.physical_flux(WR, 1.0, 0.0, 1.4))


def test_hllc_preserves_stationary_contact_and_rotates():
    WL = wl.primitive_to_conserved(1.0, 0.0, 0.3, 1.0)
    WR = wl.primitive_to_conserved(0.1, 0.0, -0.4, 1.0)
    F = osc.hllc_flux(WL, WR, 1.0, 0.0, 1.4)
    np.testing.assert_allclose(F, [0.0, 1.0, 0.0, 0.0], atol=1e-15)
    # rotating the states and the normal together rotates the flux
    rng = np.random.Generator(np.random.PCG64(10))
    WL = wl.primitive_to_conserved(1.1, 0.4, -0.3, 0.9)
    WR = wl.primitive_to_conserved(0.7, -0.2, 0.5, 0.6)
    F0 = osc.hllc_flux(WL, WR, 1.0, 0.0, 1.4)
    for _ in range(10):
        th = rng.uniform(0, 2 * np.pi)
        c, s = np.cos(th), np.sin(th)

        def rot(Wv):
            return np.array([Wv[0], c * Wv[1] - s * Wv[2], s * Wv[1] + c * Wv[2], Wv[3]])
        F = osc.hllc_flux(rot(WL), rot(WR), c, s, 1.4)
        np.testing.assert_allclose(F, rot(F0), rtol=1e-13, atol=1e-13)


def test_scalar_upwind():
    assert osc.upwind_flux(2.0, 3.0, 1.0, 0.0, 1.0, 1.0) == 2.0
    assert osc.upwind_flux(2.0, 3.0, -1.0, 0.0, 1.0, 1.0) == -3.0


@pytest.mark.parametrize("which", ["tri", "mixed"])
def test_conservation_on_periodic_mesh(which, tri_tables, mixed_tables):
    mesh, T = tri_tables if which == "tri" else mixed_tables
    W = wl.seeded_state(mesh, 4, 3)
    L = osc.residual_vectorized(T, W, EULER)
    area = np.zeros(mesh.n_cells)
    for g in T.groups.values():
        area[g.st.cells] = g.area
    tot = (L * area[None]).sum(axis=1)
    scale = np.abs(L * area[None]).sum(axis=1)
    assert (np.abs(tot) < 1e-13 * scale).all()


def test_loop_and_vectorised_residuals_agree(mixed_tables):
    mesh, T = mixed_tables
    W = wl.seeded_state(mesh, 4, 4)
    Lv = osc.residual_vectorized(T, W, EULER)
    cells = np.arange(0, mesh.n_cells, 7)
    Ll = osc.residual(T, W, EULER, cells)
    np.testing.assert_allclose(Ll, Lv[:, cells], rtol=1e-13, atol=1e-13)


def test_rk3_stability_polynomial():
    """Sec. 4: for L(W) = lambda W one step multiplies by 1 + z + z^2/2 + z^3/6,
    z = lambda dt (a complex lambda is written as a real 2x2 rotation-scaling)."""
    lam = -0.7 + 0.3j
    dt = 0.4
    Wc = 1.0 + 0.5j
    Mat = np.array([[lam.real, -lam.imag], [lam.imag, lam.real]])
    W = np.array([[Wc.real], [Wc.imag]])
    out = osc.rk3_step(None, W, None, dt, resid=lambda X: Mat @ X)
    z = lam * dt
    ref = Wc * (1 + z + z * z / 2 + z ** 3 / 6)
    np.testing.assert_allclose(out[:, 0], [ref.real, ref.imag], rtol=1e-15, atol=1e-15)


def test_rk3_stage_times_integrate_cubics_exactly():
    """The stages of a step from t sit at t, t + dt and t + dt/2 with
    effective weights 1/6, 1/6 and 2/3: for a right-hand side that depends on
    time only, a step is Simpson's rule, exact for cubics.  Other stage
    times (say t + dt for the third stage) miss y' = 4 t^3 by O(dt^3)."""
    t0, dt = 0.3, 0.2
    out = osc.rk3_step(None, np.array([[2.0]]), None, dt,
                       resid_t=lambda X, tt: np.full_like(X, 4.0 * tt ** 3), t=t0)
    assert abs(out[0, 0] - (2.0 + (t0 + dt) ** 4 - t0 ** 4)) < 1e-15
    quad = osc.rk3_step(None, np.array([[0.0]]), None, dt,
                        resid_t=lambda X, tt: np.full_like(X, 3.0 * tt ** 2), t=t0)
    assert abs(quad[0, 0] - ((t0 + dt) ** 3 - t0 ** 3)) < 1e-15


def test_cfl_on_uniform_squares():
    mesh = wl.grid_mesh(8, 8, 2.0, 2.0, "quad", 0.0, 1, True)
    T = ow.precompute(mesh)
    W = np.ones((1, mesh.n_cells))
    h = 0.25
    assert abs(osc.cfl_dt(T, W, ADV, 0.5) - 0.5 * h / 2) < 1e-15


def test_density_wave_keeps_velocity_and_pressure_uniform():
    mesh = wl.grid_mesh(10, 10, 2.0, 2.0, "quad", 0.2, 44, True)
    T = ow.precompute(mesh)
    W = wl.initial_state("c2q", mesh, q=3)
    for _ in range(3):
        W = osc.rk3_step(T, W, EULER, 0.05)
    u = W[1] / W[0]
    v = W[2] / W[0]
    p = 0.4 * (W[3] - 0.5 * W[0] * (u * u + v * v))
    assert np.abs(u - 1).max() < 1e-13 and np.abs(v - 1).max() < 1e-13
    assert np.abs(p - 1).max() < 1e-13


def test_smooth_advection_converges_at_third_order():
    """Accuracy section: third order on smooth data (scalar advection on
    jittered triangles, the linear scheme and WENO)."""
    for mode in ("linear", "weno"):
        errs = []
        for n in (10, 20, 40):
            mesh = wl.grid_mesh(n, n, 2.0, 2.0, "tri", 0.1, 1, True)
            T = ow.precompute(mesh, ow.Scheme(mode=mode))
            W = wl.cell_averages(mesh, wl.density_wave_scalar(0.0), 1, q=5)
            t, tend, dt = 0.0, 0.5, 0.15 * 2 / n
            while t < tend - 1e-12:
                d = min(dt, tend - t)
                W = osc.rk3_step(T, W, ADV, d)
                t += d
            ex = wl.cell_averages(mesh, wl.density_wave_scalar(tend), 1, q=5)
            A = np.zeros(mesh.n_cells)
            A[T.groups[3].st.cells] = T.groups[3].area
            errs.append((A * np.abs(W - ex)[0]).sum() / A.sum())
        order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
        if mode == "linear":
            assert (order > 2.7).all(), (mode, errs, order)
        else:
            assert order[-1] > 2.8, (mode, errs, order)
