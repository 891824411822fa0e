"""The seeded input generators against what they stand for: the cell counts
of the named configurations, the batch's size distribution, and the initial
data of the paper's test problems (Sec. 4) checked against the physics they
state (exact transport, isentropy, Rankine-Hugoniot jumps) rather than
against their own formulas."""
import math

import numpy as np

import workloads as wl

G = wl.GAMMA


def _primitive(U):
    rho = U[0]
    u, v = U[1] / rho, U[2] / rho
    p = (G - 1.0) * (U[3] - 0.5 * rho * (u * u + v * v))
    return rho, u, v, p


def _counts(mesh):
    tri = int((mesh.cell_nodes[:, 3] < 0).sum())
    return mesh.n_cells - tri, tri


def test_configuration_cell_counts():
    assert _counts(wl.mesh_c1()) == (0, 800)
    assert _counts(wl.mesh_c2t()) == (0, 160178)
    q, t = _counts(wl.mesh_c5(n=128, block=64))   # 2 x 2 blocks, checkerboard
    assert (q, t) == (2 * 64 * 64, 2 * 2 * 64 * 64)


def test_c3_band_splits_the_expected_share():
    """Squares whose centre lies within 0.05 of the interface (a line through
    the centre at 30 degrees, 1/cos 30 long inside the unit square) are
    split: 2 x 0.05 / cos 30 = 11.5% of them, which at h = 1/1340 gives the
    1.59M quadrilaterals and 0.41M triangles of the configuration."""
    n = 200
    q, t = _counts(wl.mesh_c3(n=n))
    share = 2 * 0.05 / math.cos(math.pi / 6)
    assert abs(t / 2 / n ** 2 - share) < 0.01
    assert q + t // 2 == n * n
    assert abs((1 - share) * 1340 ** 2 - 1.59e6) < 0.01e6
    assert abs(2 * share * 1340 ** 2 - 0.41e6) < 0.01e6


def test_batch_sizes_are_log_uniform_with_the_stated_mean():
    inst = wl.c4_instances()
    assert len(inst) == 256
    cells = np.array([n * n * (2 if kind == "tri" else 1) for kind, n, _, _ in inst], float)
    # rounding n to an integer moves a size by at most about 2 sqrt(N)
    assert cells.min() >= 2e3 - 2 * math.sqrt(2e3) * 2 and cells.max() <= 2e5 + 2 * math.sqrt(2e5) * 2
    # E[N] of a log-uniform N on [a, b] is (b - a) / ln(b / a): 11.0M for 256
    mean = (2e5 - 2e3) / math.log(100.0)
    assert abs(cells.sum() - 256 * mean) < 0.15 * 256 * mean
    # ln N uniform: mean (ln a + ln b) / 2, standard deviation ln(b/a) / sqrt(12)
    ln = np.log(cells)
    assert abs(ln.mean() - 0.5 * (math.log(2e3) + math.log(2e5))) < 4 * math.log(100) / math.sqrt(12 * 256)
    assert 96 <= sum(k == "tri" for k, _, _, _ in inst) <= 160
    assert all(0.0 <= a <= 0.3 for _, _, a, _ in inst)
    again = wl.c4_instances()
    assert [(k, n, a) for k, n, a, _ in again] == [(k, n, a) for k, n, a, _ in inst]


def test_density_wave_is_transported_exactly():
    """With u = v = p = 1 the Euler equations reduce to transport of the
    density with velocity (1, 1)."""
    rng = np.random.Generator(np.random.PCG64(3))
    x, y = rng.uniform(0, 2, 50), rng.uniform(0, 2, 50)
    t = 0.37
    rho_t, u, v, p = _primitive(wl.density_wave_euler(t)(x, y))
    rho_0 = _primitive(wl.density_wave_euler(0.0)(x - t, y - t))[0]
    assert np.allclose(rho_t, rho_0, rtol=0, atol=1e-14)
    assert np.allclose(u, 1) and np.allclose(v, 1) and np.allclose(p, 1)


def test_vortex_is_isentropic_tangential_and_decays():
    """The vortex factor keeps p / rho^gamma equal to that of the density wave
    alone, its velocity is tangential about the centre, and far from the
    centre the state is the wave with u = v = p = 1."""
    rng = np.random.Generator(np.random.PCG64(4))
    x, y = rng.uniform(0.6, 1.4, 200), rng.uniform(0.6, 1.4, 200)
    rho, u, v, p = _primitive(wl.wave_vortex_euler()(x, y))
    w = 1.0 + 0.2 * np.sin(np.pi * (x + y))
    assert np.allclose(p / rho ** G * w ** G, 1.0, rtol=1e-12)
    assert np.allclose((u - 1.0) * (x - 1.0) + (v - 1.0) * (y - 1.0), 0.0, atol=1e-13)
    assert (p < 1.0).all()                      # pressure drops towards the core
    xf, yf = np.array([0.0, 2.0, 0.0]), np.array([0.0, 0.0, 2.0])
    rf, uf, vf, pf = _primitive(wl.wave_vortex_euler()(xf, yf))
    assert np.allclose(uf, 1, atol=1e-9) and np.allclose(vf, 1, atol=1e-9)
    assert np.allclose(pf, 1, atol=1e-9)


def test_shock_tube_states():
    f = wl.rotated_sod()
    n = np.array([math.cos(math.pi / 6), math.sin(math.pi / 6)])
    a = np.array([0.5, 0.5]) - 0.1 * n
    b = np.array([0.5, 0.5]) + 0.1 * n
    assert np.allclose(_primitive(f(np.array([a[0]]), np.array([a[1]]))), [[1], [0], [0], [1]])
    assert np.allclose(_primitive(f(np.array([b[0]]), np.array([b[1]]))),
                       [[0.125], [0], [0], [0.1]])


def test_lax_states():
    mesh = wl.grid_mesh(20, 4, 1.0, 0.2, "quad", 0.0, 1, False)
    rho, u, v, p = _primitive(wl.lax_state(mesh))
    cx, _ = wl.cell_centres(mesh)
    left = cx < 0.5
    assert np.allclose(rho[left], 0.445) and np.allclose(u[left], 0.698)
    assert np.allclose(p[left], 3.528)
    assert np.allclose(rho[~left], 0.5) and np.allclose(u[~left], 0.0)
    assert np.allclose(p[~left], 0.571)


def _rh_downstream(mach, rho1, p1):
    """Post-shock (rho, p) and the jump of the normal velocity across a
    shock of Mach number `mach` into (rho1, p1), from the Rankine-Hugoniot
    relations written as mass, momentum and energy balances solved for the
    density ratio numerically (independent of the closed forms)."""
    c1 = math.sqrt(G * p1 / rho1)
    w1 = mach * c1                              # inflow speed in the shock frame
    m = rho1 * w1
    P = p1 + m * w1
    H = G / (G - 1) * p1 / rho1 + 0.5 * w1 ** 2

    def energy_residual(r):
        w2 = m / r
        p2 = P - m * w2
        return G / (G - 1) * p2 / r + 0.5 * w2 ** 2 - H

    lo, hi = rho1 * 1.0000001, rho1 * (G + 1) / (G - 1)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if energy_residual(lo) * energy_residual(mid) <= 0:
            hi = mid
        else:
            lo = mid
    r2 = 0.5 * (lo + hi)
    w2 = m / r2
    return r2, P - m * w2, w1 - w2


def test_shu_osher_left_state_is_behind_a_mach_3_shock():
    """The paper's left state (3.857134, 2.629369, 10.33333) is the state
    behind a Mach 3 shock running into (1, 0, 1): velocity and pressure to
    the printed digits; the printed density differs from the jump's 27/7 =
    3.857143 by 2.3e-6 (two digits in swapped order), and the generator keeps
    the printed value."""
    mesh, U = wl.shu_osher(nx=40, ny=2, jitter=0.0)
    rho, u, v, p = _primitive(U)
    cx, _ = wl.cell_centres(mesh)
    left = cx < 0.9
    r2, p2, du = _rh_downstream(3.0, 1.0, 1.0)
    assert abs(r2 - 27.0 / 7.0) < 1e-9
    assert np.allclose(rho[left], 3.857134, rtol=1e-12)
    assert np.allclose(rho[left], r2, rtol=3e-6)
    assert np.allclose(p[left], p2, rtol=1e-6)
    assert np.allclose(u[left], du, rtol=1e-6)
    right = cx > 1.1
    assert np.allclose(u[right], 0.0) and np.allclose(p[right], 1.0)
    assert np.allclose(mesh.inflow[0], U[:, np.argmin(cx)], rtol=1e-12)


def test_shock_vortex_shock_satisfies_rankine_hugoniot():
    """Upstream (Ma^2, sqrt(gamma), 0, 1) is Mach 1.1; the downstream state
    carries the same mass, momentum and energy fluxes (a stationary shock)."""
    mesh, U = wl.shock_vortex(n=40, jitter=0.0)
    rho, u, v, p = _primitive(U)
    cx, cy = wl.cell_centres(mesh)
    # the vortex decays as exp(mu (1 - (r/rc)^2)), mu = 0.204, rc = 0.05:
    # below 1e-6 of the state beyond r = 0.45
    far = np.hypot(cx - 0.25, cy - 0.5) > 0.45
    up = far & (cx < 0.45)
    dn = cx > 0.55                                      # cells clear of the shock
    assert up.any() and dn.any()
    r1, u1, p1 = 1.21, math.sqrt(G), 1.0
    assert np.allclose(rho[up], r1, rtol=1e-6) and np.allclose(p[up], p1, rtol=1e-6)
    assert np.allclose(u[up], u1, rtol=1e-6)
    assert abs(u1 / math.sqrt(G * p1 / r1) - 1.1) < 1e-12
    assert np.ptp(rho[dn]) < 1e-12 and np.ptp(p[dn]) < 1e-12 and np.ptp(u[dn]) < 1e-12
    r2, u2, p2 = rho[dn].mean(), u[dn].mean(), p[dn].mean()
    assert abs(r1 * u1 - r2 * u2) < 1e-12
    assert abs(r1 * u1 ** 2 + p1 - (r2 * u2 ** 2 + p2)) < 1e-12
    h1 = G / (G - 1) * p1 / r1 + 0.5 * u1 ** 2
    h2 = G / (G - 1) * p2 / r2 + 0.5 * u2 ** 2
    assert abs(h1 - h2) < 1e-12
    # the vortex: entropy of the upstream gas unchanged inside it
    near = (np.hypot(cx - 0.25, cy - 0.5) < 0.1) & (cx < 0.5)
    assert near.any()
    s = p[near] / rho[near] ** G
    assert np.allclose(s, p1 / r1 ** G, rtol=1e-3)


def test_channel_face_kinds():
    mesh = wl.channel_mesh(8, 4, "tri", 0.2, 9)
    cn = mesh.cell_nodes
    xy = mesh.node_xy
    seen = set()
    for i in range(mesh.n_cells):
        nf = 3 if cn[i, 3] < 0 else 4
        for k in range(nf):
            a, b = xy[cn[i, k]], xy[cn[i, (k + 1) % nf]]
            m = 0.5 * (a + b)
            kind = mesh.face_bc[i, k]
            if abs(m[1]) < 1e-12 or abs(m[1] - 1.0) < 1e-12:
                assert kind == wl.BC_REFLECTIVE
                seen.add("wall")
            elif abs(m[0]) < 1e-12:
                assert kind == wl.BC_INFLOW
                seen.add("inflow")
            elif abs(m[0] - 2.0) < 1e-12:
                assert kind == wl.BC_TRANSMISSIVE
                seen.add("open")
    assert seen == {"wall", "inflow", "open"}


def test_triangle_rule_integrates_polynomials_exactly():
    """The collapsed Gauss rule with q points per direction integrates every
    monomial s^i t^j of total degree <= 2q - 2 over the reference triangle:
    the integral is i! j! / (i + j + 2)!."""
    for q in (2, 3, 4):
        s, t, w = wl._triangle_rule(q)
        for i in range(2 * q - 1):
            for j in range(2 * q - 1 - i):
                exact = math.factorial(i) * math.factorial(j) / math.factorial(i + j + 2)
                assert abs((w * s ** i * t ** j).sum() - exact) < 1e-15


def test_cell_averages_of_polynomials_and_positive_seeded_states():
    """Averages over jittered quadrilaterals and triangles of a quadratic
    agree with the polygon moments computed from the vertices (Green's
    theorem); the seeded Euler state keeps density and pressure positive."""
    mesh = wl.grid_mesh(6, 5, 2.0, 1.0, np.arange(30).reshape(5, 6) % 2 == 0, 0.25, 7, False)
    avg = wl.cell_averages(mesh, lambda x, y: np.stack([np.ones_like(x), x, y * y, x * y]), 4, q=3)
    cn = mesh.cell_nodes
    for i in range(mesh.n_cells):
        nf = 3 if cn[i, 3] < 0 else 4
        P = mesh.node_xy[cn[i, :nf]]
        x0, y0 = P[:, 0], P[:, 1]
        x1, y1 = np.roll(x0, -1), np.roll(y0, -1)
        cr = x0 * y1 - x1 * y0
        A = cr.sum() / 2
        mx = ((x0 + x1) * cr).sum() / (6 * A)
        myy = ((y0 ** 2 + y0 * y1 + y1 ** 2) * cr).sum() / (12 * A)
        mxy = ((x0 * y1 + 2 * x0 * y0 + 2 * x1 * y1 + x1 * y0) * cr).sum() / (24 * A)
        assert np.allclose(avg[:, i], [1.0, mx, myy, mxy], rtol=0, atol=1e-13)
    W = wl.seeded_state(mesh, 4, 21)
    rho, u, v, p = _primitive(W)
    assert (rho > 0).all() and (p > 0).all()
