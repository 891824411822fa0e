"""Pins of the oracle's geometry, least squares and linear weights
(paper Sec. 2, 3.1-3.4)."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import mesh as om
from oracle import geometry as og
from oracle import weights as ow
from oracle import stencil as ost


# ---------------------------------------------------------------- quadrature
def _gl_triangle(q):
    """Collapsed Gauss-Legendre rule on the unit triangle, written here
    independently of the oracle and of the input generators."""
    g, w = np.polynomial.legendre.leggauss(q)
    u = (g + 1) / 2
    wu = w / 2
    pts, wts = [], []
    for a, wa in zip(u, wu):
        for b, wb in zip(u, wu):
            pts.append((a, b * (1 - a)))
            wts.append(wa * wb * (1 - a))
    return np.array(pts), np.array(wts)


def _poly_integral(P, f, q=6):
    """Integral of f over the polygon P (list of vertices, counter-clockwise)."""
    pts, wts = _gl_triangle(q)
    tot = 0.0
    for k in range(1, len(P) - 1):
        a, b, c = np.asarray(P[0]), np.asarray(P[k]), np.asarray(P[k + 1])
        J = (b[0] - a[0]) * (c[1] - a[1]) - (c[0] - a[0]) * (b[1] - a[1])
        x = a + np.outer(pts[:, 0], b - a) + np.outer(pts[:, 1], c - a)
        tot += J * (wts * f(x[:, 0], x[:, 1])).sum()
    return tot


def test_moments_match_gauss_legendre():
    rng = np.random.Generator(np.random.PCG64(3))
    for _ in range(50):
        # random convex or non-convex (dart) quadrilateral and a triangle
        base = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], float)
        P = base + rng.uniform(-0.3, 0.3, size=(4, 2))
        if rng.random() < 0.3:
            P[2] = [0.45, 0.45]                       # reflex vertex
        T = rng.uniform(-1, 1, size=(3, 2))
        if (T[1, 0] - T[0, 0]) * (T[2, 1] - T[0, 1]) - (T[2, 0] - T[0, 0]) * (T[1, 1] - T[0, 1]) < 0:
            T = T[[0, 2, 1]]
        for poly, nf in ((P, 4), (np.vstack([T, T[:1]]), 3)):
            mom = og.poly_moments(poly[None], np.array([nf]))[0]
            verts = poly[:nf]
            fs = [lambda x, y: np.ones_like(x), lambda x, y: x, lambda x, y: y,
                  lambda x, y: x * x, lambda x, y: y * y, lambda x, y: x * y]
            ref = [_poly_integral(verts, f) for f in fs]
            np.testing.assert_allclose(mom, ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("kind", ["quad", "tri"])
def test_areas_sum_to_domain_and_faces_close(kind):
    mesh = wl.grid_mesh(10, 10, 2.0, 2.0, kind, 0.3, 2, True)
    T = ow.precompute(mesh)
    total = 0.0
    for g in T.groups.values():
        total += g.area.sum()
        n = g.st.spec.n
        s = (g.length[:, :n, None] * g.normal[:, :n]).sum(axis=1)
        assert np.abs(s).max() < 1e-14
        np.testing.assert_allclose(np.linalg.norm(g.normal[:, :n], axis=-1), 1.0, atol=1e-15)
    assert abs(total - 4.0) < 1e-12


def test_two_point_gauss_rule_integrates_cubics_on_a_face():
    # eq. (quadrature): |l| (f(x1) + f(x2)) / 2 with the points
    # (3 +- sqrt3)/6 between the end points is exact for cubics
    rng = np.random.Generator(np.random.PCG64(5))
    for _ in range(20):
        a, b = rng.uniform(-1, 1, 2), rng.uniform(-1, 1, 2)
        c = rng.normal(size=4)
        f = lambda s: c[0] + c[1] * s + c[2] * s ** 2 + c[3] * s ** 3  # noqa: E731
        exact = c[0] + c[1] / 2 + c[2] / 3 + c[3] / 4          # integral over s in [0,1]
        x1 = og.GP_A * a + og.GP_B * b
        x2 = og.GP_B * a + og.GP_A * b
        s1 = np.linalg.norm(x1 - a) / np.linalg.norm(b - a)
        s2 = np.linalg.norm(x2 - a) / np.linalg.norm(b - a)
        assert abs(0.5 * (f(s1) + f(s2)) - exact) < 1e-14


# ---------------------------------------------------------------- reproduction
def _stencil_averages(mesh, g, fn):
    """Cell averages of fn over every slot polygon of every target, from the
    raw mesh (shifted periodic images, mirrored ghosts), by quadrature."""
    st = g.st
    m, S = st.cell.shape
    out = np.zeros((m, S))
    cn, xy = mesh.cell_nodes, mesh.node_xy
    for r in range(m):
        i0 = st.cells[r]
        P0 = [xy[n] for n in cn[i0] if n >= 0]
        for j in range(S):
            if not st.present[r, j]:
                continue
            if st.ghost[r, j] >= 0:
                k = st.ghost[r, j]
                a, b = np.asarray(P0[k]), np.asarray(P0[(k + 1) % len(P0)])
                d = (b - a) / np.linalg.norm(b - a)
                nrm = np.array([d[1], -d[0]])
                P = [np.asarray(p) - 2 * np.dot(np.asarray(p) - a, nrm) * nrm for p in P0][::-1]
            else:
                P = [xy[n] + st.shift[r, j] for n in cn[st.cell[r, j]] if n >= 0]
            out[r, j] = _poly_integral(P, fn) / _poly_integral(P, lambda x, y: np.ones_like(x))
    return out


def _gauss_points(mesh, g):
    st = g.st
    n = st.spec.n
    pts = np.zeros((st.cells.size, 2 * n, 2))
    for r, i0 in enumerate(st.cells):
        P = [mesh.node_xy[v] for v in mesh.cell_nodes[i0] if v >= 0]
        for k in range(n):
            a, b = P[k], P[(k + 1) % n]
            pts[r, 2 * k] = (3 + math.sqrt(3)) / 6 * a + (3 - math.sqrt(3)) / 6 * b
            pts[r, 2 * k + 1] = (3 - math.sqrt(3)) / 6 * a + (3 + math.sqrt(3)) / 6 * b
    return pts


MESHES = {
    "quad20": lambda: wl.grid_mesh(6, 6, 2.0, 2.0, "quad", 0.2, 12, True),
    "tri30": lambda: wl.grid_mesh(5, 5, 2.0, 2.0, "tri", 0.3, 13, True),
    "mixed": lambda: wl.mesh_c5(n=8, block=2, jitter=0.3, seed=14),
    "sod": lambda: wl.grid_mesh(5, 5, 1.0, 1.0,
                                np.add.outer(np.arange(5), np.arange(5)) % 2 == 0, 0.15, 15, False),
}


@pytest.mark.parametrize("name", list(MESHES))
def test_eta_and_gamma_reproduce_quadratics(name):
    """eq. (polynomial-eta) with a consistent least squares reproduces exact
    quadratic data; eq. (linRelation) then reproduces it through the
    candidates: sum_j gamma_j P_j(x_G) = P^2(x_G) = q(x_G)."""
    mesh = MESHES[name]()
    T = ow.precompute(mesh)
    rng = np.random.Generator(np.random.PCG64(21))
    c = rng.normal(size=6)
    q = lambda x, y: c[0] + c[1] * x + c[2] * y + c[3] * x * x + c[4] * y * y + c[5] * x * y  # noqa: E731
    for g in T.groups.values():
        avg = _stencil_averages(mesh, g, q)
        G = _gauss_points(mesh, g)
        exact = q(G[..., 0], G[..., 1])
        # reproduction needs a full-rank constraint matrix (5 independent rows);
        # near a boundary corner a stencil can have fewer
        A = np.where(g.st.present[:, 1:, None], g.frame.basis_avg[:, 1:, :], 0.0)
        full = np.linalg.svd(A, compute_uv=False)[:, -1] > 1e-8
        assert full.mean() > 0.8
        for eta in (g.eta_raw, g.eta):
            P2 = (eta * avg[:, None, :]).sum(-1)
            np.testing.assert_allclose(P2[full], exact[full], rtol=0, atol=2e-9)
            assert np.abs(eta.sum(-1) - 1).max() < 1e-12
            assert (np.where(~g.st.present[:, None, :], eta, 0) == 0).all()
        # candidates: P_j(G) = b_j0 W_i0 + b_ja W_a + b_jb W_b, through B; the
        # weighted sum reproduces P^2 (and so q where P^2 is exact)
        for gam, eta in ((g.gamma_raw, g.eta_raw), (g.gamma, g.eta)):
            R = np.einsum("mgsj,mgj,ms->mg", g.B, gam, avg)
            P2 = (eta * avg[:, None, :]).sum(-1)
            tol = 5e-9 * max(1, np.abs(gam).max())
            np.testing.assert_allclose(R, P2, rtol=0, atol=tol)
            np.testing.assert_allclose(R[full], exact[full], rtol=0, atol=tol)
            # sum gamma = 1 (paper Sec. 3.1) for the minimum-norm solution; the
            # regularisation moves gamma by at most zeta sqrt(M) |eta| / s_min^3
            sv = np.linalg.svd(g.B, compute_uv=False)
            smin = np.where(sv > 1e-12 * sv[..., :1], sv, np.inf).min(-1)
            bound = 1e-12 + 1e-14 * np.sqrt(sv.shape[-1]) * np.linalg.norm(eta, axis=-1) / smin ** 3
            assert (np.abs(gam.sum(-1) - 1) <= bound).all()


@pytest.mark.parametrize("name", list(MESHES))
def test_candidates_reproduce_linear_functions(name):
    mesh = MESHES[name]()
    T = ow.precompute(mesh)
    c = np.array([0.7, -1.3, 2.1])
    lin = lambda x, y: c[0] + c[1] * x + c[2] * y  # noqa: E731
    for g in T.groups.values():
        avg = _stencil_averages(mesh, g, lin)
        G = _gauss_points(mesh, g)
        exact = lin(G[..., 0], G[..., 1])
        # each column of B is one candidate P_j evaluated at G
        Pj = np.einsum("mgsj,ms->mgj", g.B, avg)
        ok = np.ones(Pj.shape[:1] + (1, Pj.shape[2]), bool)
        # a degenerate sub-stencil (third cell substituted by i0) only fits
        # the one remaining constraint; exclude those columns
        deg = (g.cand_b == 0)[:, None, :]
        ok = ok & ~deg
        err = np.where(ok, np.abs(Pj - exact[..., None]), 0)
        assert err.max() < 1e-12
        np.testing.assert_allclose(g.B.sum(axis=2), 1.0, atol=1e-13)


def test_gamma_is_the_minimum_norm_solution():
    mesh = wl.grid_mesh(6, 6, 2.0, 2.0, "quad", 0.2, 12, True)
    T = ow.precompute(mesh)
    g = T.groups[4]
    import scipy.linalg
    for r in range(0, g.B.shape[0], 7):
        for gp in range(g.B.shape[1]):
            sol = scipy.linalg.lstsq(g.B[r, gp], g.eta_raw[r, gp], lapack_driver="gelsy",
                                     cond=1e-10)[0]
            np.testing.assert_allclose(g.gamma_raw[r, gp], sol, atol=1e-9)
            # rank of B is 11 for a full quadrilateral stencil (two left null vectors)
            s = np.linalg.svd(g.B[r, gp], compute_uv=False)
            assert (s > 1e-10).sum() <= 11


def test_optimisation_tames_large_weights():
    """Sec. 3.3: on strongly perturbed meshes the optimised weights are O(1)."""
    for kind, seed in (("quad", 31), ("tri", 32)):
        mesh = wl.grid_mesh(12, 12, 2.0, 2.0, kind, 0.3, seed, True)
        d = ow.diagnostics(ow.precompute(mesh))
        assert d["max_abs_gamma_opt"] <= d["max_abs_gamma_raw"]
        assert d["max_abs_gamma_opt"] < 12.0
        if kind == "tri":       # large raw weights appear on perturbed triangles
            assert d["max_abs_gamma_raw"] > 50 * d["max_abs_gamma_opt"]
        assert d["resid_opt"] < 1e-9 and d["sum_dev"] < 1e-10


def test_tikhonov_limit_is_pseudo_inverse():
    """Remark after eq. (quadratic-2): the regularised solution differs from
    the unregularised one by O(zeta); in the limit it is the pseudo-inverse."""
    rng = np.random.Generator(np.random.PCG64(8))
    A = rng.normal(size=(12, 5))
    X = ow.tikhonov(A, 1e-14)
    ref = np.linalg.solve(A.T @ A, A.T)
    np.testing.assert_allclose(X, ref, atol=1e-12)
    Xz = ow.tikhonov(A, 1e-4)
    ref_z = np.linalg.solve(1e-4 * np.eye(5) + A.T @ A, A.T)
    np.testing.assert_allclose(Xz, ref_z, atol=1e-12)


def test_absent_slots_have_zero_rows():
    mesh = wl.grid_mesh(6, 6, 2.0, 2.0, "quad", 0.0, 1, True)
    T = ow.precompute(mesh)
    g = T.groups[4]
    assert (g.eta[:, :, 9:] == 0).all()
    assert not g.st.present[:, 9:].any()
    assert set(ost.QUAD.replace) == {0, 5, 6, 7, 8}
