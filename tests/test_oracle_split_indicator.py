"""Pins of the oracle's split of the linear weights, its new smoothness
indicator and its nonlinear weights (paper Sec. 3.4), through the oracle's
own functions.

What fixes each value here is not the formula typed again but a property
the paper states or a special case with a known answer:

* the split for theta = 3 has the closed forms (2 gamma, gamma) for gamma >= 0
  and (|gamma|, 2|gamma|) for gamma < 0; theta = 1 reduces to the positive
  and negative parts;
* with equal indicators the nonlinear weights equal the split linear ones,
  and sigma+ R+ - sigma- R- is then the linear combination sum gamma_j P_j;
* the ratio argument after the new indicator: for a candidate that crosses
  a jump and carries a very large linear weight gamma_1, delta_1 / delta_j
  falls like gamma_1^-3 (the classical indicator gives gamma_1^+1, the new
  one without its squared term gamma_1^-1);
* in smooth regions the indicator is h^2 (1 + O(h)).
"""
import numpy as np
import pytest

import workloads as wl
from oracle import weights as ow
from oracle import scheme as osc


def _gammas(seed, shape=(200, 12)):
    rng = np.random.Generator(np.random.PCG64(seed))
    gam = rng.normal(size=shape)
    gam /= gam.sum(axis=-1, keepdims=True)       # linear weights sum to one
    return gam


def test_split_theta3_closed_forms():
    gam = _gammas(4)
    gp, sp, gm, sm = osc.split_linear_weights(gam, 3.0)
    tp, tm = gp * sp, gm * sm                     # gamma~+, gamma~-
    np.testing.assert_allclose(tp, np.where(gam >= 0, 2 * gam, -gam), rtol=1e-14, atol=0)
    np.testing.assert_allclose(tm, np.where(gam >= 0, gam, -2 * gam), rtol=1e-14, atol=0)
    assert (gp >= 0).all() and (gm >= 0).all()
    np.testing.assert_allclose(gp.sum(-1), 1.0, rtol=0, atol=1e-14)
    np.testing.assert_allclose(gm.sum(-1), 1.0, rtol=0, atol=1e-14)
    # sigma+ - sigma- = sum gamma = 1, and sigma- = 1 + 3 sum |gamma<0| for theta = 3
    np.testing.assert_allclose((sp - sm)[..., 0], gam.sum(-1), atol=1e-12)
    neg = np.where(gam < 0, -gam, 0.0).sum(-1)
    np.testing.assert_allclose(sm[..., 0], 1.0 + 3.0 * neg, rtol=1e-13)


def test_split_depends_on_theta():
    """theta = 1 is the plain split into positive and negative parts; the
    theta = 3 closed forms above would then fail."""
    gam = _gammas(5)
    gp, sp, gm, sm = osc.split_linear_weights(gam, 1.0)
    np.testing.assert_allclose(gp * sp, np.maximum(gam, 0.0), atol=1e-15)
    np.testing.assert_allclose(gm * sm, np.maximum(-gam, 0.0), atol=1e-15)
    # a larger theta moves weight into both halves: sigma- grows with theta
    s = [osc.split_linear_weights(gam, th)[3][..., 0] for th in (1.0, 3.0, 5.0)]
    assert (s[0] < s[1]).all() and (s[1] < s[2]).all()


def test_all_positive_weights_split_into_equal_halves():
    """theta = 3 and gamma >= 0: gamma+ = gamma- = gamma and (sigma+,
    sigma-) = (2, 1), so R = 2 R+ - R- = R+."""
    rng = np.random.Generator(np.random.PCG64(6))
    gam = rng.uniform(0.0, 1.0, size=(50, 9))
    gam /= gam.sum(-1, keepdims=True)
    gp, sp, gm, sm = osc.split_linear_weights(gam, 3.0)
    np.testing.assert_allclose(gp, gam, rtol=1e-14)
    np.testing.assert_allclose(gm, gam, rtol=1e-14)
    np.testing.assert_allclose(sp, 2.0, rtol=1e-14)
    np.testing.assert_allclose(sm, 1.0, rtol=1e-14)


@pytest.mark.parametrize("kind,seed", [("quad", 31), ("tri", 32)])
def test_equal_indicators_give_the_linear_combination(kind, seed):
    """With every beta~_j equal, delta_j^pm = gamma_j^pm, and the split form
    sigma+ R+ - sigma- R- collapses to sum_j gamma_j P_j: this holds only
    with the factors sigma^pm and with sum gamma^pm = 1 (Sec. 3.4).  The new
    indicator depends on gamma^pm, so equal beta~ needs beta = 0 (a locally
    constant state), or an eps that swamps every beta~.  The linear weights
    are the oracle's optimised ones on a 30%-jittered mesh, negative parts
    included."""
    mesh = wl.grid_mesh(8, 8, 2.0, 2.0, kind, 0.3, seed, True)
    T = ow.precompute(mesh)
    g = T.groups[4 if kind == "quad" else 3]
    gam = g.gamma                                    # [m,G,M]
    assert (gam < -1e-3).any()
    gp, sp, gm, sm = osc.split_linear_weights(gam, 3.0)
    rng = np.random.Generator(np.random.PCG64(seed))
    d = rng.normal(size=(2,) + gam.shape)            # candidate increments, 2 fields
    ref = (gam[None] * d).sum(-1)
    for b, eps in ((0.0, 1e-3), (0.0, 1e-6), (0.37, 1e30), (5.0, 1e30)):
        beta = np.full(d.shape, b)
        got = osc._nonlinear_combination(gp, sp, gm, sm, beta, d, eps)
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * (1 + np.abs(d).max()))
    # equal beta > 0 with a small eps: beta~ differs by candidate, so the
    # result moves away from the linear combination
    got = osc._nonlinear_combination(gp, sp, gm, sm, np.full(d.shape, 5.0), d, 1e-3)
    assert np.abs(got - ref).max() > 1e-3


def _delta_ratio(g1):
    """delta_1 / delta_2 of the + half for a candidate 1 that crosses a jump
    (beta_1 = 1) with linear weight g1, against smooth candidates (beta =
    h^2, h = 0.01) of weight 1/3, from the oracle's combination with unit
    increments (d = e_k picks delta_k; sigma+ = 1, sigma- = 0)."""
    h, eps, M = 0.01, 1e-3, 4
    gw = np.array([g1, 1 / 3, 1 / 3, 1 / 3])[None, None, :]
    beta = np.array([1.0, h * h, h * h, h * h])[None, None, None, :]
    one, zero = np.ones((1, 1, 1)), np.zeros((1, 1, 1))
    out = []
    for k in (0, 1):
        d = np.zeros((1, 1, 1, M))
        d[..., k] = 1.0
        out.append(osc._nonlinear_combination(gw, one, gw, zero, beta, d, eps)[0, 0, 0])
    return out[0] / out[1]


def test_ratio_argument_of_the_new_indicator():
    """Sec. 3.4: with a very large linear weight on a jump-crossing
    candidate, delta_1 / delta_j decays like gamma_1^-3.  A dropped squared
    term gives a slope of -1, the classical indicator +1."""
    gs = np.geomspace(1e2, 1e4, 9)
    r = np.array([_delta_ratio(g) for g in gs])
    slope = np.polyfit(np.log(gs), np.log(r), 1)[0]
    assert abs(slope + 3.0) < 0.02, slope
    # and the crossing candidate is suppressed outright
    assert r[0] < 1e-4


def test_new_indicator_limits():
    """Sec. 3.4's ratio argument writes the new indicator of a candidate with
    beta = O(1) and a large weight gamma as gamma (gamma + O(1)): with
    beta = 1 it is gamma^2 (1 + O(1/gamma)).  And beta~ is the sum of the
    first three terms of the geometric series beta sum_k (gamma beta)^k,
    i.e. beta (1 - (gamma beta)^3) / (1 - gamma beta) where gamma beta != 1;
    beta~ -> beta as gamma beta -> 0."""
    g = np.geomspace(1e2, 1e6, 5)
    bt = osc.new_smoothness_indicator(np.ones_like(g), g)
    dev = np.abs(bt / g ** 2 - 1.0)
    assert (dev * g < 1.01).all() and dev[-1] < 1e-5, dev
    rng = np.random.Generator(np.random.PCG64(7))
    beta = rng.uniform(0.0, 3.0, 1000)
    gw = rng.uniform(0.0, 1.0, 1000)
    t = gw * beta
    ok = np.abs(1.0 - t) > 1e-3
    geo = beta[ok] * (1.0 - t[ok] ** 3) / (1.0 - t[ok])
    np.testing.assert_allclose(osc.new_smoothness_indicator(beta, gw)[ok], geo, rtol=1e-9)
    small = osc.new_smoothness_indicator(np.full(5, 2.0), np.geomspace(1e-12, 1e-8, 5))
    np.testing.assert_allclose(small, 2.0, rtol=1e-7)


def test_jump_crossing_candidate_loses_its_weight_on_a_mesh():
    """The same on a real stencil: a cell just left of a unit jump; every
    candidate that spans the jump gets delta far below its linear weight
    in both halves of the split."""
    mesh = wl.grid_mesh(12, 12, 2.0, 2.0, "quad", 0.1, 43, True)
    T = ow.precompute(mesh)
    W = wl.cell_averages(mesh, lambda x, y: np.where(x < 1.0, 1.0, 2.0)[None], 1, q=3)
    g = T.groups[4]
    cx = g.frame.centroid[:, 0]
    r = int(np.argmin(np.abs(cx - (1.0 - 2.0 / 24)) + np.abs(g.frame.centroid[:, 1] - 1.0)))
    rows = np.array([r])
    dW = W[:, g.st.runtime_cell[rows]] - W[:, g.st.cells[rows]][:, :, None]
    _, _, beta = osc.candidate_gradients(g, dW, rows)       # [1,1,M]
    crossing = beta[0, 0] > 0.1
    assert crossing.any() and (~crossing).any()
    gp, _, gm, _ = osc.split_linear_weights(g.gamma[rows], T.scheme.theta)
    for gw in (gp, gm):
        delta = osc.nonlinear_weights(gw[0], beta[0], T.scheme.eps)    # [G,M]
        on = gw[0][:, crossing] > 1e-6
        assert (delta[:, crossing][on] < 1e-3 * gw[0][:, crossing][on]).all()


@pytest.mark.parametrize("kind", ["quad", "tri"])
def test_indicator_is_h2_times_one_plus_order_h_in_smooth_regions(kind):
    """Sec. 3.4: IS = h^2 (1 + O(h)).  For a smooth u the candidate indicator
    is |Omega| |grad u(x_i0)|^2 (1 + O(h)): the median relative deviation
    halves with each halving of h.  The new indicator adds gamma beta (1 +
    gamma beta) = O(h^2) relative to beta."""
    f = lambda x, y: np.sin(np.pi * x) * np.cos(np.pi * y)  # noqa: E731
    med, top_new = [], []
    for n in (16, 32, 64):
        mesh = wl.grid_mesh(n, n, 2.0, 2.0, kind, 0.2, 7, True)
        T = ow.precompute(mesh)
        W = wl.cell_averages(mesh, lambda x, y: f(x, y)[None], 1, q=4)
        g = T.groups[4 if kind == "quad" else 3]
        rows = np.arange(g.st.cells.size)
        dW = W[:, g.st.runtime_cell] - W[:, g.st.cells][:, :, None]
        _, _, beta = osc.candidate_gradients(g, dW, rows)     # [1,m,M]
        c = g.frame.centroid
        gu = np.stack([np.pi * np.cos(np.pi * c[:, 0]) * np.cos(np.pi * c[:, 1]),
                       -np.pi * np.sin(np.pi * c[:, 0]) * np.sin(np.pi * c[:, 1])], -1)
        g2 = (gu ** 2).sum(-1)
        sel = g2 > 0.25 * np.pi ** 2                   # away from critical points of u
        rel = beta[0][sel] / (g.area[sel, None] * g2[sel, None]) - 1.0
        med.append(np.median(np.abs(rel)))
        gp, _, gm, _ = osc.split_linear_weights(g.gamma, T.scheme.theta)
        worst = 0.0
        for gw in (gp, gm):
            bt = osc.new_smoothness_indicator(beta[0][:, None, :], gw)   # [m,G,M]
            b = np.broadcast_to(beta[0][:, None, :], bt.shape)
            ok = b > 0
            worst = max(worst, float((bt[ok] / b[ok] - 1.0).max()))
        top_new.append(worst / (2.0 / n) ** 2)
    assert med[-1] < 0.06, med
    for a, b in zip(med, med[1:]):
        assert 1.6 < a / b < 2.5, med
    # (beta~ / beta - 1) / h^2 stays bounded under refinement
    assert max(top_new) < 50.0 and top_new[-1] < 2.0 * top_new[0] + 1.0, top_new


def test_reconstruction_uses_the_normalised_split(monkeypatch):
    """The oracle's reconstruction hands the nonlinear combination the
    scaled weights gamma^pm (non-negative, summing to one) and their sums
    sigma^pm with sigma+ - sigma- = sum gamma (not, e.g., the unscaled
    gamma~pm)."""
    mesh = wl.mesh_c5(n=12, block=3, jitter=0.3, seed=42)
    T = ow.precompute(mesh)
    seen = []
    real = osc._nonlinear_combination

    def spy(gp, sp, gm, sm, beta, d, eps):
        seen.append((gp.copy(), sp.copy(), gm.copy(), sm.copy(), eps))
        return real(gp, sp, gm, sm, beta, d, eps)

    monkeypatch.setattr(osc, "_nonlinear_combination", spy)
    W = wl.seeded_state(mesh, 4, 1)
    osc.reconstruct_face_states(T, W)
    assert len(seen) == len(T.groups)
    for gp, sp, gm, sm, eps in seen:
        assert eps == T.scheme.eps
        assert (gp >= 0).all() and (gm >= 0).all()
        np.testing.assert_allclose(gp.sum(-1), 1.0, atol=1e-13)
        np.testing.assert_allclose(gm.sum(-1), 1.0, atol=1e-13)
        np.testing.assert_allclose(sp - sm, 1.0, atol=1e-10)
        assert (sm >= 1.0 - 1e-12).all()
