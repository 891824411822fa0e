"""Pins of the exact Riemann solver used by the physics tests: the star
states of the classical test problems as tabulated in Toro's book (Riemann
Solvers and Numerical Methods for Fluid Dynamics, tests 1-3 of Sec. 4.3.3),
far-field states, and conservation of mass, momentum and energy by the
sampled self-similar solution."""
import numpy as np
import pytest

import exact_riemann as er

CASES = [  # left, right, p*, u*, rho*L, rho*R (Toro, tests 1-3)
    ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 0.30313, 0.92745, 0.42632, 0.26557),
    ((1.0, -2.0, 0.4), (1.0, 2.0, 0.4), 0.00189, 0.00000, 0.02185, 0.02185),
    ((1.0, 0.0, 1000.0), (1.0, 0.0, 0.01), 460.894, 19.5975, 0.57506, 5.99924),
]


@pytest.mark.parametrize("left,right,ps,us,rl,rr", CASES)
def test_star_states_match_the_tabulated_values(left, right, ps, us, rl, rr):
    p, u = er.star_state(left, right)
    assert p == pytest.approx(ps, rel=2e-4, abs=1e-5)
    assert u == pytest.approx(us, rel=2e-4, abs=1e-5)
    eps = 1e-9
    rho, _, _ = er.sample(left, right, np.array([u - eps, u + eps]))
    assert rho[0] == pytest.approx(rl, rel=2e-4)
    assert rho[1] == pytest.approx(rr, rel=2e-4)


@pytest.mark.parametrize("left,right", [c[:2] for c in CASES])
def test_self_similar_solution_conserves(left, right):
    """At t = 1 the integral of each conserved variable over [-X, X] equals
    its initial integral plus the net flux through the ends."""
    g = 1.4
    X = 60.0
    s = np.linspace(-X, X, 2_000_001)
    rho, u, p = er.sample(left, right, s)
    E = p / (g - 1) + 0.5 * rho * u * u

    def cons(r, v, q):
        e = q / (g - 1) + 0.5 * r * v * v
        return np.array([r, r * v, e]), np.array([r * v, r * v * v + q, (e + q) * v])

    (Ul, Fl), (Ur, Fr) = cons(*left), cons(*right)
    w = np.full(s.size, s[1] - s[0])
    w[0] = w[-1] = 0.5 * w[0]
    got = np.array([(w * rho).sum(), (w * rho * u).sum(), (w * E).sum()])
    expect = X * (Ul + Ur) + (Fl - Fr)
    np.testing.assert_allclose(got, expect, rtol=2e-5, atol=1e-4)
    # far field
    r0, u0, p0 = er.sample(left, right, np.array([-X, X]))
    assert (r0[0], u0[0], p0[0]) == pytest.approx(left)
    assert (r0[1], u0[1], p0[1]) == pytest.approx(right)
