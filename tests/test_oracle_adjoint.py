"""Pins of the oracle's source gradient: central finite differences of the
loss (central differences are exact for the quadratic L up to rounding),
and the linearity of b in the source coefficients."""
import numpy as np

from workloads import mesh as M
from workloads.problems import LegendreSource, legendre_theta
from oracle.adjoint import loss_and_grad, source_rhs
from oracle.functional import Discretization
from oracle.solve import dense_solve


def _setup():
    mesh = M.box_mesh(2, (2, 1, 1), (-1, -1, -1), (1, 0, 0))
    deg = 2
    disc = Discretization(mesh, LegendreSource(np.zeros(deg ** 3), deg))
    X = disc.dense_X()
    return disc, deg, (lambda r: dense_solve(X, r))


def test_gradient_matches_central_differences():
    disc, deg, solve = _setup()
    u_t = solve(source_rhs(disc, legendre_theta(deg, 1), deg))
    theta = legendre_theta(deg, 2)
    L, g = loss_and_grad(disc, theta, u_t, deg, solve)
    h = 1e-6
    for k in range(deg ** 3):
        e = np.zeros(deg ** 3)
        e[k] = h
        Lp = float(np.sum((solve(source_rhs(disc, theta + e, deg)) - u_t) ** 2))
        Lm = float(np.sum((solve(source_rhs(disc, theta - e, deg)) - u_t) ** 2))
        assert abs((Lp - Lm) / (2 * h) - g[k]) <= 1e-6 * np.abs(g).max()


def test_rhs_is_linear_in_theta():
    disc, deg, _ = _setup()
    t1, t2 = legendre_theta(deg, 3), legendre_theta(deg, 4)
    b12 = source_rhs(disc, 2.0 * t1 - t2, deg)
    ref = 2.0 * source_rhs(disc, t1, deg) - source_rhs(disc, t2, deg)
    assert np.linalg.norm(b12 - ref) <= 1e-12 * np.linalg.norm(ref)


def test_legendre_source_values():
    # P0 = 1, P1 = x: theta selecting P1(x1) P0 P0 gives f = x1
    deg = 2
    theta = np.zeros(deg ** 3)
    theta[1] = 1.0
    x = np.random.default_rng(0).uniform(-1, 1, (10, 3))
    np.testing.assert_allclose(LegendreSource(theta, deg).f(x), x[:, 0], rtol=0, atol=1e-15)
    theta = np.zeros(deg ** 3)
    theta[1 + deg * (1 + deg * 1)] = 1.0
    np.testing.assert_allclose(LegendreSource(theta, deg).f(x), x.prod(axis=1), rtol=0, atol=1e-15)
