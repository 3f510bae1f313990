"""Pins of the oracle's general operator (eq 2.2: variable coefficients,
first-order and zeroth-order terms, not self-adjoint):

* on an affine box element the weighted residual equals the closed form of
  L in lam (constant J = diag(h/2));
* the nodal interpolant of a polynomial solution of degree <= W with
  variable, non-polynomial coefficients makes every volume residual vanish
  at every quadrature point, so it satisfies X U = b to rounding;
* the normal equations stay symmetric and the error of the thesis's
  Table 6.14 operator (Dirichlet data) decays exponentially in W."""
import numpy as np
import pytest

from workloads import mesh as M
from workloads.problems import GeneralElliptic, Problem
from oracle.functional import Discretization
from oracle.precond import BlockPreconditioner
from oracle.solve import pcg, h1_error


class PolyWithCoefficients(Problem):
    """u = cubic in x; the Table 6.14 coefficients plus a first-order term."""

    def __init__(self):
        self.base = GeneralElliptic()

    def coefficients(self, x):
        a, beta, c = self.base.coefficients(x)
        beta = np.stack([0.3 * np.sin(x[..., 1]), -0.2 + 0 * x[..., 0], 0.1 * x[..., 0] * x[..., 2]], -1)
        return a, beta, c

    def u(self, x):
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        return 1 + X - 2 * X ** 3 + X * Y * Z + Y ** 2 * Z - Z ** 3

    def grad_u(self, x):
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        return np.stack([1 - 6 * X ** 2 + Y * Z, X * Z + 2 * Y * Z, X * Y + Y ** 2 - 3 * Z ** 2], -1)

    def f(self, x):
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        H = np.stack([-12 * X, 2 * Z, -6 * Z, Z, Y, X + 2 * Y], -1)   # xx yy zz xy xz yz
        a, beta, c = self.coefficients(x)
        lu = -(a[..., 0] * H[..., 0] + a[..., 1] * H[..., 1] + a[..., 2] * H[..., 2]
               + 2 * (a[..., 3] * H[..., 3] + a[..., 4] * H[..., 4] + a[..., 5] * H[..., 5]))
        return lu + (beta * self.grad_u(x)).sum(-1) + c * self.u(x)


def test_closed_form_on_an_affine_box():
    mesh = M.box_mesh(3, (1, 1, 1), (0.1, -0.2, 0.3), (0.6, 0.5, 1.2))
    P = PolyWithCoefficients()
    disc = Discretization(mesh, P)
    v = disc.vol[0]
    rng = np.random.default_rng(2)
    ue = rng.standard_normal((disc.n,) * 3)
    z = disc.volume_residual(ue, v)
    h = np.array([0.5, 0.7, 0.9])
    g = 2.0 / h
    d = lambda o: disc._fields(ue, o) * np.prod([g[i] ** o[i] for i in range(3)])
    a, beta, c = P.coefficients(v["x"])
    lu = -(a[:, 0] * d((2, 0, 0)) + a[:, 1] * d((0, 2, 0)) + a[:, 2] * d((0, 0, 2))
           + 2 * (a[:, 3] * d((1, 1, 0)) + a[:, 4] * d((1, 0, 1)) + a[:, 5] * d((0, 1, 1))))
    lu += beta[:, 0] * d((1, 0, 0)) + beta[:, 1] * d((0, 1, 0)) + beta[:, 2] * d((0, 0, 1))
    lu += c * d((0, 0, 0))
    ref = v["s"] * lu
    np.testing.assert_allclose(z, ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_polynomial_solution_satisfies_the_normal_equations():
    mesh = M.box_mesh(3, (2, 2, 1), (-1.0, -1.0, -1.0), (1.0, 0.4, 0.8))
    P = PolyWithCoefficients()
    disc = Discretization(mesh, P)
    n = disc.n
    A, B, C = np.meshgrid(disc.xn, disc.xn, disc.xn, indexing="ij")
    lam = np.stack([A.ravel(order="F"), B.ravel(order="F"), C.ravel(order="F")], -1)
    U = np.zeros(disc.ndof)
    for e in disc.real:
        o = disc.offset[e]
        U[o:o + n ** 3] = P.u(M.chart_points(mesh, e, lam))
    b = disc.rhs()
    assert disc.functional(U) <= 1e-20 * (b @ b)
    assert np.linalg.norm(disc.apply_X(U) - b) <= 1e-11 * np.linalg.norm(b)


def test_general_operator_symmetric_and_converging():
    P = GeneralElliptic()
    errs = []
    for W in (2, 4, 6):
        mesh = M.box_mesh(W, (2, 2, 2), (-1, -1, -1), (1, 1, 1))
        disc = Discretization(mesh, P)
        if W == 2:
            rng = np.random.default_rng(0)
            u, v = rng.standard_normal((2, disc.ndof))
            assert abs(v @ disc.apply_X(u) - u @ disc.apply_X(v)) <= 1e-12 * abs(v @ disc.apply_X(u))
        x, _, _ = pcg(disc.apply_X, disc.rhs(), BlockPreconditioner(disc).apply, 1e-12, 20000)
        errs.append(h1_error(disc, x, P))
    assert errs[0] > 10 * errs[1] and errs[1] > 20 * errs[2], errs
