"""Pins of the FP64 oracle against closed forms, printed values and invariants.

Each test checks the oracle against something other than itself: textbook
closed forms, the thesis's Table 5.1, exact integrals by brute force, the
closed-form transformed operators of Ch. 2, and structural invariants.
"""
import os

import numpy as np
import pytest
import sympy as sp

from workloads import mesh as M
from workloads.problems import SinProduct, Polynomial, Constant
from oracle import gll, charts
from oracle.functional import Discretization, SECOND, FIRST
from oracle.precond import table51_kappa, BlockPreconditioner, forms_1d, element_block
from oracle.solve import pcg, dense_solve, h1_error

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append([float(v) for v in line.split()])
    return np.array(rows)


# ---------------------------------------------------------------- 1D machinery
def test_gll_closed_form_w4():
    x, w = gll.gll(5)
    s = np.sqrt(3.0 / 7.0)
    np.testing.assert_allclose(x, [-1, -s, 0, s, 1], atol=1e-15)
    np.testing.assert_allclose(w, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], atol=1e-15)


@pytest.mark.parametrize("n", [3, 5, 7, 9, 13, 21])
def test_gll_exactness_degree(n):
    x, w = gll.gll(n)
    for k in range(2 * n - 2):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs((w * x ** k).sum() - exact) < 1e-13, k
    k = 2 * n - 2          # first even degree where the rule fails
    assert abs((w * x ** k).sum() - 2.0 / (k + 1)) > 5e-13


@pytest.mark.parametrize("W", [2, 4, 6, 10])
def test_differentiation_exact_for_degree_W(W):
    x, _ = gll.gll(W + 1)
    D = gll.diff_matrix(x)
    np.testing.assert_allclose(D @ np.ones(W + 1), 0, atol=1e-12)
    rng = np.random.default_rng(W)
    c = rng.standard_normal(W + 1)
    p = np.polynomial.Polynomial(c)
    np.testing.assert_allclose(D @ p(x), p.deriv()(x), rtol=1e-11, atol=1e-11)
    xm, _ = gll.gll(2 * W + 1)
    for d in range(3):
        Ld = gll.lagrange(x, xm, d)
        np.testing.assert_allclose(Ld @ p(x), p.deriv(d)(xm), rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("W", [2, 4, 6, 8])
def test_legendre_restriction_equals_interpolation_transpose(W):
    rng = np.random.default_rng(W)
    O = rng.standard_normal(2 * W + 1)
    G = gll.lagrange(gll.gll(W + 1)[0], gll.gll(2 * W + 1)[0])
    np.testing.assert_allclose(gll.legendre_restriction(O, W), G.T @ O, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("W", [2, 4, 6])
def test_half_norm_exact_for_polynomials(W):
    """GLL double sum = exact double integral of the difference quotient (deg <= 2W)."""
    m = 2 * W + 1
    x, _ = gll.gll(m)
    rng = np.random.default_rng(3 + W)
    p = np.polynomial.Polynomial(rng.standard_normal(2 * W + 1))
    K = gll.half_matrix(m)
    disc = p(x) @ K @ p(x)
    # brute force: quotient q(s,t) = (p(s)-p(t))/(s-t) is a polynomial in s,t
    xg, wg = np.polynomial.legendre.leggauss(2 * W + 4)
    S, T = np.meshgrid(xg, xg, indexing="ij")
    with np.errstate(invalid="ignore", divide="ignore"):
        q = (p(S) - p(T)) / (S - T)
    q[np.isclose(S, T)] = p.deriv()(S[np.isclose(S, T)])
    exact = (np.outer(wg, wg) * q ** 2).sum()
    assert abs(disc - exact) < 1e-10 * exact
    assert abs(gll.half_form_direct(p(x), m) - disc) < 1e-10 * exact
    np.testing.assert_allclose(K, K.T, atol=1e-12)
    np.testing.assert_allclose(K @ np.ones(m), 0, atol=1e-11)
    assert np.linalg.eigvalsh(K).min() > -1e-10


# ------------------------------------------------------------- Table 5.1 pin
def test_table51_condition_numbers():
    gold = _golden("table5_1.txt")
    for W, kappa in gold:
        assert abs(table51_kappa(int(W)) - kappa) < 1e-8 * kappa, W


@pytest.mark.parametrize("W", [2, 5])
def test_separable_eigenbasis(W):
    """C psi_ijk = (mu_i + mu_j + mu_k + 1) F psi_ijk (eq 5.20)."""
    F, S1, S2 = forms_1d(W)
    E = S2 + S1
    mu, V = np.linalg.eigh(np.diag(1 / np.sqrt(np.diag(F))) @ E @ np.diag(1 / np.sqrt(np.diag(F))))
    Phi = np.diag(1 / np.sqrt(np.diag(F))) @ V
    mesh = M.box_mesh(W, (1, 1, 1))
    C = element_block(mesh, 0)
    psi = np.kron(Phi[:, 1], np.kron(Phi[:, 2], Phi[:, 0]))  # i<-0, j<-2, k<-1
    FFF = np.kron(F, np.kron(F, F))
    np.testing.assert_allclose(C @ psi, (mu[0] + mu[2] + mu[1] + 1) * (FFF @ psi), rtol=1e-10, atol=1e-10)


# ------------------------------------------------ transformed operators, Ch. 2
def _single(chart, box, patch=None, region=M.REG, W=3):
    mesh = M.box_mesh(W, (1, 1, 1))
    mesh.chart[:] = chart
    mesh.region[:] = region
    mesh.box[0] = box
    if patch is not None:
        mesh.patch[0] = patch
    mesh.bc[:] = M.SKIP
    return mesh


def _lam_derivs(disc, ue):
    """lam-derivative fields at the fine points, keyed by derivative orders."""
    out = {}
    for (o, _, _) in SECOND:
        out[o] = disc._fields(ue, o)
    for (o, _) in FIRST:
        out[o] = disc._fields(ue, o)
    return out


def _check_closed_form(chart, region, box, closed):
    mesh = _single(chart, box, region=region)
    disc = Discretization(mesh)
    rng = np.random.default_rng(7)
    ue = rng.standard_normal((disc.n,) * 3)
    z = disc.volume_residual(ue, disc.vol[0])
    dv = _lam_derivs(disc, ue)
    h = box[1::2] - box[0::2]
    sc = 2.0 / h
    d = lambda o: dv[o] * np.prod([sc[i] ** o[i] for i in range(3)])
    m = disc.m
    A, B, C = np.meshgrid(disc.xm, disc.xm, disc.xm, indexing="ij")
    y = [box[2 * i] + 0.5 * (g.ravel(order="F") + 1) * h[i] for i, g in enumerate((A, B, C))]
    WA, WB, WC = np.meshgrid(disc.wm, disc.wm, disc.wm, indexing="ij")
    wq = (WA * WB * WC).ravel(order="F")
    ref = np.sqrt(wq * np.prod(h) / 8) * closed(d, y)
    np.testing.assert_allclose(z, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


def test_edge_operator_closed_form():
    """L^e u = -(u_tau tau + u_theta theta + e^{2 tau} u_33) (eq 2.35, 2.36, L = -Lap)."""
    box = np.array([np.log(0.02), np.log(0.1), 0.3, 1.1, 0.2, 0.7])
    _check_closed_form(M.EDGE_BOX, M.EDGE, box,
                       lambda d, y: -(d((2, 0, 0)) + d((0, 2, 0)) + np.exp(2 * y[0]) * d((0, 0, 2))))


def test_vertex_operator_closed_form():
    """L^v u = -e^{chi/2} sqrt(sin phi)(u_chichi + u_chi + u_phiphi + cot phi u_phi
    + u_thth / sin^2 phi) (eq 2.22, 2.23 with L = -Lap)."""
    box = np.array([0.5, 0.9, 0.2, 1.3, np.log(0.01), np.log(0.05)])

    def closed(d, y):
        ph, ch = y[0], y[2]
        return -np.exp(ch / 2) * np.sqrt(np.sin(ph)) * (
            d((0, 0, 2)) + d((0, 0, 1)) + d((2, 0, 0)) + d((1, 0, 0)) / np.tan(ph)
            + d((0, 2, 0)) / np.sin(ph) ** 2)
    _check_closed_form(M.VTX_BOX, M.VTX, box, closed)


def test_vertex_edge_operator_closed_form():
    """L^{v-e} u = -e^{zeta/2}(u_psipsi + u_thth + e^{2psi}(u_psipsi - 2u_psizeta
    + u_zetazeta + u_psi - u_zeta)) (eq 2.28 with L = -Lap)."""
    box = np.array([np.log(0.05), np.log(0.3), 0.1, 0.9, np.log(0.01), np.log(0.06)])

    def closed(d, y):
        ps, ze = y[0], y[2]
        return -np.exp(ze / 2) * (d((2, 0, 0)) + d((0, 2, 0)) + np.exp(2 * ps) * (
            d((2, 0, 0)) - 2 * d((1, 0, 1)) + d((0, 0, 2)) + d((1, 0, 0)) - d((0, 0, 1))))
    _check_closed_form(M.VE_BOX, M.VE, box, closed)


POLAR = [0, np.pi / 2, 3 * np.pi / 4, np.tan(np.pi / 6), 0.25, 0.0, 1.0, -1.0, 1.0, 0.5, 0, 0]
BILIN = [1, 0.0, 0.0, 1.0, 0.1, 0.05, 0.9, 0.95, 1.0, 0.5, 0, 0]


@pytest.mark.parametrize("chart,box,patch,region", [
    (M.COLUMN, [-1, 1, -1, 1, 0.0, 1.0], POLAR, M.REG),
    (M.COLUMN, [-1, 1, -1, 1, 0.2, 0.7], BILIN, M.REG),
    (M.VTX_PATCH, [-1, 1, -1, 1, np.log(0.1), np.log(0.5)], POLAR, M.VTX),
    (M.AFFINE, [0.1, 0.4, -0.2, 0.3, 1.0, 1.5], None, M.REG),
])
def test_chain_rule_laplacian_on_curved_maps(chart, box, patch, region):
    """Oracle coefficients applied to the lam-derivatives of u(x(lam)) give
    -Lap u(x) for a smooth u (pointwise, symbolic reference)."""
    mesh = _single(chart, np.array(box, float), patch, region)
    mesh.frame[0] = np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]], float)
    mesh.origin[0] = [0.1, -0.2, 0.05]
    disc = Discretization(mesh)
    v = disc.vol[0]
    X = sp.symbols("x0:3")
    u = sp.sin(X[0]) + X[1] ** 2 * X[2] + sp.exp(0.5 * X[2]) * X[0]
    lap = sum(sp.diff(u, xi, 2) for xi in X)
    l = charts._l
    chart_ = int(mesh.chart[0])
    ptype = int(mesh.patch[0][0]) if chart_ in (M.VTX_PATCH, M.COLUMN) else 0
    subs = dict(zip(charts._b, mesh.box[0]))
    subs.update(dict(zip(charts._p, mesh.patch[0])))
    xl = [sp.sympify(c).subs(subs) for c in charts._local_expr(chart_, ptype)]
    Rm = mesh.frame[0]
    xg = [mesh.origin[0][a] + sum(Rm[a, b] * xl[b] for b in range(3)) for a in range(3)]
    uhat = u.subs(dict(zip(X, xg)))
    rng = np.random.default_rng(1)
    for q in rng.choice(disc.m ** 3, 4, replace=False):
        lam_q = {}
        a, b, c = q % disc.m, (q // disc.m) % disc.m, q // disc.m ** 2
        lam_q = {l[0]: disc.xm[a], l[1]: disc.xm[b], l[2]: disc.xm[c]}
        Lu = 0.0
        for (o, _, _), cf in zip(SECOND, v["coef2"]):
            der = uhat
            for ax in range(3):
                if o[ax]:
                    der = sp.diff(der, l[ax], o[ax])
            Lu += cf[q] * float(der.subs(lam_q))
        for (o, _), cf in zip(FIRST, v["coef1"]):
            der = uhat
            for ax in range(3):
                if o[ax]:
                    der = sp.diff(der, l[ax], o[ax])
            Lu += cf[q] * float(der.subs(lam_q))
        xq = v["x"][q]
        ref = -float(lap.subs(dict(zip(X, xq))))
        assert abs(Lu - ref) < 1e-9 * max(1.0, abs(ref)), (q, Lu, ref)


@pytest.mark.parametrize("kind,fwd", [
    (M.VTX, lambda y: np.exp(y[2]) * np.array([np.sin(y[0]) * np.cos(y[1]),
                                               np.sin(y[0]) * np.sin(y[1]), np.cos(y[0])])),
    (M.VE, lambda y: np.array([np.exp(y[0] + y[2]) * np.cos(y[1]),
                               np.exp(y[0] + y[2]) * np.sin(y[1]), np.exp(y[2])])),
    (M.EDGE, lambda y: np.array([np.exp(y[0]) * np.cos(y[1]), np.exp(y[0]) * np.sin(y[1]), y[2]])),
])
def test_modified_jacobian_matches_forward_map(kind, fwd):
    """dx/dy from eq 2.3, 2.5, 2.8 against central differences of x(y)."""
    y = np.array([0.6, 2.1, -1.3])
    x = fwd(y)
    J = charts.modified_jacobian(kind, x[None, :])[0]
    h = 1e-6
    for k in range(3):
        dy = np.zeros(3)
        dy[k] = h
        np.testing.assert_allclose(J[:, k], (fwd(y + dy) - fwd(y - dy)) / (2 * h), rtol=1e-7, atol=1e-8)


# ------------------------------------------------ the functional and its solve
@pytest.fixture(scope="module")
def cube_w3():
    mesh = M.box_mesh(3, (2, 2, 1), (0, 0, 0), (1, 1, 0.5))
    disc = Discretization(mesh, Polynomial())
    return disc, disc.dense_X()


def test_normal_matrix_symmetric_positive_definite(cube_w3):
    disc, X = cube_w3
    assert np.abs(X - X.T).max() < 1e-13 * np.abs(X).max()
    assert np.linalg.eigvalsh(X).min() > 1e-8


def test_functional_is_the_quadratic_of_X_and_b(cube_w3):
    disc, X = cube_w3
    b = disc.rhs()
    U = np.random.default_rng(2).standard_normal(disc.ndof)
    R0 = disc.functional(np.zeros_like(U))
    assert abs(disc.functional(U) - R0 - (U @ X @ U - 2 * b @ U)) < 1e-9 * abs(U @ X @ U)


def test_polynomial_solution_reproduced(cube_w3):
    """u of degree <= W per direction is reproduced: R_h(U*) = 0."""
    disc, X = cube_w3
    b = disc.rhs()
    U = dense_solve(X, b)
    assert disc.functional(U) < 1e-18 * max(1.0, b @ U)
    assert h1_error(disc, U, Polynomial()) < 1e-10


def test_constant_solution_reproduced():
    mesh = M.box_mesh(2, (2, 1, 1), (0, 0, 0), (1, 0.5, 0.5))
    disc = Discretization(mesh, Constant(2.5))
    U = dense_solve(disc.dense_X(), disc.rhs())
    np.testing.assert_allclose(U, 2.5, rtol=1e-10)


def test_volume_term_exact_for_polynomial_data():
    """Affine elements, polynomial u and f: the (2W+1)^3 GLL sum is the exact integral."""
    W = 3
    mesh = M.box_mesh(W, (1, 1, 1), (0.2, -0.1, 0.3), (0.7, 0.5, 0.6))
    disc = Discretization(mesh, Polynomial())
    rng = np.random.default_rng(4)
    ue = rng.standard_normal((disc.n,) * 3)
    v = disc.vol[0]
    z = disc.volume_residual(ue, v, np.zeros(disc.m ** 3))
    xg, wg = np.polynomial.legendre.leggauss(W + 3)
    B = [gll.lagrange(disc.xn, xg, d) for d in range(3)]
    h = mesh.box[0][1::2] - mesh.box[0][0::2]
    from oracle.functional import tensor_apply
    lap = sum(tensor_apply(*[B[2 if a == k else 0] for a in range(3)], ue) * (2 / h[k]) ** 2
              for k in range(3))
    wq = np.einsum("a,b,c->abc", wg, wg, wg) * np.prod(h) / 8
    exact = (wq * lap ** 2).sum()
    assert abs(z @ z - exact) < 1e-11 * exact


def test_pcg_matches_dense_solve_config1():
    mesh = M.box_mesh(4, (2, 2, 2), (0, 0, 0), (1, 1, 1))
    disc = Discretization(mesh, SinProduct())
    b = disc.rhs()
    P = BlockPreconditioner(disc)
    u, it, hist = pcg(disc.apply_X, b, P.apply, 1e-12)
    X = disc.dense_X()
    ud = dense_solve(X, b)
    assert np.linalg.norm(u - ud) < 1e-10 * np.linalg.norm(ud)
    assert np.linalg.norm(b - X @ u) < 1e-11 * np.linalg.norm(b)
    assert 20 < it < 400


def test_error_decays_exponentially_on_cube():
    errs = []
    for W in (2, 4, 6):
        mesh = M.box_mesh(W, (2, 2, 2), (0, 0, 0), (1, 1, 1))
        disc = Discretization(mesh, SinProduct())
        P = BlockPreconditioner(disc)
        u, _, _ = pcg(disc.apply_X, disc.rhs(), P.apply, 1e-13)
        errs.append(h1_error(disc, u, SinProduct()))
    assert errs[0] > 20 * errs[1] > 400 * errs[2]


def test_table62_magnitudes():
    """Table 6.2 (Mesh 2 on (-1,1)^3): iterations and errors agree in magnitude."""
    gold = _golden("table6_2.txt")
    for W, _, its, err in gold[:3]:
        mesh = M.box_mesh(int(W), (2, 2, 2), (-1, -1, -1), (1, 1, 1))
        disc = Discretization(mesh, SinProduct())
        P = BlockPreconditioner(disc)
        u, it, _ = pcg(disc.apply_X, disc.rhs(), P.apply, 1e-8)
        e = 100 * h1_error(disc, u, SinProduct())
        assert 0.6 * its < it < 1.5 * its, (W, it, its)
        assert err / 10 < e < err * 1.5, (W, e, err)


def test_term_magnitude_apply_bounds_the_operator():
    """apply_X_abs(u) >= |X| |u| >= |X u| entry by entry (X assembled densely),
    and it equals |X| |u| on a single affine element whose operator entries
    are all of one sign per term chain (u >= 0 then gives |X u| only if no
    cancellation; the inequality chain is what the float bound uses)."""
    mesh = M.box_mesh(2, (2, 1, 1))
    disc = Discretization(mesh, Polynomial())
    X = disc.dense_X()
    u = np.random.default_rng(3).standard_normal(disc.ndof)
    A = disc.apply_X_abs(u)
    assert (A >= np.abs(X) @ np.abs(u) * (1 - 1e-12)).all()
    assert (np.abs(X) @ np.abs(u) >= np.abs(X @ u) * (1 - 1e-12)).all()
    # scaling: homogeneous of degree one in |u|
    np.testing.assert_allclose(disc.apply_X_abs(3 * u), 3 * A, rtol=1e-14)
