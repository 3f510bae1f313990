"""Pins of the conforming correction (Appendix C.1): it leaves conforming
functions alone, removes a jump confined to the inside of one face exactly
(half from each side), and keeps the solution's H^1 error at its size."""
import numpy as np
import pytest

from workloads import mesh as M
from workloads.problems import SinProduct
from oracle.functional import Discretization
from oracle.precond import BlockPreconditioner
from oracle.solve import pcg, h1_error
from oracle.conform import correction, face_jumps


def _interpolant(disc, fun):
    n = disc.n
    A, B, C = np.meshgrid(disc.xn, disc.xn, disc.xn, indexing="ij")
    lam = np.stack([A.ravel(order="F"), B.ravel(order="F"), C.ravel(order="F")], -1)
    U = np.zeros(disc.ndof)
    for e in disc.real:
        o = disc.offset[e]
        U[o:o + n ** 3] = fun(M.chart_points(disc.mesh, e, lam))
    return U


def test_conforming_function_is_unchanged():
    mesh = M.box_mesh(3, (2, 2, 1), (0.0, 0.0, 0.0), (1.0, 0.7, 0.4))
    disc = Discretization(mesh)
    poly = lambda x: 1 + x[..., 0] ** 3 - 2 * x[..., 0] * x[..., 1] + x[..., 2] ** 2 * x[..., 1]
    U = _interpolant(disc, poly)
    assert face_jumps(disc, U) < 1e-13
    np.testing.assert_allclose(correction(disc, U), U, rtol=0, atol=1e-14)


def test_jump_inside_one_face_is_removed_half_from_each_side():
    mesh = M.box_mesh(3, (2, 1, 1))
    disc = Discretization(mesh)
    U = _interpolant(disc, lambda x: np.cos(x[..., 0]) + x[..., 1] * x[..., 2])
    # a bubble on element 0's face lam_1 = +1 that vanishes on the face's edges
    n = disc.n
    x = disc.xn
    bub = np.einsum("i,j,k->ijk", (1 + x) / 2, 1 - x ** 2, 1 - x ** 2)
    V = U.copy()
    o = disc.offset[0]
    V[o:o + n ** 3] += bub.reshape(-1, order="F")
    assert face_jumps(disc, V) > 0.1
    Vc = correction(disc, V)
    assert face_jumps(disc, Vc) < 1e-13
    # element 0 takes back half of the bubble, element 1 gains the other half
    d0 = (Vc - V)[o:o + n ** 3].reshape((n, n, n), order="F")
    np.testing.assert_allclose(d0, -0.5 * bub, atol=1e-14)
    o1 = disc.offset[1]
    d1 = (Vc - V)[o1:o1 + n ** 3].reshape((n, n, n), order="F")
    np.testing.assert_allclose(d1, 0.5 * np.flip(bub, 0), atol=1e-14)


@pytest.mark.parametrize("W", [3, 5])
def test_corrected_solution_keeps_its_accuracy(W):
    mesh = M.box_mesh(W, (2, 2, 2), (0, 0, 0), (1, 1, 1))
    P = SinProduct()
    disc = Discretization(mesh, P)
    u, _, _ = pcg(disc.apply_X, disc.rhs(), BlockPreconditioner(disc).apply, 1e-12, 20000)
    uc = correction(disc, u)
    e0, e1 = h1_error(disc, u, P), h1_error(disc, uc, P)
    assert face_jumps(disc, uc) < face_jumps(disc, u)
    assert e1 < 2.0 * e0, (e0, e1)
