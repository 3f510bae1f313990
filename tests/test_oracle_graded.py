"""Pins of the oracle's layer-graded degrees (Sec. 2.3: W_l = [mu_1 i],
V_q = [mu_2 k]; the graded space is a subspace of the uniform-W space):

* the 1D embedding reproduces degree-w polynomials exactly (brute force at
  the fine nodes), and the projector built from it is the orthogonal
  projector onto them (idempotent, symmetric, rank w + 1, fixes degree w,
  moves degree w + 1);
* a solution of degree (3, 2, 1) in (x, y, z) is reproduced exactly on a box
  mesh with degrees (3, 2, 1) and not with (1, 2, 3): the direction order of
  the embedding;
* uniform degrees W reproduce the uniform system;
* the graded minimiser lies between the uniform minimisers of the lowest
  and the highest degree (the spaces are nested);
* the degree rule of Sec. 2.3 on the Fichera mesh;
* both graded preconditioners map into the graded space, are symmetric and
  the element-block one inverts the projected block there."""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from workloads import mesh as M
from workloads import fichera, grading
from workloads.problems import Polynomial, SinProduct
from oracle import gll
from oracle.functional import Discretization
from oracle.graded import (GradedSystem, GradedSeparablePreconditioner, GradedElementBlockPreconditioner,
                           embedding_1d, projector_1d)
from oracle.precond import kron3, element_blocks
from oracle.solve import h1_error


@pytest.mark.parametrize("W,w", [(4, 1), (4, 2), (6, 3), (8, 5), (10, 10)])
def test_embedding_reproduces_low_degree_polynomials(W, w):
    rng = np.random.default_rng(W * 10 + w)
    c = rng.standard_normal(w + 1)                     # monomial coefficients
    poly = lambda x: sum(ck * x ** k for k, ck in enumerate(c))
    xw, _ = gll.gll(w + 1)
    xW, _ = gll.gll(W + 1)
    assert np.allclose(embedding_1d(W, w) @ poly(xw), poly(xW), atol=1e-12, rtol=0)


@pytest.mark.parametrize("W,w", [(4, 1), (6, 3), (8, 7)])
def test_projector_is_the_orthogonal_projector_onto_degree_w(W, w):
    Q = projector_1d(W, w)
    assert np.abs(Q @ Q - Q).max() < 1e-13
    assert np.abs(Q - Q.T).max() < 1e-13
    assert abs(np.trace(Q) - (w + 1)) < 1e-12
    xW, _ = gll.gll(W + 1)
    for k in range(w + 1):
        v = npleg.legval(xW, np.eye(W + 1)[k])
        assert np.abs(Q @ v - v).max() < 1e-12
    v = xW ** (w + 1)
    assert np.abs(Q @ v - v).max() > 1e-3


def test_anisotropic_degrees_reproduce_a_matching_polynomial_only():
    W = 4
    mesh = M.box_mesh(W, (2, 1, 1), (0.0, 0.0, 0.0), (1.0, 0.7, 0.6))
    P = Polynomial()                                  # degree 3 in x, 2 in y, 1 in z
    disc = Discretization(mesh, P)
    right = GradedSystem(disc, np.tile([3, 2, 1], (mesh.E, 1)))
    wrong = GradedSystem(disc, np.tile([1, 2, 3], (mesh.E, 1)))
    e_right = h1_error(disc, right.solve(), P)
    e_wrong = h1_error(disc, wrong.solve(), P)
    assert e_right < 1e-11
    assert e_wrong > 1e-3
    assert right.ndof_graded == mesh.E * 4 * 3 * 2


def test_uniform_degrees_give_the_uniform_system():
    W = 3
    mesh = fichera.fichera_mesh(N=1, W=W)
    disc = Discretization(mesh, SinProduct())
    gs = GradedSystem(disc, np.full((mesh.E, 3), W))
    U = np.random.default_rng(3).standard_normal(disc.ndof)
    assert np.allclose(gs.apply_X(U), disc.apply_X(U), rtol=0, atol=1e-12 * np.abs(disc.apply_X(U)).max())
    assert np.allclose(gs.project(U), U, rtol=0, atol=1e-13)
    assert gs.ndof_graded == disc.ndof


def test_graded_minimiser_between_nested_spaces():
    W = 3
    mesh = M.box_mesh(W, (2, 2, 1))
    P = SinProduct()
    disc = Discretization(mesh, P)
    deg = np.array([[1, 2, 3], [2, 2, 2], [3, 1, 2], [3, 3, 3]])
    R = {}
    for name, d in (("low", np.ones((4, 3), int)), ("graded", deg), ("high", np.full((4, 3), W))):
        gs = GradedSystem(disc, d)
        R[name] = disc.functional(gs.solve())
    assert R["high"] < R["graded"] < R["low"]


def test_layer_degrees_follow_the_layer_rule():
    N, W = 3, 4
    mesh = fichera.fichera_mesh(N=N, W=W)
    deg = grading.layer_degrees(mesh, 1.0, 2.0)
    for e in mesh.real_elements():
        i, k = mesh.layer[e]
        r = mesh.region[e]
        if r == M.REG:
            assert tuple(deg[e]) == (W, W, W)
        elif r == M.VTX:
            assert tuple(deg[e]) == (i, i, i)
        elif r == M.EDGE:
            assert tuple(deg[e]) == (i, i, W)
        else:
            assert tuple(deg[e]) == (i, i, min(W, 2 * k))
    # every layer index of the geometric mesh is used
    assert set(mesh.layer[mesh.region == M.VTX][:, 0]) >= {1, 2, 3}
    assert grading.graded_dof(mesh, deg) < mesh.ndof()


def test_graded_preconditioners_act_on_the_graded_space():
    W = 3
    mesh = M.box_mesh(W, (2, 2, 1))
    disc = Discretization(mesh, SinProduct())
    deg = np.array([[1, 2, 3], [3, 3, 2], [2, 1, 1], [3, 3, 3]])
    gs = GradedSystem(disc, deg)
    rng = np.random.default_rng(5)
    R1 = gs.project(rng.standard_normal(disc.ndof))
    R2 = gs.project(rng.standard_normal(disc.ndof))
    for B in (GradedSeparablePreconditioner(gs), GradedElementBlockPreconditioner(gs)):
        Z1, Z2 = B.apply(R1), B.apply(R2)
        assert np.abs(gs.project(Z1) - Z1).max() < 1e-10 * np.abs(Z1).max()
        assert abs(R2 @ Z1 - R1 @ Z2) < 1e-10 * abs(R1 @ Z1)
        assert R1 @ Z1 > 0
    # element-block form: exact inverse of the projected block on the graded space
    B = GradedElementBlockPreconditioner(gs)
    blocks, _ = element_blocks(disc)
    n3 = disc.n ** 3
    e = disc.real[0]
    Q = kron3(*gs.Q[e])
    v = Q @ rng.standard_normal(n3)
    R = np.zeros(disc.ndof)
    o = disc.offset[e]
    R[o:o + n3] = Q @ blocks[0] @ Q @ v
    assert np.abs(B.apply(R)[o:o + n3] - v).max() < 1e-9 * np.abs(v).max()
