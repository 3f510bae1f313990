"""X = A^T M A assembled term by term against the matrix-free X (Sec. 5.3).

The oracle's operator apply runs every term's transposed contractions (the
adjoint of the volume fields, the transposed traces and face interpolation).
Here the normal-equation matrix is assembled instead from the forward maps
alone: for every unit vector the weighted volume residuals z_q and the face
quantities of every term give the columns of A_t, the face weights M_t
(alpha Om(x)Om + beta K(x)Om + gamma Om(x)K) are applied to them, and
X = sum_t A_t^T M_t A_t by dense products.  A wrong transpose anywhere in the
matrix-free path (a transposed operand, a dropped term, a sign) makes the two
differ.  The same forward maps pin the functional: R(U) = U^T X U - 2 b^T U
+ R(0), for the right-hand side b of the data (Dirichlet, Neumann, source).

Cases: a box with a Neumann face and the general operator of eq 2.2 (all ten
fields), and the Fichera mesh (every face kind of the singular regions,
corner elements)."""
import numpy as np
import pytest

from workloads import mesh as M
from workloads.fichera import fichera_mesh
from workloads.problems import GeneralElliptic, RhoPower
from oracle.functional import Discretization


def _columns(disc, e):
    """The unknowns an element's function depends on."""
    mesh = disc.mesh
    if mesh.kind[e] == M.REAL:
        return range(disc.offset[e], disc.offset[e] + disc.n ** 3)
    c = disc.n_real_dof + mesh.cdof[e]
    return range(c, c + 1) if mesh.kind[e] == M.CORNER_CONST else range(c, c + disc.n)


def _assembled(disc):
    N = disc.ndof
    X = np.zeros((N, N))
    U = np.zeros(N)
    # a term's columns are zero outside the unknowns of its elements
    for v in disc.vol:
        cols = list(_columns(disc, v["e"]))
        A = np.zeros((disc.m ** 3, len(cols)))
        for i, j in enumerate(cols):
            U[j] = 1
            A[:, i] = disc.volume_residual(disc.element_values(U, v["e"]), v)
            U[j] = 0
        X[np.ix_(cols, cols)] += A.T @ A
    for T in disc.faces:
        cols = list(_columns(disc, T.eA)) + (list(_columns(disc, T.eB)) if T.eB >= 0 else [])
        As = [np.zeros((disc.m ** 2, len(cols))) for _ in T.quants]
        for i, j in enumerate(cols):
            U[j] = 1
            for k, q in enumerate(disc._face_quantities(T, U)):
                As[k][:, i] = q
            U[j] = 0
        for A, (_, _, wts, _) in zip(As, T.quants):
            MA = np.stack([disc.face_weight(A[:, i], wts) for i in range(len(cols))], axis=1)
            X[np.ix_(cols, cols)] += A.T @ MA
    return X


CASES = {
    # Neumann on x3 = hi (the conormal of the general a) and every field of L
    "box_general_neumann_w2": lambda: (M.box_mesh(2, (2, 1, 1), (0.1, 0.2, 0.0), (0.9, 0.7, 0.6),
                                                  neumann=((2, 1),)), GeneralElliptic()),
    "fichera_n1w1": lambda: (fichera_mesh(N=1, W=1), RhoPower()),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_matrix_free_X_equals_term_by_term_assembly(name):
    mesh, prob = CASES[name]()
    disc = Discretization(mesh, prob)
    Xa = _assembled(disc)
    scale = np.abs(Xa).max()
    assert np.abs(Xa - Xa.T).max() < 1e-12 * scale
    rng = np.random.default_rng(7)
    for _ in range(3):
        U = rng.standard_normal(disc.ndof)
        ref = Xa @ U
        assert np.abs(disc.apply_X(U) - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("name", sorted(CASES))
def test_functional_is_the_quadratic_of_X_and_b(name):
    mesh, prob = CASES[name]()
    disc = Discretization(mesh, prob)
    rng = np.random.default_rng(8)
    U = rng.standard_normal(disc.ndof)
    R0 = disc.functional(np.zeros(disc.ndof))
    R = disc.functional(U)
    quad = U @ disc.apply_X(U) - 2 * disc.rhs() @ U + R0
    assert abs(R - quad) < 1e-10 * max(abs(R), abs(R0))
