"""Pins of the oracle on the Fichera geometric mesh (modified coordinates).

* every face of the mesh conforms: both sides map the face grid to the same
  physical points (checked while the oracle builds its face terms);
* the constant function is the exact minimiser for u = const data: the
  functional vanishes at it and X c = b (thesis: the least-squares functional
  is zero exactly at the solution when it is representable);
* X is symmetric and positive on random vectors;
* the manufactured data f = -Laplace(u) matches a finite-difference Laplacian;
* the element counts follow the geometric-mesh formulas of Sec. 2.3.
"""
import numpy as np
import pytest

from workloads import mesh as M
from workloads.fichera import fichera_mesh
from workloads.problems import Constant, RhoPower
from oracle.functional import Discretization


@pytest.fixture(scope="module")
def small():
    mesh = fichera_mesh(N=1, W=2)
    return mesh, Discretization(mesh, Constant(1.7))


def test_element_counts_follow_geometric_mesh():
    for N in (1, 2, 3):
        mesh = fichera_mesh(N=N, W=2)
        I = 6
        assert (mesh.region == M.VE).sum() == 3 * I * (N + 1) ** 2          # N_{v-e} = I (N+1)^2
        assert (mesh.region == M.EDGE).sum() == 3 * I * 1 * (N + 1)         # N_e = I J_e (N+1)
        assert (mesh.region == M.VTX).sum() == 30 * (N + 1)                 # N_v = I_v (N+1)
        assert ((mesh.region == M.VTX) & (mesh.kind == M.REAL)).sum() == 30 * N


def test_faces_conform_and_boundary_is_closed(small):
    mesh, disc = small
    # every finite face of a real element is either paired or on the boundary
    for e in mesh.real_elements():
        for f in range(6):
            assert mesh.bc[e, f] in (M.INTERIOR, M.DIRICHLET)
    assert len(disc.faces) > 0


def test_constant_is_the_minimiser(small):
    mesh, disc = small
    c = np.full(disc.ndof, 1.7)
    assert disc.functional(c) < 1e-20
    b = disc.rhs()
    assert np.linalg.norm(disc.apply_X(c) - b) < 1e-11 * np.linalg.norm(b)


def test_symmetric_positive(small):
    mesh, disc = small
    rng = np.random.default_rng(0)
    u, v = rng.standard_normal((2, disc.ndof))
    Xu, Xv = disc.apply_X(u), disc.apply_X(v)
    assert abs(v @ Xu - u @ Xv) < 1e-12 * abs(v @ Xu)
    assert u @ Xu > 0 and v @ Xv > 0


def test_manufactured_source_matches_fd_laplacian():
    p = RhoPower()
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, (20, 3))
    x = x[np.linalg.norm(x, axis=1) > 0.2]
    h = 1e-4
    lap = sum((p.u(x + h * np.eye(3)[k]) - 2 * p.u(x) + p.u(x - h * np.eye(3)[k])) / h ** 2 for k in range(3))
    np.testing.assert_allclose(-lap, p.f(x), rtol=1e-5, atol=1e-5)
    g = np.stack([(p.u(x + h * np.eye(3)[k]) - p.u(x - h * np.eye(3)[k])) / (2 * h) for k in range(3)], -1)
    np.testing.assert_allclose(g, p.grad_u(x), rtol=1e-7, atol=1e-7)


def test_restricted_oracle_rows_are_exact():
    """The oracle restricted to a few elements reproduces those elements' rows
    of X u and b of the full oracle (the basis of the full-size sampled
    parity checks)."""
    mesh = fichera_mesh(N=1, W=2)
    full = Discretization(mesh, RhoPower())
    rng = np.random.default_rng(4)
    S = [int(e) for e in rng.choice(full.real, 5, replace=False)]
    part = Discretization(mesh, RhoPower(), only=S)
    u = rng.standard_normal(full.ndof)
    Xf, Xp = full.apply_X(u), part.apply_X(u)
    bf, bp = full.rhs(), part.rhs()
    n3 = full.n ** 3
    for e in S:
        o = full.offset[e]
        np.testing.assert_allclose(Xp[o:o + n3], Xf[o:o + n3], rtol=0, atol=1e-12 * np.abs(Xf).max())
        np.testing.assert_allclose(bp[o:o + n3], bf[o:o + n3], rtol=0, atol=1e-12 * np.abs(bf).max())
