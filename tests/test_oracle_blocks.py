"""Pins of the oracle's element-block preconditioner (exact diagonal blocks
of X): the blocks are checked against X applied to single unit vectors and
against the densely assembled X, independently of the colouring that the
oracle uses to assemble them with fewer applies."""
import numpy as np
import pytest

from workloads import mesh as M
from workloads.fichera import fichera_mesh
from workloads.problems import Polynomial, RhoPower
from oracle.functional import Discretization
from oracle.precond import BlockPreconditioner, ElementBlockPreconditioner, element_blocks
from oracle.solve import pcg


@pytest.fixture(scope="module")
def fich():
    mesh = fichera_mesh(N=1, W=1)
    disc = Discretization(mesh, RhoPower())
    return disc, element_blocks(disc)


def test_blocks_equal_dense_diagonal_blocks():
    mesh = M.box_mesh(2, (2, 2, 1))
    disc = Discretization(mesh, Polynomial())
    X = disc.dense_X()
    blocks, Xcc = element_blocks(disc)
    n3 = disc.n ** 3
    for i, e in enumerate(disc.real):
        o = disc.offset[e]
        np.testing.assert_allclose(blocks[i], X[o:o + n3, o:o + n3], rtol=0, atol=1e-12 * np.abs(X).max())
    assert Xcc.size == 0


def test_blocks_are_columns_of_X(fich):
    disc, (blocks, Xcc) = fich
    n3 = disc.n ** 3
    rng = np.random.default_rng(5)
    for _ in range(6):
        i = int(rng.integers(len(disc.real)))
        j = int(rng.integers(n3))
        e = disc.real[i]
        v = np.zeros(disc.ndof)
        v[disc.offset[e] + j] = 1.0
        y = disc.apply_X(v)
        o = disc.offset[e]
        np.testing.assert_allclose(blocks[i][:, j], y[o:o + n3], rtol=0, atol=1e-13 * np.abs(y).max())
    nc = disc.ndof - disc.n_real_dof
    assert nc > 0
    for j in rng.choice(nc, 3, replace=False):
        v = np.zeros(disc.ndof)
        v[disc.n_real_dof + j] = 1.0
        y = disc.apply_X(v)[disc.n_real_dof:]
        np.testing.assert_allclose(Xcc[:, j], y, rtol=0, atol=1e-13 * np.abs(y).max())


def test_blocks_symmetric_positive_definite(fich):
    disc, (blocks, Xcc) = fich
    for B in blocks + [Xcc]:
        assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
        assert np.linalg.eigvalsh(B).min() > 0


def test_pcg_solution_independent_of_preconditioner(fich):
    disc, _ = fich
    b = disc.rhs()
    u_sep, it_sep, _ = pcg(disc.apply_X, b, BlockPreconditioner(disc).apply, 1e-12, 20000)
    u_blk, it_blk, _ = pcg(disc.apply_X, b, ElementBlockPreconditioner(disc).apply, 1e-12, 20000)
    assert np.linalg.norm(u_blk - u_sep) <= 1e-9 * np.linalg.norm(u_sep)
    assert it_blk < it_sep


def test_equal_blocks_separate_cleanly(fich):
    """Symmetry images of an element (the theta-sectors, the three edges of the
    geometric mesh) have equal diagonal blocks up to rounding, and distinct
    blocks differ by a margin far above rounding: a relative tolerance of 1e-9
    finds the same classes as exact arithmetic would, which is what lets the
    library store each class's block once."""
    disc, (blocks, Xcc) = fich
    reps, count, within = [], [], 0.0
    for B in blocks:
        scale = np.abs(B).max()
        for i, R in enumerate(reps):
            d = np.abs(R - B).max() / scale
            if d <= 1e-9:
                count[i] += 1
                within = max(within, d)
                break
        else:
            reps.append(B)
            count.append(1)
    assert within < 1e-13, within
    gap = min(np.abs(reps[i] - reps[j]).max() / np.abs(reps[i]).max()
              for i in range(len(reps)) for j in range(i))
    assert gap > 1e-3, gap
    # the mesh's symmetry: far fewer distinct blocks than elements
    assert len(reps) < len(blocks) // 2 and max(count) >= 3, (len(reps), len(blocks), max(count))


def _reversal(n, c):
    """Local index map f of an element with the lambda axes of the bits of c reversed."""
    idx = np.arange(n ** 3).reshape((n, n, n), order="F")
    for d in range(3):
        if c & (1 << d):
            idx = np.flip(idx, d)
    return idx.ravel(order="F")


def test_reversed_blocks_separate_cleanly(fich):
    """Mirror images of an element across a theta-plane (sector j and its
    image across the mesh's symmetry planes) have blocks equal to rounding up
    to a reversal of lambda axes, X_ee[a][b] = X_uu[f(a)][f(b)], and blocks of
    different classes stay far apart under every reversal: the library's
    1e-9 tolerance again finds the exact classes, now fewer of them."""
    disc, (blocks, _) = fich
    n = disc.n
    fs = [_reversal(n, c) for c in range(8)]
    reps, within = [], 0.0
    for B in blocks:
        scale = np.abs(B).max()
        hit = False
        for R in reps:
            d = min(np.abs(B - R[np.ix_(f, f)]).max() for f in fs) / scale
            if d <= 1e-9:
                within = max(within, d)
                hit = True
                break
        if not hit:
            reps.append(B)
    assert within < 1e-13, within
    gap = min(min(np.abs(reps[i] - reps[j][np.ix_(f, f)]).max() for f in fs) / np.abs(reps[i]).max()
              for i in range(len(reps)) for j in range(i))
    assert gap > 1e-3, gap
    plain = []
    for B in blocks:
        if not any(np.abs(B - R).max() <= 1e-9 * np.abs(B).max() for R in plain):
            plain.append(B)
    assert len(reps) < len(plain), (len(reps), len(plain))
