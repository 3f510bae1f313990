"""Mixed precision through the C ABI: the float operator (sem_residual_prec)
against the FP64 oracle, and the mixed-precision PCG with FP64 residual
replacement (sem_pcg_solve_mixed) against the FP64 oracle solution.

The float operator is an addition of this library (the thesis computes in
double); the bar for its solve is the FP64 solution to 1e-8 relative.
"""
import numpy as np
import pytest

from workloads import mesh as M
from workloads.fichera import fichera_mesh
from workloads.problems import Constant, RhoPower, SinProduct
from oracle.functional import Discretization
from oracle.precond import BlockPreconditioner
from oracle.solve import pcg
from tests.gpu_common import RTOL_FP32_APPLY, RTOL_MIXED, rand_vec, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

CASES = {
    "cube_w4": lambda: (M.box_mesh(4, (2, 2, 2), (0, 0, 0), (1, 1, 1)), SinProduct()),
    "box_w9": lambda: (M.box_mesh(9, (2, 1, 1), (0, 0, 0), (1, 0.6, 0.8)), SinProduct()),
    "fichera_n1w3": lambda: (fichera_mesh(N=1, W=3), RhoPower()),
    "fichera_n2w2": lambda: (fichera_mesh(N=2, W=2), RhoPower()),
}


# the float operator needs kappa(W^-1 X) x float eps well below 1; on the
# Fichera meshes that holds with the element-block preconditioner
PRECOND = {"cube_w4": "separable", "box_w9": "separable", "fichera_n1w3": "block", "fichera_n2w2": "block"}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    import torch
    from paper_1110_2316_amd import setup_problem
    print("mixed case %s" % request.param, flush=True)
    mesh, prob = CASES[request.param]()
    disc = Discretization(mesh, prob)
    ctx = setup_problem(mesh, prob)
    ctx.set_preconditioner(PRECOND[request.param])
    torch.cuda.synchronize()
    return mesh, disc, ctx


def test_float_operator_apply(case):
    import torch
    mesh, disc, ctx = case
    u = rand_vec(disc.ndof, 31)
    r = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
    ctx.residual(to_dev(u), r, precision="mixed")
    ref = disc.apply_X(u)
    err = rel(to_host(r), ref)
    assert err < RTOL_FP32_APPLY
    # and it is a float computation, not the FP64 one
    r64 = torch.zeros_like(r)
    ctx.residual(to_dev(u), r64)
    assert rel(to_host(r64), ref) < 1e-12
    assert err > 1e-12


@pytest.mark.parametrize("tile", [0, 1, 2])
def test_float_operator_entrywise_bound(case, tile):
    """Entry by entry, the float operator errs by at most (3n + 3m + 20) float
    unit roundoffs times the sum of the moduli of the terms of that entry
    (the oracle's |A|^T |M| |A| |u|): data rounded to float (one roundoff
    per value) and sums of at most n terms in each of the three forward
    stages, m terms in each transposed stage, ten fields pointwise; every
    tile, every element and face kind of the case."""
    import torch
    mesh, disc, ctx = case
    u = rand_vec(disc.ndof, 32)
    ref = disc.apply_X(u)
    bound = (3 * disc.n + 3 * disc.m + 20) * np.finfo(np.float32).eps / 2 * disc.apply_X_abs(u)
    ctx.set_tile(tile, "mixed")
    try:
        r = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
        ctx.residual(to_dev(u), r, precision="mixed")
    finally:
        ctx.set_tile(0, "mixed")
    err = np.abs(to_host(r) - ref)
    worst = float((err / bound).max())
    print("mixed: tile %d, worst entry error / bound = %.3f" % (tile, worst), flush=True)
    assert worst <= 1.0


def test_float_inhomogeneous_residual(case):
    import torch
    mesh, disc, ctx = case
    b = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
    ctx.rhs(b)
    u = rand_vec(disc.ndof, 4)
    r = torch.zeros_like(b)
    ctx.residual(to_dev(u), r, homogeneous=False, precision="mixed")
    ref = disc.apply_X(u) - disc.rhs()
    assert rel(to_host(r), ref) < RTOL_FP32_APPLY


def test_mixed_solve_matches_fp64_oracle(case):
    """Cube / box cases: against the oracle's own PCG solution.  Fichera cases
    (thousands of oracle iterations): against the oracle's normal equations;
    their oracle-solution parity is in the element-block tests on smaller
    Fichera meshes."""
    import torch
    mesh, disc, ctx = case
    b = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
    ctx.rhs(b)
    u = torch.zeros_like(b)
    info = ctx.pcg_solve(b, u, rtol=1e-12, maxit=20000, precision="mixed")
    got = to_host(u)
    if mesh.n_corner_dof == 0:
        P = BlockPreconditioner(disc)
        uref, _, _ = pcg(disc.apply_X, disc.rhs(), P.apply, 1e-13)
        assert rel(got, uref) < RTOL_MIXED
    # the stopping test is on the true FP64 residual: recompute it in the oracle
    bo = disc.rhs()
    assert np.linalg.norm(bo - disc.apply_X(got)) <= 1.5e-12 * np.linalg.norm(bo)
    assert info["status"] == 0 and info["rel_residual"] <= 1e-12
    assert info["outer"] >= 1


def test_mixed_and_fp64_solves_agree(case):
    import torch
    mesh, disc, ctx = case
    b = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
    ctx.rhs(b)
    u64 = torch.zeros_like(b)
    i64 = ctx.pcg_solve(b, u64, rtol=1e-12, maxit=20000)
    umx = torch.zeros_like(b)
    imx = ctx.pcg_solve(b, umx, rtol=1e-12, maxit=20000, precision="mixed")
    assert rel(to_host(umx), to_host(u64)) < RTOL_MIXED
    print("iterations fp64 %d mixed %d (%d replacements)" % (i64["iterations"], imx["iterations"], imx["outer"]))


def test_mixed_below_attainable_accuracy_stops_early():
    """rtol far below what double can reach: the solver escalates to FP64,
    sees the true residual stop improving and returns ENOCONV long before maxit."""
    import torch
    from paper_1110_2316_amd import setup_problem
    mesh = M.box_mesh(4, (2, 2, 2), (0, 0, 0), (1, 1, 1))
    ctx = setup_problem(mesh, SinProduct())
    b = torch.zeros(ctx.ndof, dtype=torch.float64, device="cuda")
    ctx.rhs(b)
    u = torch.zeros_like(b)
    info = ctx.pcg_solve(b, u, rtol=1e-20, maxit=20000, raise_on_fail=False, precision="mixed")
    assert info["status"] == -4 and info["iterations"] < 5000
    # far below the float operator's floor (about 1e-7): the FP64 phase ran
    assert info["rel_residual"] < 1e-10


def test_mixed_maxit_reports_no_convergence():
    import torch
    from paper_1110_2316_amd import setup_problem
    mesh = M.box_mesh(3, (2, 1, 1))
    ctx = setup_problem(mesh, SinProduct())
    b = torch.zeros(ctx.ndof, dtype=torch.float64, device="cuda")
    ctx.rhs(b)
    u = torch.zeros_like(b)
    info = ctx.pcg_solve(b, u, rtol=1e-14, maxit=5, raise_on_fail=False, precision="mixed")
    assert info["status"] == -4 and info["iterations"] == 5


def test_mixed_constant_reproduced_on_fichera():
    import torch
    from paper_1110_2316_amd import setup_problem
    mesh = fichera_mesh(N=1, W=3)
    ctx = setup_problem(mesh, Constant(1.7))
    ctx.set_preconditioner("block")
    b = torch.zeros(ctx.ndof, dtype=torch.float64, device="cuda")
    ctx.rhs(b)
    u = torch.zeros_like(b)
    ctx.pcg_solve(b, u, rtol=1e-11, maxit=20000, precision="mixed")
    assert np.abs(to_host(u) - 1.7).max() < 1e-8
