"""Parity of the HIP library (through its C ABI) with the FP64 oracle.

Every case compares element by element on the same seeded inputs:
X u (sem_residual), W^-1 r (sem_precond), b (sem_rhs), the PCG solution
(sem_pcg_solve) and the relative H^1 error (sem_error).
"""
import numpy as np
import pytest

from workloads import mesh as M
from workloads.problems import SinProduct, Polynomial
from oracle.functional import Discretization
from oracle.precond import BlockPreconditioner, element_block
from oracle.solve import pcg, h1_error
from tests.gpu_common import RTOL_APPLY, RTOL_SOLVE, rand_vec, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

CASES = [
    # (W, nel, lo, hi, problem)  -- config 1 first, then ragged / skewed boxes
    (4, (2, 2, 2), (0, 0, 0), (1, 1, 1), SinProduct()),
    (2, (3, 2, 1), (-1, 0, 0.5), (1, 0.7, 1.1), Polynomial()),
    (3, (1, 3, 2), (0.2, -1, 0), (0.9, 0.5, 1.3), Polynomial()),
    (5, (2, 1, 3), (0, 0, 0), (1, 0.5, 1.5), SinProduct()),
    (6, (2, 2, 1), (-1, -1, -1), (1, 1, 0), SinProduct()),
    (7, (1, 2, 2), (0, 0, 0), (0.5, 1, 1), SinProduct()),
    # degrees whose element kernel runs the lam1-slab LDS layout
    (8, (2, 1, 1), (0, 0, 0), (1, 0.6, 0.8), SinProduct()),
    (9, (1, 1, 2), (-0.5, 0, 0), (0.5, 1, 1.4), Polynomial()),
    (10, (1, 2, 1), (0, 0, 0), (1, 1, 0.5), SinProduct()),
    (11, (2, 1, 1), (0, -1, 0), (1.2, 0, 0.9), SinProduct()),
    (12, (1, 1, 2), (0, 0, 0), (1, 1, 1), SinProduct()),
]


def _pair(case):
    import torch
    from paper_1110_2316_amd import setup_problem
    W, nel, lo, hi, prob = case
    mesh = M.box_mesh(W, nel, lo, hi)
    print("case W=%d nel=%s" % (W, nel), flush=True)
    disc = Discretization(mesh, prob)
    ctx = setup_problem(mesh, prob)
    torch.cuda.synchronize()
    return mesh, disc, ctx, prob


@pytest.fixture(scope="module", params=range(len(CASES)), ids=lambda i: "W%d" % CASES[i][0])
def pair(request):
    return _pair(CASES[request.param])


def test_ndof_matches(pair):
    mesh, disc, ctx, _ = pair
    assert ctx.ndof == disc.ndof == mesh.ndof()


def test_operator_apply(pair):
    import torch
    mesh, disc, ctx, _ = pair
    u = rand_vec(disc.ndof, 11)
    r = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
    ctx.residual(to_dev(u), r, homogeneous=True)
    torch.cuda.synchronize()
    ref = disc.apply_X(u)
    got = to_host(r)
    assert rel(got, ref) < RTOL_APPLY
    assert np.abs(got - ref).max() < RTOL_APPLY * np.abs(ref).max()


def test_operator_apply_is_deterministic(pair):
    import torch
    mesh, disc, ctx, _ = pair
    u = to_dev(rand_vec(disc.ndof, 5))
    outs = []
    for _ in range(2):
        r = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
        ctx.residual(u, r)
        outs.append(to_host(r))
    assert np.array_equal(outs[0], outs[1])


def test_rhs(pair):
    import torch
    mesh, disc, ctx, _ = pair
    b = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
    ctx.rhs(b)
    torch.cuda.synchronize()
    ref = disc.rhs()
    assert rel(to_host(b), ref) < RTOL_APPLY


def test_inhomogeneous_residual(pair):
    import torch
    mesh, disc, ctx, _ = pair
    b = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
    ctx.rhs(b)
    u = rand_vec(disc.ndof, 3)
    r = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
    ctx.residual(to_dev(u), r, homogeneous=False)
    ref = disc.apply_X(u) - disc.rhs()
    assert rel(to_host(r), ref) < RTOL_APPLY


def test_preconditioner(pair):
    import torch
    mesh, disc, ctx, _ = pair
    P = BlockPreconditioner(disc)
    rv = rand_vec(disc.ndof, 7)
    z = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
    ctx.precond(to_dev(rv), z)
    torch.cuda.synchronize()
    # the oracle solves with a Cholesky factor, the library through the
    # separable eigenbasis: they agree to the block's conditioning times eps
    kappa = max(np.linalg.cond(element_block(mesh, e)) for e in disc.real)
    tol = max(RTOL_APPLY, 20 * kappa * np.finfo(float).eps)
    assert rel(to_host(z), P.apply(rv)) < tol


def test_pcg_solution_and_error(pair):
    import torch
    mesh, disc, ctx, prob = pair
    b = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
    ctx.rhs(b)
    u = torch.zeros_like(b)
    info = ctx.pcg_solve(b, u, rtol=1e-13, maxit=5000)
    P = BlockPreconditioner(disc)
    uref, it, _ = pcg(disc.apply_X, disc.rhs(), P.apply, 1e-13)
    got = to_host(u)
    assert rel(got, uref) < RTOL_SOLVE
    assert info["rel_residual"] <= 1e-13
    assert abs(info["iterations"] - it) <= max(3, it // 20)
    xe = ctx.error_points()
    e_gpu = ctx.error(u, prob.u(xe), prob.grad_u(xe))
    e_ref = h1_error(disc, uref, prob)
    assert abs(e_gpu - e_ref) <= 1e-8 * max(e_ref, 1e-12) + 1e-12


def test_pcg_maxit_reports_no_convergence():
    import torch
    from paper_1110_2316_amd import setup_problem
    mesh = M.box_mesh(3, (2, 1, 1))
    ctx = setup_problem(mesh, SinProduct())
    b = torch.zeros(ctx.ndof, dtype=torch.float64, device="cuda")
    ctx.rhs(b)
    u = torch.zeros_like(b)
    info = ctx.pcg_solve(b, u, rtol=1e-14, maxit=3, raise_on_fail=False)
    assert info["status"] == -4 and info["iterations"] == 3
