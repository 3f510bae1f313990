"""The element-block preconditioner (exact diagonal blocks of X, assembled on
the GPU with the operator kernels and factored there) against the oracle's
own assembly and Cholesky solves, through the C ABI."""
import numpy as np
import pytest

from workloads import mesh as M
from workloads.fichera import fichera_mesh
from workloads.problems import RhoPower, SinProduct
from oracle.functional import Discretization
from oracle.precond import ElementBlockPreconditioner
from oracle.solve import pcg
from tests.gpu_common import RTOL_APPLY, RTOL_MIXED, RTOL_SOLVE, rand_vec, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

CASES = {
    "cube_w4": lambda: (M.box_mesh(4, (2, 2, 2), (0, 0, 0), (1, 1, 1)), SinProduct()),
    # 18 elements per stored block (the inner x-positions of each of the four
    # cross-section places): more than 16, so a block's elements split into
    # two tasks of the grouped apply
    "box20_w2": lambda: (M.box_mesh(2, (20, 2, 2), (0, 0, 0), (10, 1, 1)), SinProduct()),
    # n^3 = 343: two row parts of the grouped apply, six residual chunks (the
    # last one ragged), four mirror images sharing one stored block
    "box4_w6": lambda: (M.box_mesh(6, (2, 2, 1), (0, 0, 0), (1, 1, 0.5)), SinProduct()),
    "fichera_n1w1": lambda: (fichera_mesh(N=1, W=1), RhoPower()),
    "fichera_n1w2": lambda: (fichera_mesh(N=1, W=2), RhoPower()),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    import torch
    from paper_1110_2316_amd import setup_problem
    print("block case %s" % request.param, flush=True)
    mesh, prob = CASES[request.param]()
    disc = Discretization(mesh, prob)
    P = ElementBlockPreconditioner(disc)
    ctx = setup_problem(mesh, prob)
    ctx.set_preconditioner("block")
    torch.cuda.synchronize()
    return mesh, disc, P, ctx


def test_block_preconditioner_apply(case):
    import torch
    mesh, disc, P, ctx = case
    rv = rand_vec(disc.ndof, 17)
    z = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
    ctx.precond(to_dev(rv), z)
    ref = P.apply(rv)
    # the library assembles the blocks with its own kernels and solves through
    # G = L^{-1}; the oracle through cho_solve: they agree to kappa(block) x eps
    kappa = max([np.linalg.cond(B) for B in P.blocks] + ([np.linalg.cond(P.Xcc)] if P.Xcc.size else []))
    tol = max(RTOL_APPLY, 20 * kappa * np.finfo(float).eps)
    assert rel(to_host(z), ref) < tol


def test_block_pcg_solution(case):
    import torch
    mesh, disc, P, ctx = case
    b = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
    ctx.rhs(b)
    u = torch.zeros_like(b)
    info = ctx.pcg_solve(b, u, rtol=1e-13, maxit=20000)
    uref, it, _ = pcg(disc.apply_X, disc.rhs(), P.apply, 1e-13, 20000)
    assert rel(to_host(u), uref) < RTOL_SOLVE
    assert abs(info["iterations"] - it) <= max(3, it // 20)


def test_block_mixed_solution(case):
    import torch
    mesh, disc, P, ctx = case
    b = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
    ctx.rhs(b)
    u = torch.zeros_like(b)
    info = ctx.pcg_solve(b, u, rtol=1e-12, maxit=20000, precision="mixed")
    uref, _, _ = pcg(disc.apply_X, disc.rhs(), P.apply, 1e-13, 20000)
    assert rel(to_host(u), uref) < RTOL_MIXED
    assert info["status"] == 0


def test_switch_back_to_separable(case):
    import torch
    from oracle.precond import BlockPreconditioner
    mesh, disc, P, ctx = case
    ctx.set_preconditioner("separable")
    try:
        rv = rand_vec(disc.ndof, 2)
        z = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
        ctx.precond(to_dev(rv), z)
        Ps = BlockPreconditioner(disc)
        from oracle.precond import element_block
        kappa = max(np.linalg.cond(element_block(mesh, e)) for e in disc.real)
        assert rel(to_host(z), Ps.apply(rv)) < max(RTOL_APPLY, 20 * kappa * np.finfo(float).eps)
    finally:
        ctx.set_preconditioner("block")


@pytest.mark.parametrize("name", ["box20_w2", "fichera_n1w2"])
def test_chunked_assembly(name, monkeypatch):
    """Blocks assembled with a 16 KiB chunk buffer (two blocks of n^3 = 27):
    many chunks per colour, blocks matched against stored blocks of earlier
    chunks.  The preconditioner is still the oracle's, with as many stored
    blocks as the assembly in one chunk per colour."""
    import torch
    from paper_1110_2316_amd import setup_problem
    mesh, prob = CASES[name]()
    disc = Discretization(mesh, prob)
    P = ElementBlockPreconditioner(disc)
    whole = setup_problem(mesh, prob)
    whole.set_preconditioner("block")
    monkeypatch.setenv("SEM_BLOCK_CHUNK_KB", "16")
    ctx = setup_problem(mesh, prob)
    ctx.set_preconditioner("block")
    torch.cuda.synchronize()
    assert ctx.work_counts()["block_bytes_fp64"] == whole.work_counts()["block_bytes_fp64"]
    rv = rand_vec(disc.ndof, 19)
    z = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
    ctx.precond(to_dev(rv), z)
    kappa = max([np.linalg.cond(B) for B in P.blocks] + ([np.linalg.cond(P.Xcc)] if P.Xcc.size else []))
    assert rel(to_host(z), P.apply(rv)) < max(RTOL_APPLY, 20 * kappa * np.finfo(float).eps)


def test_mirror_images_share_stored_blocks():
    """The eight elements of the 2x2x2 cube are mirror images of each other
    (reversals of lambda axes), so one stored block serves all of them, each
    element applying it through its own reversal (checked against the
    oracle's per-element blocks by test_block_preconditioner_apply)."""
    import torch
    from paper_1110_2316_amd import setup_problem
    mesh, prob = CASES["cube_w4"]()
    ctx = setup_problem(mesh, prob)
    ctx.set_preconditioner("block")
    torch.cuda.synchronize()
    n3 = mesh.n ** 3
    stored = ctx.work_counts()["block_bytes_fp64"] // (n3 * n3 * 8)
    assert stored == 1, stored
