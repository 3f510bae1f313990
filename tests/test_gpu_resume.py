"""Checkpoint and resume of a solve: the solvers start from the values in u,
so a solve stopped at maxit (SEM_ENOCONV) and written to host memory can be
resumed later, in a fresh context of the same mesh, and reaches the solution
of an uninterrupted solve; the same for the mixed path."""
import numpy as np
import pytest

from workloads.fichera import fichera_mesh
from workloads.problems import RhoPower
from tests.gpu_common import RTOL_MIXED, RTOL_SOLVE, rel, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_resume_from_a_host_checkpoint(precision, tmp_path):
    import torch
    from paper_1110_2316_amd import setup_problem
    print("resume %s" % precision, flush=True)
    mesh = fichera_mesh(N=2, W=3)
    ctx = setup_problem(mesh, RhoPower())
    ctx.set_preconditioner("block")
    b = torch.zeros(ctx.ndof, dtype=torch.float64, device="cuda")
    ctx.rhs(b)
    full = torch.zeros_like(b)
    info_full = ctx.pcg_solve(b, full, rtol=1e-11, maxit=20000, precision=precision)
    # interrupted solve: a few iterations, then a checkpoint on the host (file)
    u = torch.zeros_like(b)
    part = ctx.pcg_solve(b, u, rtol=1e-11, maxit=10, precision=precision, raise_on_fail=False)
    assert part["status"] != 0
    ck = str(tmp_path / "u.npy")
    np.save(ck, to_host(u))
    del ctx, u
    torch.cuda.synchronize()
    # a fresh context resumes from the checkpoint
    ctx2 = setup_problem(mesh, RhoPower())
    ctx2.set_preconditioner("block")
    b2 = torch.zeros_like(b)
    ctx2.rhs(b2)
    u2 = to_dev(np.load(ck))
    info = ctx2.pcg_solve(b2, u2, rtol=1e-11, maxit=20000, precision=precision)
    assert info["status"] == 0
    tol = RTOL_SOLVE if precision == "fp64" else RTOL_MIXED
    assert rel(to_host(u2), to_host(full)) < 100 * tol
    print("resume %s: %d + %d iterations (uninterrupted %d)"
          % (precision, part["iterations"], info["iterations"], info_full["iterations"]), flush=True)
