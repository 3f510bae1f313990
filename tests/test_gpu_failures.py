"""Failure paths of the PCG drivers, forced from the host with kernels that
all exit normally: a NaN in the right-hand side (SEM_ENAN), an indefinite
operator from negated face-norm weights (SEM_EBREAKDOWN: p^T X p <= 0), and
an iteration limit (SEM_ENOCONV), on the FP64 and mixed paths."""
import numpy as np
import pytest

from workloads import mesh as M
from workloads.problems import SinProduct

pytestmark = pytest.mark.gpu

ENOCONV, EBREAKDOWN, ENAN = -4, -5, -6


def _ctx():
    import torch
    from paper_1110_2316_amd import setup_problem
    ctx = setup_problem(M.box_mesh(3, (2, 2, 2), (0, 0, 0), (1, 1, 1)), SinProduct())
    b = torch.zeros(ctx.ndof, dtype=torch.float64, device="cuda")
    ctx.rhs(b)
    return ctx, b


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_nan_in_b_reports_enan(precision):
    import torch
    ctx, b = _ctx()
    b[7] = float("nan")
    u = torch.zeros_like(b)
    info = ctx.pcg_solve(b, u, rtol=1e-10, maxit=500, raise_on_fail=False, precision=precision)
    print("failures: NaN in b, %s: status %d after %d iterations" % (precision, info["status"], info["iterations"]),
          flush=True)
    assert info["status"] == ENAN


def test_negated_face_weights_report_breakdown():
    import torch
    ctx, b = _ctx()
    w = ctx.face_weights()
    assert (w[:, 0, 0] > 0).all()
    ctx.set_face_weights(-w)
    u = torch.zeros_like(b)
    info = ctx.pcg_solve(b, u, rtol=1e-10, maxit=500, raise_on_fail=False)
    print("failures: negated face weights: status %d after %d iterations" % (info["status"], info["iterations"]),
          flush=True)
    assert info["status"] == EBREAKDOWN
    # restoring the weights restores the solve
    ctx.set_face_weights(w)
    u.zero_()
    assert ctx.pcg_solve(b, u, rtol=1e-10, maxit=2000, raise_on_fail=False)["status"] == 0


def test_iteration_limit_reports_enoconv():
    import torch
    ctx, b = _ctx()
    u = torch.zeros_like(b)
    info = ctx.pcg_solve(b, u, rtol=1e-14, maxit=3, raise_on_fail=False)
    assert info["status"] == ENOCONV and info["iterations"] == 3
