"""The allocation-free entry point (sem_error_noalloc) against sem_error,
through the C ABI, on two calls in a row (the second on a smaller context,
so it reads only what it wrote itself into the scratch the first call
filled further)."""
import numpy as np
import pytest

from gpu_common import to_dev

pytestmark = pytest.mark.gpu


def _case(mesh, problem, seed):
    from paper_1110_2316_amd import setup_problem
    ctx = setup_problem(mesh, problem)
    u = to_dev(np.random.default_rng(seed).standard_normal(ctx.ndof))
    xe = ctx.error_points()
    uex, gex = problem.u(xe), problem.grad_u(xe)
    return ctx, u, uex, gex


def test_noalloc_error_matches_sem_error_twice():
    import torch
    from workloads.fichera import fichera_mesh
    from workloads.mesh import box_mesh
    from workloads.problems import RhoPower, SinProduct
    big = _case(fichera_mesh(N=2, W=3), RhoPower(), 1)
    small = _case(box_mesh(4, (2, 2, 2)), SinProduct(), 2)
    assert big[0].n_real_elements > small[0].n_real_elements
    for ctx, u, uex, gex in (big, small):
        ref = ctx.error(u, uex, gex)
        got = ctx.error_noalloc(u, to_dev(uex), to_dev(np.ascontiguousarray(gex)))
        torch.cuda.synchronize()
        print("noalloc: %d real elements, sem_error %.17g, sem_error_noalloc %.17g"
              % (ctx.n_real_elements, ref, got), flush=True)
        # the same kernels, the partials summed in the same element order
        assert abs(got - ref) <= 1e-12 * abs(ref)
