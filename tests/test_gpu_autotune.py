"""The element kernel's tile candidates give bit-identical results (same
summation order per output), and the autotuner selects one of them."""
import pytest

from workloads import mesh as M
from workloads.problems import SinProduct
from tests.gpu_common import rand_vec, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("W", [6, 8, 10])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tiles_bit_identical_and_autotune(W, precision):
    import torch
    from paper_1110_2316_amd import setup_problem
    print("autotune W=%d %s" % (W, precision), flush=True)
    mesh = M.box_mesh(W, (2, 1, 1), (0, 0, 0), (1, 0.7, 0.9))
    ctx = setup_problem(mesh, SinProduct())
    u = to_dev(rand_vec(ctx.ndof, 4))
    outs = []
    for t in range(3):
        ctx.set_tile(t, precision)
        r = torch.zeros_like(u)
        ctx.residual(u, r, precision=precision)
        outs.append(r)
    for r in outs[1:]:
        assert torch.equal(r, outs[0])
    res = ctx.autotune(precision, reps=3)
    assert res["tile"] in (0, 1, 2)
    assert res["ms"][res["tile"]] > 0
    r = torch.zeros_like(u)
    ctx.residual(u, r, precision=precision)
    assert torch.equal(r, outs[0])
