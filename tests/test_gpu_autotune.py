"""The element kernel's tile candidates: in FP64 the two with one lane per
column give bit-identical results (same summation order per output); the one
with 4 lanes per column splits the forward sums in four, the FP64 tile that
keeps stage-1 values per slab (W >= 10, where the 78 KB slab is one point)
sums the transposed stage 1 slab by slab over four lanes, and the float tile
with stage 3 on the matrix cores sums in its own order: they agree to
rounding.  The autotuner selects one of them and later applies reproduce
that tile's bits."""
import pytest

from workloads import mesh as M
from workloads.problems import SinProduct
from tests.gpu_common import rand_vec, to_dev, RTOL_FP32_APPLY

pytestmark = pytest.mark.gpu


def _case(name):
    if name.startswith("box"):
        W = int(name[5:])
        return M.box_mesh(W, (2, 1, 1), (0, 0, 0), (1, 0.7, 0.9)), SinProduct()
    # curved elements in modified coordinates: all nine coefficient fields
    from workloads.fichera import fichera_mesh
    from workloads.problems import RhoPower
    return fichera_mesh(N=1, W=int(name[-1])), RhoPower()


def _fp64_slab_tile(W):
    """FP64 tile 1 keeps stage-1 values per slab when the whole-element arrays
    plus one slab exceed 78 KB twice over (the 78 KB slab would be one point)."""
    n, m = W + 1, 2 * W + 1
    fixed = 3 * m * n + n * n + n ** 3 + 3 * n * n * m
    return (78 * 1024 // 8 - fixed) // (6 * n * m) < 2


@pytest.mark.parametrize("case", ["box_w%d" % w for w in range(2, 13)] + ["fichera_n1w4"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tiles_agree_and_autotune(case, precision):
    import torch
    from paper_1110_2316_amd import setup_problem
    print("autotune %s %s" % (case, precision), flush=True)
    mesh, prob = _case(case)
    ctx = setup_problem(mesh, prob)
    u = to_dev(rand_vec(ctx.ndof, 4))
    outs = []
    for t in range(3):
        ctx.set_tile(t, precision)
        r = torch.zeros_like(u)
        ctx.residual(u, r, precision=precision)
        outs.append(r)
    # a different split of sums of at most a few hundred terms
    tol = 1e-12 if precision == "fp64" else RTOL_FP32_APPLY
    if precision == "fp64" and not _fp64_slab_tile(mesh.W):
        assert torch.equal(outs[1], outs[0])
    for t in (1, 2):
        rel = float(torch.linalg.norm(outs[t] - outs[0]) / torch.linalg.norm(outs[0]))
        assert rel < tol, (t, rel)
    res = ctx.autotune(precision, reps=3)
    assert res["tile"] in (0, 1, 2)
    assert res["ms"][res["tile"]] > 0
    r = torch.zeros_like(u)
    ctx.residual(u, r, precision=precision)
    assert torch.equal(r, outs[res["tile"]])
