"""Batched solves (sem_pcg_solve_batch): several contexts of different degree
and several right-hand sides each in one graph-captured iteration loop,
against the single solves of the same library (identical arithmetic, so
identical bits) and against the oracle."""
import numpy as np
import pytest

from workloads import mesh as M
from workloads.fichera import fichera_mesh
from workloads.problems import FourierSource, fourier_coef
from oracle.functional import Discretization
from oracle.precond import BlockPreconditioner, ElementBlockPreconditioner
from oracle.solve import pcg
from tests.gpu_common import RTOL_APPLY, RTOL_SOLVE, rel, to_dev, to_host

pytestmark = pytest.mark.gpu


def _rhs(ctx, seed):
    import torch
    ctx.set_source_fourier(to_dev(fourier_coef(seed)))
    b = torch.zeros(ctx.ndof, dtype=torch.float64, device="cuda")
    ctx.rhs(b)
    return b


@pytest.fixture(scope="module")
def batch():
    import torch
    from paper_1110_2316_amd import Context
    print("batch: building contexts", flush=True)
    meshes = [M.box_mesh(4, (2, 2, 2), (0, 0, 0), (1, 1, 1)), M.box_mesh(7, (2, 1, 1), (0, 0, 0), (1, 0.5, 0.5)),
              fichera_mesh(N=1, W=2)]
    ctxs = [Context(m) for m in meshes]
    ctxs[2].set_preconditioner("block")
    R = [2, 3, 2]
    bs = [torch.stack([_rhs(c, 100 * i + k) for k in range(r)]) for i, (c, r) in enumerate(zip(ctxs, R))]
    torch.cuda.synchronize()
    return meshes, ctxs, R, bs


def test_fourier_source_rhs_matches_oracle():
    import torch
    from paper_1110_2316_amd import Context
    mesh = fichera_mesh(N=1, W=2)
    coef = fourier_coef(7)
    disc = Discretization(mesh, FourierSource(coef))
    ctx = Context(mesh)
    b = _rhs(ctx, 7)
    assert rel(to_host(b), disc.rhs()) < RTOL_APPLY


def test_batch_equals_single_solves(batch):
    import torch
    from paper_1110_2316_amd import pcg_solve_batch
    meshes, ctxs, R, bs = batch
    us = [torch.zeros_like(b) for b in bs]
    infos = pcg_solve_batch(ctxs, bs, us, rtol=1e-12, maxit=20000)
    o = 0
    for c, b, u in zip(ctxs, bs, us):
        for k in range(b.shape[0]):
            u1 = torch.zeros_like(b[k])
            i1 = c.pcg_solve(b[k].contiguous(), u1, rtol=1e-12, maxit=20000)
            assert infos[o]["status"] == 0
            assert infos[o]["iterations"] == i1["iterations"]
            assert torch.equal(u[k], u1)
            o += 1


def test_batch_matches_oracle(batch):
    import torch
    from paper_1110_2316_amd import pcg_solve_batch
    meshes, ctxs, R, bs = batch
    us = [torch.zeros_like(b) for b in bs]
    pcg_solve_batch(ctxs, bs, us, rtol=1e-13, maxit=20000)
    for mesh, b, u in zip(meshes, bs, us):
        disc = Discretization(mesh)
        P = BlockPreconditioner(disc) if mesh.info.get("N") is None else ElementBlockPreconditioner(disc)
        for k in range(b.shape[0]):
            uref, _, _ = pcg(disc.apply_X, to_host(b[k]), P.apply, 1e-13, 20000)
            assert rel(to_host(u[k]), uref) < RTOL_SOLVE


def test_batch_repeated_calls_and_fewer_rhs(batch):
    """Graph replays against fresh state: a second call, then one with fewer
    right-hand sides in the same buffers, give the same solutions."""
    import torch
    from paper_1110_2316_amd import pcg_solve_batch
    meshes, ctxs, R, bs = batch
    us1 = [torch.zeros_like(b) for b in bs]
    pcg_solve_batch(ctxs, bs, us1, rtol=1e-12, maxit=20000)
    us2 = [torch.zeros_like(b) for b in bs]
    pcg_solve_batch(ctxs, bs, us2, rtol=1e-12, maxit=20000)
    for a, b in zip(us1, us2):
        assert torch.equal(a, b)
    sub = [b[:1].contiguous() for b in bs]
    us3 = [torch.zeros_like(b) for b in sub]
    pcg_solve_batch(ctxs, sub, us3, rtol=1e-12, maxit=20000)
    for a, b in zip(us1, us3):
        assert torch.equal(a[:1], b)


def test_mixed_batch_matches_fp64(batch):
    """Mixed batch (FP64 refinement around float inner batches) against the
    FP64 batch: 1e-8, and every true FP64 residual at rtol."""
    import torch
    from paper_1110_2316_amd import pcg_solve_batch
    meshes, ctxs, R, bs = batch
    u64 = [torch.zeros_like(b) for b in bs]
    pcg_solve_batch(ctxs, bs, u64, rtol=1e-11, maxit=20000)
    umx = [torch.zeros_like(b) for b in bs]
    infos = pcg_solve_batch(ctxs, bs, umx, rtol=1e-11, maxit=20000, precision="mixed")
    for a, b in zip(umx, u64):
        for k in range(b.shape[0]):
            assert float(torch.linalg.norm(a[k] - b[k]) / torch.linalg.norm(b[k])) < 1e-8
    assert all(i["status"] == 0 and i["rel_residual"] <= 1e-11 and i["outer"] >= 2 for i in infos)
    # the true residual, recomputed through the single-solve ABI
    for c, b, u in zip(ctxs, bs, umx):
        for k in range(b.shape[0]):
            r = torch.zeros_like(b[k])
            c.residual(u[k].contiguous(), r)
            assert float(torch.linalg.norm(r - b[k]) / torch.linalg.norm(b[k])) <= 1.01e-11


@pytest.mark.slow
@pytest.mark.parametrize("W", [4, 8, 12])
def test_batch_workload_contexts_at_full_size(W):
    """The batched workload's Fichera contexts (N = 2 layers, element-block
    preconditioner, four Fourier right-hand sides solved together) at W = 4,
    8, 12: sampled element rows of X u and of every b against the oracle
    restricted to those elements, and every batch solution satisfying the
    oracle's normal equations on the sampled rows to the solve tolerance."""
    import torch
    from paper_1110_2316_amd import Context, pcg_solve_batch
    print("batch workload context: fichera N=2 W=%d" % W, flush=True)
    mesh = fichera_mesh(N=2, W=W)
    ctx = Context(mesh)
    ctx.set_preconditioner("block")
    coefs = [fourier_coef(1000 * (17 + W) + j) for j in range(4)]
    B = torch.stack([_rhs(ctx, 1000 * (17 + W) + j) for j in range(4)])
    U = torch.zeros_like(B)
    rtol = 1e-10
    infos = pcg_solve_batch([ctx], [B], [U], rtol=rtol, maxit=20000)
    assert all(i["status"] == 0 for i in infos)
    rng = np.random.default_rng(W)
    real = mesh.real_elements()
    S = [int(e) for e in rng.choice(real, 4, replace=False)]
    n3 = (W + 1) ** 3
    v = rng.standard_normal(ctx.ndof)
    Xv = torch.zeros(ctx.ndof, dtype=torch.float64, device="cuda")
    ctx.residual(to_dev(v), Xv)
    base = None
    for j, coef in enumerate(coefs):
        part = Discretization(mesh, FourierSource(coef), only=S)
        if base is None:
            base = part
            Xo = part.apply_X(v)
        bo = part.rhs()
        Xu = part.apply_X(to_host(U[j]))
        bnorm = float(torch.linalg.norm(B[j]))
        for e in S:
            o = part.offset[e]
            rows = slice(o, o + n3)
            if j == 0:
                assert rel(to_host(Xv)[rows], Xo[rows]) < RTOL_APPLY
            assert rel(to_host(B[j])[rows], bo[rows]) < RTOL_APPLY
            # the solution's residual on these rows, by the oracle's operator
            assert np.linalg.norm(Xu[rows] - bo[rows]) <= 10 * rtol * bnorm
