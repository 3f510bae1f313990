"""Layer-graded degrees (Sec. 2.3; sem_set_degrees) against the oracle's
graded system, through the C ABI: the projection, the projected operator and
right-hand side, both graded preconditioners, and the FP64, mixed and
batched solutions, on an anisotropic box case (degrees (3, 2, 1), exact for
a polynomial of those degrees) and on the Fichera mesh with the layer rule."""
import numpy as np
import pytest

from workloads import mesh as M
from workloads import grading
from workloads.fichera import fichera_mesh
from workloads.problems import Polynomial, RhoPower
from oracle.functional import Discretization
from oracle.graded import GradedSystem, GradedSeparablePreconditioner, GradedElementBlockPreconditioner
from oracle.solve import h1_error
from tests.gpu_common import RTOL_APPLY, RTOL_MIXED, RTOL_SOLVE, rand_vec, rel, to_dev, to_host

pytestmark = pytest.mark.gpu


def _box():
    mesh = M.box_mesh(4, (2, 1, 1), (0.0, 0.0, 0.0), (1.0, 0.7, 0.6))
    return mesh, Polynomial(), np.tile([3, 2, 1], (mesh.E, 1))


def _fichera():
    # layers 1, 2 at W = 2: degrees (1,1,1), (1,1,2), (2,2,1) and (2,2,2)
    mesh = fichera_mesh(N=2, W=2)
    return mesh, RhoPower(), grading.layer_degrees(mesh, 1.0, 1.5)


CASES = {"box_w4_321": _box, "fichera_n2w2_layers": _fichera}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    from paper_1110_2316_amd import setup_problem
    print("graded case %s" % request.param, flush=True)
    mesh, prob, deg = CASES[request.param]()
    disc = Discretization(mesh, prob)
    gs = GradedSystem(disc, deg)
    ctx = setup_problem(mesh, prob)
    ctx.set_degrees(deg)
    return request.param, mesh, prob, deg, disc, gs, ctx


_REF = {}


def _reference(name, gs):
    """(oracle element-block preconditioner, oracle graded solution): the
    dense reduced solve on the small box, PCG to 1e-14 with the oracle's
    graded element blocks on the Fichera mesh."""
    from oracle.solve import pcg
    if name not in _REF:
        P = GradedElementBlockPreconditioner(gs)
        if gs.ndof_graded <= 400:
            u = gs.solve()
        else:
            u, _, _ = pcg(gs.apply_X, gs.rhs(), P.apply, 1e-14, 20000)
        _REF[name] = (P, u)
    return _REF[name]


def test_graded_ndof(case):
    name, mesh, prob, deg, disc, gs, ctx = case
    assert ctx.graded_ndof == gs.ndof_graded == grading.graded_dof(mesh, deg)
    assert ctx.graded_ndof < ctx.ndof


def test_projection(case):
    name, mesh, prob, deg, disc, gs, ctx = case
    v = rand_vec(disc.ndof, 3)
    u = to_dev(v)
    ctx.project(u)
    assert rel(to_host(u), gs.project(v)) < RTOL_APPLY


def test_apply_and_rhs(case):
    import torch
    name, mesh, prob, deg, disc, gs, ctx = case
    v = gs.project(rand_vec(disc.ndof, 4))
    q = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
    ctx.residual(to_dev(v), q)
    assert rel(to_host(q), gs.apply_X(v)) < RTOL_APPLY
    b = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
    ctx.rhs(b)
    assert rel(to_host(b), gs.rhs()) < RTOL_APPLY


def test_separable_preconditioner(case):
    import torch
    name, mesh, prob, deg, disc, gs, ctx = case
    ctx.set_preconditioner("separable")
    r = rand_vec(disc.ndof, 5)
    z = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
    ctx.precond(to_dev(r), z)
    P = GradedSeparablePreconditioner(gs)
    ref = P.apply(r)
    # eigenbases of the reduced 1D pencils here, Cholesky of the assembled
    # reduced blocks in the oracle: they agree to kappa(block) x eps
    kappa = max(np.linalg.cond(B) for B in _blocks(P))
    assert rel(to_host(z), ref) < max(RTOL_APPLY, 20 * kappa * np.finfo(float).eps)


def test_solutions(case):
    import torch
    name, mesh, prob, deg, disc, gs, ctx = case
    _, uref = _reference(name, gs)
    b = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
    ctx.rhs(b)
    for kind in ("separable", "block"):
        ctx.set_preconditioner(kind)
        u = torch.zeros_like(b)
        info = ctx.pcg_solve(b, u, rtol=1e-13, maxit=50000)
        print("graded %s %s: %d iterations" % (name, kind, info["iterations"]), flush=True)
        assert rel(to_host(u), uref) < RTOL_SOLVE
    um = torch.zeros_like(b)
    info = ctx.pcg_solve(b, um, rtol=1e-12, maxit=50000, precision="mixed")
    assert info["status"] == 0
    assert rel(to_host(um), uref) < RTOL_MIXED
    if name == "box_w4_321":
        # the polynomial has exactly these degrees: reproduced to rounding
        xe = ctx.error_points()
        assert ctx.error(u, prob.u(xe), prob.grad_u(xe)) < 1e-10
        assert h1_error(disc, uref, prob) < 1e-10


def test_block_preconditioner(case):
    import torch
    name, mesh, prob, deg, disc, gs, ctx = case
    ctx.set_preconditioner("block")
    P, _ = _reference(name, gs)
    r = rand_vec(disc.ndof, 6)
    z = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
    ctx.precond(to_dev(r), z)
    ref = P.apply(r)
    kappa = max(np.linalg.cond(B) for B in _blocks(P))
    assert rel(to_host(z), ref) < max(RTOL_APPLY, 20 * kappa * np.finfo(float).eps)


def _blocks(P):
    """The factored blocks of an oracle graded preconditioner, reassembled
    (for their condition numbers), the corner block included."""
    out = []
    facs = list(P.fac.values()) + ([P.chol_c] if P.chol_c is not None else [])
    for c, lower in facs:
        L = np.tril(c) if lower else np.triu(c).T
        out.append(L @ L.T)
    return out


def test_batch_matches_single(case):
    import torch
    from paper_1110_2316_amd.semlib import pcg_solve_batch
    name, mesh, prob, deg, disc, gs, ctx = case
    ctx.set_preconditioner("block")
    b = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
    ctx.rhs(b)
    bs = torch.stack([b, 0.5 * b])
    us = torch.zeros_like(bs)
    pcg_solve_batch([ctx], [bs], [us], rtol=1e-12)
    u1 = torch.zeros_like(b)
    ctx.pcg_solve(b, u1, rtol=1e-12, maxit=50000)
    assert torch.equal(us[0], u1)
    assert rel(to_host(us[1]), 0.5 * to_host(u1)) < 1e-10


def test_degrees_reset_and_rejected(case):
    import torch
    from paper_1110_2316_amd.semlib import SemError
    name, mesh, prob, deg, disc, gs, ctx = case
    bad = np.array(deg)
    bad[mesh.real_elements()[0], 0] = mesh.W + 1
    with pytest.raises(SemError):
        ctx.set_degrees(bad)
    ctx.set_degrees(None)
    assert ctx.graded_ndof == ctx.ndof
    v = rand_vec(disc.ndof, 7)
    q = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
    ctx.residual(to_dev(v), q)
    assert rel(to_host(q), disc.apply_X(v)) < RTOL_APPLY
    ctx.set_degrees(deg)


def test_graded_source_gradient():
    """The autograd solve on a graded space against the oracle's gradient with
    the graded solve operator S = P (P^T X P)^-1 P^T (symmetric, so the
    oracle's lambda = S 2 (u - u_t) applies unchanged)."""
    import scipy.linalg as sla
    import torch
    from paper_1110_2316_amd import Context, solve_source
    from workloads.problems import LegendreSource, legendre_theta
    from oracle.adjoint import loss_and_grad, source_rhs
    mesh = M.box_mesh(4, (2, 2, 1), (-1, -1, -1), (1, 1, 0))
    degs = np.array([[3, 2, 4], [4, 4, 2], [2, 3, 3], [4, 1, 2]])
    deg = 3
    disc = Discretization(mesh, LegendreSource(np.zeros(deg ** 3), deg))
    gs = GradedSystem(disc, degs)
    fac = sla.cho_factor(gs.reduced_matrix())
    solve = lambda r: gs.embed(sla.cho_solve(fac, gs.restrict(r)))
    u_t = solve(source_rhs(disc, legendre_theta(deg, 1), deg))
    theta0 = legendre_theta(deg, 2)
    L_ref, g_ref = loss_and_grad(disc, theta0, u_t, deg, solve)
    ctx = Context(mesh)
    ctx.set_degrees(degs)
    ctx.set_preconditioner("block")
    theta = to_dev(theta0).requires_grad_(True)
    u = solve_source(theta, ctx, rtol=1e-14)
    loss = torch.sum((u - to_dev(u_t)) ** 2)
    loss.backward()
    assert abs(float(loss.detach()) - L_ref) <= 1e-9 * L_ref
    assert rel(to_host(theta.grad), g_ref) < 1e-8


@pytest.mark.slow
def test_graded_full_size_sampled_rows():
    """Fichera N = W = 10 with the layer rule (mu1 = 1, mu2 = 1.5) in the
    bench's launch configuration: rows of Q X Q u and Q b of sampled elements
    (every region, graded and ungraded) against the oracle restricted to
    them, and the graded FP64 and mixed solutions against each other."""
    import torch
    from paper_1110_2316_amd import setup_problem
    from oracle.functional import tensor_apply
    from oracle.graded import projector_1d
    from tests.gpu_common import RTOL_FP32_APPLY
    print("graded: fichera N=10 W=10, layer rule", flush=True)
    mesh = fichera_mesh(N=10, W=10)
    deg = grading.layer_degrees(mesh, 1.0, 1.5)
    ctx = setup_problem(mesh, RhoPower())
    ctx.set_degrees(deg)
    ctx.set_preconditioner("block")
    for p in ("fp64", "mixed"):
        ctx.autotune(p, reps=3)
    print("graded: library set up, %d of %d unknowns" % (ctx.graded_ndof, ctx.ndof), flush=True)
    assert ctx.graded_ndof == grading.graded_dof(mesh, deg)
    real = np.flatnonzero(mesh.kind == M.REAL)
    rng = np.random.default_rng(11)
    S = []
    for reg in (M.REG, M.VTX, M.VE, M.EDGE):
        cand = real[mesh.region[real] == reg]
        S += [int(e) for e in rng.choice(cand, 2, replace=False)]
    disc = Discretization(mesh, RhoPower(), only=S)
    W, n3 = mesh.W, disc.n ** 3
    Q = {e: [projector_1d(W, int(w)) for w in deg[e]] for e in S}

    def project(v, elems):
        out = np.array(v, copy=True)
        for e in elems:
            o = disc.offset[e]
            ue = v[o:o + n3].reshape((disc.n,) * 3, order="F")
            out[o:o + n3] = tensor_apply(*Q[e], ue).reshape(-1, order="F")
        return out

    ud = to_dev(rand_vec(ctx.ndof, 34))
    ctx.project(ud)                               # u in the graded space (library)
    u = to_host(ud)
    assert rel(u[disc.offset[S[0]]:disc.offset[S[0]] + n3],
               project(rand_vec(ctx.ndof, 34), [S[0]])[disc.offset[S[0]]:disc.offset[S[0]] + n3]) < RTOL_APPLY
    r = torch.zeros(ctx.ndof, dtype=torch.float64, device="cuda")
    ctx.residual(ud, r)
    rm = torch.zeros_like(r)
    ctx.residual(ud, rm, precision="mixed")
    b = torch.zeros_like(r)
    ctx.rhs(b)
    Xo = project(disc.apply_X(u), S)
    bo = project(disc.rhs(), S)
    got, gotm, gb = to_host(r), to_host(rm), to_host(b)
    for e in S:
        o = disc.offset[e]
        sl = slice(o, o + n3)
        assert rel(got[sl], Xo[sl]) < RTOL_APPLY, e
        assert rel(gb[sl], bo[sl]) < RTOL_APPLY, e
        assert rel(gotm[sl], Xo[sl]) < RTOL_FP32_APPLY, e
    u64 = torch.zeros_like(b)
    i64 = ctx.pcg_solve(b, u64, rtol=1e-10, maxit=20000)
    umx = torch.zeros_like(b)
    imx = ctx.pcg_solve(b, umx, rtol=1e-10, maxit=20000, precision="mixed")
    print("graded N=10: fp64 %d, mixed %d iterations" % (i64["iterations"], imx["iterations"]), flush=True)
    assert rel(to_host(umx), to_host(u64)) < RTOL_MIXED
