"""Neumann faces (mesh bc code 3, sem_set_neumann_data) against the oracle:
the operator apply, the right-hand side with Neumann data, and the solution,
on the thesis's mixed-boundary cube (Table 6.3) and with Neumann faces in the
vertex, vertex-edge and edge regions."""
import os

import numpy as np
import pytest

from workloads import mesh as M
from workloads.singular import vertex_mesh, edge_mesh, vertex_edge_mesh
from workloads.problems import MixedSin, VertexPower, EdgePower, VertexEdgePower
from oracle.functional import Discretization
from oracle.precond import BlockPreconditioner
from oracle.solve import pcg, h1_error
from tests.gpu_common import RTOL_APPLY, RTOL_SOLVE, rand_vec, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

CASES = {
    "cube_mixed_w4": lambda: (M.box_mesh(4, (2, 2, 2), (-1, -1, -1), (1, 1, 1), neumann=MixedSin.NEUMANN_FACES),
                              MixedSin()),
    # theta = 3 pi / 2 face and the sphere rho = 1 Neumann
    "vertex_n2w3": lambda: (vertex_mesh(2, 3, I=2, neumann=((1, 1), (2, 1))), VertexPower()),
    # x3 = 1 and theta = pi / 2 faces Neumann
    "edge_n2w3": lambda: (edge_mesh(2, 3, neumann=((2, 1), (1, 1))), EdgePower()),
    # the cone phi = phi_v Neumann
    "vertex_edge_n2w3": lambda: (vertex_edge_mesh(2, 3, neumann=((0, 1),)), VertexEdgePower()),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    from paper_1110_2316_amd import setup_problem
    print("neumann case %s" % request.param, flush=True)
    mesh, prob = CASES[request.param]()
    assert (mesh.bc == M.NEUMANN).any()
    return request.param, mesh, prob, Discretization(mesh, prob), setup_problem(mesh, prob)


def test_apply_and_rhs(case):
    import torch
    name, mesh, prob, disc, ctx = case
    v = rand_vec(disc.ndof, 8)
    q = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
    ctx.residual(to_dev(v), q)
    assert rel(to_host(q), disc.apply_X(v)) < RTOL_APPLY
    b = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
    ctx.rhs(b)
    assert rel(to_host(b), disc.rhs()) < RTOL_APPLY


def test_solution(case):
    import torch
    name, mesh, prob, disc, ctx = case
    b = torch.zeros(disc.ndof, dtype=torch.float64, device="cuda")
    ctx.rhs(b)
    u = torch.zeros_like(b)
    ctx.pcg_solve(b, u, rtol=1e-13, maxit=20000)
    uref, _, _ = pcg(disc.apply_X, disc.rhs(), BlockPreconditioner(disc).apply, 1e-13, 20000)
    assert rel(to_host(u), uref) < RTOL_SOLVE
    if name == "cube_mixed_w4":
        xe = ctx.error_points()
        err = 100 * ctx.error(u, prob.u(xe), prob.grad_u(xe))
        ref = 100 * h1_error(disc, uref, prob)
        print("neumann: Table 6.3 W=4 error %.4e %% (oracle %.4e %%, printed 0.540972 %%)" % (err, ref), flush=True)
        assert abs(err - ref) <= 1e-6 * ref
