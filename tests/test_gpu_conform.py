"""The conforming correction (sem_conforming_correction, Appendix C.1)
against the oracle's, element by element, through the C ABI: random
non-conforming vectors on a box mesh and on the Fichera mesh (real, corner
and cross-region neighbours, every orientation code it uses), and a
solution on the unit cube."""
import numpy as np
import pytest

from workloads import mesh as M
from workloads.fichera import fichera_mesh
from workloads.problems import SinProduct
from oracle.conform import correction, face_jumps
from oracle.functional import Discretization
from tests.gpu_common import rand_vec, to_dev, to_host

pytestmark = pytest.mark.gpu


def _gpu_correction(mesh, U):
    import torch
    from paper_1110_2316_amd import Context
    ctx = Context(mesh)
    uc = torch.zeros(ctx.ndof, dtype=torch.float64, device="cuda")
    ctx.conforming_correction(to_dev(U), uc)
    torch.cuda.synchronize()
    return to_host(uc)


@pytest.mark.parametrize("name", ["box_w3", "fichera_n1w2", "fichera_n2w3"])
def test_correction_matches_oracle(name):
    mesh = {"box_w3": lambda: M.box_mesh(3, (3, 2, 2), (0, 0, 0), (1.5, 1.0, 0.7)),
            "fichera_n1w2": lambda: fichera_mesh(N=1, W=2),
            "fichera_n2w3": lambda: fichera_mesh(N=2, W=3)}[name]()
    print("conform case %s" % name, flush=True)
    disc = Discretization(mesh)
    U = rand_vec(disc.ndof, 3)
    ref = correction(disc, U)
    got = _gpu_correction(mesh, U)
    # one product and a sum of at most six terms per unknown
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14 * np.abs(ref).max() * 10)


def test_corrected_solution_on_the_cube():
    import torch
    from paper_1110_2316_amd import setup_problem
    mesh = M.box_mesh(4, (2, 2, 2), (0, 0, 0), (1, 1, 1))
    prob = SinProduct()
    ctx = setup_problem(mesh, prob)
    b = torch.zeros(ctx.ndof, dtype=torch.float64, device="cuda")
    ctx.rhs(b)
    u = torch.zeros_like(b)
    ctx.pcg_solve(b, u, rtol=1e-12, maxit=5000)
    uc = torch.zeros_like(u)
    ctx.conforming_correction(u, uc)
    disc = Discretization(mesh, prob)
    np.testing.assert_allclose(to_host(uc), correction(disc, to_host(u)), rtol=0, atol=1e-13)
    assert face_jumps(disc, to_host(uc)) < face_jumps(disc, to_host(u))
    xe = ctx.error_points()
    e0 = ctx.error(u, prob.u(xe), prob.grad_u(xe))
    e1 = ctx.error(uc, prob.u(xe), prob.grad_u(xe))
    print("conform: H1 error %.3e uncorrected, %.3e corrected" % (e0, e1), flush=True)
    assert e1 < 2.0 * e0
