"""Staged validations of the oracle on the thesis's single-singularity domains.

Sec. 6.3 solves three model problems whose exact solutions carry one kind
of singularity each: a vertex (Table 6.16), an edge (Table 6.18) and a
vertex-edge (Table 6.20).  The oracle solves the same problems on geometric
meshes built from the same neighbourhood definitions (workloads.singular)
and is checked for

* exponential decay of the relative H^1 error as N = W grows (Thm 4.3.2);
* the printed errors and iteration counts in magnitude, at the thesis's
  layer count N = W - 1 (inferred from its N_dof column).

The thesis's errors are smaller than the oracle's (factors 3-110 at
W = 2-4).  The functional at the interpolant of the exact solution is
dominated by the face between the corner element (whose shared function
cannot follow the exact solution's angular variation) and the first real
layer, so the literal functional trades accuracy in the real elements
against that jump, while the printed errors sit at the level of the real
elements' best approximation (e.g. Omega^(v), W = 4: interpolation error
5.0e-5, thesis 3.1e-5, oracle 1.6e-3).  The magnitude check therefore
only bounds the ratio to the printed values (two decades); decay and the
interpolation-level agreement carry the pin.
"""
import os

import numpy as np
import pytest

from workloads import mesh as M
from workloads.singular import vertex_mesh, edge_mesh, vertex_edge_mesh
from workloads.problems import VertexPower, EdgePower, VertexEdgePower
from oracle.functional import Discretization
from oracle.precond import BlockPreconditioner
from oracle.solve import pcg, h1_error

GOLD = os.path.join(os.path.dirname(__file__), "golden")

DOMAINS = {
    "vertex": (vertex_mesh, VertexPower, "table6_16.txt"),
    "edge": (edge_mesh, EdgePower, "table6_18.txt"),
    "vertex_edge": (vertex_edge_mesh, VertexEdgePower, "table6_20.txt"),
}


def _golden(name):
    rows = {}
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            W, ndof, its, err = line.split()
            rows[int(W)] = (int(ndof), int(its), float(err))
    return rows


def _solve(domain, N, W):
    gen, prob, _ = DOMAINS[domain]
    mesh = gen(N, W)
    P = prob()
    disc = Discretization(mesh, P)
    u, its, _ = pcg(disc.apply_X, disc.rhs(), BlockPreconditioner(disc).apply, 1e-11, 20000)
    return disc, u, its, 100 * h1_error(disc, u, P)


@pytest.mark.parametrize("domain", sorted(DOMAINS))
def test_error_decays_with_layers_and_degree(domain):
    errs = [_solve(domain, W, W)[3] for W in (2, 3, 4)]
    assert errs[0] > errs[1] > errs[2], errs
    # corner-limited on the edge domain (about mu^(N/3) per layer), faster elsewhere
    assert errs[0] / errs[2] > (2.5 if domain == "edge" else 8.0), errs


@pytest.mark.parametrize("domain", sorted(DOMAINS))
def test_thesis_tables_in_magnitude(domain):
    gold = _golden(DOMAINS[domain][2])
    for W in (2, 4) if domain != "vertex_edge" else (2, 3, 4):
        _, its, err = gold[W]
        _, _, our_its, our_err = _solve(domain, W - 1, W)
        assert 1.0 <= our_err / err < 150.0, (domain, W, our_err, err)
        assert its / 10 < our_its < 10 * its, (domain, W, our_its, its)


def test_vertex_interpolant_at_the_printed_error_level():
    """The thesis's Omega^(v) error at W = 4 (N = 3) is at the level of the
    nodal interpolant of the exact solution in the real elements."""
    gen, prob, table = DOMAINS["vertex"]
    mesh = gen(3, 4)
    P = prob()
    disc = Discretization(mesh, P)
    n = disc.n
    A, B, C = np.meshgrid(disc.xn, disc.xn, disc.xn, indexing="ij")
    lam = np.stack([A.ravel(order="F"), B.ravel(order="F"), C.ravel(order="F")], -1)
    UI = np.zeros(disc.ndof)
    for e in disc.real:
        o = disc.offset[e]
        UI[o:o + n ** 3] = P.u(M.chart_points(mesh, e, lam))
    err_i = 100 * h1_error(disc, UI, P)
    printed = _golden(table)[4][2]
    assert 0.5 < err_i / printed < 3.0, (err_i, printed)
