"""Conforming correction of the non-conforming solution (thesis Appendix C.1,
proof of Lemma 3.3.1; the remark after Thm 4.3.2).

ORACLE: test infrastructure only.

For a real element with master-cube coordinates lam and faces lam_d = -1,
+1, the correction is

    nu(lam) = sum over the element's interior faces f of
              (1 -/+ lam_d) / 2 * c_f * [u]_f(face coordinates)

where [u]_f is the jump across f, the neighbour's value minus the
element's own, as a function of the face coordinates (so that u + [u]/2 is
the average of the two sides), c_f = 1/2, except c_f = 1 when the neighbour
is a corner element (the corrected function takes the corner's value on
that face).  Corner elements are not corrected.  The corrected unknowns
are the nodal values of u + nu (nu lies in the same polynomial space: degree
W along the face, linear across it); the corner unknowns are kept.

Reading where the appendix is silent: faces on the boundary (Dirichlet) are
not corrected (the lemma concerns the interior jumps).
"""
import numpy as np

from workloads import mesh as M
from . import gll


def _neighbour_value(disc, U, e2, f2, o, a, b):
    """Neighbour e2's function at the points of its face f2 whose face
    coordinates are orient_map(o, a, b) (a, b: this side's face coordinates)."""
    mesh = disc.mesh
    a2, b2 = M.orient_map(o, a, b)
    lam = M.face_lam(f2, a2, b2)
    ue = disc.element_values(U, e2)
    L = [gll.lagrange(disc.xn, lam[:, d]) for d in range(3)]
    return np.einsum("ijk,pi,pj,pk->p", ue, L[0], L[1], L[2])


def correction(disc, U):
    """The corrected unknown vector (same layout as U)."""
    mesh = disc.mesh
    n = disc.n
    x = disc.xn
    out = np.array(U, float, copy=True)
    for e in disc.real:
        ue = disc.element_values(U, e)
        nu = np.zeros((n, n, n))
        for f in range(6):
            if mesh.bc[e, f] != M.INTERIOR:
                continue
            d, s = divmod(f, 2)
            t0, t1 = M.FACE_TANGENT[d]
            e2, f2, o = int(mesh.nbr[e, f]), int(mesh.nbr_face[e, f]), int(mesh.orient[e, f])
            A, B = np.meshgrid(x, x, indexing="ij")          # face nodes (t0 index, t1 index)
            a, b = A.ravel(), B.ravel()
            own_idx = [slice(None)] * 3
            own_idx[d] = n - 1 if s else 0
            own = ue[tuple(own_idx)]                          # [n, n] over (t0, t1)
            nb = _neighbour_value(disc, U, e2, f2, o, a, b).reshape(n, n)
            c = 1.0 if mesh.kind[e2] != M.REAL else 0.5
            jump = c * (nb - own)
            blend = (1 + x) / 2 if s else (1 - x) / 2         # along lam_d at the nodes
            shape = [1, 1, 1]
            shape[d] = n
            jt = np.zeros((n, n, n))
            idx = [slice(None)] * 3
            for i in range(n):
                idx[d] = i
                jt[tuple(idx)] = jump
            nu += blend.reshape(shape) * jt
        o0 = disc.offset[e]
        out[o0:o0 + n ** 3] = (ue + nu).reshape(-1, order="F")
    return out


def face_jumps(disc, U, npts=5, seed=0):
    """Largest jump of the element functions across the interior faces between
    real elements, at random points of each face (a check of conformity)."""
    mesh = disc.mesh
    rng = np.random.default_rng(seed)
    worst = 0.0
    for e in disc.real:
        for f in range(6):
            if mesh.bc[e, f] != M.INTERIOR:
                continue
            e2, f2, o = int(mesh.nbr[e, f]), int(mesh.nbr_face[e, f]), int(mesh.orient[e, f])
            a, b = rng.uniform(-1, 1, npts), rng.uniform(-1, 1, npts)
            own = _neighbour_value(disc, U, e, f, 0, a, b)
            nb = _neighbour_value(disc, U, e2, f2, o, a, b)
            worst = max(worst, np.abs(nb - own).max())
    return worst
