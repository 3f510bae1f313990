"""Per-element polynomial degrees of a layer-graded mesh (thesis Sec. 2.3).

Input generator only: the degree triple (w1, w2, w3) of every element, one
per master-cube direction lam_d, from the mesh's geometric layer indices
(``Mesh.layer``: (i, k), 0 where the region has no such layer):

* regular region:          (W, W, W)
* vertex layers  i:        ([mu1 i], [mu1 i], [mu1 i])          (phi, theta, chi)
* edge layers    i:        ([mu1 i], [mu1 i], W)                (tau, theta, x3)
* vertex-edge    (i, k):   ([mu1 i], [mu1 i], [mu2 k])          (psi, theta, zeta)

[a] is the largest integer <= a, clipped to 1..W.  Corner elements get W
(their functions keep the mesh's degree).
"""
import numpy as np

from . import mesh as M


def layer_degrees(mesh, mu1, mu2=None):
    """[E, 3] int32 degrees."""
    W = mesh.W
    mu2 = mu1 if mu2 is None else mu2
    deg = np.full((mesh.E, 3), W, np.int32)
    if mesh.layer is None:
        return deg
    clip = lambda a: int(min(W, max(1, np.floor(a + 1e-12))))
    for e in range(mesh.E):
        if mesh.kind[e] != M.REAL:
            continue
        i, k = (int(v) for v in mesh.layer[e])
        reg = mesh.region[e]
        if reg == M.VTX:
            deg[e] = clip(mu1 * i)
        elif reg == M.EDGE:
            deg[e, :2] = clip(mu1 * i)
        elif reg == M.VE:
            deg[e, :2] = clip(mu1 * i)
            deg[e, 2] = clip(mu2 * k)
    return deg


def graded_dof(mesh, deg):
    """Unknowns of the graded space: sum over real elements of prod (w_d + 1),
    plus the corner unknowns."""
    real = mesh.kind == M.REAL
    return int(np.prod(np.asarray(deg)[real] + 1, axis=1).sum()) + mesh.n_corner_dof
