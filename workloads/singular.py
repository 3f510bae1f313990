"""Geometric meshes of the thesis's single-singularity test domains (Sec. 6.3).

Input generators only (element maps and connectivity).  Every element is a
box in the modified coordinates of its neighbourhood (Sec. 2.2-2.3):

* ``vertex_mesh``: Omega^(v) = {pi/6 <= phi <= pi/3, 0 <= theta <= 3 pi/2,
  rho <= 1} (Table 6.16) in vertex coordinates (phi, theta, chi = ln rho);
  geometric layers rho_k = mu^(N+1-k), the innermost a corner element
  carrying the vertex constant.
* ``edge_mesh``: Omega^(e)_1 = {r <= 1, 0 <= theta <= pi/2, 0 <= x3 <= 1}
  (Table 6.18) in edge coordinates (tau = ln r, theta, x3); geometric layers
  r_i = mu^(N+1-i), the innermost a corner element carrying one polynomial in
  x3 per x3-interval.
* ``vertex_edge_mesh``: the vertex-edge neighbourhood {0 < phi < phi_v,
  0 < x3 < delta_v} with rho_v = 1, phi_v = pi/6 (Table 6.20's domain, whose
  cap rho = 1 is replaced by the plane x3 = delta_v = cos phi_v, so that every
  element is a box) in (psi = ln tan phi, theta, zeta = ln x3); geometric in
  phi (tan phi_i = mu^(N+1-i) tan phi_v) and in x3 ((x3)_k = delta_v
  mu^(N+1-k)); corner elements: the vertex constant for x3 < (x3)_1, one
  polynomial in zeta per x3-layer for phi < phi_1.

Faces between boxes of one neighbourhood share their face coordinates
(orientation 0).  Faces of infinite measure in modified coordinates are
SKIP; the outer faces of the real elements are Dirichlet.  mu = 0.15 as in
the thesis's runs.
"""
import numpy as np

from . import mesh as M

MU = 0.15


class _Grid:
    """Elements indexed by (i, j, k), linked along lam directions."""

    def __init__(self):
        self.rows = []
        self.idx = {}

    def add(self, key, region, kind, chart, box, cdof=-1, cdir=0, layer=(0, 0)):
        self.idx[key] = len(self.rows)
        self.rows.append(dict(region=region, kind=kind, chart=chart, box=np.asarray(box, float),
                              cdof=cdof, cdir=cdir, layer=layer))

    def build(self, W, ncd, name, info):
        E = len(self.rows)
        eye = np.tile(np.eye(3), (E, 1, 1))
        return M.Mesh(W=W,
                      region=np.array([r["region"] for r in self.rows], np.int32),
                      kind=np.array([r["kind"] for r in self.rows], np.int32),
                      chart=np.array([r["chart"] for r in self.rows], np.int32),
                      frame=eye.copy(), mframe=eye.copy(), origin=np.zeros((E, 3)),
                      box=np.array([r["box"] for r in self.rows]), patch=np.zeros((E, 12)),
                      nbr=-np.ones((E, 6), np.int32), nbr_face=-np.ones((E, 6), np.int32),
                      orient=np.zeros((E, 6), np.int32), bc=np.full((E, 6), M.SKIP, np.int32),
                      cdof=np.array([r["cdof"] for r in self.rows], np.int32),
                      cdir=np.array([r["cdir"] for r in self.rows], np.int32),
                      n_corner_dof=ncd, name=name, info=info,
                      layer=np.array([r["layer"] for r in self.rows], np.int32))


def _link(mesh, e, f, e2, f2):
    mesh.nbr[e, f], mesh.nbr_face[e, f], mesh.bc[e, f] = e2, f2, M.INTERIOR
    mesh.nbr[e2, f2], mesh.nbr_face[e2, f2], mesh.bc[e2, f2] = e, f, M.INTERIOR


def _stitch(mesh, idx, shape, finite, neumann=()):
    """Link neighbours along lam direction d (faces 2d+1 / 2d) when the face
    has finite measure (finite(key, d)); every other real face left SKIP
    lies on the outer boundary and becomes Dirichlet, or Neumann when its
    lambda direction and side (d, s) are listed in neumann."""
    for key, e in idx.items():
        for d in range(3):
            nxt = list(key)
            nxt[d] += 1
            if nxt[d] < shape[d] and finite(key, d) and finite(tuple(nxt), d):
                _link(mesh, e, 2 * d + 1, idx[tuple(nxt)], 2 * d)
    for key, e in idx.items():
        if mesh.kind[e] != M.REAL:
            continue
        for d in range(3):
            for s in (0, 1):
                f = 2 * d + s
                if mesh.bc[e, f] != M.SKIP:
                    continue
                edge = key[d] == (shape[d] - 1 if s else 0)
                if not edge:
                    raise ValueError("unlinked inner face %s/%d" % (key, f))
                mesh.bc[e, f] = M.NEUMANN if (d, s) in neumann else M.DIRICHLET


def vertex_mesh(N, W=None, I=1, J=1, mu=MU, phi=(np.pi / 6, np.pi / 3), theta=(0.0, 1.5 * np.pi), rho=1.0,
                neumann=()):
    """Omega^(v): J phi-sectors x I theta-sectors x (N+1) rho-layers (layer 0 the corner)."""
    W = N if W is None else W
    ph = np.linspace(phi[0], phi[1], J + 1)
    th = np.linspace(theta[0], theta[1], I + 1)
    chi = [None] + [np.log(rho * mu ** (N + 1 - k)) for k in range(1, N + 2)]
    g = _Grid()
    for k in range(N + 1):
        c0, c1 = (chi[k], chi[k + 1]) if k else (chi[1] - 1.0, chi[1])
        for j in range(I):
            for i in range(J):
                box = (ph[i], ph[i + 1], th[j], th[j + 1], c0, c1)
                if k:
                    g.add((i, j, k), M.VTX, M.REAL, M.VTX_BOX, box, layer=(k, 0))
                else:
                    g.add((i, j, k), M.VTX, M.CORNER_CONST, M.VTX_BOX, box, cdof=0)
    mesh = g.build(W, 1, "vertex N=%d W=%d" % (N, W), dict(N=N, W=W, I=I, J=J, mu=mu))
    # the corner layer only meets the first real layer (its other faces are semi-infinite)
    _stitch(mesh, g.idx, (J, I, N + 1), lambda key, d: key[2] >= 1 or d == 2, neumann)
    return mesh


def edge_mesh(N, W=None, I=1, Je=1, mu=MU, theta=(0.0, 0.5 * np.pi), Z=1.0, x3=(0.0, 1.0), neumann=()):
    """Omega^(e)_1: (N+1) r-layers (layer 0 the corner) x I theta-sectors x Je x3-intervals."""
    W = N if W is None else W
    n = W + 1
    th = np.linspace(theta[0], theta[1], I + 1)
    zs = np.linspace(x3[0], x3[1], Je + 1)
    tau = [None] + [np.log(Z * mu ** (N + 1 - i)) for i in range(1, N + 2)]
    g = _Grid()
    for l in range(Je):
        for j in range(I):
            for i in range(N + 1):
                t0, t1 = (tau[i], tau[i + 1]) if i else (tau[1] - 1.0, tau[1])
                box = (t0, t1, th[j], th[j + 1], zs[l], zs[l + 1])
                if i:
                    g.add((i, j, l), M.EDGE, M.REAL, M.EDGE_BOX, box, layer=(i, 0))
                else:
                    g.add((i, j, l), M.EDGE, M.CORNER_POLY, M.EDGE_BOX, box, cdof=l * n, cdir=2)
    mesh = g.build(W, Je * n, "edge N=%d W=%d" % (N, W), dict(N=N, W=W, I=I, Je=Je, mu=mu))
    _stitch(mesh, g.idx, (N + 1, I, Je), lambda key, d: key[0] >= 1 or d == 0, neumann)
    return mesh


def vertex_edge_mesh(N, W=None, I=1, mu=MU, phi_v=np.pi / 6, theta=(0.0, 1.5 * np.pi), rho_v=1.0, neumann=()):
    """Vertex-edge neighbourhood: (N+1) phi-layers x I theta-sectors x (N+1)
    x3-layers; phi-layer 0 and x3-layer 0 are corner elements."""
    W = N if W is None else W
    n = W + 1
    dv = rho_v * np.cos(phi_v)
    th = np.linspace(theta[0], theta[1], I + 1)
    psi = [None] + [np.log(mu ** (N + 1 - i) * np.tan(phi_v)) for i in range(1, N + 2)]
    zeta = [None] + [np.log(dv * mu ** (N + 1 - k)) for k in range(1, N + 2)]
    g = _Grid()
    for k in range(N + 1):
        for j in range(I):
            for i in range(N + 1):
                p0, p1 = (psi[i], psi[i + 1]) if i else (psi[1] - 1.0, psi[1])
                z0, z1 = (zeta[k], zeta[k + 1]) if k else (zeta[1] - 1.0, zeta[1])
                box = (p0, p1, th[j], th[j + 1], z0, z1)
                if k == 0:
                    g.add((i, j, k), M.VE, M.CORNER_CONST, M.VE_BOX, box, cdof=0)
                elif i == 0:
                    g.add((i, j, k), M.VE, M.CORNER_POLY, M.VE_BOX, box, cdof=1 + (k - 1) * n, cdir=2)
                else:
                    g.add((i, j, k), M.VE, M.REAL, M.VE_BOX, box, layer=(i, k))
    mesh = g.build(W, 1 + N * n, "vertex-edge N=%d W=%d" % (N, W), dict(N=N, W=W, I=I, mu=mu))

    def finite(key, d):
        i, _, k = key
        if i >= 1 and k >= 1:
            return True
        # corner polynomials (i = 0) meet the real elements across psi;
        # the vertex constant (k = 0) meets them across zeta
        return (i == 0 and k >= 1 and d == 0) or (k == 0 and i >= 1 and d == 2)
    _stitch(mesh, g.idx, (N + 1, I, N + 1), finite, neumann)
    return mesh
