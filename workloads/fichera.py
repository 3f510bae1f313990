"""Geometric mesh of the Fichera corner  Omega = (-1,1)^3 minus [0,1)^3.

Input generator only (element maps and connectivity), following the domain
decomposition of the thesis, Sec. 2.2-2.3, at the re-entrant vertex v = 0 and
the three re-entrant edges along +e_1, +e_2, +e_3:

* vertex neighbourhood  Omega^v = {rho < rho_v} minus the cones phi < phi_v
  around the three edges (Sec. 2.2.1); geometric layers
  rho_k = rho_v mu^(N+1-k) (Sec. 2.3), the innermost layer a corner element
  carrying the vertex constant h_v;
* vertex-edge neighbourhoods {phi < phi_v, 0 < x3 < delta_v} in (psi, theta,
  zeta) (eq 2.8), geometric in phi (tan phi_i = mu^(N+1-i) tan phi_v) and in
  x3 ((x3)_k = delta_v mu^(N+1-k)), N_{v-e} = I (N+1)^2 elements;
* edge neighbourhoods {r < Z, delta_v < x3 < 1} in (tau, theta, x3) (eq 2.5),
  r_i = Z mu^(N+1-i), J_e intervals in x3, N_e = I J_e (N+1);
* the regular region: one "column" per sphere patch, blending the sphere
  rho = rho_v to the outer faces of the cube (and, next to an edge, the
  cylinder r = Z).

The sphere S^v (seven octants of it, minus the three cone caps) is split by
the cube-face partition: in each octant the part where |x_b| is largest is
mapped gnomonically to the plane x_b = +-1.  On a positive face the cone cap
is a quarter disc of radius tan(phi_v) around the edge; the rest is split
into two polar patches per octant (theta sectors of pi/4), so every edge sees
I = 6 theta-sectors over its 3 pi/2 opening.  Negative faces are squares.

rho_v = 1/2, phi_v = pi/6 (Z = rho_v sin phi_v = 1/4, delta_v = rho_v cos
phi_v), mu_v = mu_e = 0.15 (the thesis's choice, Sec. 6.3).
"""
import numpy as np

from . import mesh as M

RHO_V = 0.5
PHI_V = np.pi / 6
MU = 0.15


def axis_frame(a):
    """Columns = images of the local X, Y, Z axes; Z = +e_a, cyclic X, Y."""
    R = np.zeros((3, 3))
    R[(a + 1) % 3, 0] = 1.0
    R[(a + 2) % 3, 1] = 1.0
    R[a, 2] = 1.0
    return R


def neg_frame(b):
    """Z = -e_b, X = e_{b+1}, Y = -e_{b+2} (right-handed)."""
    R = np.zeros((3, 3))
    R[(b + 1) % 3, 0] = 1.0
    R[(b + 2) % 3, 1] = -1.0
    R[b, 2] = -1.0
    return R


def _ray_hit(th):
    """Where the ray at angle th leaves the square max(|X|, |Y|) = 1."""
    c, s = np.cos(th), np.sin(th)
    t = 1.0 / max(abs(c), abs(s))
    snap = lambda v: 0.0 if abs(v) < 1e-14 else (np.sign(v) if abs(abs(v) - 1) < 1e-14 else v)
    return snap(c * t), snap(s * t)


class _Builder:
    def __init__(self, W):
        self.W = W
        self.rows = []

    def add(self, region, kind, chart, frame, box, patch=None, mframe=None, cdof=-1, cdir=0, key=None, layer=(0, 0)):
        self.rows.append(dict(region=region, kind=kind, chart=chart, frame=frame,
                              mframe=frame if mframe is None else mframe,
                              box=np.asarray(box, float), patch=np.zeros(12) if patch is None else np.asarray(patch, float),
                              cdof=cdof, cdir=cdir, key=key, layer=layer))
        return len(self.rows) - 1


def fichera_mesh(N=6, W=None, Je=1, mu=MU, rho_v=RHO_V, phi_v=PHI_V):
    W = N if W is None else W
    n = W + 1
    Z = rho_v * np.sin(phi_v)
    dv = rho_v * np.cos(phi_v)
    B = _Builder(W)
    idx = {}
    # corner DOF layout: h_v, then per axis the vertex-edge polynomials
    # (layers k = 1..N), then per axis the edge polynomials (intervals)
    hv = 0
    ve_poly = lambda a, k: 1 + (a * N + (k - 1)) * n
    ed_poly = lambda a, l: 1 + 3 * N * n + (a * Je + l) * n
    ncd = 1 + 3 * N * n + 3 * Je * n

    psi = [None] + [np.log(mu ** (N + 1 - i) * np.tan(phi_v)) for i in range(1, N + 2)]
    zeta = [None] + [np.log(dv * mu ** (N + 1 - k)) for k in range(1, N + 2)]
    tau = [None] + [np.log(Z * mu ** (N + 1 - i)) for i in range(1, N + 2)]
    chi = [None] + [np.log(rho_v * mu ** (N + 1 - k)) for k in range(1, N + 2)]
    th = [np.pi / 2 + j * np.pi / 4 for j in range(7)]
    x3e = [dv + (1 - dv) * l / Je for l in range(Je + 1)]

    # ---------------------------------------------------- vertex-edge regions
    for a in range(3):
        R = axis_frame(a)
        for k in range(N + 1):
            for j in range(6):
                for i in range(N + 1):
                    p0 = psi[i] if i else psi[1] - 1.0
                    p1 = psi[i + 1] if i else psi[1]
                    z0 = zeta[k] if k else zeta[1] - 1.0
                    z1 = zeta[k + 1] if k else zeta[1]
                    box = (p0, p1, th[j], th[j + 1], z0, z1)
                    if i >= 1 and k >= 1:
                        e = B.add(M.VE, M.REAL, M.VE_BOX, R, box, layer=(i, k))
                    elif i == 0 and k >= 1:
                        e = B.add(M.VE, M.CORNER_POLY, M.VE_BOX, R, box, cdof=ve_poly(a, k), cdir=2)
                    else:
                        e = B.add(M.VE, M.CORNER_CONST, M.VE_BOX, R, box, cdof=hv)
                    idx[("ve", a, i, j, k)] = e
    # ---------------------------------------------------- edge regions
    for a in range(3):
        R = axis_frame(a)
        for l in range(Je):
            for j in range(6):
                for i in range(N + 1):
                    t0 = tau[i] if i else tau[1] - 1.0
                    t1 = tau[i + 1] if i else tau[1]
                    box = (t0, t1, th[j], th[j + 1], x3e[l], x3e[l + 1])
                    if i >= 1:
                        e = B.add(M.EDGE, M.REAL, M.EDGE_BOX, R, box, layer=(i, 0))
                    else:
                        e = B.add(M.EDGE, M.CORNER_POLY, M.EDGE_BOX, R, box, cdof=ed_poly(a, l), cdir=2)
                    idx[("ed", a, i, j, l)] = e
    # ---------------------------------------------------- sphere patches
    patches = []   # (frame, mframe, patch row, (cone axis, theta sector) or -1)
    for s in [(s1, s2, s3) for s1 in (1, -1) for s2 in (1, -1) for s3 in (1, -1)]:
        if s == (1, 1, 1):
            continue
        for b in range(3):
            if s[b] > 0:
                R = axis_frame(b)
                sx, sy = s[(b + 1) % 3], s[(b + 2) % 3]
                q0 = {(-1, 1): np.pi / 2, (-1, -1): np.pi, (1, -1): 1.5 * np.pi}[(sx, sy)]
                for h in range(2):
                    ta, tb = q0 + h * np.pi / 4, q0 + (h + 1) * np.pi / 4
                    oa, ob = _ray_hit(ta), _ray_hit(tb)
                    row = [0, ta, tb, np.tan(phi_v), Z, oa[0], oa[1], ob[0], ob[1], rho_v, 0, 0]
                    patches.append((R, R, row, (b, int(round((ta - np.pi / 2) / (np.pi / 4))))))
            else:
                R = neg_frame(b)
                sx, sy = s[(b + 1) % 3], -s[(b + 2) % 3]
                row = [1, 0.0, 0.0, sx, 0.0, 0.0, sy, sx, sy, rho_v, 0, 0]
                mf = axis_frame((b + 1) % 3)
                patches.append((R, mf, row, -1))
    for p, (R, mf, row, cone) in enumerate(patches):
        for k in range(N + 1):
            c0 = chi[k] if k else chi[1] - 1.0
            c1 = chi[k + 1] if k else chi[1]
            box = (-1, 1, -1, 1, c0, c1)
            kind = M.REAL if k else M.CORNER_CONST
            e = B.add(M.VTX, kind, M.VTX_PATCH, R, box, row, mframe=mf, cdof=-1 if k else hv, layer=(k, 0))
            idx[("vx", p, k)] = e
        for l in range(Je):
            e = B.add(M.REG, M.REAL, M.COLUMN, R, (-1, 1, -1, 1, l / Je, (l + 1) / Je), row)
            idx[("col", p, l)] = e

    rows = B.rows
    E = len(rows)
    mesh = M.Mesh(W=W,
                  region=np.array([r["region"] for r in rows], np.int32),
                  kind=np.array([r["kind"] for r in rows], np.int32),
                  chart=np.array([r["chart"] for r in rows], np.int32),
                  frame=np.array([r["frame"] for r in rows]),
                  mframe=np.array([r["mframe"] for r in rows]),
                  origin=np.zeros((E, 3)),
                  box=np.array([r["box"] for r in rows]),
                  patch=np.array([r["patch"] for r in rows]),
                  nbr=-np.ones((E, 6), np.int32), nbr_face=-np.ones((E, 6), np.int32),
                  orient=np.zeros((E, 6), np.int32), bc=np.full((E, 6), M.SKIP, np.int32),
                  cdof=np.array([r["cdof"] for r in rows], np.int32),
                  cdir=np.array([r["cdir"] for r in rows], np.int32),
                  n_corner_dof=ncd, name="fichera N=%d W=%d" % (N, W),
                  info=dict(N=N, W=W, Je=Je, mu=mu, rho_v=rho_v, phi_v=phi_v, I=6, patches=len(patches)),
                  layer=np.array([r["layer"] for r in rows], np.int32))

    def link(e, f, e2, f2, o=None):
        if o is None:
            o = M.find_orientation(mesh, e, f, e2, f2)
            if o is None:
                raise ValueError("faces do not conform: %d/%d - %d/%d" % (e, f, e2, f2))
        mesh.nbr[e, f], mesh.nbr_face[e, f], mesh.orient[e, f] = e2, f2, o
        mesh.bc[e, f] = M.INTERIOR
        inv = [oo for oo in range(8)
               if np.allclose(M.orient_map(oo, *M.orient_map(o, 0.3, -0.7)), (0.3, -0.7))][0]
        mesh.nbr[e2, f2], mesh.nbr_face[e2, f2], mesh.orient[e2, f2] = e, f, inv
        mesh.bc[e2, f2] = M.INTERIOR

    # Structured connectivity of the neighbourhoods: the boxes share exact
    # modified-coordinate values, so the faces coincide with orientation 0
    # (the thin elements next to the edge defeat any physical-point matching).
    polar = {cone: p for p, (_, _, _, cone) in enumerate(patches) if cone != -1}
    for a in range(3):
        for j in range(6):
            for k in range(1, N + 1):
                link(idx[("ve", a, 0, j, k)], 1, idx[("ve", a, 1, j, k)], 0, 0)
            for i in range(1, N + 1):
                link(idx[("ve", a, i, j, 0)], 5, idx[("ve", a, i, j, 1)], 4, 0)
            for l in range(Je):
                link(idx[("ed", a, 0, j, l)], 1, idx[("ed", a, 1, j, l)], 0, 0)
            for i in range(1, N + 1):
                for k in range(1, N + 1):
                    e = idx[("ve", a, i, j, k)]
                    if i < N:
                        link(e, 1, idx[("ve", a, i + 1, j, k)], 0, 0)
                    else:
                        link(e, 1, idx[("vx", polar[(a, j)], k)], 2, 0)
                    if j < 5:
                        link(e, 3, idx[("ve", a, i, j + 1, k)], 2, 0)
                    if k < N:
                        link(e, 5, idx[("ve", a, i, j, k + 1)], 4, 0)
                    else:
                        link(e, 5, idx[("ed", a, i, j, 0)], 4, 0)
                    if j == 0:
                        mesh.bc[e, 2] = M.DIRICHLET
                    if j == 5:
                        mesh.bc[e, 3] = M.DIRICHLET
                for l in range(Je):
                    e = idx[("ed", a, i, j, l)]
                    if i < N:
                        link(e, 1, idx[("ed", a, i + 1, j, l)], 0, 0)
                    else:
                        link(e, 1, idx[("col", polar[(a, j)], l)], 2, 0)
                    if j < 5:
                        link(e, 3, idx[("ed", a, i, j + 1, l)], 2, 0)
                    if l < Je - 1:
                        link(e, 5, idx[("ed", a, i, j, l + 1)], 4, 0)
                    else:
                        mesh.bc[e, 5] = M.DIRICHLET
                    if j == 0:
                        mesh.bc[e, 2] = M.DIRICHLET
                    if j == 5:
                        mesh.bc[e, 3] = M.DIRICHLET
    for p in range(len(patches)):
        link(idx[("vx", p, 0)], 5, idx[("vx", p, 1)], 4, 0)

    # real elements: match faces by their physical points (tolerance relative
    # to the face size: faces near the vertex are ~mu^N small)
    from scipy.spatial import cKDTree
    real = np.nonzero(mesh.kind == M.REAL)[0]
    cand = [(e, f) for e in real for f in range(6)
            if mesh.bc[e, f] == M.SKIP and mesh.region[e] in (M.VTX, M.REG)]
    cen = np.array([M.chart_points(mesh, e, M.face_lam(f, 0.0, 0.0)) for e, f in cand])
    dia = np.array([np.linalg.norm(M.chart_points(mesh, e, M.face_lam(f, 1.0, 1.0))
                                   - M.chart_points(mesh, e, M.face_lam(f, -1.0, -1.0))) for e, f in cand])
    tree = cKDTree(cen)
    done = np.zeros(len(cand), bool)
    for i, (e, f) in enumerate(cand):
        if done[i]:
            continue
        js = [j for j in tree.query_ball_point(cen[i], 1e-6 * dia[i]) if j != i and not done[j]]
        js = [j for j in js if M.find_orientation(mesh, e, f, *cand[j]) is not None]
        if len(js) == 1:
            link(e, f, *cand[js[0]])
            done[i] = done[js[0]] = True
        elif not js:
            pts = M.chart_points(mesh, e, M.face_lam(f, np.array([0.0, -0.8, 0.6]), np.array([0.0, 0.5, -0.9])))
            if not all(_on_boundary(x) for x in pts):
                raise ValueError("unmatched interior face %d/%d at %s" % (e, f, pts[0]))
            mesh.bc[e, f] = M.DIRICHLET
            done[i] = True
        else:
            raise ValueError("face %d/%d matched %d times" % (e, f, len(js)))
    return mesh


def _on_boundary(x, tol=1e-9):
    """On the boundary of (-1,1)^3 minus [0,1)^3."""
    if np.max(np.abs(x)) > 1 - tol:
        return True
    for a in range(3):
        others = [x[(a + 1) % 3], x[(a + 2) % 3]]
        if abs(x[a]) < tol and min(others) > -tol:
            return True
    return False
