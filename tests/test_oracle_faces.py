"""Face terms of the oracle against the thesis's norms evaluated by brute force.

For one face of every kind the oracle's discrete face term (GLL double sums
on the (2W+1) x (2W+1) face grid of side A, extents folded into constant
factors, jumps through its trace matrices) is compared with the norm as the
thesis prints it:

* regular faces, eq 2.16 with the norms of eq 2.17b on the master square;
  regular Dirichlet faces, eq 2.18 (the 3/2-norm) with data, eq 4.2;
* vertex faces, eq 2.25 / 4.3: the same norms scaled by R = sup e^chi;
* vertex-edge faces, eq 2.27a-c inside eq 2.29 / 4.5 (E, F, G);
* edge faces, eq 2.34a-c inside eq 2.38 / 4.7 (G, H);
* the readings for faces between regions (counted once, in the coordinates
  of the more singular side, derivatives of the other side transformed)
  and for Dirichlet faces of the neighbourhoods (tangential derivatives,
  the third one weighted like its jump, the L2 weight of the interior term).

The brute-force side shares nothing with the oracle's face machinery: the
element functions are evaluated from the unknown vector by their own
Lagrange interpolation; the face is parametrised by the coordinates its
norm is written in (the master square of side A for regular and vertex
faces, the actual rectangle in modified coordinates for vertex-edge and
edge faces); derivatives in modified coordinates come from complex-step
differentiation of the element maps composed with the closed-form
modified coordinates of the neighbourhood (Newton inversion of the
neighbour's map); the sups R, E, F, G, H are maxima over sampled physical
face points; the L2 integrals and the double integrals of the difference
quotients are Gauss-Legendre sums over the actual extents (two different
rules for s and s', so no point pair coincides).

Where every jump is a polynomial of degree <= W in the coordinates of the
norm (boxes in one neighbourhood, or the regular affine mesh) the GLL double
sum is exact (pinned in test_oracle_pins) and the two agree to rounding.
Where a side is curved the traces are smooth but not polynomial and the two
agree to the quadrature error of the (2W+1)-point rule; that tolerance
still separates every plausible misreading (a swapped extent, a misplaced
E, F, G, H or R) by orders of magnitude, which the planted-mistake test
checks.
"""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from workloads import mesh as M
from workloads.fichera import fichera_mesh
from workloads.singular import vertex_mesh, edge_mesh, vertex_edge_mesh
from workloads.problems import Problem, Polynomial
from oracle.functional import Discretization

H_CS = 1e-20          # complex step
PRIO = {M.REG: 0, M.VTX: 1, M.EDGE: 2, M.VE: 3}


class Zero(Problem):
    """Homogeneous data: the Dirichlet terms are the norms of the trace itself."""

    def u(self, x):
        return np.zeros(np.asarray(x).shape[:-1])

    def grad_u(self, x):
        return np.zeros(np.asarray(x).shape)

    def f(self, x):
        return np.zeros(np.asarray(x).shape[:-1])


# ------------------------------------------------------------ element functions
def gll_nodes(n):
    """n GLL nodes: -1, the roots of P'_{n-1}, 1."""
    inner = npleg.Legendre.basis(n - 1).deriv().roots()
    return np.concatenate([[-1.0], np.sort(inner.real), [1.0]])


def lagrange_polys(nodes):
    out = []
    for j, xj in enumerate(nodes):
        others = np.delete(nodes, j)
        p = np.polynomial.Polynomial.fromroots(others)
        out.append(p / p(xj))
    return out


class ElementFunctions:
    """u_e(lam) and grad_lam u_e from the unknown vector (layout: real
    elements in mesh order, n^3 values each, i fastest; then the corner
    unknowns, the constant or the n nodal values of the 1D polynomial)."""

    def __init__(self, mesh, U):
        self.mesh, self.U = mesh, U
        self.n = mesh.W + 1
        self.polys = lagrange_polys(gll_nodes(self.n))
        self.dpolys = [p.deriv() for p in self.polys]
        real = mesh.real_elements()
        self.off = {int(e): i * self.n ** 3 for i, e in enumerate(real)}
        self.nreal = len(real) * self.n ** 3

    def coeffs(self, e):
        n, mesh = self.n, self.mesh
        if mesh.kind[e] == M.REAL:
            o = self.off[e]
            return self.U[o:o + n ** 3].reshape((n, n, n), order="F")
        c = self.nreal + mesh.cdof[e]
        if mesh.kind[e] == M.CORNER_CONST:
            return np.full((n, n, n), self.U[c])
        shape = [1, 1, 1]
        shape[mesh.cdir[e]] = n
        return np.broadcast_to(self.U[c:c + n].reshape(shape), (n, n, n))

    def value_grad(self, e, lam):
        """u [P] and du/dlam [P, 3] at real points lam [P, 3]."""
        C = self.coeffs(e)
        L = [np.stack([p(lam[:, d]) for p in self.polys], -1) for d in range(3)]
        D = [np.stack([p(lam[:, d]) for p in self.dpolys], -1) for d in range(3)]
        val = np.einsum("ijk,pi,pj,pk->p", C, L[0], L[1], L[2])
        g = np.stack([np.einsum("ijk,pi,pj,pk->p", C, D[0], L[1], L[2]),
                      np.einsum("ijk,pi,pj,pk->p", C, L[0], D[1], L[2]),
                      np.einsum("ijk,pi,pj,pk->p", C, L[0], L[1], D[2])], -1)
        return val, g


# ------------------------------------------------------------ geometry by complex steps
def modified_coords(region, R, o, x, th_ref):
    """Closed-form modified coordinates of the neighbourhood frame (R, o)
    (vertex: phi, theta, chi = ln rho; vertex-edge: psi = ln tan phi,
    theta, zeta = ln x3; edge: tau = ln r, theta, x3; regular: x), complex
    capable.  theta by the half-angle formula about th_ref."""
    if region == M.REG:
        return x
    xl = (x - o) @ R
    a, b, c = xl[..., 0], xl[..., 1], xl[..., 2]
    ca, sa = np.cos(th_ref), np.sin(th_ref)
    ar, br = ca * a + sa * b, -sa * a + ca * b
    r = np.sqrt(a * a + b * b)
    th = th_ref + 2 * np.arctan(br / (r + ar))
    if region == M.VTX:
        rho = np.sqrt(r * r + c * c)
        return np.stack([np.arccos(c / rho), th, np.log(rho)], -1)
    if region == M.VE:
        return np.stack([np.log(r / c), th, np.log(c)], -1)
    return np.stack([np.log(r), th, c], -1)


def chart_jacobian(mesh, e, lam):
    """dx/dlam [P, 3, 3] by complex steps."""
    return np.stack([M.chart_points(mesh, e, lam + 1j * H_CS * np.eye(3)[c]).imag / H_CS
                     for c in range(3)], -1)


def chart_inverse(mesh, e, x, lam0, iters=60):
    """lam with chart(e, lam) = x (complex x allowed): Newton with the
    Jacobian at the real part."""
    lam = np.asarray(lam0, complex).copy()
    for _ in range(iters):
        F = M.chart_points(mesh, e, lam) - x
        J = chart_jacobian(mesh, e, lam.real)
        lam = lam - np.linalg.solve(J, F[..., None])[..., 0]
    err = np.abs(M.chart_points(mesh, e, lam.real) - x.real).max()
    assert err < 1e-13, err
    return lam


def face_evaluator(mesh, fun, eA, fA, eB, fB, region, s, t, param):
    """Values and derivatives in the norm's coordinates of both sides at the
    face points given by parameters (s, t) [P].

    param = ("lam",): (s, t) are side A's face coordinates on the master square;
            ("y",): (s, t) are the two tangential modified coordinates
            (face normal fixed by fA), y mapped to side A's lam affinely.
    Returns dict with uA, gA [P,3] (derivatives in the modified coordinates
    of the chosen region, x for regular), uB, gB (None for Dirichlet), x [P,3]."""
    d = fA // 2
    t0, t1 = M.FACE_TANGENT[d]
    P = s.size
    lamA = np.zeros((P, 3))
    lamA[:, d] = 1.0 if fA % 2 else -1.0
    if param[0] == "lam":
        lamA[:, t0], lamA[:, t1] = s, t
    else:
        box = mesh.box[eA]
        for c, v in ((t0, s), (t1, t)):
            lamA[:, c] = 2 * (v - box[2 * c]) / (box[2 * c + 1] - box[2 * c]) - 1
    R = mesh.mframe[eA] if region == M.VTX else mesh.frame[eA]
    o = mesh.origin[eA]
    x = M.chart_points(mesh, eA, lamA)
    xl = (x - o) @ R
    th_ref = float(np.mean(np.arctan2(xl[:, 1], xl[:, 0])))
    # dY/dlamA and its inverse
    dY = np.stack([modified_coords(region, R, o, M.chart_points(mesh, eA, lamA + 1j * H_CS * np.eye(3)[c]),
                                   th_ref).imag / H_CS for c in range(3)], -1)     # [P, k, c]
    dlamA_dY = np.linalg.inv(dY)                                                  # [P, c, k]
    out = dict(x=x)
    uA, glA = fun.value_grad(eA, lamA)
    out["uA"] = uA
    out["gA"] = np.einsum("pck,pc->pk", dlamA_dY, glA)
    if eB < 0:
        out["uB"] = out["gB"] = None
        return out
    # side B: lamB(lamA) by Newton from the mesh's face correspondence
    o_ab = mesh.orient[eA, fA]
    a, b = M.orient_map(o_ab, lamA[:, t0], lamA[:, t1])
    guess = M.face_lam(fB, a, b)
    lamB = chart_inverse(mesh, eB, x, guess).real
    dlamB_dlamA = np.stack([chart_inverse(mesh, eB, M.chart_points(mesh, eA, lamA + 1j * H_CS * np.eye(3)[c]),
                                          lamB).imag / H_CS for c in range(3)], -1)   # [P, b, c]
    dlamB_dY = np.einsum("pbc,pck->pbk", dlamB_dlamA, dlamA_dY)
    uB, glB = fun.value_grad(eB, lamB)
    out["uB"] = uB
    out["gB"] = np.einsum("pbk,pb->pk", dlamB_dY, glB)
    return out


# ------------------------------------------------------------ brute-force norms
def rules(a, b, q):
    """Two Gauss-Legendre rules on [a, b] with q and q + 1 points."""
    out = []
    for k in (q, q + 1):
        xg, wg = npleg.leggauss(k)
        out.append((a + (b - a) * (xg + 1) / 2, wg * (b - a) / 2))
    return out


class FaceQuadrature:
    """Evaluates integrands on the union grid of two rules per direction."""

    def __init__(self, s_rng, t_rng, q):
        (self.s1, self.ws1), (self.s2, self.ws2) = rules(*s_rng, q)
        (self.t1, self.wt1), (self.t2, self.wt2) = rules(*t_rng, q)
        self.S = np.concatenate([self.s1, self.s2])
        self.T = np.concatenate([self.t1, self.t2])
        self.n1s, self.n1t = len(self.s1), len(self.t1)
        SS, TT = np.meshgrid(self.S, self.T, indexing="ij")
        self.s, self.t = SS.ravel(), TT.ravel()

    def grid(self, v):
        return v.reshape(len(self.S), len(self.T))

    def l2(self, v):
        g = self.grid(v)[:self.n1s, :self.n1t]
        return np.einsum("i,j,ij->", self.ws1, self.wt1, g ** 2)

    def quotient_s(self, v):
        """int dt int int (w(s,t) - w(s',t))^2 / (s - s')^2 ds ds'."""
        g = self.grid(v)
        a, b = g[:self.n1s, :self.n1t], g[self.n1s:, :self.n1t]
        diff = (a[:, None, :] - b[None, :, :]) / (self.s1[:, None, None] - self.s2[None, :, None])
        return np.einsum("i,k,j,ikj->", self.ws1, self.ws2, self.wt1, diff ** 2)

    def quotient_t(self, v):
        g = self.grid(v)
        a, b = g[:self.n1s, :self.n1t], g[:self.n1s, self.n1t:]
        diff = (a[:, :, None] - b[:, None, :]) / (self.t1[:, None] - self.t2[None, :])[None]
        return np.einsum("i,j,k,ijk->", self.ws1, self.wt1, self.wt2, diff ** 2)


def sup_weights(region, R, o, x):
    """R = sup e^chi (vertex); E = sup sin phi, F = sup e^zeta (vertex-edge);
    G = sup e^tau (edge): maxima over the sampled physical face points."""
    xl = (x - o) @ R
    r = np.hypot(xl[:, 0], xl[:, 1])
    rho = np.linalg.norm(xl, axis=1)
    if region == M.VTX:
        return dict(R=rho.max())
    if region == M.VE:
        return dict(E=(r / rho).max(), F=xl[:, 2].max())
    if region == M.EDGE:
        return dict(G=r.max())
    return {}


def brute_face(mesh, fun, eA, fA, eB, fB, region, problem=None, q=None, sample=41):
    """The face's contribution to the functional, from the norms as printed."""
    W = mesh.W
    d = fA // 2
    t0, t1 = M.FACE_TANGENT[d]
    curved = any(mesh.chart[e] in (M.VTX_PATCH, M.COLUMN) for e in (eA, eB) if e >= 0)
    q = q or (24 if curved else W + 3)
    if region in (M.REG, M.VTX):
        param = ("lam",)
        s_rng = t_rng = (-1.0, 1.0)
    else:
        box = mesh.box[eA]
        s_rng, t_rng = (box[2 * t0], box[2 * t0 + 1]), (box[2 * t1], box[2 * t1 + 1])
        param = ("y",)
    Q = FaceQuadrature(s_rng, t_rng, q)
    ev = face_evaluator(mesh, fun, eA, fA, eB, fB, region, Q.s, Q.t, param)
    # sups over a fine sample of the face (corners included)
    ss, tt = np.meshgrid(np.linspace(*s_rng, sample), np.linspace(*t_rng, sample), indexing="ij")
    R = mesh.mframe[eA] if region == M.VTX else mesh.frame[eA]
    xs = face_evaluator(mesh, fun, eA, fA, -1, -1, region, ss.ravel(), tt.ravel(), param)["x"]
    sw = sup_weights(region, R, mesh.origin[eA], xs)

    dirichlet = eB < 0
    if dirichlet:
        g = problem.u(ev["x"]) if problem is not None else 0.0
        jump = ev["uA"] - g
    else:
        jump = ev["uA"] - ev["uB"]

    if region in (M.REG, M.VTX):
        scale = sw.get("R", 1.0)
        half = lambda w: Q.l2(w) + Q.quotient_s(w) + Q.quotient_t(w)   # eq 2.17b, sigma = 1/2
        if not dirichlet:
            # eq 2.16 / 2.25: ||[u]||_0^2 + sum_k ||[u_{x_k}]||_{1/2}^2
            total = Q.l2(jump) + sum(half(ev["gA"][:, k] - ev["gB"][:, k]) for k in range(3))
        else:
            # eq 2.18 with sigma = 1/2: ||w||_0^2 + sum_i ||dw/dlam_i||_{1/2}^2,
            # lam_i the face's own coordinates of side A
            lamA = np.zeros((Q.s.size, 3))
            lamA[:, d] = 1.0 if fA % 2 else -1.0
            lamA[:, t0], lamA[:, t1] = Q.s, Q.t
            _, glA = fun.value_grad(eA, lamA)
            total = Q.l2(jump)
            for i, c in enumerate((t0, t1)):
                dg = 0.0
                if problem is not None:
                    JA = chart_jacobian(mesh, eA, lamA)
                    dg = np.einsum("pa,pa->p", problem.grad_u(ev["x"]), JA[:, :, c])
                total += half(glA[:, c] - dg)
        return scale * total

    # vertex-edge and edge faces: |||.||| of eq 2.27 / 2.34 on the actual rectangle
    if region == M.VE:
        E, F = sw["E"], sw["F"]
        # eq 2.27a (zeta-face): E F (L2 + Q_psi + Q_theta); 2.27b (psi-face):
        # F (L2 + Q_theta + E Q_zeta); 2.27c (theta-face): F (L2 + Q_psi + E Q_zeta)
        outer = E * F if d == 2 else F
        wq = {c: (E if c == 2 else 1.0) for c in (t0, t1)}
        l2w = F * (E if d == 2 else 1.0)          # F G, G = E on zeta-faces (eq 2.29)
        third = E                                  # E [u_{x3}] (eq 2.29)
    else:
        G = sw["G"]
        # eq 2.34a (x3-face): G (L2 + Q_tau + Q_theta); 2.34b (tau-face):
        # L2 + Q_theta + G Q_x3; 2.34c (theta-face): L2 + Q_tau + G Q_x3
        outer = G if d == 2 else 1.0
        wq = {c: (G if c == 2 else 1.0) for c in (t0, t1)}
        l2w = G if d == 2 else 1.0                 # H (eq 2.38)
        third = G                                  # G [u_{x3}] (eq 2.38)

    def triple(w):
        return outer * (Q.l2(w) + wq[t0] * Q.quotient_s(w) + wq[t1] * Q.quotient_t(w))

    total = l2w * Q.l2(jump)
    if not dirichlet:
        comps = range(3)
        dwk = lambda k: ev["gA"][:, k] - ev["gB"][:, k]
    else:
        comps = (t0, t1)
        if problem is not None:
            # data derivatives in the same modified coordinates, by the chain rule
            # through the (real) map of side A
            lamA = np.zeros((Q.s.size, 3))
            lamA[:, d] = 1.0 if fA % 2 else -1.0
            box = mesh.box[eA]
            for c, v in ((t0, Q.s), (t1, Q.t)):
                lamA[:, c] = 2 * (v - box[2 * c]) / (box[2 * c + 1] - box[2 * c]) - 1
            JA = chart_jacobian(mesh, eA, lamA)
            dlam_dy = 2.0 / (box[1::2] - box[0::2])
            dg = np.einsum("pa,pac->pc", problem.grad_u(ev["x"]), JA) * dlam_dy
        else:
            dg = np.zeros((Q.s.size, 3))
        dwk = lambda k: ev["gA"][:, k] - dg[:, k]
    for k in comps:
        sc = third ** 2 if k == 2 else 1.0
        total += sc * triple(dwk(k))
    return total


def oracle_face(disc, U, eA, fA, eB, fB):
    for T in disc.faces:
        pair = {(T.eA, T.fA), (T.eB, T.fB)}
        if pair == {(eA, fA), (eB, fB)}:
            qs = disc._face_quantities(T, U)
            if T.eB < 0:
                qs = [qv - gv for qv, gv in zip(qs, disc.face_data(T))]
            return sum(qv @ disc.face_weight(qv, wts) for qv, (_, _, wts, _) in zip(qs, T.quants)), T
    raise KeyError((eA, fA, eB, fB))


def side_A(mesh, e, f):
    """The reading for faces between regions: the real side, then the more
    singular region (vertex-edge > edge > vertex > regular), then the lower
    element index; the face is normed in side A's region."""
    e2, f2 = int(mesh.nbr[e, f]), int(mesh.nbr_face[e, f])
    if e2 < 0 or mesh.bc[e, f] != M.INTERIOR:
        return e, f, -1, -1, int(mesh.region[e])
    key = lambda el: (mesh.kind[el] == M.REAL, PRIO[int(mesh.region[el])], -el)
    if key(e2) > key(e):
        e, f, e2, f2 = e2, f2, e, f
    reg = int(mesh.region[e])
    if mesh.kind[e2] == M.REAL and PRIO[int(mesh.region[e2])] > PRIO[reg]:
        reg = int(mesh.region[e2])
    return e, f, e2, f2, reg


def face_kinds(mesh):
    """One representative face (e, f) per (region of A, regions/kinds of
    both sides, normal direction in A, Dirichlet)."""
    seen = {}
    for e in range(mesh.E):
        for f in range(6):
            if mesh.bc[e, f] == M.SKIP:
                continue
            eA, fA, eB, fB, reg = side_A(mesh, e, f)
            if eB >= 0:
                kB = (int(mesh.region[eB]), int(mesh.kind[eB]), int(mesh.chart[eB]))
            else:
                kB = None
            key = (reg, int(mesh.chart[eA]), fA // 2, kB)
            seen.setdefault(key, (eA, fA, eB, fB, reg))
    return list(seen.values())


def check_mesh(mesh, problem, tol_poly, tol_curved, seed=0):
    fun_U = np.random.default_rng(seed).standard_normal(mesh.ndof())
    fun = ElementFunctions(mesh, fun_U)
    rows = []
    for (eA, fA, eB, fB, reg) in face_kinds(mesh):
        only = [e for e in (eA, eB) if e >= 0 and mesh.kind[e] == M.REAL]
        disc = Discretization(mesh, problem, only=only)
        val, T = oracle_face(disc, fun_U, eA, fA, eB, fB)
        assert T.eA == eA and T.region == reg, (T.eA, eA, T.region, reg)
        ref = brute_face(mesh, fun, eA, fA, eB, fB, reg, problem if eB < 0 else None)
        curved = any(mesh.chart[e] in (M.VTX_PATCH, M.COLUMN) for e in (eA, eB) if e >= 0)
        rows.append((eA, fA, eB, fB, reg, curved, val, ref))
        tol = tol_curved if curved else tol_poly
        assert abs(val - ref) <= tol * abs(ref), (eA, fA, eB, fB, reg, val, ref, abs(val - ref) / abs(ref))
    return rows


# ------------------------------------------------------------ the pins
def test_regular_faces_affine_mesh_with_data():
    """Regular interior faces (eq 2.16, 2.17b) and Dirichlet faces with
    polynomial data (eq 2.18, 4.2) on boxes of unequal sides: exact."""
    mesh = M.box_mesh(3, (2, 2, 2), (0.0, 0.0, 0.0), (1.0, 0.6, 1.4))
    rows = check_mesh(mesh, Polynomial(), 1e-11, None)
    kinds = {(r[4], r[1] // 2, r[2] >= 0) for r in rows}
    assert {(M.REG, d, i) for d in range(3) for i in (True, False)} <= kinds


def test_vertex_faces_spherical_boxes():
    """Vertex faces (eq 2.25, 4.3): R-weighted master-square norms, on
    spherical boxes with theta- and phi-neighbours and the vertex constant."""
    mesh = vertex_mesh(2, 3, I=2, J=2)
    rows = check_mesh(mesh, Zero(), 1e-11, None)
    kinds = {(r[1] // 2, r[2] >= 0) for r in rows}
    assert {(0, True), (1, True), (2, True), (0, False), (1, False), (2, False)} <= kinds


def test_vertex_edge_faces():
    """Vertex-edge faces: zeta-, psi- and theta-faces (eq 2.27a-c in eq
    2.29), the corner polynomial and the vertex constant, Dirichlet theta-,
    psi- and zeta-faces (eq 4.5)."""
    mesh = vertex_edge_mesh(2, 3, I=2)
    rows = check_mesh(mesh, Zero(), 1e-11, None)
    kinds = {(r[1] // 2, r[2] >= 0) for r in rows}
    assert {(d, i) for d in range(3) for i in (True, False)} <= kinds


def test_edge_faces():
    """Edge faces: x3-, tau- and theta-faces (eq 2.34a-c in eq 2.38), the
    corner polynomial, Dirichlet faces of every direction (eq 4.7)."""
    mesh = edge_mesh(2, 3, I=2, Je=2)
    rows = check_mesh(mesh, Zero(), 1e-11, None)
    kinds = {(r[1] // 2, r[2] >= 0) for r in rows}
    assert {(d, i) for d in range(3) for i in (True, False)} <= kinds


def test_fichera_every_face_kind():
    """Every kind of face of the Fichera mesh, including those between
    regions (vertex-edge | edge, vertex-edge | vertex patch, edge | regular
    column, vertex patch | column) and curved vertex patches.  Box faces
    agree to rounding; faces with a curved side to the quadrature error of
    the (2W+1)-point rule on their smooth chart factors (at most 8e-5 at
    W = 4)."""
    mesh = fichera_mesh(N=2, W=4, Je=2)
    rows = check_mesh(mesh, Zero(), 1e-11, 5e-4)
    regions = {(r[4], mesh.chart[r[0]], mesh.chart[r[2]] if r[2] >= 0 else -1) for r in rows}
    assert (M.VE, M.VE_BOX, M.EDGE_BOX) in regions
    assert (M.VE, M.VE_BOX, M.VTX_PATCH) in regions
    assert (M.EDGE, M.EDGE_BOX, M.COLUMN) in regions
    assert (M.VTX, M.VTX_PATCH, M.COLUMN) in regions
    assert (M.VTX, M.VTX_PATCH, M.VTX_PATCH) in regions


def _term_value(disc, T, U, quants):
    import copy
    T2 = copy.copy(T)
    T2.quants = quants
    qs = disc._face_quantities(T2, U)
    return sum(qv @ disc.face_weight(qv, qd[2]) for qv, qd in zip(qs, quants))


def test_planted_weight_mistakes_are_caught():
    """Mistakes of the kinds a misreading would make, planted in the oracle's
    face weights, move the face term far outside the tolerances above: the
    extents of the two difference-quotient terms exchanged (h0/2 for h1/2),
    the third derivative's E^2 / G^2 left off, the L2 weight without its G
    (vertex-edge) or H (edge) factor."""
    cases = [(vertex_edge_mesh(2, 3, I=2), (5, 1, 3)), (edge_mesh(2, 3, I=2, Je=2), (5, 1, 3))]
    for mesh, faces in cases:
        U = np.random.default_rng(1).standard_normal(mesh.ndof())
        fun = ElementFunctions(mesh, U)
        e = int(mesh.real_elements()[0])
        for f in faces:
            eA, fA, eB, fB, reg = side_A(mesh, e, f)
            disc = Discretization(mesh, Zero(), only=[x for x in (eA, eB) if x >= 0 and mesh.kind[x] == M.REAL])
            val, T = oracle_face(disc, U, eA, fA, eB, fB)
            ref = brute_face(mesh, fun, eA, fA, eB, fB, reg)
            assert abs(val - ref) <= 1e-11 * abs(ref)
            base = [list(qd) for qd in T.quants]
            plants = []
            swapped = [list(qd) for qd in base]
            for qd in swapped[1:]:
                a, b, c = qd[2]
                qd[2] = (a, c, b)
            plants.append(("extents exchanged", swapped))
            third = [list(qd) for qd in base]
            third[3][2] = base[1][2] if fA // 2 != 0 else base[2][2]
            plants.append(("third derivative unweighted", third))
            if fA // 2 == 2:
                l2 = [list(qd) for qd in base]
                a, b, c = l2[0][2]
                w3 = base[3][2][0] / base[1][2][0]          # E^2 or G^2
                l2[0][2] = (a / np.sqrt(w3), b, c)
                plants.append(("L2 weight without G / H", l2))
            for name, qd in plants:
                bad = _term_value(disc, T, U, [tuple(x) for x in qd])
                assert abs(bad - ref) > 1e-3 * abs(ref), (mesh.name, f, name, bad, ref)
