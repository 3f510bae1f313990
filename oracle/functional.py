"""The discrete least-squares functional R^{N,W} and its normal equations.

ORACLE: test infrastructure only.

R^{N,W}(U) (thesis eq 4.1-4.8) evaluated by GLL quadrature as in Sec. 5.3:

Volume term, every element of finite measure (eq 4.2, 4.3, 4.5, 4.7 first
lines).  With the transformed operators of eq 2.22, 2.28, 2.35 and the data
transforms F^r, F^v, F^{v-e}, F^e, each equals
    sum_q  w_q |J(lam_q)| omega(x_q)^2 (L u(x_q) - f(x_q))^2
over the (2W+1)^3 GLL points lam_q of Q, where J is the Jacobian of the map
lam -> x and omega = 1 (regular region), rho (vertex neighbourhood), r =
distance to the edge (edge and vertex-edge neighbourhoods).  L = -Laplace.
L u(x) comes from the chain rule: grad_x u = J^-T grad_lam u and
Hess_x u = J^-T (Hess_lam u - sum_b (grad_x u)_b H^b) J^-1.

General operators (eq 2.2) come from the problem's ``coefficients(x)``:
L u = -sum_ij a_ij u_{x_i x_j} + sum_j beta_j u_{x_j} + c u (a symmetric,
beta_j = b_j - sum_i d a_ij / d x_i); without it L = -Laplace.  Then
Hess_x u gives the lam-fields the coefficients J^-1 a J^-T (second order),
sum_b J^-1[a, b] (tr(J^-1 a J^-T H^b) + beta_b) (first order) and c (the
value).

Face terms (eq 4.2, 4.3, 4.5, 4.7; norms eq 2.17b, 2.18, 2.27, 2.34) on the
(2W+1)x(2W+1) GLL grid of the face, parametrised by the face coordinates of
side A.  The discrete H^{1/2} seminorm is the GLL double sum of Sec. 5.3.
Each face contributes sum_k Q_k^T M_k Q_k with M_k = alpha Om(x)Om +
beta K(x)Om + gamma Om(x)K, Om = diag(GLL weights), K = ``gll.half_matrix``.

Readings where the thesis leaves a choice: a face between two regions is counted once,
in the coordinates and weights of the more singular region (vertex-edge >
edge > vertex > regular); faces of a corner element take the real
neighbour as side A; ties take the lower element index.  Vertex-region
derivatives are taken in the modified-coordinate frame (mframe) of side A.
"""
import numpy as np

from workloads import mesh as M
from . import gll
from . import charts

PRIO = {M.REG: 0, M.VTX: 1, M.EDGE: 2, M.VE: 3}
# derivative orders per direction for the fields of the volume operator
SECOND = [((2, 0, 0), 0, 0), ((0, 2, 0), 1, 1), ((0, 0, 2), 2, 2),
          ((1, 1, 0), 0, 1), ((1, 0, 1), 0, 2), ((0, 1, 1), 1, 2)]
FIRST = [((1, 0, 0), 0), ((0, 1, 0), 1), ((0, 0, 1), 2)]
ZERO = (0, 0, 0)


def _weight_omega(mesh, e, x):
    """Volume weight omega(x) of eq 2.22, 2.28, 2.35 (1, rho or r)."""
    reg = mesh.region[e]
    if reg == M.REG:
        return np.ones(x.shape[0])
    xl = (x - mesh.origin[e]) @ mesh.frame[e]
    if reg == M.VTX:
        return np.linalg.norm(xl, axis=-1)
    return np.sqrt(xl[:, 0] ** 2 + xl[:, 1] ** 2)


def tensor_apply(M0, M1, M2, u):
    """(M0 (x) M1 (x) M2) applied to u[i, j, k]: out[a, b, c] = sum M0[a,i] M1[b,j] M2[c,k] u[i,j,k]."""
    t = np.tensordot(M0, u, axes=(1, 0))            # a j k
    t = np.tensordot(M1, t, axes=(1, 1))            # b a k
    t = np.tensordot(M2, t, axes=(1, 2))            # c b a
    return t.transpose(2, 1, 0)


class FaceTerm:
    pass


class Discretization:
    def __init__(self, mesh, problem=None, only=None):
        """only: optional set of real elements.  Then only their volume terms
        and the face terms touching them are set up, so that the rows of
        apply_X and rhs belonging to those elements are exact (X couples an
        element only through its own volume term and the face terms on its
        faces) and the other rows are partial sums."""
        self.mesh = mesh
        self.problem = problem
        self.only = None if only is None else set(int(e) for e in only)
        W = mesh.W
        self.W, self.n, self.m = W, W + 1, 2 * W + 1
        n, m = self.n, self.m
        self.xn, self.wn = gll.gll(n)
        self.xm, self.wm = gll.gll(m)
        # fine-grid evaluation of the Lagrange basis and its derivatives
        self.B = [gll.lagrange(self.xn, self.xm, d) for d in range(3)]
        self.K = gll.half_matrix(m)
        self.real = mesh.real_elements()
        self.offset = -np.ones(mesh.E, np.int64)
        self.offset[self.real] = np.arange(len(self.real)) * n ** 3
        self.n_real_dof = len(self.real) * n ** 3
        self.ndof = self.n_real_dof + mesh.n_corner_dof
        self._volume_setup()
        self._face_setup()

    # ------------------------------------------------------------------
    # unknown layout: real elements (mesh order), n^3 each, i fastest;
    # then the corner DOFs.  u_e[i, j, k] = U[off + i + n j + n^2 k].
    # ------------------------------------------------------------------
    def element_values(self, U, e):
        n = self.n
        mesh = self.mesh
        if mesh.kind[e] == M.REAL:
            o = self.offset[e]
            return U[o:o + n ** 3].reshape((n, n, n), order="F")
        c = self.n_real_dof + mesh.cdof[e]
        if mesh.kind[e] == M.CORNER_CONST:
            return np.full((n, n, n), U[c])
        p = U[c:c + n]
        shape = [1, 1, 1]
        shape[mesh.cdir[e]] = n
        return np.broadcast_to(p.reshape(shape), (n, n, n)).copy()

    def element_accumulate(self, R, e, ue):
        n = self.n
        mesh = self.mesh
        if mesh.kind[e] == M.REAL:
            o = self.offset[e]
            R[o:o + n ** 3] += ue.reshape(-1, order="F")
            return
        c = self.n_real_dof + mesh.cdof[e]
        if mesh.kind[e] == M.CORNER_CONST:
            R[c] += ue.sum()
            return
        axes = tuple(a for a in range(3) if a != mesh.cdir[e])
        R[c:c + n] += ue.sum(axis=axes)

    # ------------------------------------------------------------------
    # volume term
    # ------------------------------------------------------------------
    def _volume_setup(self):
        mesh, m = self.mesh, self.m
        xm, wm = self.xm, self.wm
        A, Bb, C = np.meshgrid(xm, xm, xm, indexing="ij")
        lam = np.stack([A.ravel(order="F"), Bb.ravel(order="F"), C.ravel(order="F")], -1)
        WA, WB, WC = np.meshgrid(wm, wm, wm, indexing="ij")
        wq = (WA * WB * WC).ravel(order="F")
        self.vol = []
        for e in self.real:
            if self.only is not None and e not in self.only:
                continue
            x, J, H = charts.geometry(mesh, e, lam)
            detJ = np.abs(np.linalg.det(J))
            Ji = np.linalg.inv(J)
            if self.problem is not None and hasattr(self.problem, "coefficients"):
                a6, beta, c0 = self.problem.coefficients(x)
                A = np.empty((x.shape[0], 3, 3))
                for k, (i, j) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
                    A[:, i, j] = A[:, j, i] = a6[:, k]
            else:
                A = np.broadcast_to(np.eye(3), (x.shape[0], 3, 3))
                beta = np.zeros((x.shape[0], 3))
                c0 = None
            G = np.einsum("pci,pij,pdj->pcd", Ji, A, Ji)
            a1 = np.einsum("pab,pb->pa", Ji, np.einsum("pbcd,pcd->pb", H, G) + beta)
            s = np.sqrt(wq * detJ) * _weight_omega(mesh, e, x)
            coef2 = [-G[:, c, d] * (1 if c == d else 2) for (_, c, d) in SECOND]
            coef1 = [a1[:, a] for (_, a) in FIRST]
            coef0 = None if c0 is None or not np.any(c0) else np.asarray(c0, float)
            self.vol.append(dict(e=e, x=x, s=s, coef2=coef2, coef1=coef1, coef0=coef0))

    def _fields(self, ue, orders):
        B = self.B
        return tensor_apply(B[orders[0]], B[orders[1]], B[orders[2]], ue).ravel(order="F")

    def _fields_T(self, z, orders):
        B = self.B
        m = self.m
        z3 = z.reshape((m, m, m), order="F")
        return tensor_apply(B[orders[0]].T, B[orders[1]].T, B[orders[2]].T, z3)

    def volume_residual(self, ue, v, f_vals=None):
        """z_q = s_q (L u_q - f_q) for one element."""
        Lu = np.zeros(self.m ** 3)
        for (o, _, _), cf in zip(SECOND, v["coef2"]):
            Lu += cf * self._fields(ue, o)
        for (o, _), cf in zip(FIRST, v["coef1"]):
            Lu += cf * self._fields(ue, o)
        if v["coef0"] is not None:
            Lu += v["coef0"] * self._fields(ue, ZERO)
        if f_vals is not None:
            Lu = Lu - f_vals
        return v["s"] * Lu

    def volume_adjoint(self, z, v):
        zs = v["s"] * z
        out = 0
        for (o, _, _), cf in zip(SECOND, v["coef2"]):
            out = out + self._fields_T(cf * zs, o)
        for (o, _), cf in zip(FIRST, v["coef1"]):
            out = out + self._fields_T(cf * zs, o)
        if v["coef0"] is not None:
            out = out + self._fields_T(v["coef0"] * zs, ZERO)
        return out

    # ------------------------------------------------------------------
    # face terms
    # ------------------------------------------------------------------
    def _face_setup(self):
        mesh = self.mesh
        self.faces = []
        for e in range(mesh.E):
            for f in range(6):
                bc = mesh.bc[e, f]
                if bc == M.INTERIOR:
                    e2, f2 = int(mesh.nbr[e, f]), int(mesh.nbr_face[e, f])
                    if (e2, f2) < (e, f):
                        continue
                    if self.only is not None and e not in self.only and e2 not in self.only:
                        continue
                    self.faces.append(self._make_face(e, f, e2, f2, int(mesh.orient[e, f])))
                elif bc in (M.DIRICHLET, M.NEUMANN):
                    if self.only is not None and e not in self.only:
                        continue
                    self.faces.append(self._make_face(e, f, -1, -1, 0, neumann=bc == M.NEUMANN))

    def _choose_A(self, e, f, e2, f2, o):
        mesh = self.mesh
        keep = True
        ka, kb = mesh.kind[e] != M.REAL, mesh.kind[e2] != M.REAL
        if ka != kb:
            keep = not ka
        else:
            pa, pb = PRIO[int(mesh.region[e])], PRIO[int(mesh.region[e2])]
            if pa != pb:
                keep = pa > pb
            else:
                keep = e < e2
        if keep:
            return e, f, e2, f2, o
        # reverse orientation: coordinates of e2's face -> e's face
        inv = None
        for oo in range(8):
            a, b = M.orient_map(o, 0.3, -0.7)
            if np.allclose(M.orient_map(oo, a, b), (0.3, -0.7)):
                inv = oo
        return e2, f2, e, f, inv

    def _face_grid(self, f, o=0):
        """lam points [P,3] on face f for A's face-grid points after orientation o."""
        xm = self.xm
        a, b = np.meshgrid(xm, xm, indexing="ij")
        a, b = a.ravel(order="F"), b.ravel(order="F")
        a, b = M.orient_map(o, a, b)
        return M.face_lam(f, a, b)

    def _trace_setup(self, f, o):
        """Trace evaluation data of face f whose points, in A's face-grid order,
        sit at face coordinates orient_map(o, a, b) on this side."""
        xm = self.xm
        m = self.m
        d, s = divmod(f, 2)
        a, b = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
        a, b = a.ravel(order="F"), b.ravel(order="F")
        ca, cb = M.orient_map(o, xm[a], xm[b])
        ia = np.array([np.argmin(np.abs(xm - v)) for v in ca])
        ib = np.array([np.argmin(np.abs(xm - v)) for v in cb])
        perm = ia + m * ib            # index into this side's own (t0, t1) grid
        end = np.array([1.0 if s else -1.0])
        mats = []
        for c in range(4):
            per_axis = []
            for ax in range(3):
                order = 1 if (c > 0 and c - 1 == ax) else 0
                pts = end if ax == d else xm
                per_axis.append(gll.lagrange(self.xn, pts, order))
            mats.append(per_axis)
        return dict(d=d, perm=perm, mats=mats)

    def _make_face(self, e, f, e2, f2, o, neumann=False):
        mesh = self.mesh
        T = FaceTerm()
        if e2 >= 0:
            e, f, e2, f2, o = self._choose_A(e, f, e2, f2, o)
        T.eA, T.fA, T.eB, T.fB, T.orient = e, f, e2, f2, o
        reg = int(mesh.region[e])
        if e2 >= 0:
            reg = max(reg, int(mesh.region[e2]), key=lambda r: PRIO[r]) \
                if mesh.kind[e2] == M.REAL else reg
        T.region = reg
        lamA = self._face_grid(f)
        T.xA, JA, _ = charts.geometry(mesh, e, lamA, second=False)
        T.trA = self._trace_setup(f, 0)
        JiA = np.linalg.inv(JA)
        if e2 >= 0:
            lamB = self._face_grid(f2, o)
            xB, JB, _ = charts.geometry(mesh, e2, lamB, second=False)
            if np.abs(xB - T.xA).max() > 1e-9 * max(1, np.abs(T.xA).max()):
                raise ValueError("non-conforming face %d/%d - %d/%d" % (e, f, e2, f2))
            T.trB = self._trace_setup(f2, o)
            JiB = np.linalg.inv(JB)
        d = f // 2
        t0, t1 = M.FACE_TANGENT[d]
        box = mesh.box[e]
        h = box[1::2] - box[0::2]
        face_val = box[2 * d + (f % 2)]
        dir_ = e2 < 0
        P = T.xA.shape[0]

        def grad_coeffs(Ji, Jy):
            # PS[k, c] for d u/d y_k = sum_c u_c (Ji @ Jy)[c, k]
            return np.einsum("pcl,plk->pkc", Ji, Jy)

        if reg == M.REG:
            Jy = np.broadcast_to(np.eye(3), (P, 3, 3))
        else:
            xl = (T.xA - mesh.origin[e]) @ mesh.mframe[e]
            Jy = np.einsum("ab,pbk->pak", mesh.mframe[e], charts.modified_jacobian(reg, xl))
        quants = []   # (PA [P,4], PB [P,4] or None, (alpha, beta, gamma), data kind)
        one = np.zeros((P, 4))
        one[:, 0] = 1.0

        def unit(c):
            u = np.zeros((P, 4))
            u[:, c + 1] = 1.0
            return u

        if reg in (M.REG, M.VTX):
            R = 1.0
            if reg == M.VTX:
                chi_max = face_val if d == 2 else box[5]
                R = np.exp(chi_max)
            if not dir_:
                gA = grad_coeffs(JiA, Jy)
                gB = grad_coeffs(JiB, Jy)
                quants.append((one, one, (R, 0.0, 0.0), None))
                for k in range(3):
                    PA = np.zeros((P, 4))
                    PA[:, 1:] = gA[:, k, :]
                    PB = np.zeros((P, 4))
                    PB[:, 1:] = gB[:, k, :]
                    quants.append((PA, PB, (R, R, R), None))
            else:
                quants.append((one, None, (R, 0.0, 0.0), ("value",)))
                for c in (t0, t1):
                    quants.append((unit(c), None, (R, R, R), ("dlam", c)))
        else:
            if reg == M.VE:
                psi_max = face_val if d == 0 else box[1]
                tpsi = np.exp(psi_max)
                Eg = tpsi / np.sqrt(1 + tpsi ** 2)
                Fg = np.exp(face_val if d == 2 else box[5])
                if d == 2:
                    norm = (Eg * Fg * h[0] * h[1] / 4, Eg * Fg * h[1] / 2, Eg * Fg * h[0] / 2)
                    l2 = Fg * Eg * h[0] * h[1] / 4
                elif d == 0:
                    norm = (Fg * h[1] * h[2] / 4, Fg * h[2] / 2, Fg * Eg * h[1] / 2)
                    l2 = Fg * h[1] * h[2] / 4
                else:
                    norm = (Fg * h[0] * h[2] / 4, Fg * h[2] / 2, Fg * Eg * h[0] / 2)
                    l2 = Fg * h[0] * h[2] / 4
                w3 = Eg ** 2
            else:
                Gg = np.exp(face_val if d == 0 else box[1])
                if d == 2:
                    norm = (Gg * h[0] * h[1] / 4, Gg * h[1] / 2, Gg * h[0] / 2)
                    l2 = Gg * h[0] * h[1] / 4
                elif d == 0:
                    norm = (h[1] * h[2] / 4, h[2] / 2, Gg * h[1] / 2)
                    l2 = h[1] * h[2] / 4
                else:
                    norm = (h[0] * h[2] / 4, h[2] / 2, Gg * h[0] / 2)
                    l2 = h[0] * h[2] / 4
                w3 = Gg ** 2
            gA = grad_coeffs(JiA, Jy)
            if not dir_:
                gB = grad_coeffs(JiB, Jy)
                quants.append((one, one, (l2, 0.0, 0.0), None))
                for k in range(3):
                    PA = np.zeros((P, 4))
                    PA[:, 1:] = gA[:, k, :]
                    PB = np.zeros((P, 4))
                    PB[:, 1:] = gB[:, k, :]
                    sc = w3 if k == 2 else 1.0
                    quants.append((PA, PB, tuple(sc * v for v in norm), None))
            else:
                quants.append((one, None, (l2, 0.0, 0.0), ("value",)))
                for k in (t0, t1):
                    PA = np.zeros((P, 4))
                    PA[:, 1:] = gA[:, k, :]
                    sc = w3 if k == 2 else 1.0
                    quants.append((PA, None, tuple(sc * v for v in norm), ("dy", k)))
        if neumann:
            quants = self._neumann_quantity(T, f, JA, reg, quants)
        T.quants = quants
        T.JA, T.Jy = JA, Jy
        return T

    def _neumann_quantity(self, T, f, JA, reg, quants):
        """Neumann face (eq 2.16, 4.2 regular; 4.3 vertex; 4.5 vertex-edge;
        4.7 edge): one quantity, the conormal derivative (du/dnu)_a = nu^T a
        grad_x u with nu the outward unit normal, times the factor the thesis
        applies to the data in the neighbourhoods (e^chi / sin phi, e^zeta
        e^psi = r, e^tau = r), normed like the face's derivative jumps
        (||.||_{1/2} on the master square, R-weighted in the vertex region;
        |||.||| of eq 2.27 / 2.34).  The data term is that factor times h."""
        mesh = self.mesh
        e = T.eA
        d, s = divmod(f, 2)
        Ji = np.linalg.inv(JA)                       # [P, c, j] = d lam_c / d x_j
        nu = Ji[:, d, :] * (1.0 if s else -1.0)
        nu = nu / np.linalg.norm(nu, axis=1)[:, None]
        if self.problem is not None and hasattr(self.problem, "coefficients"):
            a6 = self.problem.coefficients(T.xA)[0]
            A = np.empty((nu.shape[0], 3, 3))
            for k, (i, j) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
                A[:, i, j] = A[:, j, i] = a6[:, k]
            anu = np.einsum("pij,pj->pi", A, nu)
        else:
            anu = nu
        if reg == M.REG:
            wfac = np.ones(nu.shape[0])
        else:
            xl = (T.xA - mesh.origin[e]) @ mesh.mframe[e]
            r = np.hypot(xl[:, 0], xl[:, 1])
            rho = np.linalg.norm(xl, axis=1)
            wfac = rho * rho / r if reg == M.VTX else r          # e^chi / sin(phi) = rho^2 / r
        PA = np.zeros((nu.shape[0], 4))
        PA[:, 1:] = wfac[:, None] * np.einsum("pcj,pj->pc", Ji, anu)
        # the face's derivative-jump weights: quantity 1 of the face's interior-type norm
        wts = quants[1][2]
        T.nu, T.wfac = nu, wfac
        return [(PA, None, wts, ("neumann",))]

    def _trace(self, tr, ue):
        """[P, 4]: u and its three lam-derivatives at the face points."""
        out = []
        for (M0, M1, M2) in tr["mats"]:
            v = tensor_apply(M0, M1, M2, ue)
            out.append(v.reshape(self.m * self.m, order="F")[tr["perm"]])
        return np.stack(out, -1)

    def _trace_T(self, tr, w):
        """Adjoint of _trace: w [P,4] -> n^3 array."""
        d = tr["d"]
        shape = [self.m, self.m, self.m]
        shape[d] = 1
        tot = 0
        for c, (M0, M1, M2) in enumerate(tr["mats"]):
            g = np.zeros(self.m * self.m)
            g[tr["perm"]] = w[:, c]
            g = g.reshape(shape, order="F")
            tot = tot + tensor_apply(M0.T, M1.T, M2.T, g)
        return tot

    def face_weight(self, q, wts):
        m = self.m
        al, be, ga = wts
        Q = q.reshape((m, m), order="F")
        w = self.wm
        out = al * (w[:, None] * w[None, :]) * Q
        if be:
            out = out + be * (self.K @ Q) * w[None, :]
        if ga:
            out = out + ga * w[:, None] * (Q @ self.K)
        return out.ravel(order="F")

    def face_data(self, T):
        """Data values g_k at A's face points for a Dirichlet term."""
        x = T.xA
        g = self.problem.u(x)
        dg = self.problem.grad_u(x)
        out = []
        for (_, _, _, kind) in T.quants:
            if kind[0] == "neumann":
                out.append(T.wfac * self.problem.neumann(x, T.nu))
            elif kind[0] == "value":
                out.append(g)
            elif kind[0] == "dlam":
                out.append(np.einsum("pa,pa->p", dg, T.JA[:, :, kind[1]]))
            else:
                out.append(np.einsum("pa,pa->p", dg, T.Jy[:, :, kind[1]]))
        return out

    # ------------------------------------------------------------------
    # operator, right-hand side, functional
    # ------------------------------------------------------------------
    def _face_quantities(self, T, U):
        uA = self.element_values(U, T.eA)
        trA = self._trace(T.trA, uA)
        qs = [np.einsum("pc,pc->p", PA, trA) for (PA, _, _, _) in T.quants]
        if T.eB >= 0:
            uB = self.element_values(U, T.eB)
            trB = self._trace(T.trB, uB)
            qs = [q - np.einsum("pc,pc->p", PB, trB) for q, (_, PB, _, _) in zip(qs, T.quants)]
        return qs

    def _face_scatter(self, T, Ws, out):
        wA = sum(PA * Wk[:, None] for Wk, (PA, _, _, _) in zip(Ws, T.quants))
        self.element_accumulate(out, T.eA, self._trace_T(T.trA, wA))
        if T.eB >= 0:
            wB = sum(PB * Wk[:, None] for Wk, (_, PB, _, _) in zip(Ws, T.quants))
            self.element_accumulate(out, T.eB, -self._trace_T(T.trB, wB))

    def apply_volume(self, U):
        out = np.zeros(self.ndof)
        for v in self.vol:
            ue = self.element_values(U, v["e"])
            z = self.volume_residual(ue, v)
            self.element_accumulate(out, v["e"], self.volume_adjoint(z, v))
        return out

    def apply_faces(self, U):
        out = np.zeros(self.ndof)
        for T in self.faces:
            qs = self._face_quantities(T, U)
            Ws = [self.face_weight(q, wts) for q, (_, _, wts, _) in zip(qs, T.quants)]
            self._face_scatter(T, Ws, out)
        return out

    def apply_X(self, U):
        """X U with X = A^T M A, the normal-equation matrix (Sec. 5.3)."""
        U = np.asarray(U, float)
        return self.apply_volume(U) + self.apply_faces(U)

    def rhs(self):
        """b = A^T M d (data: f in the volume, g on Dirichlet faces)."""
        out = np.zeros(self.ndof)
        for v in self.vol:
            fv = self.problem.f(v["x"])
            z = v["s"] * fv
            self.element_accumulate(out, v["e"], self.volume_adjoint(z, v))
        for T in self.faces:
            if T.eB >= 0:
                continue
            gs = self.face_data(T)
            Ws = [self.face_weight(g, wts) for g, (_, _, wts, _) in zip(gs, T.quants)]
            self._face_scatter(T, Ws, out)
        return out

    def functional(self, U):
        """R_h(U) = ||A U - d||_M^2 (eq 4.1 discretised)."""
        tot = 0.0
        for v in self.vol:
            ue = self.element_values(U, v["e"])
            z = self.volume_residual(ue, v, self.problem.f(v["x"]))
            tot += z @ z
        for T in self.faces:
            qs = self._face_quantities(T, U)
            if T.eB < 0:
                qs = [q - g for q, g in zip(qs, self.face_data(T))]
            for q, (_, _, wts, _) in zip(qs, T.quants):
                tot += q @ self.face_weight(q, wts)
        return tot

    def apply_X_abs(self, U):
        """|A|^T |M| |A| |U|: X U with every operator entry, weight and unknown
        replaced by its modulus, the sum of the moduli of the terms that make
        up each entry of X U.  A floating-point evaluation of X U in unit
        roundoff eps through sums of at most K terms per step errs, entry by
        entry, by at most about K eps times this (rounded data included)."""
        U = np.abs(np.asarray(U, float))
        out = np.zeros(self.ndof)
        B = [np.abs(b) for b in self.B]

        def fields(ue, o):
            return tensor_apply(B[o[0]], B[o[1]], B[o[2]], ue).ravel(order="F")

        def fields_T(z, o):
            z3 = z.reshape((self.m,) * 3, order="F")
            return tensor_apply(B[o[0]].T, B[o[1]].T, B[o[2]].T, z3)

        for v in self.vol:
            ue = self.element_values(U, v["e"])
            terms = [(o, np.abs(cf)) for (o, _, _), cf in zip(SECOND, v["coef2"])]
            terms += [(o, np.abs(cf)) for (o, _), cf in zip(FIRST, v["coef1"])]
            if v["coef0"] is not None:
                terms.append((ZERO, np.abs(v["coef0"])))
            s = np.abs(v["s"])
            z = s * sum(cf * fields(ue, o) for o, cf in terms)
            self.element_accumulate(out, v["e"], sum(fields_T(cf * s * z, o) for o, cf in terms))
        K = np.abs(self.K)
        w = self.wm
        for T in self.faces:
            trA = self._trace_abs(T.trA, self.element_values(U, T.eA))
            qs = [np.einsum("pc,pc->p", np.abs(PA), trA) for (PA, _, _, _) in T.quants]
            if T.eB >= 0:
                trB = self._trace_abs(T.trB, self.element_values(U, T.eB))
                qs = [q + np.einsum("pc,pc->p", np.abs(PB), trB) for q, (_, PB, _, _) in zip(qs, T.quants)]
            Ws = []
            for q, (_, _, (al, be, ga), _) in zip(qs, T.quants):
                Q = q.reshape((self.m, self.m), order="F")
                r = abs(al) * (w[:, None] * w[None, :]) * Q + abs(be) * (K @ Q) * w[None, :] \
                    + abs(ga) * w[:, None] * (Q @ K)
                Ws.append(r.ravel(order="F"))
            wA = sum(np.abs(PA) * Wk[:, None] for Wk, (PA, _, _, _) in zip(Ws, T.quants))
            self.element_accumulate(out, T.eA, self._trace_T_abs(T.trA, wA))
            if T.eB >= 0:
                wB = sum(np.abs(PB) * Wk[:, None] for Wk, (_, PB, _, _) in zip(Ws, T.quants))
                self.element_accumulate(out, T.eB, self._trace_T_abs(T.trB, wB))
        return out

    def _trace_abs(self, tr, ue):
        out = []
        for (M0, M1, M2) in tr["mats"]:
            v = tensor_apply(np.abs(M0), np.abs(M1), np.abs(M2), ue)
            out.append(v.reshape(self.m * self.m, order="F")[tr["perm"]])
        return np.stack(out, -1)

    def _trace_T_abs(self, tr, wv):
        d = tr["d"]
        shape = [self.m, self.m, self.m]
        shape[d] = 1
        tot = 0
        for c, (M0, M1, M2) in enumerate(tr["mats"]):
            g = np.zeros(self.m * self.m)
            g[tr["perm"]] = wv[:, c]
            g = g.reshape(shape, order="F")
            tot = tot + tensor_apply(np.abs(M0).T, np.abs(M1).T, np.abs(M2).T, g)
        return tot

    def dense_X(self):
        N = self.ndof
        X = np.zeros((N, N))
        e = np.zeros(N)
        for i in range(N):
            e[:] = 0
            e[i] = 1
            X[:, i] = self.apply_X(e)
        return X
