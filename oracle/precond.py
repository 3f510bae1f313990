"""Block-diagonal preconditioner (thesis Sec. 5.2).

ORACLE: test infrastructure only.

1D forms (eq 5.11-5.14, 5.31-5.34) in the nodal basis of the W+1 GLL points,
every integral taken with the (W+1)-point GLL rule:
    F  = int v^2         -> diag(w)          (GLL-lumped)
    S1 = int v'^2        -> D^T diag(w) D
    S2 = int v''^2       -> (DD)^T diag(w) (DD)
This reading reproduces Table 5.1 (kappa of C against the H^2(Q) form B,
mixed derivatives counted once) to 9-10 digits, which pins it.

Element blocks: the separable forms C (eq 5.19) and C* (eq 5.30) written, like
the U-forms they stand for (eq 2.19 on the master cube; eq 2.26, 2.32, 2.40
in the element's modified coordinates), with the element's extents h_d:
    C_e = s_e (h1 h2 h3 / 8) [E1 (x) F (x) F + F (x) E2 (x) F + F (x) F (x) E3
                              + F (x) F (x) F]
    E_d = g_d^4 S2 + g_d^2 S1,  g_d = 2 / h_d  (times eta in the zeta / x3
    direction of vertex-edge and edge elements, eq 5.33).
Readings: h = 2 (regular), box extents (boxes in modified coordinates),
2 |dy/dlam_d| at the centre (curved sphere patches); s_e = 1 (regular, edge),
sup e^chi (vertex), sup e^zeta (vertex-edge); eta = sup sin(phi)
(vertex-edge), sup e^tau (edge).

Corner DOFs (U-form corner terms, eq 2.26, 2.32, 2.40, integrals with the
(W+1)-point GLL rule in the polynomial direction):
    h_v      : sum over vertex corners of e^{chi_1} |S_j|_(phi,theta)
               + sum over vertex-edge corners below zeta_1 of
                 e^{zeta_1} |psi-range cap [psi_1 - 1, inf)| h_theta
    edge p   : sum over sectors of h_theta (h_x3/2) diag(w)
    v-e  p   : sum over sectors of h_theta (h_zeta/2) diag(w e^{zeta_i})
The oracle applies C_e^{-1} by a dense Cholesky solve of the assembled block.
"""
import numpy as np
import scipy.linalg as sla

from workloads import mesh as M
from . import gll
from . import charts


def forms_1d(W):
    n = W + 1
    x, w = gll.gll(n)
    D = gll.diff_matrix(x)
    F = np.diag(w)
    S1 = D.T @ np.diag(w) @ D
    D2 = D @ D
    S2 = D2.T @ np.diag(w) @ D2
    return F, S1, S2


def kron3(A1, A2, A3):
    """Matrix acting on index i + n j + n^2 k with A1 on i, A2 on j, A3 on k."""
    return np.kron(A3, np.kron(A2, A1))


def table51_kappa(W):
    """kappa(C^-1 B) on Q for the H^2(Q) form B and the separable C (eq 5.7, 5.19)."""
    F, S1, S2 = forms_1d(W)
    C = kron3(F, F, F) + kron3(S1, F, F) + kron3(F, S1, F) + kron3(F, F, S1) \
        + kron3(S2, F, F) + kron3(F, S2, F) + kron3(F, F, S2)
    B = C + kron3(S1, S1, F) + kron3(S1, F, S1) + kron3(F, S1, S1)
    ev = sla.eigh(B, C, eigvals_only=True)
    return ev.max() / ev.min()


def modified_extents(mesh, e):
    """Extents h_d of the element along its modified coordinates.

    Box charts: the box.  Curved sphere patches: 2 |d y / d lam_d| at the
    element centre, y = (phi, theta, chi) of the element's modified frame.
    Regular region: 2 (the U-form there is on the master cube, eq 2.19)."""
    b = mesh.box[e]
    reg = mesh.region[e]
    if reg == M.REG:
        return np.array([2.0, 2.0, 2.0])
    if mesh.chart[e] != M.VTX_PATCH:
        return b[1::2] - b[0::2]
    x, J, _ = charts.geometry(mesh, e, np.zeros((1, 3)), second=False)
    xl = (x - mesh.origin[e]) @ mesh.mframe[e]
    Jy = np.einsum("ab,pbk->pak", mesh.mframe[e], charts.modified_jacobian(M.VTX, xl))
    dyl = np.linalg.solve(Jy, J)[0]          # d y / d lam
    return 2.0 * np.linalg.norm(dyl, axis=0)


def element_params(mesh, e):
    """(s_e, h [3], eta_e or None) for a real element (see module doc)."""
    reg = mesh.region[e]
    b = mesh.box[e]
    h = modified_extents(mesh, e)
    if reg == M.REG:
        return 1.0, h, None
    if reg == M.VTX:
        return float(np.exp(b[5])), h, None
    if reg == M.VE:
        t = np.exp(b[1])
        return float(np.exp(b[5])), h, float(t / np.sqrt(1 + t * t))
    return 1.0, h, float(np.exp(b[1]))


def element_block(mesh, e):
    W = mesh.W
    F, S1, S2 = forms_1d(W)
    s, h, eta = element_params(mesh, e)
    Ed = []
    for d in range(3):
        g = 2.0 / h[d]
        if d == 2 and eta is not None:
            g = g * eta
        Ed.append(g ** 4 * S2 + g ** 2 * S1)
    C = kron3(Ed[0], F, F) + kron3(F, Ed[1], F) + kron3(F, F, Ed[2]) + kron3(F, F, F)
    return s * np.prod(h) / 8 * C


def patch_area(mesh, e):
    """(phi, theta)-area of a vertex corner's sphere patch, (2W+1)^2 GLL rule."""
    b = mesh.box[e]
    if mesh.chart[e] == M.VTX_BOX:
        return (b[1] - b[0]) * (b[3] - b[2])
    m = 2 * mesh.W + 1
    xm, wm = gll.gll(m)
    A, B = np.meshgrid(xm, xm, indexing="ij")
    lam = np.stack([A.ravel(), B.ravel(), np.ones(A.size)], -1)
    x, J, _ = charts.geometry(mesh, e, lam, second=False)
    xl = (x - mesh.origin[e]) @ mesh.mframe[e]
    Jy = np.einsum("ab,pbk->pak", mesh.mframe[e], charts.modified_jacobian(M.VTX, xl))
    dyl = np.linalg.solve(Jy, J)          # d y / d lam
    det = np.abs(dyl[:, 0, 0] * dyl[:, 1, 1] - dyl[:, 0, 1] * dyl[:, 1, 0])
    return float((np.outer(wm, wm).ravel() * det).sum())


def corner_blocks(mesh):
    """Dense matrix of the corner-DOF block (n_corner_dof square)."""
    nc = mesh.n_corner_dof
    Cc = np.zeros((nc, nc))
    n = mesh.n
    x, w = gll.gll(n)
    for e in range(mesh.E):
        k = mesh.kind[e]
        if k == M.REAL:
            continue
        b = mesh.box[e]
        o = mesh.cdof[e]
        reg = mesh.region[e]
        if k == M.CORNER_CONST:
            if reg == M.VTX:
                Cc[o, o] += np.exp(b[5]) * patch_area(mesh, e)
            elif reg == M.VE:
                Cc[o, o] += np.exp(b[5]) * (b[1] - b[0]) * (b[3] - b[2])
            else:
                raise ValueError("constant corner in region %d" % reg)
        else:
            d = mesh.cdir[e]
            hth = b[3] - b[2]
            hp = b[2 * d + 1] - b[2 * d]
            yk = b[2 * d] + 0.5 * (x + 1) * hp
            if reg == M.VE:
                diag = hth * hp / 2 * w * np.exp(yk)
            else:
                diag = hth * hp / 2 * w
            Cc[o:o + n, o:o + n] += np.diag(diag)
    return Cc


class BlockPreconditioner:
    def __init__(self, disc):
        self.disc = disc
        mesh = disc.mesh
        self.chol = []
        for e in disc.real:
            self.chol.append(sla.cho_factor(element_block(mesh, e)))
        self.Cc = corner_blocks(mesh)
        self.chol_c = sla.cho_factor(self.Cc) if mesh.n_corner_dof else None

    def apply(self, R):
        disc = self.disc
        n3 = disc.n ** 3
        Z = np.zeros_like(R)
        for i, e in enumerate(disc.real):
            o = disc.offset[e]
            Z[o:o + n3] = sla.cho_solve(self.chol[i], R[o:o + n3])
        if self.chol_c is not None:
            Z[disc.n_real_dof:] = sla.cho_solve(self.chol_c, R[disc.n_real_dof:])
        return Z


class ElementBlockPreconditioner:
    """W = the exact block diagonal of X: one n^3 x n^3 block per real element
    (its diagonal block of X = A^T M A) and one dense block for all corner
    unknowns; W^{-1} by Cholesky solves.  A stronger member of the block-
    diagonal family of Sec. 5.2 (the thesis approximates these blocks by the
    separable forms above).

    Columns of X are X applied to unit vectors.  To use fewer applies, the
    unit vectors at one local index of several elements that share no face
    term are applied together: X couples two real elements only through a
    face term between them, so the part of the result on each of those
    elements is its own column."""

    def __init__(self, disc):
        self.disc = disc
        self.blocks, self.Xcc = element_blocks(disc)
        self.chol = [sla.cho_factor(B) for B in self.blocks]
        self.chol_c = sla.cho_factor(self.Xcc) if self.Xcc.size else None

    def apply(self, R):
        disc = self.disc
        n3 = disc.n ** 3
        Z = np.zeros_like(R)
        for i, e in enumerate(disc.real):
            o = disc.offset[e]
            Z[o:o + n3] = sla.cho_solve(self.chol[i], R[o:o + n3])
        if self.chol_c is not None:
            Z[disc.n_real_dof:] = sla.cho_solve(self.chol_c, R[disc.n_real_dof:])
        return Z


def element_blocks(disc):
    """(list of the real elements' diagonal blocks of X, corner block of X)."""
    n3 = disc.n ** 3
    real = list(disc.real)
    nbr = {e: set() for e in real}
    for F in disc.faces:
        if F.eB is not None and F.eB >= 0 and F.eA in nbr and F.eB in nbr:
            nbr[F.eA].add(F.eB)
            nbr[F.eB].add(F.eA)
    colour = {}
    for e in real:
        taken = {colour[x] for x in nbr[e] if x in colour}
        c = 0
        while c in taken:
            c += 1
        colour[e] = c
    blocks = {e: np.zeros((n3, n3)) for e in real}
    for c in range(max(colour.values()) + 1 if real else 0):
        group = [e for e in real if colour[e] == c]
        for j in range(n3):
            v = np.zeros(disc.ndof)
            for e in group:
                v[disc.offset[e] + j] = 1.0
            y = disc.apply_X(v)
            for e in group:
                o = disc.offset[e]
                blocks[e][:, j] = y[o:o + n3]
    nc = disc.ndof - disc.n_real_dof
    Xcc = np.zeros((nc, nc))
    for j in range(nc):
        v = np.zeros(disc.ndof)
        v[disc.n_real_dof + j] = 1.0
        Xcc[:, j] = disc.apply_X(v)[disc.n_real_dof:]
    return [blocks[e] for e in real], Xcc
