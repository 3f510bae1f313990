"""Layer-graded polynomial degrees (thesis Sec. 2.3).

ORACLE: test infrastructure only.

Sec. 2.3 lets the degree of the spectral element functions on the real
elements of a geometric mesh grow with the layer: W_l = [mu_1 i] in the
vertex layers (all three directions), W_q = [mu_1 i] in the (tau, theta)
directions of the edge layers (degree W along x3), W_q = [mu_1 i] in (psi,
theta) and V_q = [mu_2 k] in zeta in the vertex-edge layers, all clipped to
1..W; the regular region keeps W.  An element's degrees are a triple w =
(w1, w2, w3), one per master-cube direction lam_d.

The functions of degree w on an element form a subspace of those of degree
W.  The graded discretisation minimises the same functional R^{N,W} over
that subspace.  With P the embedding (the degree-w nodal basis on the
(w_d + 1)-point GLL nodes, evaluated at the degree-W GLL nodes, one factor
per direction; corner unknowns unchanged), the normal equations are
P^T X P c = P^T b and the solution is u = P c.

Readings where the thesis is silent (it ran uniform degrees only):
* every element is integrated with the mesh's rule (2W+1 GLL points per
  direction, W the largest degree), which is exact or more accurate for the
  lower-degree functions;
* corner functions keep degree W (the vertex-edge corner polynomials too).

Vectors keep the uniform layout ((W+1)^3 values per real element); a
vector of the graded space is P c.  Q = P (P^T P)^{-1} P^T is the orthogonal
projector onto that space; on it the graded normal equations read
Q X Q u = Q b, whose solution is the same u = P c.  The oracle computes the
reduced system literally and maps back; ``apply_X`` and ``rhs`` return the
projected quantities Q X u and Q b for comparisons in the uniform layout.

Preconditioners of the graded system (both act as P (.)^{-1} P^T-type maps
onto the graded space):
* separable form (Sec. 5.2 restricted): B_e = P_e (P_e^T C_e P_e)^{-1} P_e^T;
* exact element blocks: B_e = (Q_e X_ee Q_e + s_e (I - Q_e))^{-1},
  s_e = tr(X_ee) / n^3: the inverse of the projected block on the graded
  space, and on its complement the identity scaled like the block.
"""
import numpy as np
import scipy.linalg as sla

from workloads import mesh as M
from . import gll
from . import precond as PC


def embedding_1d(W, w):
    """P[i, j] = l^(w)_j(x^(W)_i): the degree-w Lagrange basis on the
    (w+1)-point GLL nodes at the (W+1)-point GLL nodes (n x (w+1))."""
    if not 1 <= w <= W:
        raise ValueError("degree %d outside 1..%d" % (w, W))
    xw, _ = gll.gll(w + 1)
    xW, _ = gll.gll(W + 1)
    return gll.lagrange(xw, xW)


def element_embedding(W, deg):
    """Embedding of one element's degree-(w1, w2, w3) space (uniform layout,
    i fastest along lam_1)."""
    return PC.kron3(*(embedding_1d(W, int(w)) for w in deg))


def projector_1d(W, w):
    """Orthogonal projector onto the degree-w polynomials in the nodal values
    at the degree-W GLL nodes: P (P^T P)^{-1} P^T by least squares."""
    P = embedding_1d(W, w)
    return P @ np.linalg.lstsq(P, np.eye(W + 1), rcond=None)[0]


class GradedSystem:
    """The graded normal equations on a Discretization at the mesh's W."""

    def __init__(self, disc, deg):
        self.disc = disc
        mesh = disc.mesh
        W = disc.W
        deg = np.asarray(deg, int).reshape(mesh.E, 3)
        self.deg = deg
        self.P = {}
        self.Q = {}
        self.roff = {}
        o = 0
        for e in disc.real:
            self.P[e] = element_embedding(W, deg[e])
            self.Q[e] = [projector_1d(W, int(w)) for w in deg[e]]
            self.roff[e] = o
            o += self.P[e].shape[1]
        self.n_real_graded = o
        self.ncd = mesh.n_corner_dof
        self.ndof_graded = o + self.ncd

    # graded coefficients c <-> uniform-layout vectors
    def embed(self, c):
        disc = self.disc
        U = np.zeros(disc.ndof)
        for e in disc.real:
            P, r0, o = self.P[e], self.roff[e], disc.offset[e]
            U[o:o + P.shape[0]] = P @ c[r0:r0 + P.shape[1]]
        U[disc.n_real_dof:] = c[self.n_real_graded:]
        return U

    def restrict(self, U):
        """P^T U."""
        disc = self.disc
        c = np.zeros(self.ndof_graded)
        for e in disc.real:
            P, r0, o = self.P[e], self.roff[e], disc.offset[e]
            c[r0:r0 + P.shape[1]] = P.T @ U[o:o + P.shape[0]]
        c[self.n_real_graded:] = U[disc.n_real_dof:]
        return c

    def project(self, U):
        """Q U (real elements; corner unknowns unchanged)."""
        from .functional import tensor_apply
        disc = self.disc
        out = np.array(U, float, copy=True)
        for e in disc.real:
            ue = disc.element_values(U, e)
            Q = self.Q[e]
            o = disc.offset[e]
            out[o:o + disc.n ** 3] = tensor_apply(Q[0], Q[1], Q[2], ue).reshape(-1, order="F")
        return out

    def apply_X(self, U):
        """Q X U."""
        return self.project(self.disc.apply_X(U))

    def rhs(self):
        """Q b."""
        return self.project(self.disc.rhs())

    def reduced_matrix(self):
        """P^T X P (dense, small meshes)."""
        Xr = np.zeros((self.ndof_graded, self.ndof_graded))
        c = np.zeros(self.ndof_graded)
        for j in range(self.ndof_graded):
            c[:] = 0
            c[j] = 1
            Xr[:, j] = self.restrict(self.disc.apply_X(self.embed(c)))
        return Xr

    def solve(self):
        """u = P (P^T X P)^{-1} P^T b (dense Cholesky)."""
        Xr = self.reduced_matrix()
        c = sla.cho_solve(sla.cho_factor(Xr), self.restrict(self.disc.rhs()))
        return self.embed(c)


class GradedSeparablePreconditioner:
    """B_e = P_e (P_e^T C_e P_e)^{-1} P_e^T with the separable block C_e of
    Sec. 5.2 at the mesh's W; corner block as in the uniform case."""

    def __init__(self, gs):
        self.gs = gs
        disc = gs.disc
        mesh = disc.mesh
        self.fac = {}
        for e in disc.real:
            P = gs.P[e]
            self.fac[e] = sla.cho_factor(P.T @ PC.element_block(mesh, e) @ P)
        Cc = PC.corner_blocks(mesh)
        self.chol_c = sla.cho_factor(Cc) if mesh.n_corner_dof else None

    def apply(self, R):
        gs, disc = self.gs, self.gs.disc
        n3 = disc.n ** 3
        Z = np.zeros_like(R)
        for e in disc.real:
            o, P = disc.offset[e], gs.P[e]
            Z[o:o + n3] = P @ sla.cho_solve(self.fac[e], P.T @ R[o:o + n3])
        if self.chol_c is not None:
            Z[disc.n_real_dof:] = sla.cho_solve(self.chol_c, R[disc.n_real_dof:])
        return Z


class GradedElementBlockPreconditioner:
    """B_e = (Q_e X_ee Q_e + s_e (I - Q_e))^{-1}, s_e = tr(X_ee) / n^3;
    corner block of X as in the uniform case."""

    def __init__(self, gs):
        self.gs = gs
        disc = gs.disc
        blocks, Xcc = PC.element_blocks(disc)
        n3 = disc.n ** 3
        self.fac = {}
        for e, Xe in zip(disc.real, blocks):
            Q = PC.kron3(*gs.Q[e])
            s = np.trace(Xe) / n3
            self.fac[e] = sla.cho_factor(Q @ Xe @ Q + s * (np.eye(n3) - Q))
        self.chol_c = sla.cho_factor(Xcc) if Xcc.size else None

    def apply(self, R):
        disc = self.gs.disc
        n3 = disc.n ** 3
        Z = np.zeros_like(R)
        for e in disc.real:
            o = disc.offset[e]
            Z[o:o + n3] = sla.cho_solve(self.fac[e], R[o:o + n3])
        if self.chol_c is not None:
            Z[disc.n_real_dof:] = sla.cho_solve(self.chol_c, R[disc.n_real_dof:])
        return Z
