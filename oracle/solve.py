"""Solvers for the normal equations X U = b and the relative H^1 error.

ORACLE: test infrastructure only.

* ``pcg``: preconditioned conjugate gradients (Ch. 5 intro; Ch. 6 intro),
  u0 = 0, stopped when ||b - X u_k||_2 / ||b||_2 < eps on the recursively
  updated residual (reading: the thesis states only "relative norm of the
  residual vector for the normal equations").
* ``dense_solve``: Cholesky of the assembled X (small meshes).
* ``h1_error``: ||u_h - u_ex||_{H^1} / ||u_ex||_{H^1} (Ch. 6 intro), broken
  over the real elements, Gauss-Legendre with W+6 points per direction in lam.
"""
import numpy as np
import scipy.linalg as sla

from workloads import mesh as M
from . import gll
from . import charts


def pcg(apply_X, b, precond, rtol=1e-12, maxit=10000, x0=None):
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_X(x) if x0 is not None else b.copy()
    z = precond(r)
    p = z.copy()
    rz = r @ z
    bn = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / bn]
    it = 0
    while hist[-1] > rtol and it < maxit:
        q = apply_X(p)
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = precond(r)
        rz_new = r @ z
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
        it += 1
        hist.append(np.linalg.norm(r) / bn)
    return x, it, np.array(hist)


def dense_solve(X, b):
    return sla.cho_solve(sla.cho_factor(X), b)


def h1_error(disc, U, problem, nq=None):
    """Relative broken H^1 error over the real elements."""
    mesh = disc.mesh
    nq = nq or disc.W + 6
    xg, wg = gll.gauss(nq)
    A, B, C = np.meshgrid(xg, xg, xg, indexing="ij")
    lam = np.stack([A.ravel(), B.ravel(), C.ravel()], -1)
    WA, WB, WC = np.meshgrid(wg, wg, wg, indexing="ij")
    wq = (WA * WB * WC).ravel()
    L = [[gll.lagrange(disc.xn, lam[:, d], k) for k in range(2)] for d in range(3)]
    num = den = 0.0
    for e in disc.real:
        ue = disc.element_values(U, e)
        x, J, _ = charts.geometry(mesh, e, lam, second=False)
        det = np.abs(np.linalg.det(J))
        val = np.einsum("pi,pj,pk,ijk->p", L[0][0], L[1][0], L[2][0], ue, optimize=True)
        gl = np.stack([np.einsum("pi,pj,pk,ijk->p", L[0][1], L[1][0], L[2][0], ue, optimize=True),
                       np.einsum("pi,pj,pk,ijk->p", L[0][0], L[1][1], L[2][0], ue, optimize=True),
                       np.einsum("pi,pj,pk,ijk->p", L[0][0], L[1][0], L[2][1], ue, optimize=True)], -1)
        gx = np.einsum("pca,pc->pa", np.linalg.inv(J), gl)
        ux = problem.u(x)
        gux = problem.grad_u(x)
        num += (wq * det * ((val - ux) ** 2 + ((gx - gux) ** 2).sum(-1))).sum()
        den += (wq * det * (ux ** 2 + (gux ** 2).sum(-1))).sum()
    return np.sqrt(num / den)
