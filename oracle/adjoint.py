"""Gradient of a misfit of the least-squares solution with respect to source
coefficients, from its plain definition.

ORACLE: test infrastructure only.

The solution of the normal equations is u(theta) = X^{-1} b(theta) (Sec. 5.3)
with b(theta) = A^T M d(theta) linear in the source coefficients.  For
L(theta) = ||u(theta) - u_t||_2^2 over the unknowns,
    dL/dtheta_k = 2 (u - u_t)^T X^{-1} b(e_k) = lambda^T b(e_k),
    lambda = X^{-1} 2 (u - u_t)       (X is symmetric),
and b(e_k) is the right-hand side of the k-th source basis function alone,
assembled here column by column.
"""
import numpy as np

from workloads.problems import LegendreSource


def source_rhs(disc, theta, deg):
    """b(theta) for the Legendre source with homogeneous Dirichlet data."""
    saved = disc.problem
    disc.problem = LegendreSource(theta, deg)
    try:
        return disc.rhs()
    finally:
        disc.problem = saved


def source_rhs_columns(disc, deg):
    """[ndof, deg^3]: b(e_k) for every basis function."""
    K = deg ** 3
    B = np.zeros((disc.ndof, K))
    for k in range(K):
        e = np.zeros(K)
        e[k] = 1.0
        B[:, k] = source_rhs(disc, e, deg)
    return B


def loss_and_grad(disc, theta, u_target, deg, solve):
    """(L, dL/dtheta) with solve(rhs) -> X^{-1} rhs."""
    u = solve(source_rhs(disc, theta, deg))
    res = u - u_target
    lam = solve(2.0 * res)
    B = source_rhs_columns(disc, deg)
    return float(res @ res), B.T @ lam
