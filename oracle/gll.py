"""1D Gauss-Lobatto-Legendre machinery (thesis Sec. 5.3).

ORACLE: test infrastructure only.

* ``gll(n)``: the n-point GLL rule: nodes -1, 1 and the roots of P'_{n-1};
  weights 2 / (n (n-1) P_{n-1}(xi)^2).  Exact for polynomials of degree
  <= 2n-3 (used with n = W+1 for the solution nodes and m = 2W+1 for the
  quadrature nodes; the thesis calls the latter the "2N+1" grid).
* ``lagrange(nodes, x, d)``: d-th derivative of the Lagrange basis at x,
  built from the Legendre Vandermonde matrix.
* ``diff_matrix``: the collocation differentiation matrix of eq 5.47.
* ``half_matrix``: the matrix of the discrete 1D H^{1/2} difference-quotient
  double integral on the GLL grid, written out from the GLL double-sum
  formula of Sec. 5.3 (the pairs i != i' give w_i w_i' times the squared
  difference quotient; the diagonal limit gives w_i^2 times the squared
  derivative).
* ``legendre_restriction``: the five-step discrete-Legendre-transform
  procedure of Sec. 5.3 that maps a vector on the fine grid to the coarse
  grid; it equals the transpose of fine-from-coarse interpolation.
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def legendre_vander(x, N, deriv=0):
    """V[q, k] = d^deriv/dx^deriv P_k(x_q), k = 0..N."""
    x = np.asarray(x, float)
    V = np.zeros((x.size, N + 1))
    for k in range(N + 1):
        c = np.zeros(N + 1)
        c[k] = 1.0
        if deriv:
            c = npleg.legder(c, deriv)
        V[:, k] = npleg.legval(x, c)
    return V


def gll(n):
    """n-point Gauss-Lobatto-Legendre nodes and weights (ascending)."""
    if n < 2:
        raise ValueError("GLL needs n >= 2")
    cN = np.zeros(n)
    cN[-1] = 1.0  # P_{n-1}
    interior = np.sort(npleg.legroots(npleg.legder(cN))) if n > 2 else np.zeros(0)
    x = np.concatenate([[-1.0], interior, [1.0]])
    # one Newton polish on the interior roots of P'_{n-1}
    if n > 2:
        d1 = npleg.legder(cN)
        d2 = npleg.legder(cN, 2)
        xi = x[1:-1]
        xi = xi - npleg.legval(xi, d1) / npleg.legval(xi, d2)
        x[1:-1] = xi
    w = 2.0 / (n * (n - 1) * npleg.legval(x, cN) ** 2)
    return x, w


def gauss(n):
    """n-point Gauss-Legendre rule (error quadrature)."""
    return npleg.leggauss(n)


def lagrange(nodes, x, deriv=0):
    """M[q, j] = l_j^(deriv)(x_q) for the Lagrange basis on ``nodes``."""
    nodes = np.asarray(nodes, float)
    N = nodes.size - 1
    V = legendre_vander(nodes, N)
    C = np.linalg.inv(V)            # l_j = sum_k C[k, j] P_k
    return legendre_vander(np.atleast_1d(x), N, deriv) @ C


def diff_matrix(nodes):
    """D[i, j] = l_j'(xi_i) (eq 5.47)."""
    return lagrange(nodes, nodes, 1)


def half_matrix(n):
    """K with l^T K l = discrete 1D H^{1/2} double integral on the n-point GLL grid.

    l^T K l = sum_{i != i'} w_i w_i' ((l_i - l_i')/(xi_i - xi_i'))^2
            + sum_i w_i^2 (sum_k d_ik l_k)^2            (Sec. 5.3)
    """
    x, w = gll(n)
    D = diff_matrix(x)
    K = np.zeros((n, n))
    for i in range(n):
        for ip in range(n):
            if i == ip:
                continue
            c = w[i] * w[ip] / (x[i] - x[ip]) ** 2
            v = np.zeros(n)
            v[i] += 1.0
            v[ip] -= 1.0
            K += c * np.outer(v, v)
    K += D.T @ np.diag(w ** 2) @ D
    return K


def half_form_direct(l_vals, n):
    """The same double sum evaluated directly for one vector (for pins)."""
    x, w = gll(n)
    D = diff_matrix(x)
    s = 0.0
    for i in range(n):
        for ip in range(n):
            if i != ip:
                s += w[i] * w[ip] * ((l_vals[i] - l_vals[ip]) / (x[i] - x[ip])) ** 2
    s += np.sum(w ** 2 * (D @ l_vals) ** 2)
    return s


def legendre_restriction(O, W):
    """Sec. 5.3 steps 1-5 in 1D: fine-grid vector O (2W+1) -> coarse (W+1).

    gamma_k^M = (k + 1/2)^-1 for k < M, 2/M for k = M (discrete norms).
    The "Legendre transform" is the discrete Legendre coefficient transform
    Delta_k = (1/gamma_k) sum_i w_i f_i P_k(xi_i).
    """
    M = 2 * W
    xf, wf = gll(M + 1)
    xc, wc = gll(W + 1)

    def gam(k, Mm):
        return 2.0 / Mm if k == Mm else 1.0 / (k + 0.5)

    O = np.asarray(O, float) / wf                                   # step 1
    Pf = legendre_vander(xf, M)
    Delta = np.array([(wf * O * Pf[:, k]).sum() / gam(k, M) for k in range(M + 1)])
    Delta = np.array([gam(k, M) * Delta[k] for k in range(M + 1)])  # step 2
    mu = np.array([Delta[k] / gam(k, W) for k in range(W + 1)])     # step 3
    Pc = legendre_vander(xc, W)
    eps = Pc @ mu                                                   # step 4
    return wc * eps                                                 # step 5
