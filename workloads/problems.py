"""Manufactured Poisson problems  -Laplace(u) = f, u = g on the boundary.

Each problem supplies numpy callables on points x [..., 3]:
  u(x), grad_u(x) [..., 3], f(x) = -Laplace(u)(x).
The Dirichlet data is g = u on the boundary, grad g = grad u.
"""
import numpy as np


class Problem:
    name = "problem"

    def neumann(self, x, nu):
        """Neumann data h = (du/dnu)_A = nu^T a grad u at points x with outward
        unit normals nu (a from ``coefficients`` when the problem has them)."""
        g = self.grad_u(x)
        if hasattr(self, "coefficients"):
            a = self.coefficients(x)[0]
            A = np.empty(a.shape[:-1] + (3, 3))
            for k, (i, j) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
                A[..., i, j] = A[..., j, i] = a[..., k]
            g = np.einsum("...ij,...j->...i", A, g)
        return (np.asarray(nu) * g).sum(-1)

    def u(self, x):
        raise NotImplementedError

    def grad_u(self, x):
        raise NotImplementedError

    def f(self, x):
        raise NotImplementedError


class SinProduct(Problem):
    """u = sin(pi x) sin(pi y) sin(pi z); f = 3 pi^2 u (thesis Table 6.2 data)."""
    name = "sin_product"

    def u(self, x):
        x = np.asarray(x)
        return np.sin(np.pi * x[..., 0]) * np.sin(np.pi * x[..., 1]) * np.sin(np.pi * x[..., 2])

    def grad_u(self, x):
        x = np.asarray(x)
        s = np.sin(np.pi * x)
        c = np.cos(np.pi * x)
        return np.pi * np.stack([c[..., 0] * s[..., 1] * s[..., 2],
                                 s[..., 0] * c[..., 1] * s[..., 2],
                                 s[..., 0] * s[..., 1] * c[..., 2]], -1)

    def f(self, x):
        return 3.0 * np.pi ** 2 * self.u(x)


class Polynomial(Problem):
    """u = a cubic-by-quadratic tensor polynomial (reproduced exactly when W >= 3)."""
    name = "polynomial"

    def u(self, x):
        x = np.asarray(x)
        return (1 + x[..., 0] - 2 * x[..., 0] ** 3) * (2 - x[..., 1] + x[..., 1] ** 2) * (1 + 3 * x[..., 2])

    def grad_u(self, x):
        x = np.asarray(x)
        a = 1 + x[..., 0] - 2 * x[..., 0] ** 3
        b = 2 - x[..., 1] + x[..., 1] ** 2
        c = 1 + 3 * x[..., 2]
        return np.stack([(1 - 6 * x[..., 0] ** 2) * b * c, a * (-1 + 2 * x[..., 1]) * c, a * b * 3], -1)

    def f(self, x):
        x = np.asarray(x)
        a = 1 + x[..., 0] - 2 * x[..., 0] ** 3
        b = 2 - x[..., 1] + x[..., 1] ** 2
        c = 1 + 3 * x[..., 2]
        return -((-12 * x[..., 0]) * b * c + a * 2 * c)


class Constant(Problem):
    """u = const, f = 0."""
    name = "constant"

    def __init__(self, c=1.7):
        self.c = c

    def u(self, x):
        return np.full(np.asarray(x).shape[:-1], self.c)

    def grad_u(self, x):
        return np.zeros(np.asarray(x).shape)

    def f(self, x):
        return np.zeros(np.asarray(x).shape[:-1])


class RhoPower(Problem):
    """u = rho^a * s(x), s = prod cos(pi x_i / 4), rho = |x| (Fichera data).

    f = -Laplace(u) = -[a(a+1) rho^(a-2) s + 2 a rho^(a-2) (x . grad s) - 3 k^2 rho^a s],
    k = pi/4.
    """
    name = "rho_power"

    def __init__(self, a=2.0 / 3.0):
        self.a = a
        self.k = np.pi / 4

    def _s(self, x):
        c = np.cos(self.k * x)
        return c[..., 0] * c[..., 1] * c[..., 2]

    def _grad_s(self, x):
        c = np.cos(self.k * x)
        s = np.sin(self.k * x)
        return -self.k * np.stack([s[..., 0] * c[..., 1] * c[..., 2],
                                   c[..., 0] * s[..., 1] * c[..., 2],
                                   c[..., 0] * c[..., 1] * s[..., 2]], -1)

    def u(self, x):
        x = np.asarray(x)
        rho = np.linalg.norm(x, axis=-1)
        return rho ** self.a * self._s(x)

    def grad_u(self, x):
        x = np.asarray(x)
        rho = np.linalg.norm(x, axis=-1)
        return (self.a * rho ** (self.a - 2) * self._s(x))[..., None] * x + (rho ** self.a)[..., None] * self._grad_s(x)

    def f(self, x):
        x = np.asarray(x)
        rho = np.linalg.norm(x, axis=-1)
        a, k = self.a, self.k
        s = self._s(x)
        xs = (x * self._grad_s(x)).sum(-1)
        lap = a * (a + 1) * rho ** (a - 2) * s + 2 * a * rho ** (a - 2) * xs - 3 * k ** 2 * rho ** a * s
        return -lap


class LegendreSource(Problem):
    """Source-parametrised data: f(x) = sum_{a,b,c < deg} theta[a + deg (b + deg c)]
    P_a(x1) P_b(x2) P_c(x3) (Legendre polynomials), homogeneous Dirichlet
    data g = 0.  The exact solution is not known (u, grad_u give g = 0)."""
    name = "legendre_source"

    def __init__(self, theta, deg):
        self.theta = np.asarray(theta, float).reshape(deg, deg, deg)   # [c, b, a]
        self.deg = deg

    def u(self, x):
        return np.zeros(np.asarray(x).shape[:-1])

    def grad_u(self, x):
        return np.zeros(np.asarray(x).shape)

    def f(self, x):
        from numpy.polynomial import legendre
        x = np.asarray(x)
        eye = np.eye(self.deg)
        P = [np.stack([legendre.legval(x[..., d], eye[k]) for k in range(self.deg)], -1) for d in range(3)]
        return np.einsum("cba,...a,...b,...c->...", self.theta, P[0], P[1], P[2])


def legendre_theta(deg, seed):
    """Seeded source coefficients, N(0, 1)."""
    return np.random.default_rng(seed).standard_normal(deg ** 3)


class FourierSource(Problem):
    """Smooth random data of the batched workload: f(x) = sum_k a_k cos(pi kappa_k . x
    + phi_k), homogeneous Dirichlet data.  coef [nmodes, 5] = (a, kappa_1..3, phi)."""
    name = "fourier_source"

    def __init__(self, coef):
        self.coef = np.asarray(coef, float).reshape(-1, 5)

    def u(self, x):
        return np.zeros(np.asarray(x).shape[:-1])

    def grad_u(self, x):
        return np.zeros(np.asarray(x).shape)

    def f(self, x):
        x = np.asarray(x)
        c = self.coef
        arg = np.pi * (x @ c[:, 1:4].T) + c[:, 4]
        return np.cos(arg) @ c[:, 0]


def fourier_coef(seed, nmodes=8):
    """a ~ N(0, 1), kappa in {0..3}^3, phi ~ U[0, 2 pi), seeded."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(nmodes)
    kappa = rng.integers(0, 4, (nmodes, 3)).astype(float)
    phi = rng.uniform(0, 2 * np.pi, nmodes)
    return np.column_stack([a, kappa, phi])


def _spherical(x):
    """rho, phi (from +x3), theta in [0, 2 pi), r = distance to the x3 axis."""
    x = np.asarray(x)
    r = np.hypot(x[..., 0], x[..., 1])
    rho = np.sqrt(r ** 2 + x[..., 2] ** 2)
    phi = np.arctan2(r, x[..., 2])
    th = np.mod(np.arctan2(x[..., 1], x[..., 0]), 2 * np.pi)
    return rho, phi, th, r


def _frame(phi, th):
    """Unit vectors rho-hat, phi-hat, theta-hat [..., 3]."""
    sp, cp, st, ct = np.sin(phi), np.cos(phi), np.sin(th), np.cos(th)
    e_rho = np.stack([sp * ct, sp * st, cp], -1)
    e_phi = np.stack([cp * ct, cp * st, -sp], -1)
    e_th = np.stack([-st, ct, np.zeros_like(st)], -1)
    return e_rho, e_phi, e_th


class VertexPower(Problem):
    """u = rho^(1/2) sin(phi/2) on Omega^(v) (thesis Table 6.16 data).

    -Laplace(u) = -rho^(-3/2) (sin(phi/2)/2 + cos(phi) / (4 sin(phi/2)))."""
    name = "vertex_power"

    def u(self, x):
        rho, phi, _, _ = _spherical(x)
        return np.sqrt(rho) * np.sin(phi / 2)

    def grad_u(self, x):
        rho, phi, th, _ = _spherical(x)
        e_rho, e_phi, _ = _frame(phi, th)
        u_rho = 0.5 / np.sqrt(rho) * np.sin(phi / 2)
        u_phi = 0.5 * np.sqrt(rho) * np.cos(phi / 2)
        return u_rho[..., None] * e_rho + (u_phi / rho)[..., None] * e_phi

    def f(self, x):
        rho, phi, _, _ = _spherical(x)
        return -rho ** -1.5 * (np.sin(phi / 2) / 2 + np.cos(phi) / (4 * np.sin(phi / 2)))


class EdgePower(Problem):
    """u = r^(1/3) sin(theta/3) x3, harmonic (thesis Table 6.18 data)."""
    name = "edge_power"

    def u(self, x):
        x = np.asarray(x)
        _, _, th, r = _spherical(x)
        return np.cbrt(r) * np.sin(th / 3) * x[..., 2]

    def grad_u(self, x):
        x = np.asarray(x)
        _, _, th, r = _spherical(x)
        st, ct = np.sin(th), np.cos(th)
        u_r = np.cbrt(r) / (3 * r) * np.sin(th / 3) * x[..., 2]
        u_th_over_r = np.cbrt(r) / (3 * r) * np.cos(th / 3) * x[..., 2]
        u_3 = np.cbrt(r) * np.sin(th / 3)
        return np.stack([u_r * ct - u_th_over_r * st, u_r * st + u_th_over_r * ct, u_3], -1)

    def f(self, x):
        return np.zeros(np.asarray(x).shape[:-1])


class VertexEdgePower(Problem):
    """u = rho^(3/4) (sin phi)^(1/2) sin(theta/2) (thesis Table 6.20 data).

    -Laplace(u) = -(9/16) rho^-2 u."""
    name = "vertex_edge_power"

    def u(self, x):
        rho, phi, th, _ = _spherical(x)
        return rho ** 0.75 * np.sqrt(np.sin(phi)) * np.sin(th / 2)

    def grad_u(self, x):
        rho, phi, th, _ = _spherical(x)
        e_rho, e_phi, e_th = _frame(phi, th)
        s = np.sin(phi)
        u_rho = 0.75 * rho ** -0.25 * np.sqrt(s) * np.sin(th / 2)
        u_phi_over_rho = rho ** -0.25 * 0.5 / np.sqrt(s) * np.cos(phi) * np.sin(th / 2)
        u_th_over = rho ** -0.25 * 0.5 / np.sqrt(s) * np.cos(th / 2)
        return u_rho[..., None] * e_rho + u_phi_over_rho[..., None] * e_phi + u_th_over[..., None] * e_th

    def f(self, x):
        rho = _spherical(x)[0]
        return -(9.0 / 16.0) * self.u(x) / rho ** 2


class GeneralElliptic(Problem):
    """A non-self-adjoint elliptic operator with variable coefficients (the
    thesis's Sec. 6.2 example of Table 6.14, with Dirichlet data on the whole
    boundary):

        L u = -(0.50 + 0.05 e^{x y z}) u_xx - (1.00 + 0.015 cos(x + y)) u_yy
              - (2.50 + 0.02 e^{y + z}) u_zz - 0.001 sin(pi (x + y + z)) (u_xy + u_yz + u_zx)
              + (4.05 + 0.045 cos(pi (x + y + z) / 2)) u,

    u = (sin(pi x) + sin(pi y / 2)) cos(pi z), f = L u.  ``coefficients``
    gives L in the form L u = -sum_ij a_ij u_{x_i x_j} + sum_j beta_j u_{x_j}
    + c u (a symmetric: a_12 = a_21 carry half the mixed term each; beta = 0;
    eq 2.2 with b_j = beta_j + sum_i d a_ij / d x_i)."""
    name = "general_elliptic"

    def coefficients(self, x):
        x = np.asarray(x)
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        s = X + Y + Z
        a = np.zeros(x.shape[:-1] + (6,))          # a11 a22 a33 a12 a13 a23
        a[..., 0] = 0.50 + 0.05 * np.exp(X * Y * Z)
        a[..., 1] = 1.00 + 0.015 * np.cos(X + Y)
        a[..., 2] = 2.50 + 0.02 * np.exp(Y + Z)
        a[..., 3:6] = (0.001 * np.sin(np.pi * s) / 2)[..., None]
        beta = np.zeros(x.shape[:-1] + (3,))
        c = 4.05 + 0.045 * np.cos(np.pi * s / 2)
        return a, beta, c

    def u(self, x):
        x = np.asarray(x)
        return (np.sin(np.pi * x[..., 0]) + np.sin(np.pi * x[..., 1] / 2)) * np.cos(np.pi * x[..., 2])

    def grad_u(self, x):
        x = np.asarray(x)
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        s = np.sin(np.pi * X) + np.sin(np.pi * Y / 2)
        return np.stack([np.pi * np.cos(np.pi * X) * np.cos(np.pi * Z),
                         np.pi / 2 * np.cos(np.pi * Y / 2) * np.cos(np.pi * Z),
                         -np.pi * s * np.sin(np.pi * Z)], -1)

    def hess_u(self, x):
        """[..., 6]: u_xx u_yy u_zz u_xy u_xz u_yz."""
        x = np.asarray(x)
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        s = np.sin(np.pi * X) + np.sin(np.pi * Y / 2)
        cz, sz = np.cos(np.pi * Z), np.sin(np.pi * Z)
        return np.stack([-np.pi ** 2 * np.sin(np.pi * X) * cz,
                         -(np.pi / 2) ** 2 * np.sin(np.pi * Y / 2) * cz,
                         -np.pi ** 2 * s * cz,
                         np.zeros_like(X),
                         -np.pi ** 2 * np.cos(np.pi * X) * sz,
                         -np.pi ** 2 / 2 * np.cos(np.pi * Y / 2) * sz], -1)

    def f(self, x):
        a, beta, c = self.coefficients(x)
        H = self.hess_u(x)
        lu = -(a[..., 0] * H[..., 0] + a[..., 1] * H[..., 1] + a[..., 2] * H[..., 2]
               + 2 * (a[..., 3] * H[..., 3] + a[..., 4] * H[..., 4] + a[..., 5] * H[..., 5]))
        return lu + (beta * self.grad_u(x)).sum(-1) + c * self.u(x)


class MixedSin(Problem):
    """u = (2 / pi^2) sin(pi x / 2) (cos(pi y / 2) - sin(pi z / 2)) on (-1,1)^3,
    Dirichlet on x = -1, 1 and y = -1, Neumann on y = 1, z = -1, 1 (thesis
    Table 6.3 data)."""
    name = "mixed_sin"
    NEUMANN_FACES = ((1, 1), (2, 0), (2, 1))

    def u(self, x):
        x = np.asarray(x)
        k = np.pi / 2
        return 2 / np.pi ** 2 * np.sin(k * x[..., 0]) * (np.cos(k * x[..., 1]) - np.sin(k * x[..., 2]))

    def grad_u(self, x):
        x = np.asarray(x)
        k = np.pi / 2
        c = 2 / np.pi ** 2
        sx, cx = np.sin(k * x[..., 0]), np.cos(k * x[..., 0])
        t = np.cos(k * x[..., 1]) - np.sin(k * x[..., 2])
        return np.stack([c * k * cx * t, -c * k * sx * np.sin(k * x[..., 1]), -c * k * sx * np.cos(k * x[..., 2])], -1)

    def f(self, x):
        return 2 * (np.pi / 2) ** 2 * self.u(x)
