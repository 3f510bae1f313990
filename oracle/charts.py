"""Element maps and their derivatives (thesis Ch. 2: analytic maps M_l from the
master cube Q to each element, in standard coordinates in the regular region
and in the modified coordinates of eq 2.3, 2.5, 2.8 in the neighbourhoods).

ORACLE: test infrastructure only.

The first and second derivatives of every map are obtained symbolically with
sympy from the chart formulas written below, then evaluated with numpy.
"""
import functools
import numpy as np
import sympy as sp

from workloads import mesh as M

_l = sp.symbols("l1 l2 l3", real=True)
_b = sp.symbols("b0:6", real=True)
_p = sp.symbols("p0:12", real=True)


def _aff(i):
    return _b[2 * i] + (_l[i] + 1) / 2 * (_b[2 * i + 1] - _b[2 * i])


def _planar(ptype, inner):
    u = (_l[0] + 1) / 2
    v = (_l[1] + 1) / 2
    if ptype == 0:
        th = _p[1] + u * (_p[2] - _p[1])
        r_in = _p[3] if inner == "S" else _p[4]
        ax, ay = r_in * sp.cos(th), r_in * sp.sin(th)
        ox = _p[5] + u * (_p[7] - _p[5])
        oy = _p[6] + u * (_p[8] - _p[6])
        return (1 - v) * ax + v * ox, (1 - v) * ay + v * oy
    c = _p[1:9]
    px = (1 - u) * (1 - v) * c[0] + u * (1 - v) * c[2] + (1 - u) * v * c[4] + u * v * c[6]
    py = (1 - u) * (1 - v) * c[1] + u * (1 - v) * c[3] + (1 - u) * v * c[5] + u * v * c[7]
    return px, py


def _local_expr(chart, ptype):
    y1, y2, y3 = _aff(0), _aff(1), _aff(2)
    if chart == M.AFFINE:
        return [y1, y2, y3]
    if chart == M.VTX_BOX:
        rho = sp.exp(y3)
        return [rho * sp.sin(y1) * sp.cos(y2), rho * sp.sin(y1) * sp.sin(y2), rho * sp.cos(y1)]
    if chart == M.VE_BOX:
        r = sp.exp(y1 + y3)
        return [r * sp.cos(y2), r * sp.sin(y2), sp.exp(y3)]
    if chart == M.EDGE_BOX:
        r = sp.exp(y1)
        return [r * sp.cos(y2), r * sp.sin(y2), y3]
    if chart == M.VTX_PATCH:
        px, py = _planar(ptype, "S")
        nrm = sp.sqrt(px ** 2 + py ** 2 + 1)
        rho = sp.exp(y3)
        return [rho * px / nrm, rho * py / nrm, rho / nrm]
    if chart == M.COLUMN:
        sx, sy = _planar(ptype, "S")
        nrm = sp.sqrt(sx ** 2 + sy ** 2 + 1)
        tx, ty = _planar(ptype, "T")
        t = y3
        rs = _p[9]
        return [(1 - t) * rs * sx / nrm + t * tx, (1 - t) * rs * sy / nrm + t * ty,
                (1 - t) * rs / nrm + t]
    raise ValueError(chart)


@functools.lru_cache(maxsize=None)
def _compiled(chart, ptype):
    X = _local_expr(chart, ptype)
    J = [[sp.diff(X[a], _l[c]) for c in range(3)] for a in range(3)]
    H = [[[sp.diff(X[a], _l[c], _l[d]) for d in range(3)] for c in range(3)] for a in range(3)]
    args = list(_l) + list(_b) + list(_p)
    fx = sp.lambdify(args, X, "numpy")
    fj = sp.lambdify(args, J, "numpy")
    fh = sp.lambdify(args, H, "numpy")
    return fx, fj, fh


def _bcast(v, shape):
    return np.broadcast_to(np.asarray(v, float), shape)


def geometry(mesh, e, lam, second=True):
    """x [P,3], J [P,3,3] (J[a,c] = dx_a/dlam_c), H [P,3,3,3] (H[a,c,d]) at lam [P,3]."""
    lam = np.asarray(lam, float).reshape(-1, 3)
    P = lam.shape[0]
    chart = int(mesh.chart[e])
    ptype = int(mesh.patch[e][0]) if chart in (M.VTX_PATCH, M.COLUMN) else 0
    fx, fj, fh = _compiled(chart, ptype)
    args = [lam[:, 0], lam[:, 1], lam[:, 2]] + list(mesh.box[e]) + list(mesh.patch[e])
    xl = np.stack([_bcast(v, (P,)) for v in fx(*args)], -1)
    Jl = np.stack([np.stack([_bcast(v, (P,)) for v in row], -1) for row in fj(*args)], -2)
    R = mesh.frame[e]
    x = mesh.origin[e] + xl @ R.T
    J = np.einsum("ab,pbc->pac", R, Jl)
    if not second:
        return x, J, None
    Hl = np.stack([np.stack([np.stack([_bcast(v, (P,)) for v in r2], -1) for r2 in r1], -2)
                   for r1 in fh(*args)], -3)
    H = np.einsum("ab,pbcd->pacd", R, Hl)
    return x, J, H


# --------------------------------------------------------------------------
# Modified coordinates of a neighbourhood frame (eq 2.3, 2.5, 2.8):
# dx_local/dy as a function of the local point, written from the inverse
# relations x(y).
# --------------------------------------------------------------------------

def modified_jacobian(kind, xl):
    """Jy[p, a, k] = d x_local_a / d y_k for y the modified coordinates."""
    x, y, z = xl[..., 0], xl[..., 1], xl[..., 2]
    r = np.sqrt(x ** 2 + y ** 2)
    ct, st = x / r, y / r
    Jy = np.zeros(xl.shape + (3,))
    if kind == M.VTX:      # (phi, theta, chi): x = e^chi (sin phi cos th, sin phi sin th, cos phi)
        rho = np.sqrt(r ** 2 + z ** 2)
        cp, sp_ = z / rho, r / rho
        Jy[..., 0, 0] = rho * cp * ct
        Jy[..., 1, 0] = rho * cp * st
        Jy[..., 2, 0] = -rho * sp_
        Jy[..., 0, 1] = -rho * sp_ * st
        Jy[..., 1, 1] = rho * sp_ * ct
        Jy[..., :, 2] = xl
    elif kind == M.VE:     # (psi, theta, zeta): x3 = e^zeta, r = e^(psi+zeta)
        Jy[..., 0, 0] = x
        Jy[..., 1, 0] = y
        Jy[..., 0, 1] = -y
        Jy[..., 1, 1] = x
        Jy[..., 0, 2] = x
        Jy[..., 1, 2] = y
        Jy[..., 2, 2] = z
    elif kind == M.EDGE:   # (tau, theta, x3): r = e^tau
        Jy[..., 0, 0] = x
        Jy[..., 1, 0] = y
        Jy[..., 0, 1] = -y
        Jy[..., 1, 1] = x
        Jy[..., 2, 2] = 1.0
    else:
        raise ValueError(kind)
    return Jy
