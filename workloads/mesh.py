"""Mesh descriptions for the least-squares h-p spectral element method.

A mesh is plain arrays, so that it can cross a C ABI unchanged.  It says
which elements exist, the analytic map of each from the master cube
Q = (-1,1)^3, and which faces touch.  It holds none of the method's
arithmetic (no quadrature, no operator, no norm): the oracle and the HIP
library each derive the discrete functional from it on their own.

``mframe`` is the frame of the modified coordinates in which the derivative
jumps of the vertex region are taken (its poles must lie outside the
element); for the other regions it equals ``frame``.

Element maps (thesis Ch. 2, Sec. 2.3: every element is the image of Q under
an analytic map; in the neighbourhoods the map goes to modified
coordinates, eq 2.3, 2.5, 2.8).  ``frame`` R and ``origin`` o place the
chart: x = o + R @ x_local.

  AFFINE     x_local = lo + (lam+1)/2 (hi-lo)
  VTX_BOX    (phi, theta, chi) affine in lam;  x_local = e^chi (sin phi cos theta,
             sin phi sin theta, cos phi)
  VE_BOX     (psi, theta, zeta) affine in lam; x3 = e^zeta, r = e^(psi+zeta)
  EDGE_BOX   (tau, theta, x3) affine in lam;   r = e^tau
  VTX_PATCH  (lam1, lam2) -> planar point P in the plane z_local = 1 (a
             "gnomonic" patch, see below); chi affine in lam3;
             x_local = e^chi (P,1)/|(P,1)|
  COLUMN     t affine in lam3 on [t0, t1];  x_local = (1-t) S + t T with
             S = rho_s (P_S,1)/|(P_S,1)| on the sphere of radius rho_s and
             T = (P_T, 1) on the plane z_local = 1

Planar patches (``patch`` row): ptype 0 = polar ruled patch between the arc
r = r_in, theta in [th0, th1] (theta affine in lam1) and the segment O0->O1
(affine in lam1), blended linearly in lam2; S uses r_in = patch[3], T uses
r_in = patch[4].  ptype 1 = bilinear patch through the four corners
C00, C10, C01, C11 (first index lam1, second lam2), same for S and T.

Faces: face f = 2 d + s is lam_d = -1 (s=0) or +1 (s=1).  Its face
coordinates are the two remaining lam's in increasing order.  ``orient``
maps the face coordinates (a, b) of this element to those of the
neighbour: bit0 swaps them, bit1 negates the first, bit2 the second.

Boundary codes: INTERIOR (neighbour given), DIRICHLET (on the boundary,
finite measure in modified coordinates), NEUMANN (the same, with a
conormal-derivative condition), SKIP (a face of infinite measure
in modified coordinates; the thesis sums only over faces with finite
measure, eq 2.25, 2.29, 2.38).

Corner elements (thesis Sec. 2.3): a semi-infinite element in modified
coordinates carries a shared function, either the vertex constant h_v
(CORNER_CONST) or a polynomial in one modified coordinate shared over the
theta-sectors (CORNER_POLY, along lam direction ``cdir``).  Their ``box``
is truncated to a finite box on the side of the infinite direction; that
is harmless, because the corner function does not vary along it.  Their
unknowns live in a separate corner-DOF array at offset ``cdof``.
"""
from dataclasses import dataclass
import numpy as np

REG, VTX, VE, EDGE = 0, 1, 2, 3
REAL, CORNER_CONST, CORNER_POLY = 0, 1, 2
AFFINE, VTX_BOX, VE_BOX, EDGE_BOX, VTX_PATCH, COLUMN = 0, 1, 2, 3, 4, 5
INTERIOR, DIRICHLET, SKIP, NEUMANN = 0, 1, 2, 3

FACE_TANGENT = ((1, 2), (0, 2), (0, 1))


@dataclass
class Mesh:
    W: int
    region: np.ndarray      # [E] int32
    kind: np.ndarray        # [E] int32
    chart: np.ndarray       # [E] int32
    frame: np.ndarray       # [E,3,3] float64
    mframe: np.ndarray      # [E,3,3] frame of the modified coordinates (derivative jumps)
    origin: np.ndarray      # [E,3]
    box: np.ndarray         # [E,6] lo1,hi1,lo2,hi2,lo3,hi3 in chart coordinates
    patch: np.ndarray       # [E,12] patch descriptor (see module doc)
    nbr: np.ndarray         # [E,6] int32, -1 if none
    nbr_face: np.ndarray    # [E,6] int32
    orient: np.ndarray      # [E,6] int32
    bc: np.ndarray          # [E,6] int32
    cdof: np.ndarray        # [E] int32 corner-DOF offset, -1 for real elements
    cdir: np.ndarray        # [E] int32 polynomial direction of CORNER_POLY
    n_corner_dof: int
    name: str = ""
    info: dict = None
    layer: np.ndarray = None  # [E,2] int32 geometric layer indices (i, k) of Sec. 2.3, 0 = none

    @property
    def E(self):
        return len(self.region)

    @property
    def n(self):
        return self.W + 1

    def real_elements(self):
        return np.nonzero(self.kind == REAL)[0]

    def ndof(self):
        return int((self.kind == REAL).sum()) * self.n ** 3 + self.n_corner_dof

    def as_arrays(self):
        """Contiguous arrays in the layout the C ABI expects."""
        return dict(
            region=np.ascontiguousarray(self.region, np.int32),
            kind=np.ascontiguousarray(self.kind, np.int32),
            chart=np.ascontiguousarray(self.chart, np.int32),
            frame=np.ascontiguousarray(self.frame, np.float64),
            mframe=np.ascontiguousarray(self.mframe, np.float64),
            origin=np.ascontiguousarray(self.origin, np.float64),
            box=np.ascontiguousarray(self.box, np.float64),
            patch=np.ascontiguousarray(self.patch, np.float64),
            nbr=np.ascontiguousarray(self.nbr, np.int32),
            nbr_face=np.ascontiguousarray(self.nbr_face, np.int32),
            orient=np.ascontiguousarray(self.orient, np.int32),
            bc=np.ascontiguousarray(self.bc, np.int32),
            cdof=np.ascontiguousarray(self.cdof, np.int32),
            cdir=np.ascontiguousarray(self.cdir, np.int32),
        )


def orient_map(o, a, b):
    """Face coordinates on the neighbour for face coordinates (a, b) here."""
    if o & 1:
        a, b = b, a
    if o & 2:
        a = -a
    if o & 4:
        b = -b
    return a, b


# --------------------------------------------------------------------------
# Chart evaluation (positions only).  This is the definition of the element
# maps; the oracle and the library each differentiate their own copy.
# --------------------------------------------------------------------------

def _planar(p, a, s, inner):
    """Planar patch point for lam1 = a, lam2 = s (arrays)."""
    ptype = int(p[0])
    u = 0.5 * (a + 1.0)
    v = 0.5 * (s + 1.0)
    if ptype == 0:
        th0, th1, r_s, r_t = p[1], p[2], p[3], p[4]
        r_in = r_s if inner == "S" else r_t
        th = th0 + u * (th1 - th0)
        ax, ay = r_in * np.cos(th), r_in * np.sin(th)
        ox = p[5] + u * (p[7] - p[5])
        oy = p[6] + u * (p[8] - p[6])
        return (1 - v) * ax + v * ox, (1 - v) * ay + v * oy
    c = p[1:9]
    px = (1 - u) * (1 - v) * c[0] + u * (1 - v) * c[2] + (1 - u) * v * c[4] + u * v * c[6]
    py = (1 - u) * (1 - v) * c[1] + u * (1 - v) * c[3] + (1 - u) * v * c[5] + u * v * c[7]
    return px, py


def chart_points(mesh, e, lam):
    """Physical points x for master-cube points lam [..., 3] of element e.

    Complex lam is kept complex (every chart is analytic), so that callers
    can differentiate the maps by complex steps."""
    lam = np.asarray(lam)
    lam = lam.astype(complex if np.iscomplexobj(lam) else float)
    l1, l2, l3 = lam[..., 0], lam[..., 1], lam[..., 2]
    b = mesh.box[e]
    y1 = b[0] + 0.5 * (l1 + 1) * (b[1] - b[0])
    y2 = b[2] + 0.5 * (l2 + 1) * (b[3] - b[2])
    y3 = b[4] + 0.5 * (l3 + 1) * (b[5] - b[4])
    c = mesh.chart[e]
    if c == AFFINE:
        xl = np.stack([y1, y2, y3], -1)
    elif c == VTX_BOX:
        rho = np.exp(y3)
        xl = np.stack([rho * np.sin(y1) * np.cos(y2), rho * np.sin(y1) * np.sin(y2),
                       rho * np.cos(y1)], -1)
    elif c == VE_BOX:
        x3 = np.exp(y3)
        r = np.exp(y1 + y3)
        xl = np.stack([r * np.cos(y2), r * np.sin(y2), x3], -1)
    elif c == EDGE_BOX:
        r = np.exp(y1)
        xl = np.stack([r * np.cos(y2), r * np.sin(y2), y3], -1)
    elif c == VTX_PATCH:
        px, py = _planar(mesh.patch[e], l1, l2, "S")
        nrm = np.sqrt(px ** 2 + py ** 2 + 1.0)
        rho = np.exp(y3)
        xl = np.stack([rho * px / nrm, rho * py / nrm, rho / nrm], -1)
    elif c == COLUMN:
        p = mesh.patch[e]
        rho_s = p[9]
        t = y3
        sx, sy = _planar(p, l1, l2, "S")
        nrm = np.sqrt(sx ** 2 + sy ** 2 + 1.0)
        tx, ty = _planar(p, l1, l2, "T")
        xl = np.stack([(1 - t) * rho_s * sx / nrm + t * tx,
                       (1 - t) * rho_s * sy / nrm + t * ty,
                       (1 - t) * rho_s / nrm + t * 1.0], -1)
    else:
        raise ValueError("unknown chart %d" % c)
    return mesh.origin[e] + xl @ mesh.frame[e].T


def face_lam(f, a, b):
    """Master-cube points on face f for face coordinates a, b (arrays)."""
    d, s = divmod(f, 2)
    t0, t1 = FACE_TANGENT[d]
    a = np.asarray(a, float)
    lam = np.zeros(a.shape + (3,))
    lam[..., d] = 1.0 if s else -1.0
    lam[..., t0] = a
    lam[..., t1] = b
    return lam


def find_orientation(mesh, e, f, e2, f2, tol=1e-7):
    """Orientation code mapping face coordinates of (e,f) to those of (e2,f2),
    or None if the faces do not coincide (tolerance relative to the face size)."""
    pa = np.array([-0.61, 0.23, 0.77, 1.0, -1.0])
    pb = np.array([-0.37, 0.81, -0.52, 1.0, -1.0])
    xa = chart_points(mesh, e, face_lam(f, pa, pb))
    size = np.linalg.norm(xa[3] - xa[4])
    best = None
    for o in range(8):
        qa, qb = orient_map(o, pa, pb)
        xb = chart_points(mesh, e2, face_lam(f2, qa, qb))
        err = np.abs(xa - xb).max()
        if best is None or err < best[1]:
            best = (o, err)
    if best[1] > tol * size:
        return None
    return best[0]


# --------------------------------------------------------------------------
# Uniform hexahedral mesh of a box (thesis Sec. 6.2, the unit-cube tests).
# --------------------------------------------------------------------------

def box_mesh(W, nel=(2, 2, 2), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), name="cube", neumann=()):
    """neumann: outer faces (d, s) of the box (x_d = lo_d for s = 0, hi_d for
    s = 1) that carry Neumann instead of Dirichlet conditions."""
    nx, ny, nz = nel
    E = nx * ny * nz
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    h = (hi - lo) / np.array(nel)
    box = np.zeros((E, 6))
    nbr = -np.ones((E, 6), np.int32)
    nbr_face = -np.ones((E, 6), np.int32)
    orient = np.zeros((E, 6), np.int32)
    bc = np.zeros((E, 6), np.int32)
    idx = lambda i, j, k: i + nx * (j + ny * k)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                e = idx(i, j, k)
                c = (i, j, k)
                for d in range(3):
                    box[e, 2 * d] = lo[d] + c[d] * h[d]
                    box[e, 2 * d + 1] = lo[d] + (c[d] + 1) * h[d]
                    for s in (0, 1):
                        cc = list(c)
                        cc[d] += 1 if s else -1
                        f = 2 * d + s
                        if 0 <= cc[d] < nel[d]:
                            nbr[e, f] = idx(*cc)
                            nbr_face[e, f] = 2 * d + (1 - s)
                        else:
                            bc[e, f] = NEUMANN if (d, s) in neumann else DIRICHLET
    return Mesh(W=W,
                region=np.full(E, REG, np.int32), kind=np.full(E, REAL, np.int32),
                chart=np.full(E, AFFINE, np.int32),
                frame=np.tile(np.eye(3), (E, 1, 1)), mframe=np.tile(np.eye(3), (E, 1, 1)),
                origin=np.zeros((E, 3)),
                box=box, patch=np.zeros((E, 12)),
                nbr=nbr, nbr_face=nbr_face, orient=orient, bc=bc,
                cdof=-np.ones(E, np.int32), cdir=np.zeros(E, np.int32),
                n_corner_dof=0, name=name, info=dict(nel=tuple(nel)))
