"""ctypes binding of libsem.so (the C ABI in include/sem.h).

Argument marshalling only: every step of the method runs in the library.
Device vectors are torch CUDA tensors of dtype float64 (HIP device memory);
host arrays are numpy float64 arrays.  Loading fails loudly when the HIP
library has not been built; there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsem.so")

SEM_OK = 0
STATUS = {0: "SEM_OK", -1: "SEM_EINVAL", -2: "SEM_ENOMEM", -3: "SEM_EHIP", -4: "SEM_ENOCONV",
          -5: "SEM_EBREAKDOWN", -6: "SEM_ENAN", -7: "SEM_ENODATA"}

_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)


class SemMesh(ctypes.Structure):
    _fields_ = [("W", ctypes.c_int32), ("nelem", ctypes.c_int32), ("n_corner_dof", ctypes.c_int32),
                ("region", _i32p), ("kind", _i32p), ("chart", _i32p),
                ("frame", _f64p), ("mframe", _f64p), ("origin", _f64p), ("box", _f64p), ("patch", _f64p),
                ("nbr", _i32p), ("nbr_face", _i32p), ("orient", _i32p), ("bc", _i32p),
                ("cdof", _i32p), ("cdir", _i32p)]


class SemPcgInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("outer", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("status", ctypes.c_int32)]


class SemError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


_lib = None

PRECISIONS = {"fp64": 0, "mixed": 1}


def _prec(name):
    if name not in PRECISIONS:
        raise ValueError("precision must be one of %s" % sorted(PRECISIONS))
    return PRECISIONS[name]

EXPORTS = {
    "sem_setup": (ctypes.c_int, [ctypes.POINTER(SemMesh), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "sem_destroy": (None, [ctypes.c_void_p]),
    "sem_last_error": (ctypes.c_char_p, []),
    "sem_ndof": (ctypes.c_int64, [ctypes.c_void_p]),
    "sem_num_real_elements": (ctypes.c_int64, [ctypes.c_void_p]),
    "sem_num_volume_points": (ctypes.c_int64, [ctypes.c_void_p]),
    "sem_num_dirichlet_points": (ctypes.c_int64, [ctypes.c_void_p]),
    "sem_volume_points": (ctypes.c_int, [ctypes.c_void_p, _f64p]),
    "sem_dirichlet_points": (ctypes.c_int, [ctypes.c_void_p, _f64p]),
    "sem_set_data": (ctypes.c_int, [ctypes.c_void_p, _f64p, _f64p, _f64p]),
    "sem_rhs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sem_residual": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                    ctypes.c_void_p]),
    "sem_residual_prec": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_void_p]),
    "sem_set_preconditioner": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "sem_precond": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sem_pcg_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                     ctypes.c_int, ctypes.POINTER(SemPcgInfo), ctypes.c_void_p]),
    "sem_pcg_solve_mixed": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                           ctypes.c_int, ctypes.POINTER(SemPcgInfo), ctypes.c_void_p]),
    "sem_set_source_legendre": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "sem_source_adjoint": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p]),
    "sem_set_source_fourier": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "sem_pcg_solve_batch": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int),
                                           ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.POINTER(SemPcgInfo), ctypes.c_void_p]),
    "sem_num_error_points": (ctypes.c_int64, [ctypes.c_void_p]),
    "sem_error_points": (ctypes.c_int, [ctypes.c_void_p, _f64p]),
    "sem_error": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, _f64p, _f64p, _f64p, ctypes.c_void_p]),
    "sem_num_neumann_points": (ctypes.c_int64, [ctypes.c_void_p]),
    "sem_neumann_points": (ctypes.c_int, [ctypes.c_void_p, _f64p, _f64p]),
    "sem_set_neumann_data": (ctypes.c_int, [ctypes.c_void_p, _f64p]),
    "sem_num_face_terms": (ctypes.c_int64, [ctypes.c_void_p]),
    "sem_face_weights": (ctypes.c_int, [ctypes.c_void_p, _f64p]),
    "sem_set_face_weights": (ctypes.c_int, [ctypes.c_void_p, _f64p]),
    "sem_set_coefficients": (ctypes.c_int, [ctypes.c_void_p, _f64p, _f64p, _f64p]),
    "sem_conforming_correction": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sem_set_degrees": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]),
    "sem_graded_ndof": (ctypes.c_int64, [ctypes.c_void_p]),
    "sem_project": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sem_error_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, _f64p,
                                         ctypes.c_void_p]),
    "sem_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _f64p,
                                    ctypes.c_void_p]),
    "sem_set_tile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "sem_work_counts": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "sem_kernel_times": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _f64p,
                                        ctypes.c_void_p]),
}


def lib():
    """The loaded library (raises if libsem.so is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsem.so not built: run paper_1110_2316_amd/build.py (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != SEM_OK:
        raise SemError(status, lib().sem_last_error().decode())


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(_f64p)


def _dev(t):
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(int(stream))


class Context:
    """Owns one sem_ctx; methods map one-to-one on the C ABI calls."""

    def __init__(self, mesh, stream=None):
        L = lib()
        arrs = mesh.as_arrays()
        self._keep = arrs
        m = SemMesh()
        m.W = mesh.W
        m.nelem = mesh.E
        m.n_corner_dof = mesh.n_corner_dof
        for k in ("region", "kind", "chart", "nbr", "nbr_face", "orient", "bc", "cdof", "cdir"):
            setattr(m, k, arrs[k].ctypes.data_as(_i32p))
        for k in ("frame", "mframe", "origin", "box", "patch"):
            setattr(m, k, arrs[k].ctypes.data_as(_f64p))
        h = ctypes.c_void_p()
        _check(L.sem_setup(ctypes.byref(m), _stream(stream), ctypes.byref(h)))
        self.h = h
        self.W = mesh.W
        self.E = mesh.E

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().sem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def ndof(self):
        return int(lib().sem_ndof(self.h))

    @property
    def n_real_elements(self):
        return int(lib().sem_num_real_elements(self.h))

    def volume_points(self):
        n = int(lib().sem_num_volume_points(self.h))
        x = np.zeros((n, 3))
        _check(lib().sem_volume_points(self.h, _ptr(x)))
        return x

    def dirichlet_points(self):
        n = int(lib().sem_num_dirichlet_points(self.h))
        x = np.zeros((n, 3))
        if n:
            _check(lib().sem_dirichlet_points(self.h, _ptr(x)))
        return x

    def error_points(self):
        n = int(lib().sem_num_error_points(self.h))
        x = np.zeros((n, 3))
        _check(lib().sem_error_points(self.h, _ptr(x)))
        return x

    def set_data(self, f, g=None, gradg=None):
        f = _f64(f)
        g = None if g is None else _f64(g)
        gradg = None if gradg is None else _f64(gradg)
        _check(lib().sem_set_data(self.h, _ptr(f), None if g is None else _ptr(g),
                                  None if gradg is None else _ptr(gradg)))

    def rhs(self, b, stream=None):
        _check(lib().sem_rhs(self.h, _dev(b), _stream(stream)))

    def residual(self, u, r, homogeneous=True, precision="fp64", stream=None):
        """r = X u (homogeneous) or X u - b; precision "fp64" or "mixed" (float contractions)."""
        if precision == "fp64":
            _check(lib().sem_residual(self.h, _dev(u), _dev(r), int(bool(homogeneous)), _stream(stream)))
        else:
            _check(lib().sem_residual_prec(self.h, _dev(u), _dev(r), int(bool(homogeneous)), _prec(precision),
                                           _stream(stream)))

    def set_preconditioner(self, kind, stream=None):
        """"separable" (thesis Sec. 5.2, default) or "block" (exact element blocks of X)."""
        kinds = {"separable": 0, "block": 1}
        if kind not in kinds:
            raise ValueError("preconditioner kind must be one of %s" % sorted(kinds))
        _check(lib().sem_set_preconditioner(self.h, kinds[kind], _stream(stream)))

    def precond(self, r, z, stream=None):
        _check(lib().sem_precond(self.h, _dev(r), _dev(z), _stream(stream)))

    def pcg_solve(self, b, u, rtol=1e-12, maxit=10000, stream=None, raise_on_fail=True, precision="fp64"):
        """PCG on X u = b; precision "mixed" = float operator with FP64 residual replacement."""
        info = SemPcgInfo()
        fn = lib().sem_pcg_solve if _prec(precision) == 0 else lib().sem_pcg_solve_mixed
        st = fn(self.h, _dev(b), _dev(u), float(rtol), int(maxit), ctypes.byref(info), _stream(stream))
        if raise_on_fail:
            _check(st)
        return dict(iterations=info.iterations, outer=info.outer, rel_residual=info.rel_residual,
                    status=info.status)

    def set_source_legendre(self, theta, stream=None):
        """Source f = sum theta[a + d (b + d c)] P_a(x1) P_b(x2) P_c(x3), g = 0; theta: device [d^3] float64."""
        deg = round(theta.numel() ** (1.0 / 3.0))
        if deg ** 3 != theta.numel():
            raise ValueError("theta must hold deg^3 coefficients")
        _check(lib().sem_set_source_legendre(self.h, deg, _dev(theta), _stream(stream)))

    def set_source_fourier(self, coef, stream=None):
        """Source f = sum_k a_k cos(pi kappa_k . x + phi_k), g = 0; coef: device [nmodes, 5] float64."""
        if coef.dim() != 2 or coef.shape[1] != 5:
            raise ValueError("coef must be [nmodes, 5]")
        _check(lib().sem_set_source_fourier(self.h, int(coef.shape[0]), _dev(coef), _stream(stream)))

    def source_adjoint(self, lam, grad, stream=None):
        """grad[k] = d (lam^T b(theta)) / d theta_k; grad: device [d^3] float64."""
        deg = round(grad.numel() ** (1.0 / 3.0))
        _check(lib().sem_source_adjoint(self.h, deg, _dev(lam), _dev(grad), _stream(stream)))

    def error(self, u, uex, graduex, stream=None):
        out = ctypes.c_double()
        uex = _f64(uex)
        graduex = _f64(graduex)
        _check(lib().sem_error(self.h, _dev(u), _ptr(uex), _ptr(graduex), ctypes.byref(out), _stream(stream)))
        return out.value

    def face_weights(self):
        """[face terms, 4, 3] norm weights (alpha, beta, gamma) per quantity."""
        w = np.zeros((int(lib().sem_num_face_terms(self.h)), 4, 3))
        _check(lib().sem_face_weights(self.h, _ptr(w)))
        return w

    def set_face_weights(self, w):
        w = _f64(w)
        if w.size != int(lib().sem_num_face_terms(self.h)) * 12:
            raise ValueError("set_face_weights: expected [face terms, 4, 3]")
        _check(lib().sem_set_face_weights(self.h, _ptr(w)))

    def neumann_points(self):
        """(points [P, 3], outward unit normals [P, 3]) of the Neumann faces."""
        n = int(lib().sem_num_neumann_points(self.h))
        x = np.zeros((n, 3))
        nu = np.zeros((n, 3))
        if n:
            _check(lib().sem_neumann_points(self.h, _ptr(x), _ptr(nu)))
        return x, nu

    def set_neumann_data(self, h):
        h = _f64(h)
        if h.size != int(lib().sem_num_neumann_points(self.h)):
            raise ValueError("set_neumann_data: one value per Neumann point")
        self._neu_keep = h
        _check(lib().sem_set_neumann_data(self.h, _ptr(h)))

    def set_coefficients(self, a=None, beta=None, c=None):
        """Operator coefficients at the volume points (numpy [P, 6], [P, 3],
        [P]; None: the Laplacian's)."""
        npts = int(lib().sem_num_volume_points(self.h))
        args = []
        for v, k in ((a, 6), (beta, 3), (c, 1)):
            if v is None:
                args.append(None)
                continue
            v = _f64(v)
            if v.size != npts * k:
                raise ValueError("set_coefficients: expected %d values, got %d" % (npts * k, v.size))
            args.append(v)
        self._coef_keep = args
        _check(lib().sem_set_coefficients(self.h, *[None if v is None else _ptr(v) for v in args]))

    def set_degrees(self, deg=None):
        """Per-element degrees [E, 3] (int, mesh element order; None: W everywhere)."""
        if deg is None:
            _check(lib().sem_set_degrees(self.h, None))
            return
        d = np.ascontiguousarray(deg, dtype=np.int32).reshape(-1)
        if d.size != 3 * self.E:
            raise ValueError("set_degrees: expected [E, 3] = [%d, 3]" % self.E)
        _check(lib().sem_set_degrees(self.h, d.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))

    @property
    def graded_ndof(self):
        return int(lib().sem_graded_ndof(self.h))

    def project(self, u, stream=None):
        """u <- Q u in place (device float64 [ndof]): the graded space's projection."""
        if u.numel() != self.ndof:
            raise ValueError("project: u must have ndof entries")
        _check(lib().sem_project(self.h, _dev(u), _stream(stream)))

    def conforming_correction(self, u, uc, stream=None):
        """uc = the conforming correction of u (device float64 [ndof] each)."""
        if u.numel() != self.ndof or uc.numel() != self.ndof:
            raise ValueError("conforming_correction: u and uc must have ndof entries")
        _check(lib().sem_conforming_correction(self.h, _dev(u), _dev(uc), _stream(stream)))

    def error_noalloc(self, u, uex, graduex, stream=None):
        """sem_error with the exact values as device tensors (float64, [P] and
        [P, 3]); the library allocates nothing for this call."""
        npts = int(lib().sem_num_error_points(self.h))
        if uex.numel() != npts or graduex.numel() != 3 * npts or u.numel() != self.ndof:
            raise ValueError("error_noalloc: expected u [%d], uex [%d], graduex [%d, 3]" % (self.ndof, npts, npts))
        out = ctypes.c_double()
        _check(lib().sem_error_noalloc(self.h, _dev(u), _dev(uex), _dev(graduex), ctypes.byref(out),
                                       _stream(stream)))
        return out.value


    def autotune(self, precision="fp64", reps=10, stream=None):
        """Select the fastest element-kernel tile; returns dict(tile, slabs, ms)."""
        t = (ctypes.c_int * 4)()
        ms = np.zeros(3)
        _check(lib().sem_autotune(self.h, _prec(precision), int(reps), t, _ptr(ms), _stream(stream)))
        return dict(tile=int(t[0]), slabs=[int(t[1]), int(t[2]), int(t[3])], ms=[float(v) for v in ms])

    def set_tile(self, tile, precision="fp64"):
        _check(lib().sem_set_tile(self.h, _prec(precision), int(tile)))

    def work_counts(self):
        c = (ctypes.c_int64 * 10)()
        _check(lib().sem_work_counts(self.h, c))
        keys = ("real_elements", "elements", "fields", "general_elements", "slots", "faces",
                "face_coef_doubles", "ndof", "block_bytes_fp64", "block_bytes_mixed")
        return dict(zip(keys, [int(v) for v in c]))

    def kernel_times(self, u, reps=20, precision="fp64", stream=None):
        """Mean ms per launch of [volume, face, gather, update], HIP events on the stream."""
        ms = np.zeros(4)
        _check(lib().sem_kernel_times(self.h, _dev(u), int(reps), _prec(precision), _ptr(ms), _stream(stream)))
        return ms


def setup_problem(mesh, problem, stream=None):
    """Context with the data of a manufactured problem loaded (f, g = u, grad g)."""
    ctx = Context(mesh, stream)
    xv = ctx.volume_points()
    xd = ctx.dirichlet_points()
    if hasattr(problem, "coefficients"):
        a, beta, c = problem.coefficients(xv)
        ctx.set_coefficients(a, beta, c)
    xn, nu = ctx.neumann_points()
    if len(xn):
        ctx.set_neumann_data(problem.neumann(xn, nu))
    ctx.set_data(problem.f(xv), problem.u(xd) if len(xd) else None,
                 problem.grad_u(xd) if len(xd) else None)
    return ctx


def pcg_solve_batch(ctxs, bs, us, rtol=1e-12, maxit=100000, check=8, stream=None, raise_on_fail=True,
                    precision="fp64"):
    """One batched solve over several contexts: bs[c], us[c] are device [R_c, ndof_c]
    float64 tensors (R_c right-hand sides of context c).  Returns one info dict per
    right-hand side, in context order."""
    n = len(ctxs)
    if not (len(bs) == len(us) == n):
        raise ValueError("one b and one u per context")
    for c, b, u in zip(ctxs, bs, us):
        if b.dim() != 2 or b.shape != u.shape or b.shape[1] != c.ndof:
            raise ValueError("b and u must be [R, ndof] of their context")
    R = [int(b.shape[0]) for b in bs]
    hs = (ctypes.c_void_p * n)(*[c.h.value for c in ctxs])
    rr = (ctypes.c_int * n)(*R)
    bp = (ctypes.c_void_p * n)(*[_dev(b).value for b in bs])
    up = (ctypes.c_void_p * n)(*[_dev(u).value for u in us])
    infos = (SemPcgInfo * sum(R))()
    st = lib().sem_pcg_solve_batch(n, hs, rr, bp, up, float(rtol), int(maxit), int(check), _prec(precision), infos,
                                   _stream(stream))
    if raise_on_fail:
        _check(st)
    return [dict(iterations=i.iterations, outer=i.outer, rel_residual=i.rel_residual, status=i.status) for i in infos]
