"""MI355X-native Fast Gravitational Approach (FGA) for rigid point set registration.

A thin ctypes binding over ``libfga.so`` (the C ABI declared in
``include/fga.h``). PyTorch supplies device memory and the current HIP
stream; every step of the method runs in the library's HIP kernels. The
functions here only marshal arguments and convert status codes into
exceptions. There is no CPU fallback: if the library or a GPU is missing the
calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

__all__ = [
    "FGAError", "Params", "Report", "lib", "default_params", "masses", "forces",
    "register", "register_batch", "register_2d", "register_sequence",
    "State", "Tree", "kabsch", "version", "energy", "forces_2d", "forces_direct_noalloc",
    "group_runs",
    "F32", "F64", "DAMP_FRACTION", "DAMP_LITERAL", "VEL_RIGID", "VEL_PARTICLE",
    "MASS_NIV", "MASS_UNIFORM", "PREC_FP32", "PREC_FP32_KAHAN", "PREC_FP64",
    "PREC_FP32_ALL",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfga.so")

F32, F64 = 0, 1
DAMP_FRACTION, DAMP_LITERAL = 0, 1
VEL_RIGID, VEL_PARTICLE = 0, 1
MASS_NIV, MASS_UNIFORM = 0, 1
PREC_FP32, PREC_FP32_KAHAN, PREC_FP64, PREC_FP32_ALL = 0, 1, 2, 3

STATUS = {0: "OK", 1: "INVALID_ARG", 2: "NOMEM", 3: "DEVICE", 4: "NONFINITE",
          5: "DEGENERATE", 6: "UNSUPPORTED"}


class FGAError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"fga status {STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class Params(ctypes.Structure):
    """Mirror of ``fga_params``."""
    _fields_ = [
        ("G", ctypes.c_double), ("eps", ctypes.c_double), ("eta", ctypes.c_double),
        ("dt", ctypes.c_double), ("theta", ctypes.c_double), ("a", ctypes.c_double),
        ("b", ctypes.c_double), ("rho", ctypes.c_int), ("max_depth", ctypes.c_int),
        ("max_iter", ctypes.c_int), ("tol", ctypes.c_double), ("damping", ctypes.c_int),
        ("velocity", ctypes.c_int), ("mass_mode", ctypes.c_int), ("precision", ctypes.c_int),
        ("leaf_size", ctypes.c_int), ("tile", ctypes.c_int), ("check_every", ctypes.c_int),
        ("group_width", ctypes.c_int), ("rbf_sigma", ctypes.c_double),
        ("rbf_weight", ctypes.c_double),
        ("reserved", ctypes.c_int * 4),
    ]

    def replace(self, **kw) -> "Params":
        q = Params()
        ctypes.pointer(q)[0] = self
        for k, v in kw.items():
            setattr(q, k, v)
        return q

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class _CReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("converged", ctypes.c_int),
                ("last_dT2", ctypes.c_double), ("interactions", ctypes.c_longlong),
                ("ms_total", ctypes.c_double), ("traversal", ctypes.c_int),
                ("leaf_size", ctypes.c_int)]


@dataclass
class Report:
    iters: int
    converged: bool
    last_dT2: float
    interactions: int
    ms_total: float
    traversal: int = 0
    leaf_size: int = 0

    @staticmethod
    def _from(c: _CReport) -> "Report":
        return Report(c.iters, bool(c.converged), c.last_dT2, c.interactions, c.ms_total, c.traversal,
                      c.leaf_size)


_lib = None


def lib():
    """Loads libfga.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime with the same soname; loading torch
        # first makes libfga bind to that one runtime, so device pointers and
        # streams from torch are valid inside the library
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise FGAError(3, f"{LIB_PATH} is missing; build it with paper_2009_14005_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, dt, st = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int
        P = ctypes.POINTER(Params)
        dp = ctypes.POINTER(ctypes.c_double)
        sig = {
            "fga_default_params": (st, [P]),
            "fga_trim_cache": (st, []),
            "fga_last_error": (ctypes.c_char_p, []),
            "fga_version": (ctypes.c_char_p, []),
            "fga_masses": (st, [vp, dt, i64, P, ctypes.c_int, vp, vp]),
            "fga_masses_landmarks": (st, [vp, dt, i64, ctypes.POINTER(i64), ctypes.c_int, P,
                                          ctypes.c_int, vp, vp]),
            "fga_state_create_landmarks": (st, [vp, i64, vp, i64, dt, ctypes.POINTER(i64),
                                                ctypes.POINTER(i64), ctypes.c_int, P, vp,
                                                ctypes.POINTER(vp)]),
            "fga_register_landmarks": (st, [vp, i64, vp, i64, dt, ctypes.POINTER(i64),
                                            ctypes.POINTER(i64), ctypes.c_int, P, dp, dp,
                                            ctypes.POINTER(_CReport), vp]),
            "fga_forces": (st, [vp, i64, vp, i64, vp, vp, dt, ctypes.c_double, P, vp,
                                ctypes.POINTER(ctypes.c_longlong), vp]),
            "fga_forces_direct_noalloc": (st, [vp, i64, vp, i64, vp, vp, dt, P, vp, vp]),
            "fga_state_create": (st, [vp, i64, vp, i64, dt, P, vp, ctypes.POINTER(vp)]),
            "fga_step": (st, [vp, ctypes.c_int]),
            "fga_step_profile": (st, [vp, ctypes.c_int, dp]),
            "fga_state_get": (st, [vp, dp, dp, ctypes.POINTER(_CReport)]),
            "fga_state_get_normalised": (st, [vp, dp, dp]),
            "fga_state_save": (st, [vp, vp, ctypes.POINTER(ctypes.c_size_t)]),
            "fga_state_load": (st, [vp, vp, ctypes.c_size_t]),
            "fga_state_destroy": (None, [vp]),
            "fga_register": (st, [vp, i64, vp, i64, dt, P, dp, dp, ctypes.POINTER(_CReport), vp]),
            "fga_register_batch": (st, [ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(i64),
                                        ctypes.POINTER(vp), ctypes.POINTER(i64), dt, P, dp, dp,
                                        ctypes.POINTER(_CReport), vp]),
            "fga_register_sequence": (st, [ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(i64), dt,
                                           P, dp, dp, dp, dp, ctypes.POINTER(_CReport), vp]),
            "fga_energy": (st, [vp, i64, vp, i64, vp, vp, dt, ctypes.c_double, P, dp,
                                ctypes.POINTER(ctypes.c_longlong), vp]),
            "fga_forces_2d": (st, [vp, i64, vp, i64, vp, vp, dt, ctypes.c_double, P, vp,
                                   ctypes.POINTER(ctypes.c_longlong), vp]),
            "fga_register_2d": (st, [vp, i64, vp, i64, dt, P, dp, dp, ctypes.POINTER(_CReport), vp]),
            "fga_tree_create": (st, [vp, vp, i64, dt, P, vp, ctypes.POINTER(vp)]),
            "fga_tree_info": (st, [vp, ctypes.POINTER(ctypes.c_int64)]),
            "fga_tree_export": (st, [vp, vp, vp, vp]),
            "fga_tree_destroy": (None, [vp]),
            "fga_kabsch": (st, [dp, dp]),
            "fga_group_runs": (st, [vp, i64, ctypes.c_int, ctypes.c_double, vp, i64,
                                    ctypes.POINTER(i64), vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise FGAError(status, lib().fga_last_error().decode())


def version() -> str:
    return lib().fga_version().decode()


def default_params(**kw) -> Params:
    p = Params()
    _check(lib().fga_default_params(ctypes.byref(p)))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


# ------------------------------------------------------------ marshalling
def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError(f"points must be float32 or float64, got {t.dtype}")


def _dev(t, name, cols=3):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device (cuda) tensor")
    if cols and (t.dim() != 2 or t.shape[1] != cols):
        raise ValueError(f"{name} must have shape (n, {cols})")
    return t.contiguous()


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _idx(a):
    """Host int64 index array for the C ABI (None for no landmarks)."""
    import numpy as np
    if a is None:
        return None, 0
    a = np.ascontiguousarray(a, dtype=np.int64)
    return (ctypes.c_int64 * len(a))(*a.tolist()), len(a)


def masses(pts, params: Params = None, norm: int = 0, landmarks=None):
    """Masses of one point set (sum 1 for norm=0, mean 1 for norm=1): NIV, or
    with ``landmarks`` (point indices) the SPM product with the RBF weights."""
    torch = _torch()
    pts = _dev(pts, "pts")
    p = params or default_params()
    out = torch.empty(pts.shape[0], dtype=pts.dtype, device=pts.device)
    if landmarks is None:
        _check(lib().fga_masses(_ptr(pts), _dtype_code(pts), pts.shape[0], ctypes.byref(p), norm,
                                _ptr(out), _stream()))
    else:
        idx, k = _idx(landmarks)
        _check(lib().fga_masses_landmarks(_ptr(pts), _dtype_code(pts), pts.shape[0], idx, k,
                                          ctypes.byref(p), norm, _ptr(out), _stream()))
    return out


def trim_cache():
    """Returns the library's idle cached device buffers to the device."""
    _check(lib().fga_trim_cache())


def forces(Y, X, mX, mY=None, theta: float = 0.0, params: Params = None):
    """Eq. (GAForce) on every template point; theta > 0 uses Barnes-Hut.
    Returns (F, interactions)."""
    torch = _torch()
    Y, X = _dev(Y, "Y"), _dev(X, "X")
    mX = _dev(mX, "mX", cols=0)
    mY = _dev(mY, "mY", cols=0) if mY is not None else None
    p = params or default_params()
    F = torch.empty_like(Y)
    cnt = ctypes.c_longlong(0)
    _check(lib().fga_forces(_ptr(Y), Y.shape[0], _ptr(X), X.shape[0], _ptr(mX), _ptr(mY),
                            _dtype_code(Y), float(theta), ctypes.byref(p), _ptr(F),
                            ctypes.byref(cnt), _stream()))
    return F, cnt.value


def forces_direct_noalloc(Y, X, mX, F, mY=None, params: Params = None):
    """The direct sum of Eq. (GAForce) into the caller's F (m x 3, Y's dtype),
    with the library's static device scratch: no allocation; queued on the
    current stream."""
    Y, X, F = _dev(Y, "Y"), _dev(X, "X"), _dev(F, "F")
    mX = _dev(mX, "mX", cols=0)
    mY = _dev(mY, "mY", cols=0) if mY is not None else None
    p = params or default_params()
    _check(lib().fga_forces_direct_noalloc(_ptr(Y), Y.shape[0], _ptr(X), X.shape[0], _ptr(mX),
                                           _ptr(mY), _dtype_code(Y), ctypes.byref(p), _ptr(F),
                                           _stream()))
    return F


def energy(Y, X, mX, mY=None, theta: float = 0.0, params: Params = None):
    """Plummer energy of the template in the reference's field (direct or
    Barnes-Hut). Returns (E, interactions)."""
    Y, X = _dev(Y, "Y"), _dev(X, "X")
    mX = _dev(mX, "mX", cols=0)
    mY = _dev(mY, "mY", cols=0) if mY is not None else None
    p = params or default_params()
    E = ctypes.c_double(0.0)
    cnt = ctypes.c_longlong(0)
    _check(lib().fga_energy(_ptr(Y), Y.shape[0], _ptr(X), X.shape[0], _ptr(mX), _ptr(mY),
                            _dtype_code(Y), float(theta), ctypes.byref(p), ctypes.byref(E),
                            ctypes.byref(cnt), _stream()))
    return E.value, cnt.value


def forces_2d(Y, X, mX, mY=None, theta: float = 0.0, params: Params = None):
    """Eq. (GAForce) for planar point sets (n x 2); quadtree when theta > 0.
    Returns (F m x 2, interactions)."""
    torch = _torch()
    Y, X = _dev(Y, "Y", cols=2), _dev(X, "X", cols=2)
    mX = _dev(mX, "mX", cols=0)
    mY = _dev(mY, "mY", cols=0) if mY is not None else None
    p = params or default_params()
    F = torch.empty_like(Y)
    cnt = ctypes.c_longlong(0)
    _check(lib().fga_forces_2d(_ptr(Y), Y.shape[0], _ptr(X), X.shape[0], _ptr(mX), _ptr(mY),
                               _dtype_code(Y), float(theta), ctypes.byref(p), _ptr(F),
                               ctypes.byref(cnt), _stream()))
    return F, cnt.value


def register_2d(X, Y, params: Params = None):
    """Alg. 2 for planar point sets (n x 2). Returns (R 2 x 2, t (2), Report)."""
    import numpy as np
    X, Y = _dev(X, "X", cols=2), _dev(Y, "Y", cols=2)
    if X.dtype != Y.dtype:
        raise TypeError("X and Y must have the same dtype")
    p = params or default_params()
    R = (ctypes.c_double * 4)()
    t = (ctypes.c_double * 2)()
    rep = _CReport()
    _check(lib().fga_register_2d(_ptr(X), X.shape[0], _ptr(Y), Y.shape[0], _dtype_code(X),
                                 ctypes.byref(p), R, t, ctypes.byref(rep), _stream()))
    return np.array(R[:]).reshape(2, 2), np.array(t[:]), Report._from(rep)


def _mat(a):
    import numpy as np
    return np.array(a[:9]).reshape(3, 3), np.array(a[9:12])


def register(X, Y, params: Params = None, landmarks=None):
    """Alg. 2 end to end. Returns (R, t, Report) with X ~= R Y + t.
    ``landmarks = (idx_X, idx_Y)``: prior correspondences X[idx_X[k]] <->
    Y[idx_Y[k]] for the RBF masses."""
    import numpy as np
    X, Y = _dev(X, "X"), _dev(Y, "Y")
    if X.dtype != Y.dtype:
        raise TypeError("X and Y must have the same dtype")
    p = params or default_params()
    R = (ctypes.c_double * 9)()
    t = (ctypes.c_double * 3)()
    rep = _CReport()
    if landmarks is None:
        _check(lib().fga_register(_ptr(X), X.shape[0], _ptr(Y), Y.shape[0], _dtype_code(X),
                                  ctypes.byref(p), R, t, ctypes.byref(rep), _stream()))
    else:
        ix, k = _idx(landmarks[0])
        iy, k2 = _idx(landmarks[1])
        if k != k2:
            raise ValueError("landmark index lists differ in length")
        _check(lib().fga_register_landmarks(_ptr(X), X.shape[0], _ptr(Y), Y.shape[0], _dtype_code(X),
                                            ix, iy, k, ctypes.byref(p), R, t, ctypes.byref(rep),
                                            _stream()))
    return np.array(R[:]).reshape(3, 3), np.array(t[:]), Report._from(rep)


def register_batch(Xs, Ys, params: Params = None):
    """Independent registrations run together. Returns (R[k,3,3], t[k,3], reports)."""
    import numpy as np
    if len(Xs) != len(Ys) or not Xs:
        raise ValueError("need equally many (>= 1) references and templates")
    Xs = [_dev(x, "X[k]") for x in Xs]
    Ys = [_dev(y, "Y[k]") for y in Ys]
    dt = _dtype_code(Xs[0])
    for a in Xs + Ys:
        if _dtype_code(a) != dt:
            raise TypeError("all clouds must share one dtype")
    k = len(Xs)
    p = params or default_params()
    xp = (ctypes.c_void_p * k)(*[x.data_ptr() for x in Xs])
    yp = (ctypes.c_void_p * k)(*[y.data_ptr() for y in Ys])
    n = (ctypes.c_int64 * k)(*[x.shape[0] for x in Xs])
    m = (ctypes.c_int64 * k)(*[y.shape[0] for y in Ys])
    R = (ctypes.c_double * (9 * k))()
    t = (ctypes.c_double * (3 * k))()
    reps = (_CReport * k)()
    _check(lib().fga_register_batch(k, xp, n, yp, m, dt, ctypes.byref(p), R, t, reps, _stream()))
    return (np.array(R[:]).reshape(k, 3, 3), np.array(t[:]).reshape(k, 3),
            [Report._from(r) for r in reps])


def register_sequence(frames, params: Params = None):
    """Frame-to-frame registration of a scan sequence: returns the relative
    transforms (R_rel[k], t_rel[k]) with frame_k ~= R_rel frame_{k+1} + t_rel,
    the composed poses (R_abs[k], t_abs[k]) of every frame in frame 0's
    coordinates, and the per-pair reports."""
    import numpy as np
    if len(frames) < 2:
        raise ValueError("need at least 2 frames")
    frames = [_dev(f, "frames[k]") for f in frames]
    dt = _dtype_code(frames[0])
    for f in frames:
        if _dtype_code(f) != dt:
            raise TypeError("all frames must share one dtype")
    k = len(frames)
    p = params or default_params()
    fp = (ctypes.c_void_p * k)(*[f.data_ptr() for f in frames])
    n = (ctypes.c_int64 * k)(*[f.shape[0] for f in frames])
    Rr = (ctypes.c_double * (9 * (k - 1)))()
    tr = (ctypes.c_double * (3 * (k - 1)))()
    Ra = (ctypes.c_double * (9 * k))()
    ta = (ctypes.c_double * (3 * k))()
    reps = (_CReport * (k - 1))()
    _check(lib().fga_register_sequence(k, fp, n, dt, ctypes.byref(p), Rr, tr, Ra, ta, reps, _stream()))
    return (np.array(Rr[:]).reshape(k - 1, 3, 3), np.array(tr[:]).reshape(k - 1, 3),
            np.array(Ra[:]).reshape(k, 3, 3), np.array(ta[:]).reshape(k, 3),
            [Report._from(r) for r in reps])


class State:
    """Registration state of Alg. 2 (normalised clouds, masses, tree, FP64
    rigid state) for step-wise driving, checkpoint and resume."""

    def __init__(self, X, Y, params: Params = None, landmarks=None):
        X, Y = _dev(X, "X"), _dev(Y, "Y")
        if X.dtype != Y.dtype:
            raise TypeError("X and Y must have the same dtype")
        self.params = params or default_params()
        self._h = ctypes.c_void_p()
        if landmarks is None:
            _check(lib().fga_state_create(_ptr(X), X.shape[0], _ptr(Y), Y.shape[0], _dtype_code(X),
                                          ctypes.byref(self.params), _stream(), ctypes.byref(self._h)))
        else:
            ix, k = _idx(landmarks[0])
            iy, k2 = _idx(landmarks[1])
            if k != k2:
                raise ValueError("landmark index lists differ in length")
            _check(lib().fga_state_create_landmarks(_ptr(X), X.shape[0], _ptr(Y), Y.shape[0],
                                                    _dtype_code(X), ix, iy, k, ctypes.byref(self.params),
                                                    _stream(), ctypes.byref(self._h)))

    def step(self, n_iters: int = 1):
        _check(lib().fga_step(self._h, int(n_iters)))

    def step_profile(self, n_iters: int):
        """Runs n_iters iterations; returns the summed milliseconds of the
        force launches and of the reduction launches (HIP events)."""
        ms = (ctypes.c_double * 2)()
        _check(lib().fga_step_profile(self._h, int(n_iters), ms))
        return ms[0], ms[1]

    def get(self):
        import numpy as np
        R = (ctypes.c_double * 9)()
        t = (ctypes.c_double * 3)()
        rep = _CReport()
        _check(lib().fga_state_get(self._h, R, t, ctypes.byref(rep)))
        return np.array(R[:]).reshape(3, 3), np.array(t[:]), Report._from(rep)

    def get_normalised(self):
        import numpy as np
        R = (ctypes.c_double * 9)()
        t = (ctypes.c_double * 3)()
        _check(lib().fga_state_get_normalised(self._h, R, t))
        return np.array(R[:]).reshape(3, 3), np.array(t[:])

    def save(self) -> bytes:
        n = ctypes.c_size_t(0)
        _check(lib().fga_state_save(self._h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(lib().fga_state_save(self._h, buf, ctypes.byref(n)))
        return buf.raw[: n.value]

    def load(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(lib().fga_state_load(self._h, buf, len(blob)))

    def close(self):
        if self._h:
            lib().fga_state_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tree:
    """Compressed Alg. 1 octree on a reference set (inspection)."""

    def __init__(self, X, mX, params: Params = None):
        X = _dev(X, "X")
        mX = _dev(mX, "mX", cols=0)
        p = params or default_params()
        self.n = X.shape[0]
        self._h = ctypes.c_void_p()
        _check(lib().fga_tree_create(_ptr(X), _ptr(mX), X.shape[0], _dtype_code(X),
                                     ctypes.byref(p), _stream(), ctypes.byref(self._h)))

    def info(self):
        a = (ctypes.c_int64 * 4)()
        _check(lib().fga_tree_info(self._h, a))
        return dict(nodes=a[0], leaves=a[1], internal=a[2], max_depth=a[3])

    def export(self):
        import numpy as np
        nn = self.info()["nodes"]
        cm = np.zeros((nn, 4), np.float32)
        ints = np.zeros((nn, 4), np.int32)
        order = np.zeros(self.n, np.int32)
        _check(lib().fga_tree_export(self._h, cm.ctypes.data_as(ctypes.c_void_p),
                                     ints.ctypes.data_as(ctypes.c_void_p),
                                     order.ctypes.data_as(ctypes.c_void_p)))
        return dict(com_mass=cm, skip=ints[:, 0], first=ints[:, 1], last=ints[:, 2],
                    depth=ints[:, 3], order=order)

    def close(self):
        if self._h:
            lib().fga_tree_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def group_runs(Y, G=64, f=0.0):
    """The group walk's runs of the FP32 points Y (m x 3, device), in their
    order: an (n_runs x 2) int32 array of (first, count)."""
    import numpy as np
    Y = _dev(Y, "Y")
    if Y.dtype != _torch().float32:
        raise TypeError("Y must be float32")
    m = Y.shape[0]
    out = np.zeros((m, 2), np.int32)  # at most one run per point
    n = ctypes.c_int64()
    _check(lib().fga_group_runs(_ptr(Y), m, int(G), float(f), out.ctypes.data_as(ctypes.c_void_p), m,
                                ctypes.byref(n), _stream()))
    return out[: n.value].copy()


def kabsch(C):
    """Host evaluation of the library's FP64 Kabsch solver (Eq. R_Kabsch)."""
    import numpy as np
    C = np.ascontiguousarray(C, dtype=np.float64).reshape(9)
    R = np.zeros(9)
    _check(lib().fga_kabsch(C.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            R.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return R.reshape(3, 3)
