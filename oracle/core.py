"""FP64 oracle of the FGA registration loop and its steps.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Each function cites the part of the paper it writes out:

  normalise / denormalise_t : Appendix A, Eqs. (A.1)-(A.3) and the derivation
                              of dnorm(t) that follows them.
  niv_masses                : Sec. "Normalized Intrinsic Volume Measure",
                              Eq. (Normalized_IntrinsicVol); SPM Eq. (FinalSPM)
                              with B = 1 when there are no landmarks.
  rbf_weights / masses      : Sec. "RBF Mass Interpolation", Eq. (RBF_function),
                              and the Hadamard product S = N o B of Eq. (FinalSPM)
                              when landmark correspondences are given.
  direct_forces             : Eq. (GAForce), in C (fga_oracle.c).
  BHTree / bh_forces        : Alg. 1 and the BHForce function of Alg. 2, in C.
  kabsch                    : Eq. (R_Kabsch) and Eq. (transEst).
  register / Stepper        : Alg. 2, with Eqs. (GAForceDissipative),
                              (TotalGAForce), (PreviousVelocity) and the
                              displacement d = dt * v.
  D = 2                     : every step takes n x 2 point sets as well: the
                              quadtree of Alg. 1's 2^D split, Eq. (GAForce) in
                              the plane, the 2 x 2 Kabsch step, and NIV with
                              the 2D lattice (rho^2 cells) and disc areas.
  BHTree.gpe / gpe          : the Plummer energy (diagnostic), direct and with
                              the BHForce traversal.

Readings of places where the paper is silent or garbled (kept identical in
the design notes):
  * Masses: reference weights sum to 1, template masses have mean 1.
  * Damping "fraction" (default): v' = (1 - eta) v + dt g, the friction that
    removes the fraction eta of the momentum per step. "literal": Eqs.
    (GAForceDissipative)-(PreviousVelocity) as printed, v' = v + dt (F - eta v)/m_Y.
  * Velocity "rigid" (default): after each Kabsch step the velocity state is
    the realised rigid displacement divided by dt. "particle": the
    unconstrained per-particle velocity v' is kept.
  * Stop rule: iterate until ||T_k - T_{k-1}||_F^2 < tol on a step smaller
    than the one before (the motion starts from rest, so the first steps are
    small too); tol <= 0 runs exactly max_iter steps. The paper's threshold
    1e-4 is read as a bound on the norm, i.e. tol = 1e-8 on its square.
  * dnorm(t): the centroid term that has to be added is (mean X - mean Y).
  * RBF masses (Eq. RBF_function is garbled: its weights carry a point index
    and the collocation targets are not stated): B interpolates a landmark
    weight beta at the landmark points and returns to the landmark-free value 1
    away from them, B(p) = 1 + sum_c lambda_c Phi(|p - a_c|) with
    Phi(s) = exp(-s^2 / sigma^2) and lambda solving the m x m collocation
    system sum_c' lambda_c' Phi(|a_c - a_c'|) = beta - 1 at every anchor a_c.
    The anchors of B(Y) are the template points of the correspondences, those
    of B(X) the reference points; sigma is taken in the normalised frame.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "build", "lib", "Params", "normalise", "denormalise_t", "niv_masses",
    "direct_forces", "BHTree", "kabsch", "Stepper", "register", "gpe",
    "angular_deviation_deg", "masses", "rbf_weights",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "fga_oracle.c")


def build(force: bool = True) -> str:
    """Compile the C part of the oracle (gcc, -O2, OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", _SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        d, l, v = ctypes.c_double, ctypes.c_long, ctypes.c_void_p
        L.oracle_direct_forces.argtypes = [v, l, v, l, v, v, d, d, v]
        L.oracle_direct_forces.restype = None
        L.oracle_gpe.argtypes = [v, l, v, l, v, v, d, d]
        L.oracle_gpe.restype = d
        L.oracle_bh_build.argtypes = [v, v, l]
        L.oracle_bh_build.restype = v
        L.oracle_bh_build_leaf.argtypes = [v, v, l, l]
        L.oracle_bh_build_leaf.restype = v
        L.oracle_bh_build_dims.argtypes = [v, v, l, l, ctypes.c_int]
        L.oracle_bh_build_dims.restype = v
        L.oracle_direct_forces_2d.argtypes = [v, l, v, l, v, v, d, d, v]
        L.oracle_direct_forces_2d.restype = None
        L.oracle_bh_gpe.argtypes = [v, v, l, v, d, d, d, v]
        L.oracle_bh_gpe.restype = d
        L.oracle_bh_free.argtypes = [v]
        L.oracle_bh_stats.argtypes = [v, v]
        L.oracle_bh_root.argtypes = [v, v]
        L.oracle_bh_leaves.argtypes = [v, v]
        L.oracle_bh_leaves.restype = l
        L.oracle_bh_quant.argtypes = [v, v]
        L.oracle_bh_forces.argtypes = [v, v, l, v, d, d, d, v, v]
        L.oracle_bh_forces.restype = None
        _lib = L
    return _lib


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


@dataclass
class Params:
    """Method parameters; defaults are the paper's settings (Sec. Experimental
    Results, "Baseline Methods and Parameter Settings")."""
    G: float = 66.7
    eps: float = 0.2
    eta: float = 0.2
    dt: float = 0.1
    theta: float = 0.0          # 0 = direct all-pairs sum
    a: float = -5.0
    b: float = 5.0
    rho: int = 16               # NIV lattice resolution
    depth: int = 20             # tree depth limit, also the d of the NIV ball radius
    max_iter: int = 200
    tol: float = 0.0            # <= 0: run exactly max_iter iterations
    damping: str = "fraction"   # or "literal"
    velocity: str = "rigid"     # or "particle"
    masses: str = "niv"         # or "uniform"
    rbf_sigma: float = 0.03     # RBF kernel width (normalised frame)
    rbf_weight: float = 100.0   # B at a landmark point (the landmark-free value is 1)
    extras: dict = field(default_factory=dict)


# --------------------------------------------------------------- Appendix A
def normalise(X, Y, a=-5.0, b=5.0):
    """Eqs. (A.1)-(A.3): subtract each cloud's mean, take the scalar minimum l
    and maximum r over all coordinates of both centred clouds, and map
    (p - mean - l) (b - a) / (r - l) + a. Returns (Xn, Yn, info)."""
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64)
    xbar = X.mean(axis=0)
    ybar = Y.mean(axis=0)
    Xc, Yc = X - xbar, Y - ybar
    l = min(Xc.min(), Yc.min())
    r = max(Xc.max(), Yc.max())
    Xn = (Xc - l) * (b - a) / (r - l) + a
    Yn = (Yc - l) * (b - a) / (r - l) + a
    return Xn, Yn, dict(xbar=xbar, ybar=ybar, l=l, r=r, a=a, b=b)


def denormalise_t(R, t_n, info):
    """Translation in the caller's coordinates for X ~= R Y + t, given
    Xn ~= R Yn + t_n in the normalised frame (dnorm(t) of Appendix A, with the
    centroid term taken as mean(X) - mean(Y)). Inverting (A.3) gives
    X = s (Xn - a) + mean(X) + l and Y = s (Yn - a) + mean(Y) + l with
    s = (r - l)/(b - a); substituting Xn = R Yn + t_n yields the expression
    below."""
    s = (info["r"] - info["l"]) / (info["b"] - info["a"])
    D = len(t_n)
    a1 = np.full(D, info["a"])
    l1 = np.full(D, info["l"])
    return info["xbar"] - R @ info["ybar"] + s * (R @ a1 + t_n - a1) + l1 - R @ l1


# ----------------------------------------------------------------- masses
def niv_masses(P, rho=16, a=-5.0, b=5.0, depth=20):
    """Eq. (Normalized_IntrinsicVol) with the reading below; returns the raw
    NIV value of every point (before the sum/mean normalisation).

    The cloud's own bounding box is split into rho cells per axis (a
    zero-extent axis counts as extent 1). Point p lies in cell
    min(floor(rho (p - lo) / ext), rho - 1) per axis. Each point carries a
    ball of radius (b - a) / (2 depth rho) (a disc in D = 2); the volume of
    the union of the balls in a cell of n_c points is taken as
    min(n_c V_ball, V_cell) (disjoint balls, capped at full cover). The NIV
    value is V_cell / V(union); the constant integral over the occupied
    lattice is dropped because the masses are normalised afterwards."""
    P = np.asarray(P, np.float64)
    D = P.shape[1]
    lo = P.min(axis=0)
    ext = P.max(axis=0) - lo
    ext = np.where(ext > 0, ext, 1.0)
    cell = np.minimum(np.floor(rho * (P - lo) / ext), rho - 1).astype(np.int64)
    flat = np.zeros(len(P), np.int64)
    for ax in range(D):
        flat = flat * rho + cell[:, ax]
    counts = np.bincount(flat, minlength=rho ** D)
    n_c = counts[flat].astype(np.float64)
    r_ball = (b - a) / (2.0 * depth * rho)
    v_ball = np.pi * r_ball ** 2 if D == 2 else 4.0 / 3.0 * np.pi * r_ball ** 3
    v_cell = float(np.prod(ext / rho))
    v_union = np.minimum(n_c * v_ball, v_cell)
    return v_cell / v_union


def rbf_weights(P, anchors, sigma, beta):
    """Eq. (RBF_function) for the points P (n x 3) and the landmark anchors
    (m x 3), with the reading in the module docstring: the m x m collocation
    system for lambda, then B at every point. No anchors: B = 1 (the
    equation's second case)."""
    P = np.asarray(P, np.float64)
    A = np.asarray(anchors, np.float64).reshape(-1, P.shape[1])
    if len(A) == 0:
        return np.ones(len(P))

    def phi(U, V):
        d2 = ((U[:, None, :] - V[None, :, :]) ** 2).sum(-1)
        return np.exp(-d2 / sigma ** 2)
    lam = np.linalg.solve(phi(A, A), np.full(len(A), beta - 1.0))
    return 1.0 + phi(P, A) @ lam


def masses(Xn, Yn, p: Params, landmarks=None):
    """SPM masses S = N o B (Eq. FinalSPM): N the NIV values (1 in ``uniform``
    mode), B the RBF weights of Eq. (RBF_function) for the landmark
    correspondences ``landmarks = (idx_X, idx_Y)`` (B = 1 without them).
    Reference weights normalised to sum 1, template masses to mean 1; without
    landmarks ``uniform`` gives exactly 1/N and 1 (the constant-NIV case)."""
    if p.masses == "uniform":
        nx, ny = np.ones(len(Xn)), np.ones(len(Yn))
    else:
        nx = niv_masses(Xn, p.rho, p.a, p.b, p.depth)
        ny = niv_masses(Yn, p.rho, p.a, p.b, p.depth)
    if landmarks is not None and len(landmarks[0]) > 0:
        ix, iy = (np.asarray(a, np.int64) for a in landmarks)
        nx = nx * rbf_weights(Xn, Xn[ix], p.rbf_sigma, p.rbf_weight)
        ny = ny * rbf_weights(Yn, Yn[iy], p.rbf_sigma, p.rbf_weight)
    elif p.masses == "uniform":
        return np.full(len(Xn), 1.0 / len(Xn)), np.ones(len(Yn))
    return nx / nx.sum(), ny / ny.mean()


# ----------------------------------------------------------------- forces
def direct_forces(Y, X, mX, mY=None, G=66.7, eps=0.2):
    """Eq. (GAForce) summed over all reference points (C loop); n x 3 or
    n x 2 point sets."""
    Y, X, mX = _c(Y), _c(X), _c(mX)
    mY = None if mY is None else _c(mY)
    F = np.empty_like(Y)
    f = lib().oracle_direct_forces_2d if Y.shape[1] == 2 else lib().oracle_direct_forces
    f(_p(Y), len(Y), _p(X), len(X), _p(mX), _p(mY), G, eps, _p(F))
    return F


def gpe(Y, X, mX, mY=None, G=66.7, eps=0.2):
    """Plummer potential energy (diagnostic; -grad is Eq. GAForce)."""
    Y, X, mX = _c(Y), _c(X), _c(mX)
    mY = None if mY is None else _c(mY)
    return lib().oracle_gpe(_p(Y), len(Y), _p(X), len(X), _p(mX), _p(mY), G, eps)


class BHTree:
    """Alg. 1 tree on (X, mX), uncompressed, built once (X is static).
    ``leaf`` > 1 stops the split at cells of at most that many points (the
    leaf-size variant; 1 is Alg. 1 itself)."""

    def __init__(self, X, mX, leaf=1):
        self.X = _c(X)
        self.mX = _c(mX)
        self.dims = self.X.shape[1]
        self.h = lib().oracle_bh_build_dims(_p(self.X), _p(self.mX), len(self.X), int(leaf),
                                            int(self.dims))
        if not self.h:
            raise ValueError("empty reference")

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.oracle_bh_free(self.h)
            self.h = None

    def stats(self):
        out = np.zeros(5, np.int64)
        lib().oracle_bh_stats(self.h, _p(out))
        return dict(nodes=int(out[0]), leaves=int(out[1]), internal=int(out[2]),
                    branching=int(out[3]), max_depth=int(out[4]))

    def root(self):
        out = np.zeros(4)
        lib().oracle_bh_root(self.h, _p(out))
        return out[0], out[1:]

    def leaves(self):
        ids = np.zeros(len(self.X), np.int64)
        n = lib().oracle_bh_leaves(self.h, _p(ids))
        return int(n), ids

    def quant(self):
        q = np.zeros((len(self.X), self.dims), np.uint32)
        lib().oracle_bh_quant(self.h, _p(q))
        return q

    def forces(self, Y, mY=None, G=66.7, eps=0.2, theta=0.5, count=False):
        Y = _c(Y)
        mY = None if mY is None else _c(mY)
        F = np.empty_like(Y)
        cnt = ctypes.c_long(0)
        lib().oracle_bh_forces(self.h, _p(Y), len(Y), _p(mY), G, eps, theta, _p(F),
                               ctypes.byref(cnt))
        return (F, int(cnt.value)) if count else F

    def gpe(self, Y, mY=None, G=66.7, eps=0.2, theta=0.5, count=False):
        """Plummer energy -G sum_i mY_i sum over the Alg. 2 traversal of
        M / sqrt(r^2 + eps^2) (diagnostic)."""
        Y = _c(Y)
        mY = None if mY is None else _c(mY)
        cnt = ctypes.c_long(0)
        e = lib().oracle_bh_gpe(self.h, _p(Y), len(Y), _p(mY), G, eps, theta, ctypes.byref(cnt))
        return (e, int(cnt.value)) if count else e


# ----------------------------------------------------------------- Kabsch
def kabsch(Y, YD):
    """Eq. (R_Kabsch) and Eq. (transEst): C = hat(YD)^T hat(Y) = U S V^T,
    R = U diag(1, 1, sgn det(U V^T)) V^T (sgn 0 taken as +1), t = mu_D - R mu.
    R maps the centred Y onto the centred YD."""
    mu = Y.mean(axis=0)
    muD = YD.mean(axis=0)
    C = (YD - muD).T @ (Y - mu)
    U, _, Vt = np.linalg.svd(C)
    d = np.sign(np.linalg.det(U @ Vt))
    if d == 0:
        d = 1.0
    R = U @ np.diag([1.0] * (C.shape[0] - 1) + [d]) @ Vt
    return R, muD - R @ mu


def angular_deviation_deg(R_gt, R):
    """Eq. (GroundTruthAngularDev) (the rotation angle of R_gt^T R; in 2D the
    trace is 2 cos phi)."""
    if R.shape[0] == 2:
        return float(np.degrees(abs(np.arctan2(R_gt[0, 0] * R[1, 0] - R_gt[1, 0] * R[0, 0],
                                               R_gt[0, 0] * R[0, 0] + R_gt[1, 0] * R[1, 0]))))
    c = np.clip(0.5 * (np.trace(R_gt.T @ R) - 1.0), -1.0, 1.0)
    return float(np.degrees(np.arccos(c)))


# ----------------------------------------------------------------- Alg. 2
class Stepper:
    """The loop body of Alg. 2 on normalised clouds, one iteration per call.

    State: current template Y (M x 3), per-particle velocity V, accumulated
    transform (R, t) with Y = R Yn + t."""

    def __init__(self, Xn, Yn, mX, mY, p: Params):
        self.p = p
        self.X = _c(Xn)
        self.Y = _c(Yn).copy()
        self.mX = _c(mX)
        self.mY = _c(mY)
        self.V = np.zeros_like(self.Y)
        D = self.Y.shape[1]
        self.R = np.eye(D)
        self.t = np.zeros(D)
        self.iters = 0
        self.last_dT2 = np.inf
        self.tree = BHTree(self.X, self.mX) if p.theta > 0 else None
        self.interactions = 0

    def accel(self):
        """g_i = F_i / m_Yi from Eq. (GAForce) (direct) or Alg. 2 BHForce."""
        p = self.p
        if self.tree is None:
            self.interactions += len(self.Y) * len(self.X)
            return direct_forces(self.Y, self.X, self.mX, None, p.G, p.eps)
        g, cnt = self.tree.forces(self.Y, None, p.G, p.eps, p.theta, count=True)
        self.interactions += cnt
        return g

    def step(self):
        p = self.p
        g = self.accel()
        if p.damping == "fraction":
            Vn = (1.0 - p.eta) * self.V + p.dt * g
        elif p.damping == "literal":
            F = self.mY[:, None] * g                      # Eq. (GAForce)
            f = F - p.eta * self.V                        # Eqs. (GAForceDissipative), (TotalGAForce)
            Vn = self.V + p.dt * f / self.mY[:, None]     # Eq. (PreviousVelocity)
        else:
            raise ValueError(p.damping)
        D = p.dt * Vn                                     # displacement
        Rs, ts = kabsch(self.Y, self.Y + D)
        Ynew = self.Y @ Rs.T + ts
        if p.velocity == "rigid":
            self.V = (Ynew - self.Y) / p.dt
        elif p.velocity == "particle":
            self.V = Vn
        else:
            raise ValueError(p.velocity)
        Rn = Rs @ self.R
        tn = ts + Rs @ self.t
        self.last_dT2 = float(np.sum((Rn - self.R) ** 2) + np.sum((tn - self.t) ** 2))
        self.R, self.t, self.Y = Rn, tn, Ynew
        self.iters += 1
        return self.last_dT2


def register(X, Y, p: Params = None, trace=False, landmarks=None):
    """Alg. 2 end to end: normalise, masses, (tree), iterate, de-normalise.
    ``landmarks = (idx_X, idx_Y)`` are prior correspondences X[idx_X[k]] <->
    Y[idx_Y[k]] for the RBF masses. Returns dict(R, t, R_n, t_n, iters,
    converged, info, ...) with X ~= R Y + t in the caller's coordinates."""
    p = p or Params()
    Xn, Yn, info = normalise(X, Y, p.a, p.b)
    mX, mY = masses(Xn, Yn, p, landmarks)
    st = Stepper(Xn, Yn, mX, mY, p)
    hist = []
    converged = False
    prev = np.inf
    while st.iters < p.max_iter:
        dT2 = st.step()
        if trace:
            hist.append((st.R.copy(), st.t.copy(), dT2))
        # stop rule of Alg. 2 (reading): the step has fallen below tol while
        # shrinking; the test is skipped while the motion is still speeding up
        # from rest, where the first steps are also small, and at the first
        # iteration, which has no earlier step to compare with
        if p.tol > 0 and st.iters >= 2 and dT2 < p.tol and dT2 < prev:
            converged = True
            break
        prev = dT2
    t = denormalise_t(st.R, st.t, info)
    return dict(R=st.R, t=t, R_n=st.R, t_n=st.t, iters=st.iters, converged=converged,
                info=info, mX=mX, mY=mY, Xn=Xn, Yn=Yn, history=hist,
                interactions=st.interactions)
