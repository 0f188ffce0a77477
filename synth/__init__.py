"""Seeded synthetic point clouds shaped like the FGA paper's workloads.

This module creates inputs only. It holds none of the registration method's
arithmetic (no forces, masses, normalisation or Kabsch steps), so the FP64
oracle and the HIP path can both be fed from it without sharing method code.

Every generator returns float64 NumPy arrays plus the ground-truth rigid
transform (R_gt, t_gt) with X ~= R_gt @ Y + t_gt, where X is the reference and
Y the template.

Workload recipes (the paper's datasets are not available; these stand in):
  * ``mixture_pair``   : Gaussian-mixture reference + rotated/noisy template
                         subset (bunny-scale runs of the runtime/robustness
                         experiments).
  * ``lidar_pair``     : two 64-beam ring scans of one seeded scene from two
                         sensor poses (KITTI/Ford-like odometry pairs).
  * ``mesh_pair``      : two independent large samples of a weighted triangle
                         mesh (the large-scan experiments).
  * ``precision_pair`` : the mixture scaled to [0,100]^3 (precision study).
  * ``batch_pairs``    : 256 mixture pairs with log-uniform sizes.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "random_rotation", "mixture", "mixture_pair", "lidar_pair", "mesh_pair",
    "precision_pair", "batch_pairs", "batch_pair", "config_seed",
    "BATCH_PAIRS", "uniform_grid_pair", "misaligned_pair", "landmark_picks", "lidar_sequence",
    "planar_pair",
]

BATCH_PAIRS = 256


def config_seed(k: int) -> int:
    """Seed of configuration ``k`` (0..6)."""
    return 14005 + k


def random_rotation(rng: np.random.Generator, max_deg: float) -> np.ndarray:
    """Rotation about an axis uniform on S^2 by an angle uniform in [0, max_deg]."""
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    ang = np.deg2rad(rng.uniform(0.0, max_deg))
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * (K @ K)


def mixture(rng: np.random.Generator, n_comp: int, per_comp: int,
            means=None, sigmas=None):
    """Gaussian mixture: means U[0,1]^3, per-axis sigma U[0.02, 0.1]."""
    if means is None:
        means = rng.uniform(0.0, 1.0, size=(n_comp, 3))
    if sigmas is None:
        sigmas = rng.uniform(0.02, 0.1, size=(n_comp, 3))
    pts = np.concatenate([means[c] + sigmas[c] * rng.normal(size=(per_comp, 3))
                          for c in range(n_comp)], axis=0)
    return pts, means, sigmas


def _pose_template(rng, ref_pts, max_deg, t_half, noise):
    """Y = R_y P + t_y + noise; returns Y and the GT mapping Y back onto P."""
    Ry = random_rotation(rng, max_deg)
    ty = rng.uniform(-t_half, t_half, size=3)
    Y = ref_pts @ Ry.T + ty
    if noise > 0:
        Y = Y + noise * rng.normal(size=Y.shape)
    return Y, Ry.T, -Ry.T @ ty


def mixture_pair(seed: int = config_seed(0), n_comp: int = 8, per_comp: int = 128,
                 m: int = 900, max_deg: float = 30.0, t_half: float = 0.1,
                 noise: float = 0.005, return_index: bool = False, min_deg: float = 0.0):
    """Reference: ``n_comp`` x ``per_comp`` mixture points. Template: an
    ``m``-point subset without replacement, rotated (angle U[min_deg,
    max_deg]), translated and noised. With ``return_index`` the subset's
    reference indices are returned too (template point i is a noisy copy of
    reference point index[i]: the true correspondences)."""
    rng = np.random.default_rng(seed)
    X, _, _ = mixture(rng, n_comp, per_comp)
    idx = rng.choice(X.shape[0], size=m, replace=False)
    if min_deg > 0.0:
        Ry = _rotation_between(rng, min_deg, max_deg)
        ty = rng.uniform(-t_half, t_half, size=3)
        Y = X[idx] @ Ry.T + ty + noise * rng.normal(size=(m, 3))
        R_gt, t_gt = Ry.T, -Ry.T @ ty
    else:
        Y, R_gt, t_gt = _pose_template(rng, X[idx], max_deg, t_half, noise)
    return (X, Y, R_gt, t_gt, idx) if return_index else (X, Y, R_gt, t_gt)


def _rotation_between(rng, min_deg, max_deg):
    """Rotation about a uniform axis by an angle uniform in [min_deg, max_deg]."""
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    ang = np.deg2rad(rng.uniform(min_deg, max_deg))
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * (K @ K)


def uniform_grid_pair(seed: int, n_side: int = 8, max_deg: float = 30.0,
                      t_half: float = 0.1):
    """Noise-free full overlap: X is a jittered grid, Y = R_y X + t_y exactly."""
    rng = np.random.default_rng(seed)
    g = (np.arange(n_side) + 0.5) / n_side
    X = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    X = X + rng.uniform(-0.2, 0.2, size=X.shape) / n_side
    Y, R_gt, t_gt = _pose_template(rng, X, max_deg, t_half, 0.0)
    return X, Y, R_gt, t_gt


def misaligned_pair(seed: int, per_comp: int = 236, max_deg: float = 135.0):
    """Full overlap under large misalignment (the robustness experiment's
    third case): a noise-free 8-component mixture (1,888 points) and the same
    points in shuffled order, rotated by Euler angles about x, y and z each
    uniform in [0, max_deg] and translated U[-0.1, 0.1]^3. Returns X, Y,
    R_gt, t_gt and the correspondences: Y[i] is the image of X[index[i]]."""
    rng = np.random.default_rng([14010, seed])
    X, _, _ = mixture(rng, 8, per_comp)
    idx = rng.permutation(X.shape[0])
    a = np.deg2rad(rng.uniform(0.0, max_deg, size=3))
    Rx = np.array([[1, 0, 0], [0, np.cos(a[0]), -np.sin(a[0])], [0, np.sin(a[0]), np.cos(a[0])]])
    Ry = np.array([[np.cos(a[1]), 0, np.sin(a[1])], [0, 1, 0], [-np.sin(a[1]), 0, np.cos(a[1])]])
    Rz = np.array([[np.cos(a[2]), -np.sin(a[2]), 0], [np.sin(a[2]), np.cos(a[2]), 0], [0, 0, 1]])
    Rt = Rz @ Ry @ Rx
    tt = rng.uniform(-0.1, 0.1, size=3)
    Y = X[idx] @ Rt.T + tt
    return X, Y, Rt.T, -Rt.T @ tt, idx


def landmark_picks(seed: int, k: int, m: int) -> np.ndarray:
    """k distinct template indices (of m) whose true correspondences serve as
    prior matches for misaligned pair `seed`."""
    return np.random.default_rng([7, seed]).choice(m, k, replace=False)


def planar_pair(seed: int = config_seed(6), per_comp: int = 32768, m: int = 196608,
                max_deg: float = 30.0, t_half: float = 0.1, noise: float = 0.005):
    """The mixture recipe in the plane (D = 2): the x, y coordinates of an
    8-component mixture (262,144 points by default) as reference; the
    template an m-point subset without replacement, rotated about z by an
    angle U[0, max_deg], translated U[-t_half, t_half]^2 and noised. Returns
    X, Y (n x 2, m x 2), R_gt (2 x 2), t_gt."""
    rng = np.random.default_rng(seed)
    X, _, _ = mixture(rng, 8, per_comp)
    X = X[:, :2]
    idx = rng.choice(X.shape[0], size=m, replace=False)
    a = np.deg2rad(rng.uniform(0.0, max_deg))
    Ry = np.array([[np.cos(a), -np.sin(a)], [np.sin(a), np.cos(a)]])
    ty = rng.uniform(-t_half, t_half, size=2)
    Y = X[idx] @ Ry.T + ty + noise * rng.normal(size=(m, 2))
    return X, Y, Ry.T, -Ry.T @ ty


def precision_pair(seed: int = config_seed(3), per_comp: int = 16384):
    """Mixture of 8 components scaled x100 into ~[0,100]^3; the template is an
    independent draw of the same mixture, rotated U[0,30] deg, translated
    U[-10,10]^3, noise sigma 0.5."""
    rng = np.random.default_rng(seed)
    X, means, sig = mixture(rng, 8, per_comp)
    P, _, _ = mixture(rng, 8, per_comp, means, sig)
    X = 100.0 * X
    Y, R_gt, t_gt = _pose_template(rng, 100.0 * P, 30.0, 10.0, 0.5)
    return X, Y, R_gt, t_gt


def batch_pair(p: int):
    """Pair ``p`` of the batched workload: N_p log-uniform in [2048, 65536],
    M_p = round(0.88 N_p); mixture reference, rotated/noisy subset template."""
    rng = np.random.default_rng([14009, p])
    n = int(round(np.exp(rng.uniform(np.log(2048), np.log(65536)))))
    m = int(round(0.88 * n))
    per = [n // 8 + (1 if c < n % 8 else 0) for c in range(8)]
    means = rng.uniform(0.0, 1.0, size=(8, 3))
    sig = rng.uniform(0.02, 0.1, size=(8, 3))
    X = np.concatenate([means[c] + sig[c] * rng.normal(size=(per[c], 3)) for c in range(8)])
    idx = rng.choice(n, size=m, replace=False)
    Y, R_gt, t_gt = _pose_template(rng, X[idx], 30.0, 0.1, 0.005)
    return X, Y, R_gt, t_gt


def batch_pairs(count: int = BATCH_PAIRS):
    return [batch_pair(p) for p in range(count)]


# ---------------------------------------------------------------- LiDAR scene
def _scene(rng):
    boxes = []
    for _ in range(12):
        rng_r = rng.uniform(5.0, 40.0)
        ang = rng.uniform(-np.pi, np.pi)
        c = np.array([rng_r * np.cos(ang), rng_r * np.sin(ang)])
        half = rng.uniform(0.5, 2.5, size=2)
        h = rng.uniform(1.0, 3.0)
        yaw = rng.uniform(-np.pi, np.pi)
        boxes.append((c, half, h, yaw))
    cyls = []
    for _ in range(8):
        rng_r = rng.uniform(5.0, 40.0)
        ang = rng.uniform(-np.pi, np.pi)
        cyls.append((np.array([rng_r * np.cos(ang), rng_r * np.sin(ang)]),
                     rng.uniform(0.2, 1.0), rng.uniform(2.0, 6.0)))
    return boxes, cyls


def _cast(origin, dirs, boxes, cyls, wall_r=80.0, wall_h=30.0):
    """Nearest hit distance of each ray with the scene (ground z=0, yawed
    boxes, vertical cylinders, enclosing cylindrical wall)."""
    n = dirs.shape[0]
    best = np.full(n, np.inf)
    ox, oy, oz = origin
    dx, dy, dz = dirs[:, 0], dirs[:, 1], dirs[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        tg = np.where(dz < 0, -oz / dz, np.inf)
    best = np.minimum(best, tg)
    # enclosing wall: origin inside the cylinder, so the positive root always exists
    a = dx * dx + dy * dy
    b = 2 * (ox * dx + oy * dy)
    c = ox * ox + oy * oy - wall_r * wall_r
    tw = (-b + np.sqrt(b * b - 4 * a * c)) / (2 * a)
    zw = oz + tw * dz
    best = np.minimum(best, np.where((zw >= 0) & (zw <= wall_h), tw, np.inf))
    for (cc, rad, h) in cyls:
        px, py = ox - cc[0], oy - cc[1]
        bb = 2 * (px * dx + py * dy)
        cq = px * px + py * py - rad * rad
        disc = bb * bb - 4 * a * cq
        with np.errstate(invalid="ignore"):
            t1 = (-bb - np.sqrt(disc)) / (2 * a)
        z1 = oz + t1 * dz
        ok = (disc >= 0) & (t1 > 1e-6) & (z1 >= 0) & (z1 <= h)
        best = np.minimum(best, np.where(ok, t1, np.inf))
    for (cc, half, h, yaw) in boxes:
        cs, sn = np.cos(-yaw), np.sin(-yaw)
        px, py = ox - cc[0], oy - cc[1]
        lx, ly = cs * px - sn * py, sn * px + cs * py
        ldx, ldy = cs * dx - sn * dy, sn * dx + cs * dy
        tmin = np.full(n, -np.inf)
        tmax = np.full(n, np.inf)
        for o, d, lo, hi in ((lx, ldx, -half[0], half[0]), (ly, ldy, -half[1], half[1]),
                             (np.full(n, oz), dz, 0.0, h)):
            with np.errstate(divide="ignore", invalid="ignore"):
                ta = (lo - o) / d
                tb = (hi - o) / d
            t_lo = np.where(d != 0, np.minimum(ta, tb), np.where((o >= lo) & (o <= hi), -np.inf, np.inf))
            t_hi = np.where(d != 0, np.maximum(ta, tb), np.where((o >= lo) & (o <= hi), np.inf, -np.inf))
            tmin = np.maximum(tmin, t_lo)
            tmax = np.minimum(tmax, t_hi)
        ok = (tmax >= tmin) & (tmin > 1e-6)
        best = np.minimum(best, np.where(ok, tmin, np.inf))
    return best


def _scan(rng, pose_R, pose_t, boxes, cyls, beams, azimuths, height, range_noise):
    elev = np.deg2rad(np.linspace(-24.8, 2.0, beams))
    az = np.linspace(-np.pi, np.pi, azimuths, endpoint=False)
    E, A = np.meshgrid(elev, az, indexing="ij")
    local = np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], -1).reshape(-1, 3)
    dirs = local @ pose_R.T
    origin = pose_t + np.array([0.0, 0.0, height])
    rng_hit = _cast(origin, dirs, boxes, cyls)
    assert np.all(np.isfinite(rng_hit)), "every ray must hit the enclosed scene"
    rng_hit = rng_hit + range_noise * rng.normal(size=rng_hit.shape)
    return local * rng_hit[:, None] + np.array([0.0, 0.0, height])  # sensor-base frame


def lidar_pair(seed: int = config_seed(1), beams: int = 64, azimuths: int = 1024,
               height: float = 1.73, range_noise: float = 0.02):
    """Two ring scans of one seeded scene. Scan 1 (reference) is taken at the
    world origin; scan 2 (template) from a pose offset by yaw U[-20,20] deg and
    xy translation U[-2,2] m. Points are in each scan's own base frame, so
    X ~= R_gt Y + t_gt with (R_gt, t_gt) the second pose."""
    rng = np.random.default_rng(seed)
    boxes, cyls = _scene(rng)
    yaw = np.deg2rad(rng.uniform(-20.0, 20.0))
    R2 = np.array([[np.cos(yaw), -np.sin(yaw), 0.0], [np.sin(yaw), np.cos(yaw), 0.0], [0, 0, 1.0]])
    t2 = np.array([rng.uniform(-2, 2), rng.uniform(-2, 2), 0.0])
    X = _scan(rng, np.eye(3), np.zeros(3), boxes, cyls, beams, azimuths, height, range_noise)
    Y = _scan(rng, R2, t2, boxes, cyls, beams, azimuths, height, range_noise)
    return X, Y, R2, t2


def lidar_sequence(frames: int = 32, seed: int = config_seed(5), step: float = 1.0,
                   beams: int = 64, azimuths: int = 1024, height: float = 1.73,
                   range_noise: float = 0.02):
    """A drive through one seeded scene (the LiDAR pair's scene recipe): the
    sensor advances ``step`` metres per frame along its heading, which turns by
    U[-3, 3] degrees per frame, and takes one ring scan per frame. Returns the
    scans (each in its own sensor-base frame) and the world poses (R_k, t_k)
    of every frame; frame k+1 registered to frame k has the ground truth
    R_k^T R_{k+1}, R_k^T (t_{k+1} - t_k)."""
    rng = np.random.default_rng(seed)
    boxes, cyls = _scene(rng)
    yaw = rng.uniform(-np.pi, np.pi)
    pos = np.zeros(3)
    scans, poses = [], []
    for k in range(frames):
        R = np.array([[np.cos(yaw), -np.sin(yaw), 0.0], [np.sin(yaw), np.cos(yaw), 0.0], [0, 0, 1.0]])
        scans.append(_scan(rng, R, pos.copy(), boxes, cyls, beams, azimuths, height, range_noise))
        poses.append((R, pos.copy()))
        yaw += np.deg2rad(rng.uniform(-3.0, 3.0))
        pos = pos + step * np.array([np.cos(yaw), np.sin(yaw), 0.0])
    return scans, poses


# ---------------------------------------------------------------- weighted mesh
def _torus_mesh(rng, nu=25, nv=40):
    u = np.linspace(0, 2 * np.pi, nu, endpoint=False)
    v = np.linspace(0, 2 * np.pi, nv, endpoint=False)
    U, V = np.meshgrid(u, v, indexing="ij")
    bump = np.zeros_like(U)
    for _ in range(6):
        a, fu, fv, pu, pv = rng.uniform(0.02, 0.08), rng.integers(1, 4), rng.integers(1, 4), \
            rng.uniform(0, 2 * np.pi), rng.uniform(0, 2 * np.pi)
        bump += a * np.sin(fu * U + pu) * np.cos(fv * V + pv)
    Rm, rm = 1.0, 0.35 + bump
    P = np.stack([(Rm + rm * np.cos(V)) * np.cos(U), (Rm + rm * np.cos(V)) * np.sin(U),
                  rm * np.sin(V) * 0.8], -1).reshape(-1, 3)
    P = P + rng.uniform(-0.01, 0.01, size=P.shape)
    P = (P - P.min(0)) / (P.max(0) - P.min(0)).max()
    tris = []
    for i in range(nu):
        for j in range(nv):
            a = i * nv + j
            b = ((i + 1) % nu) * nv + j
            c = ((i + 1) % nu) * nv + (j + 1) % nv
            d = i * nv + (j + 1) % nv
            tris.append((a, b, c))
            tris.append((a, c, d))
    return P, np.array(tris)


def _sample_mesh(rng, P, T, w, n):
    A, B, C = P[T[:, 0]], P[T[:, 1]], P[T[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(B - A, C - A), axis=1)
    p = w * area
    counts = rng.multinomial(n, p / p.sum())
    tri = np.repeat(np.arange(T.shape[0]), counts)
    r1, r2 = rng.uniform(size=n), rng.uniform(size=n)
    s = np.sqrt(r1)
    b0, b1, b2 = 1 - s, s * (1 - r2), s * r2
    return b0[:, None] * A[tri] + b1[:, None] * B[tri] + b2[:, None] * C[tri]


def mesh_pair(seed: int = config_seed(2), n: int = 1 << 20, m: int = 1 << 20):
    """Two independent draws from a bumpy 2,000-triangle torus mesh with
    per-triangle density weights 10^U[0,2]; template rotated U[0,45] deg and
    translated U[-0.2,0.2]^3."""
    rng = np.random.default_rng(seed)
    P, T = _torus_mesh(rng)
    w = 10.0 ** rng.uniform(0.0, 2.0, size=T.shape[0])
    X = _sample_mesh(rng, P, T, w, n)
    S = _sample_mesh(rng, P, T, w, m)
    Y, R_gt, t_gt = _pose_template(rng, S, 45.0, 0.2, 0.0)
    return X, Y, R_gt, t_gt
