"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these checks re-types the oracle's own formula: each uses a closed
form evaluated independently (extended precision), an invariant, a special
case with a known answer, a library routine, or an independent construction.
"""
import json
import os

import mpmath as mp
import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
G, EPS = 66.7, 0.2


def rot(rng, deg=180.0):
    return synth.random_rotation(rng, deg)


# ----------------------------------------------------------- Eq. (GAForce)
def test_two_particle_closed_form(oracle_lib):
    cases = json.load(open(os.path.join(GOLDEN, "two_particle_force.json")))["cases"]
    for c in cases:
        F = oracle.direct_forces(np.array([c["y"]]), np.array([c["x"]]), np.array([c["mX"]]),
                                 np.array([c["mY"]]), c["G"], c["eps"])[0]
        ref = np.array([float(v) for v in c["F"]])
        assert np.allclose(F, ref, rtol=1e-14, atol=1e-14), (F, ref)


def _mp_forces(Y, X, mX, mY, G, eps):
    mp.mp.dps = 50
    out = []
    for i in range(len(Y)):
        acc = [mp.mpf(0)] * 3
        for j in range(len(X)):
            d = [mp.mpf(float(Y[i, a])) - mp.mpf(float(X[j, a])) for a in range(3)]
            r2 = d[0] ** 2 + d[1] ** 2 + d[2] ** 2 + mp.mpf(eps) ** 2
            w = mp.mpf(float(mX[j])) * mp.mpf(float(mY[i])) / (r2 * mp.sqrt(r2))
            for a in range(3):
                acc[a] += w * d[a]
        out.append([float(-mp.mpf(G) * acc[a]) for a in range(3)])
    return np.array(out)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_brute_force_extended_precision(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    n, m = rng.integers(1, 9), rng.integers(1, 9)
    X = rng.uniform(-2, 2, size=(n, 3))
    Y = rng.uniform(-2, 2, size=(m, 3))
    mX = rng.uniform(0.1, 1.0, size=n)
    mY = rng.uniform(0.5, 2.0, size=m)
    F = oracle.direct_forces(Y, X, mX, mY, G, EPS)
    ref = _mp_forces(Y, X, mX, mY, G, EPS)
    assert np.allclose(F, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


def test_pair_antisymmetry(oracle_lib):
    """Force on a from b equals minus force on b from a (swapped masses)."""
    rng = np.random.default_rng(5)
    a, b = rng.normal(size=(1, 3)), rng.normal(size=(1, 3))
    ma, mb = np.array([0.7]), np.array([1.3])
    Fab = oracle.direct_forces(a, b, mb, ma, G, EPS)
    Fba = oracle.direct_forces(b, a, ma, mb, G, EPS)
    assert np.allclose(Fab, -Fba, rtol=1e-14)
    # attraction: the force on a points from a towards b
    assert np.dot(Fab[0], (b - a)[0]) > 0


def test_rigid_equivariance(oracle_lib):
    rng = np.random.default_rng(7)
    X = rng.normal(size=(50, 3))
    Y = rng.normal(size=(40, 3))
    mX = rng.uniform(0.1, 1, size=50)
    Q = rot(rng)
    c = rng.normal(size=3) * 3
    F = oracle.direct_forces(Y, X, mX, None, G, EPS)
    F2 = oracle.direct_forces(Y @ Q.T + c, X @ Q.T + c, mX, None, G, EPS)
    assert np.allclose(F2, F @ Q.T, rtol=1e-12, atol=1e-12 * np.abs(F).max())


def test_superposition(oracle_lib):
    rng = np.random.default_rng(8)
    X1, X2 = rng.normal(size=(30, 3)), rng.normal(size=(20, 3)) + 1
    m1, m2 = rng.uniform(0.1, 1, 30), rng.uniform(0.1, 1, 20)
    Y = rng.normal(size=(25, 3))
    F = oracle.direct_forces(Y, np.vstack([X1, X2]), np.concatenate([m1, m2]), None, G, EPS)
    F1 = oracle.direct_forces(Y, X1, m1, None, G, EPS)
    F2 = oracle.direct_forces(Y, X2, m2, None, G, EPS)
    assert np.allclose(F, F1 + F2, rtol=1e-12, atol=1e-13)


def test_force_is_minus_gradient_of_plummer_energy(oracle_lib):
    """Eq. (GAForce) is -grad of E = -G sum mY mX / sqrt(r^2 + eps^2); central
    differences in extended precision of the energy agree with the force."""
    rng = np.random.default_rng(9)
    X = rng.normal(size=(6, 3))
    mX = rng.uniform(0.2, 1, 6)
    y = rng.normal(size=3)
    mp.mp.dps = 40
    h = mp.mpf("1e-12")

    def E(p):
        s = mp.mpf(0)
        for j in range(6):
            r2 = sum((p[a] - mp.mpf(float(X[j, a]))) ** 2 for a in range(3)) + mp.mpf(EPS) ** 2
            s += mp.mpf(float(mX[j])) / mp.sqrt(r2)
        return -mp.mpf(G) * s

    p0 = [mp.mpf(float(v)) for v in y]
    grad = []
    for a in range(3):
        pp, pm = list(p0), list(p0)
        pp[a] += h
        pm[a] -= h
        grad.append(float((E(pp) - E(pm)) / (2 * h)))
    F = oracle.direct_forces(y[None], X, mX, None, G, EPS)[0]
    assert np.allclose(F, -np.array(grad), rtol=1e-10)
    # and the oracle's own energy matches the mpmath energy
    assert np.isclose(oracle.gpe(y[None], X, mX, None, G, EPS), float(E(p0)), rtol=1e-13)


# ------------------------------------------------------- Alg. 1 / Alg. 2 BH
def test_bh_theta_zero_is_direct(oracle_lib):
    X, Y, _, _ = synth.mixture_pair(11, per_comp=64, m=300)
    mX = np.random.default_rng(1).uniform(0.5, 1.5, len(X))
    mX /= mX.sum()
    t = oracle.BHTree(X, mX)
    Fd = oracle.direct_forces(Y, X, mX, None, G, EPS)
    Fb, cnt = t.forces(Y, None, G, EPS, theta=0.0, count=True)
    assert cnt == len(X) * len(Y)
    assert np.allclose(Fb, Fd, rtol=1e-12, atol=1e-12 * np.abs(Fd).max())


def test_bh_huge_theta_is_single_body(oracle_lib):
    rng = np.random.default_rng(12)
    X = rng.normal(size=(200, 3))
    mX = rng.uniform(0.1, 1, 200)
    Y = rng.normal(size=(50, 3)) * 3
    t = oracle.BHTree(X, mX)
    F, cnt = t.forces(Y, None, G, EPS, theta=1e12, count=True)
    M = mX.sum()
    com = (mX[:, None] * X).sum(0) / M
    d = Y - com
    r2 = (d ** 2).sum(1) + EPS ** 2
    ref = -G * M * d / (r2 * np.sqrt(r2))[:, None]
    assert cnt == len(Y)
    assert np.allclose(F, ref, rtol=1e-12)


def test_bh_mac_uses_box_diagonal_and_strict_less(oracle_lib):
    """Two unit masses at (0,0,0) and (a,b,c); query on the far side at
    distance r from their CoM. The root box diagonal is l = |(a,b,c)|. With
    theta just above l/r the root is accepted (force of mass 2 at the CoM),
    just below it the root is opened (exact pair sum)."""
    p = np.array([[0.0, 0.0, 0.0], [0.3, 0.2, 0.1]])
    m = np.array([1.0, 1.0])
    com = p.mean(0)
    l = np.linalg.norm(p[1] - p[0])
    y = com + np.array([0.0, 0.0, 4.0])
    r = 4.0
    t = oracle.BHTree(p, m)
    F_hi = t.forces(y[None], None, G, EPS, theta=l / r * (1 + 1e-9))[0]
    F_lo = t.forces(y[None], None, G, EPS, theta=l / r * (1 - 1e-9))[0]
    d = y - com
    r2 = d @ d + EPS ** 2
    acc_node = -G * 2 * d / r2 ** 1.5
    exact = oracle.direct_forces(y[None], p, m, None, G, EPS)[0]
    assert np.allclose(F_hi, acc_node, rtol=1e-14)
    assert np.allclose(F_lo, exact, rtol=1e-14)
    assert not np.allclose(acc_node, exact, rtol=1e-8)


def test_bh_root_mass_and_com(oracle_lib):
    rng = np.random.default_rng(13)
    X = rng.normal(size=(500, 3))
    mX = rng.uniform(0.1, 1, 500)
    t = oracle.BHTree(X, mX)
    M, com = t.root()
    assert np.isclose(M, mX.sum(), rtol=1e-14)
    assert np.allclose(com, (mX[:, None] * X).sum(0) / mX.sum(), rtol=1e-13)


def _independent_leaves(X):
    """Leaf sets from prefixes of the quantised coordinates, built without
    recursion: a point's leaf is the shortest octal prefix it shares with no
    other point, or its full 20-digit code when duplicates exist."""
    lo, hi = X.min(0), X.max(0)
    ext = hi - lo
    q = np.zeros(X.shape, dtype=np.int64)
    for a in range(3):
        if ext[a] > 0:
            q[:, a] = np.minimum(np.floor((X[:, a] - lo[a]) / ext[a] * 2.0 ** 20), 2 ** 20 - 1)
    digits = []
    for k in range(20):
        b = 19 - k
        digits.append(((q[:, 0] >> b) & 1) * 4 + ((q[:, 1] >> b) & 1) * 2 + ((q[:, 2] >> b) & 1))
    digits = np.stack(digits, 1)
    keys = [tuple(r) for r in digits]
    leaves = {}
    for j, key in enumerate(keys):
        for k in range(0, 21):
            pre = key[:k]
            others = [i for i in range(len(keys)) if i != j and keys[i][:k] == pre]
            if not others or k == 20:
                leaves.setdefault(pre, []).append(j)
                break
    return sorted(tuple(sorted(v)) for v in leaves.values()), q


def test_bh_leaves_match_independent_prefix_grouping(oracle_lib):
    rng = np.random.default_rng(14)
    X = np.vstack([rng.normal(size=(120, 3)), rng.normal(size=(5, 3)) * 1e-7])
    X = np.vstack([X, X[:3]])  # exact duplicates end in depth-20 leaves
    t = oracle.BHTree(X, np.ones(len(X)))
    n, ids = t.leaves()
    got = sorted(tuple(sorted(np.flatnonzero(ids == k))) for k in range(n))
    ref, q = _independent_leaves(X)
    assert got == ref
    assert np.array_equal(t.quant(), q.astype(np.uint32))
    assert t.stats()["max_depth"] == 20


def test_bh_error_shrinks_with_theta(oracle_lib):
    X, Y, _, _ = synth.mixture_pair(15, per_comp=256, m=400)
    mX = np.full(len(X), 1.0 / len(X))
    t = oracle.BHTree(X, mX)
    Fd = oracle.direct_forces(Y, X, mX, None, G, EPS)
    errs, cnts = [], []
    for th in (0.8, 0.5, 0.3):
        F, c = t.forces(Y, None, G, EPS, th, count=True)
        errs.append(np.median(np.linalg.norm(F - Fd, axis=1) / np.linalg.norm(Fd, axis=1)))
        cnts.append(c)
    assert errs[0] > errs[1] > errs[2] and errs[1] < 1e-2
    assert cnts[0] < cnts[1] < cnts[2] < len(X) * len(Y)


# --------------------------------------------------------- Eq. (R_Kabsch)
def test_kabsch_recovers_known_transform():
    rng = np.random.default_rng(16)
    for _ in range(20):
        Y = rng.normal(size=(30, 3))
        R0, t0 = rot(rng), rng.normal(size=3)
        R, t = oracle.kabsch(Y, Y @ R0.T + t0)
        assert np.allclose(R, R0, atol=1e-12) and np.allclose(t, t0, atol=1e-12)


def test_kabsch_reflection_gives_proper_rotation():
    rng = np.random.default_rng(17)
    Y = rng.normal(size=(40, 3))
    YD = Y * np.array([1.0, 1.0, -1.0])  # mirror image: best orthogonal map is a reflection
    R, _ = oracle.kabsch(Y, YD)
    assert np.isclose(np.linalg.det(R), 1.0)
    assert np.allclose(R @ R.T, np.eye(3), atol=1e-12)


def test_kabsch_planar_template():
    rng = np.random.default_rng(18)
    Y = np.c_[rng.normal(size=(25, 2)), np.zeros(25)]
    R0 = rot(rng)
    R, t = oracle.kabsch(Y, Y @ R0.T)
    assert np.allclose(R, R0, atol=1e-10)


# ------------------------------------------------------------- Appendix A
def test_normalisation_range_and_ground_truth_round_trip():
    rng = np.random.default_rng(19)
    X = rng.normal(size=(200, 3)) * [3.0, 1.0, 0.5] + [10, -4, 2]
    R0, t0 = rot(rng, 40), rng.normal(size=3) * 5
    Y = (X - t0) @ R0  # X = R0 Y + t0 exactly
    Xn, Yn, info = oracle.normalise(X, Y)
    both = np.concatenate([Xn.ravel(), Yn.ravel()])
    assert np.isclose(both.min(), -5.0) and np.isclose(both.max(), 5.0)
    # in the normalised frame the same rotation holds: Xn = R0 Yn + t_n
    t_n = Xn.mean(0) - R0 @ Yn.mean(0)
    assert np.allclose(Xn, Yn @ R0.T + t_n, atol=1e-12)
    assert np.allclose(oracle.denormalise_t(R0, t_n, info), t0, atol=1e-12)


def test_denormalisation_sign_matters():
    """The centroid term must be mean(X) - mean(Y); the opposite sign printed
    in the appendix misses the translation by twice the centroid gap."""
    rng = np.random.default_rng(20)
    X = rng.normal(size=(100, 3)) + [20, 0, 0]
    Y = X - [3, 1, 2]
    Xn, Yn, info = oracle.normalise(X, Y)
    t_n = Xn.mean(0) - Yn.mean(0)
    t = oracle.denormalise_t(np.eye(3), t_n, info)
    assert np.allclose(t, [3, 1, 2], atol=1e-12)


# ------------------------------------------------------- Eq. (NIV)
def test_niv_one_point_per_cell_is_uniform():
    rho = 4
    g = (np.arange(rho) + 0.5) / rho
    P = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    w = oracle.niv_masses(P, rho=rho)
    assert np.allclose(w, w[0])


def test_niv_two_cells_inverse_count_ratio():
    rng = np.random.default_rng(21)
    n1, n2 = 3, 7
    A = rng.uniform(0.0, 0.4, size=(n1, 3))
    B = rng.uniform(0.6, 1.0, size=(n2, 3))
    P = np.vstack([A, B, [[0, 0, 0], [1, 1, 1]]])  # pins the box to [0,1]^3
    w = oracle.niv_masses(P, rho=2)
    # cell (0,0,0) holds A + the corner (n1 + 1), cell (1,1,1) holds B + corner
    assert np.isclose(w[0] / w[n1], (n2 + 1) / (n1 + 1))
    # each occupied cell carries equal total weight
    assert np.isclose(w[: n1].sum() + w[-2], w[n1: n1 + n2].sum() + w[-1])


def test_niv_invariances():
    rng = np.random.default_rng(22)
    P = rng.normal(size=(300, 3))
    w = oracle.niv_masses(P)
    perm = rng.permutation(300)
    assert np.allclose(oracle.niv_masses(P[perm]), w[perm])
    w2 = oracle.niv_masses(P * 2.0 + 7.0)  # power-of-two scale keeps cells exact
    assert np.allclose(w2 / w2.sum(), w / w.sum())


def test_niv_cap_binds_at_full_cover():
    """A cell whose balls would exceed its volume is treated as fully covered."""
    P = np.vstack([np.zeros((5, 3)), np.ones((1, 3))])
    w = oracle.niv_masses(P, rho=1, a=-5, b=5, depth=20)
    r = 10.0 / (2 * 20 * 1)
    vb = 4 / 3 * np.pi * r ** 3
    assert np.isclose(w[0], 1.0 / (6 * vb)) if 6 * vb < 1 else np.isclose(w[0], 1.0)


# --------------------------------------------------------------- Alg. 2
def test_fixed_point_identical_clouds(oracle_lib):
    """With equal reference masses and Y = X the net force and torque vanish
    by pair antisymmetry, and sum_i g_i y_i^T is symmetric, so the Kabsch step
    is the identity at every iteration. (Unequal masses break the symmetry.)"""
    X, _, _, _ = synth.mixture_pair(23, per_comp=32, m=10)
    res = oracle.register(X, X.copy(), oracle.Params(max_iter=200, masses="uniform"))
    assert np.allclose(res["R"], np.eye(3), atol=1e-12)
    assert np.allclose(res["t"], 0, atol=1e-11)


@pytest.mark.parametrize("theta", [0.0, 0.5])
def test_exact_recovery_full_overlap(oracle_lib, theta):
    """Noise-free, fully overlapping data with uniform masses converges to the
    ground-truth transform."""
    X, Y, R_gt, t_gt = synth.uniform_grid_pair(24, n_side=7, max_deg=30.0)
    res = oracle.register(X, Y, oracle.Params(max_iter=400, masses="uniform", theta=theta))
    phi = oracle.angular_deviation_deg(R_gt, res["R"])
    assert phi < 1e-3, phi
    assert np.linalg.norm(res["t"] - t_gt) < 1e-4


def test_literal_damping_reduces_to_fraction(oracle_lib):
    """With m_Y = 1, literal damping eta_l equals fractional damping eta_l*dt."""
    X, Y, _, _ = synth.mixture_pair(25, per_comp=32, m=200)
    Xn, Yn, _ = oracle.normalise(X, Y)
    mX = np.full(len(Xn), 1 / len(Xn))
    mY = np.ones(len(Yn))
    pa = oracle.Params(damping="literal", eta=2.0)
    pb = oracle.Params(damping="fraction", eta=0.2)
    a, b = oracle.Stepper(Xn, Yn, mX, mY, pa), oracle.Stepper(Xn, Yn, mX, mY, pb)
    for _ in range(10):
        a.step()
        b.step()
    assert np.allclose(a.R, b.R, atol=1e-13) and np.allclose(a.t, b.t, atol=1e-13)


def test_stationary_at_convergence(oracle_lib):
    X, Y, _, _ = synth.uniform_grid_pair(26, n_side=6)
    Xn, Yn, _ = oracle.normalise(X, Y)
    st = oracle.Stepper(Xn, Yn, np.full(len(Xn), 1 / len(Xn)), np.ones(len(Yn)),
                        oracle.Params())
    for _ in range(300):
        dT2 = st.step()
    assert dT2 < 1e-20
    g = oracle.direct_forces(st.Y, st.X, st.mX, None, 66.7, 0.2)
    # net force and torque of the field on the registered template vanish
    assert np.linalg.norm(g.sum(0)) < 1e-6 * np.abs(g).sum()
    tau = np.cross(st.Y - st.Y.mean(0), g).sum(0)
    assert np.linalg.norm(tau) < 1e-6 * np.abs(g).sum()


def test_config0_registration_is_close(oracle_lib):
    X, Y, R_gt, t_gt = synth.mixture_pair()
    res = oracle.register(X, Y, oracle.Params(max_iter=200))
    assert oracle.angular_deviation_deg(R_gt, res["R"]) < 2.0


# ------------------------------------------ the pins catch planted mistakes
def test_planted_mistakes_are_caught(oracle_lib, monkeypatch):
    rng = np.random.default_rng(27)
    Y = rng.normal(size=(30, 3))
    R0 = rot(rng)
    good = oracle.kabsch
    monkeypatch.setattr(oracle.core, "kabsch", lambda a, b: (good(a, b)[0].T, good(a, b)[1]))
    R, _ = oracle.core.kabsch(Y, Y @ R0.T)
    assert not np.allclose(R, R0, atol=1e-6)  # transposed rotation fails the recovery pin
    monkeypatch.undo()
    # a dropped softening term fails the closed form
    c = json.load(open(os.path.join(GOLDEN, "two_particle_force.json")))["cases"][0]
    F_noeps = oracle.direct_forces(np.array([c["y"]]), np.array([c["x"]]), np.array([1.0]),
                                   np.array([1.0]), 66.7, 0.0)[0]
    assert not np.isclose(F_noeps[0], float(c["F"][0]), rtol=1e-6)


def test_stop_rule_waits_for_shrinking_steps(oracle_lib):
    """Alg. 2's stop rule with the motion starting from rest: the first steps
    are below the threshold too, so the test only fires on a shrinking step."""
    X, Y, _, _ = synth.mixture_pair()
    res = oracle.register(X, Y, oracle.Params(max_iter=300, tol=1e-8), trace=True)
    h = [x[2] for x in res["history"]]
    assert res["converged"] and 20 < res["iters"] < 150
    assert h[0] < h[5]                       # accelerating start
    assert h[-1] < 1e-8 and h[-1] < h[-2]    # stopped on a shrinking, small step
    assert all(not (h[k] < 1e-8 and h[k] < h[k - 1]) for k in range(1, len(h) - 1))


# ------------------------------------- node length below the root (Alg. 1)
# Four unit masses: A at the origin and B1, B2, B3 on the main diagonal. The
# root box is [0, 8]^3 (diagonal 8 sqrt 3). By the midpoint splits of Alg. 1,
# B1 = (8,8,8), B2 = (5,5,5), B3 = (6.5,6.5,6.5) share the depth-1 cell
# [4,8]^3; B1 and B3 share the depth-2 cell [6,8]^3 and part at depth 3; A and
# B2 end up alone. The query sits far out on the other side of the origin, so
# that each internal cell flips between accepted and opened at its own
# theta = l_k / r_k with l_k the root diagonal halved k times.
_NODE_PTS = np.array([[0.0, 0, 0], [8.0, 8, 8], [5.0, 5, 5], [6.5, 6.5, 6.5]])
_NODE_Y = np.array([[-20.0, -20.0, -20.0]])


def _single_body(y, pts):
    """Eq. (GAForce) of unit masses `pts` merged into one body at their mean."""
    d = y - pts.mean(0)
    r2 = d @ d + EPS ** 2
    return -G * len(pts) * d / r2 ** 1.5


def _point_sum(y, pts):
    return sum(_single_body(y, p[None]) for p in pts)


def _check_node_lengths(bh_force):
    """bh_force(theta) -> force on _NODE_Y[0]. Raises AssertionError when the
    accept/open flips do not happen at l_k = diag(root) 2^-k."""
    y = _NODE_Y[0]
    A, B1, B2, B3 = _NODE_PTS
    diag = 8.0 * np.sqrt(3.0)
    c1 = np.array([B1, B2, B3])
    c2 = np.array([B1, B3])
    th1 = (diag / 2) / np.linalg.norm(y - c1.mean(0))
    th2 = (diag / 4) / np.linalg.norm(y - c2.mean(0))
    fA = _point_sum(y, A[None])
    cases = [
        (th1 * (1 + 1e-9), fA + _single_body(y, c1)),                       # depth-1 cell accepted
        (th1 * (1 - 1e-9), fA + _point_sum(y, B2[None]) + _single_body(y, c2)),  # opened; depth 2 accepted
        (th2 * (1 + 1e-9), fA + _point_sum(y, B2[None]) + _single_body(y, c2)),
        (th2 * (1 - 1e-9), _point_sum(y, _NODE_PTS)),                       # everything exact
    ]
    for th, ref in cases:
        got = bh_force(th)
        assert np.allclose(got, ref, rtol=1e-13, atol=0), (th, got, ref)
    # the four cases are distinct, so a shifted threshold cannot pass by accident
    refs = [c[1] for c in cases]
    assert not np.allclose(refs[0], refs[1], rtol=1e-8)
    assert not np.allclose(refs[2], refs[3], rtol=1e-8)


def test_bh_node_length_halves_per_level(oracle_lib):
    t = oracle.BHTree(_NODE_PTS, np.ones(4))
    assert t.stats()["internal"] == 3  # root, [4,8]^3, [6,8]^3
    _check_node_lengths(lambda th: t.forces(_NODE_Y, None, G, EPS, th)[0])


def _mutated_oracle(tmp_path, old, new):
    """The oracle's C source with one planted change, built into a separate
    library (the planted mistake lives in the oracle, on the CPU)."""
    import ctypes
    import subprocess
    src = open(os.path.join(os.path.dirname(oracle.core.__file__), "fga_oracle.c")).read()
    assert old in src
    path = tmp_path / "mut.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", str(path), "-o", str(so), "-lm"])
    L = ctypes.CDLL(str(so))
    v, l, d = ctypes.c_void_p, ctypes.c_long, ctypes.c_double
    L.oracle_bh_build.argtypes = [v, v, l]
    L.oracle_bh_build.restype = v
    L.oracle_bh_forces.argtypes = [v, v, l, v, d, d, d, v, v]
    X = np.ascontiguousarray(_NODE_PTS)
    m = np.ones(4)
    h = L.oracle_bh_build(X.ctypes.data, m.ctypes.data, 4)

    def force(th):
        F = np.zeros((1, 3))
        Y = np.ascontiguousarray(_NODE_Y)
        L.oracle_bh_forces(h, Y.ctypes.data, 1, None, G, EPS, th, F.ctypes.data, None)
        return F[0]
    return force


@pytest.mark.parametrize("old,new", [
    # one level off: the root's children get the root's length
    ("nd->l = ldexp(diag_root, -nd->depth);", "nd->l = ldexp(diag_root, 1 - nd->depth);"),
    # one level too short
    ("nd->l = ldexp(diag_root, -nd->depth);", "nd->l = ldexp(diag_root, -nd->depth - 1);"),
    # the longest side instead of the diagonal
    ("for (int a = 0; a < t->dims; ++a) d2 += (t->hi[a] - t->lo[a]) * (t->hi[a] - t->lo[a]);",
     "for (int a = 0; a < t->dims; ++a) d2 = fmax(d2, (t->hi[a] - t->lo[a]) * (t->hi[a] - t->lo[a]));"),
])
def test_node_length_pin_catches_planted_mistakes(oracle_lib, tmp_path, old, new):
    force = _mutated_oracle(tmp_path, old, new)
    with pytest.raises(AssertionError):
        _check_node_lengths(force)


# --------------------------------------------- leaf-size variant of Alg. 1
def _independent_leaves_cap(X, L):
    """Leaf sets of the tree whose cells of at most L points are not split:
    a point's leaf is the shortest octal prefix of its quantised code shared
    by at most L points (or the full 20 digits)."""
    lo, hi = X.min(0), X.max(0)
    ext = hi - lo
    q = np.zeros(X.shape, dtype=np.int64)
    for a in range(3):
        if ext[a] > 0:
            q[:, a] = np.minimum(np.floor((X[:, a] - lo[a]) / ext[a] * 2.0 ** 20), 2 ** 20 - 1)
    digits = np.stack([((q[:, 0] >> b) & 1) * 4 + ((q[:, 1] >> b) & 1) * 2 + ((q[:, 2] >> b) & 1)
                       for b in range(19, -1, -1)], 1)
    keys = [tuple(r) for r in digits]
    leaves = {}
    for j, key in enumerate(keys):
        for k in range(0, 21):
            pre = key[:k]
            share = sum(1 for kk in keys if kk[:k] == pre)
            if share <= L or k == 20:
                leaves.setdefault(pre, []).append(j)
                break
    return sorted(tuple(sorted(v)) for v in leaves.values())


@pytest.mark.parametrize("L", [2, 5, 16])
def test_leaf_size_tree_leaves(oracle_lib, L):
    rng = np.random.default_rng(40 + L)
    X = np.vstack([rng.normal(size=(150, 3)), rng.normal(size=(6, 3)) * 1e-6])
    X = np.vstack([X, X[:2], X[:2]])  # triplicates: depth-20 leaves above L = 2
    t = oracle.BHTree(X, np.ones(len(X)), leaf=L)
    n, ids = t.leaves()
    got = sorted(tuple(sorted(np.flatnonzero(ids == k))) for k in range(n))
    assert got == _independent_leaves_cap(X, L)


def test_leaf_size_one_is_alg1(oracle_lib):
    X, Y, _, _ = synth.mixture_pair(41, per_comp=64, m=200)
    mX = np.random.default_rng(2).uniform(0.5, 1.5, len(X))
    a = oracle.BHTree(X, mX).forces(Y, None, G, EPS, 0.5, count=True)
    b = oracle.BHTree(X, mX, leaf=1).forces(Y, None, G, EPS, 0.5, count=True)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1]


@pytest.mark.parametrize("L", [4, 16])
def test_leaf_size_theta_zero_is_direct(oracle_lib, L):
    X, Y, _, _ = synth.mixture_pair(42, per_comp=64, m=200)
    mX = np.full(len(X), 1.0 / len(X))
    F, cnt = oracle.BHTree(X, mX, leaf=L).forces(Y, None, G, EPS, 0.0, count=True)
    Fd = oracle.direct_forces(Y, X, mX, None, G, EPS)
    assert cnt == len(X) * len(Y)
    assert np.allclose(F, Fd, rtol=1e-12, atol=1e-12 * np.abs(Fd).max())


def test_leaf_size_whole_set_is_one_leaf(oracle_lib):
    """With L >= n the root is the only node: a query it does not accept gets
    the exact sum over every point, one it accepts the single-body term."""
    rng = np.random.default_rng(43)
    X = rng.normal(size=(40, 3))
    m = np.ones(40)
    t = oracle.BHTree(X, m, leaf=40)
    assert t.stats()["nodes"] == 1
    near, far = rng.normal(size=(1, 3)), np.array([[300.0, 0, 0]])
    F, c = t.forces(near, None, G, EPS, 0.5, count=True)
    assert c == 40 and np.allclose(F[0], _point_sum(near[0], X), rtol=1e-12)
    F, c = t.forces(far, None, G, EPS, 0.5, count=True)
    assert c == 1 and np.allclose(F[0], _single_body(far[0], X), rtol=1e-12)


# ------------------------------- mass normalisation (Eq. FinalSPM, B = 1)
def test_masses_normalisation_two_cells():
    """Three points in one lattice cell and one in another: NIV is inversely
    proportional to the cell count (1/3, 1/3, 1/3, 1), so the reference weights
    normalised to sum 1 are (1/6, 1/6, 1/6, 1/2) and the template masses
    normalised to mean 1 are (2/3, 2/3, 2/3, 2)."""
    P = np.array([[0.0, 0, 0], [0.01, 0, 0], [0, 0.01, 0.01], [1.0, 1, 1]])
    mX, mY = oracle.masses(P, P.copy(), oracle.Params())
    assert np.allclose(mX, [1 / 6, 1 / 6, 1 / 6, 1 / 2], rtol=1e-14)
    assert np.allclose(mY, [2 / 3, 2 / 3, 2 / 3, 2.0], rtol=1e-14)
    assert np.isclose(mX.sum(), 1.0, rtol=1e-15) and np.isclose(mY.mean(), 1.0, rtol=1e-15)
    uX, uY = oracle.masses(P, P[:3], oracle.Params(masses="uniform"))
    assert np.allclose(uX, 0.25) and np.allclose(uY, 1.0) and len(uY) == 3


def test_masses_pin_catches_swapped_normalisation(monkeypatch):
    P = np.array([[0.0, 0, 0], [0.01, 0, 0], [0, 0.01, 0.01], [1.0, 1, 1]])
    real = oracle.core.niv_masses
    # planted: template masses normalised to sum 1 like the reference weights
    monkeypatch.setattr(oracle.core, "masses",
                        lambda a, b, p: (real(a) / real(a).sum(), real(b) / real(b).sum()))
    with pytest.raises(AssertionError):
        mX, mY = oracle.core.masses(P, P.copy(), oracle.Params())
        assert np.allclose(mY, [2 / 3, 2 / 3, 2 / 3, 2.0], rtol=1e-14)


# ------------------------------- per-particle velocity (Eq. PreviousVelocity)
def _particle_velocity_unrolled(velocity):
    """With fraction damping and no projection of the velocity, v after k
    steps is the damped sum of the past accelerations:
    v_2 = (1 - eta) dt g(Y_0) + dt g(Y_1). Returns (stepper V, unrolled sum)."""
    X, Y, _, _ = synth.mixture_pair(44, per_comp=32, m=150)
    Xn, Yn, _ = oracle.normalise(X, Y)
    mX = np.full(len(Xn), 1 / len(Xn))
    p = oracle.Params(velocity=velocity)
    st = oracle.Stepper(Xn, Yn, mX, np.ones(len(Yn)), p)
    Y0 = st.Y.copy()
    st.step()
    Y1 = st.Y.copy()
    st.step()
    g0 = oracle.direct_forces(Y0, Xn, mX, None, p.G, p.eps)
    g1 = oracle.direct_forces(Y1, Xn, mX, None, p.G, p.eps)
    return st.V, (1 - p.eta) * p.dt * g0 + p.dt * g1


def test_particle_velocity_is_damped_sum_of_accelerations(oracle_lib):
    V, ref = _particle_velocity_unrolled("particle")
    assert np.allclose(V, ref, rtol=1e-12, atol=1e-14)
    # the rigid reading carries a different state: the planted swap fails the pin
    Vr, refr = _particle_velocity_unrolled("rigid")
    assert not np.allclose(Vr, refr, rtol=1e-6)


def test_particle_velocity_exact_recovery(oracle_lib):
    """Noise-free full overlap with uniform masses: the per-particle velocity
    reading converges to the ground-truth transform like the rigid one."""
    X, Y, R_gt, t_gt = synth.uniform_grid_pair(24, n_side=7, max_deg=30.0)
    res = oracle.register(X, Y, oracle.Params(max_iter=400, masses="uniform", velocity="particle"))
    assert oracle.angular_deviation_deg(R_gt, res["R"]) < 1e-3
    assert np.linalg.norm(res["t"] - t_gt) < 1e-4


def test_stop_rule_never_fires_at_the_first_iteration(oracle_lib):
    """A threshold above every step size (1e-4 on the squared norm, the
    printed value read as a bound on the square): the first iteration has no
    earlier step to be smaller than, so the earliest stop is the second
    iteration, and then only if that step is smaller than the first."""
    X, Y, _, _ = synth.mixture_pair()
    res = oracle.register(X, Y, oracle.Params(max_iter=300, tol=1e-4), trace=True)
    h = [x[2] for x in res["history"]]
    assert res["converged"] and res["iters"] >= 2
    k = next(k for k in range(1, len(h)) if h[k] < 1e-4 and h[k] < h[k - 1])
    assert res["iters"] == k + 1


# ------------------------------------ RBF landmark masses (Eq. RBF_function)
SIG, BETA = 0.03, 100.0


def test_rbf_without_landmarks_is_one():
    P = np.random.default_rng(50).normal(size=(20, 3))
    assert np.array_equal(oracle.rbf_weights(P, np.zeros((0, 3)), SIG, BETA), np.ones(20))
    X, Y, _, _ = synth.mixture_pair(51, per_comp=16, m=100)
    a = oracle.masses(X, Y, oracle.Params())
    b = oracle.masses(X, Y, oracle.Params(), landmarks=(np.zeros(0, int), np.zeros(0, int)))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_rbf_single_anchor_closed_form():
    rng = np.random.default_rng(52)
    a = rng.normal(size=3)
    P = a + rng.normal(size=(30, 3)) * 0.05
    B = oracle.rbf_weights(P, a[None], SIG, BETA)
    ref = 1.0 + (BETA - 1.0) * np.exp(-((P - a) ** 2).sum(1) / SIG ** 2)
    assert np.allclose(B, ref, rtol=1e-14)


def test_rbf_two_anchors_closed_form():
    """Two anchors at distance s: the 2 x 2 collocation system gives
    lambda_1 = lambda_2 = (beta - 1) / (1 + exp(-s^2 / sigma^2))."""
    a1, a2 = np.zeros(3), np.array([0.04, 0.0, 0.0])
    e = np.exp(-0.04 ** 2 / SIG ** 2)
    rng = np.random.default_rng(53)
    P = rng.normal(size=(25, 3)) * 0.05
    B = oracle.rbf_weights(P, np.stack([a1, a2]), SIG, BETA)
    phi = lambda c: np.exp(-((P - c) ** 2).sum(1) / SIG ** 2)
    ref = 1.0 + (BETA - 1.0) / (1.0 + e) * (phi(a1) + phi(a2))
    assert np.allclose(B, ref, rtol=1e-13)
    # interpolation: B equals beta at both anchors; a planted lambda = beta - 1
    # (no collocation solve) misses it where the anchors overlap
    assert np.allclose(oracle.rbf_weights(np.stack([a1, a2]), np.stack([a1, a2]), SIG, BETA), BETA, rtol=1e-13)
    wrong = 1.0 + (BETA - 1.0) * (np.exp(-0.0) + e)
    assert not np.isclose(wrong, BETA, rtol=1e-3)


def test_rbf_interpolates_and_is_rigid_invariant():
    rng = np.random.default_rng(54)
    A = rng.normal(size=(5, 3))
    P = np.vstack([A, rng.normal(size=(40, 3)), A[0] + 10.0])
    B = oracle.rbf_weights(P, A, 0.8, BETA)
    assert np.allclose(B[:5], BETA, rtol=1e-10)
    assert np.isclose(B[-1], 1.0, atol=1e-12)   # far from every landmark
    Q = synth.random_rotation(rng, 180.0)
    c = rng.normal(size=3)
    B2 = oracle.rbf_weights(P @ Q.T + c, A @ Q.T + c, 0.8, BETA)
    assert np.allclose(B, B2, rtol=1e-10)


def test_spm_hadamard_two_cells_with_landmark():
    """The two-cell set of the NIV pin with a landmark on point 0 (its
    neighbours lie far outside sigma): S is proportional to
    (beta/3, 1/3, 1/3, 1) for both clouds."""
    P = np.array([[0.0, 0, 0], [0.01, 0, 0], [0, 0.01, 0.01], [1.0, 1, 1]])
    p = oracle.Params(rbf_sigma=1e-3)
    mX, mY = oracle.masses(P, P.copy(), p, landmarks=(np.array([0]), np.array([0])))
    raw = np.array([BETA / 3, 1 / 3, 1 / 3, 1.0])
    assert np.allclose(mX, raw / raw.sum(), rtol=1e-12)
    assert np.allclose(mY, raw / raw.mean(), rtol=1e-12)
    uX, uY = oracle.masses(P, P.copy(), oracle.Params(rbf_sigma=1e-3, masses="uniform"),
                           landmarks=(np.array([3]), np.array([3])))
    ru = np.array([1.0, 1.0, 1.0, BETA])
    assert np.allclose(uX, ru / ru.sum(), rtol=1e-12) and np.allclose(uY, ru / ru.mean(), rtol=1e-12)


# ------------------------------------------- D = 2 (quadtree, 2 x 2 Kabsch)
def _rot2(deg):
    a = np.deg2rad(deg)
    return np.array([[np.cos(a), -np.sin(a)], [np.sin(a), np.cos(a)]])


def test_2d_two_particle_closed_form():
    c = json.load(open(os.path.join(GOLDEN, "two_particle_force.json")))["cases"][0]
    F = oracle.direct_forces(np.array([c["y"][:2]]), np.array([c["x"][:2]]), np.array([c["mX"]]),
                             np.array([c["mY"]]), c["G"], c["eps"])[0]
    assert c["y"][2] == c["x"][2] == 0.0
    assert np.allclose(F, [float(v) for v in c["F"][:2]], rtol=1e-14, atol=1e-14)


def test_2d_brute_force_extended_precision():
    rng = np.random.default_rng(70)
    X, Y = rng.uniform(-2, 2, size=(7, 2)), rng.uniform(-2, 2, size=(5, 2))
    mX, mY = rng.uniform(0.1, 1, 7), rng.uniform(0.5, 2, 5)
    F = oracle.direct_forces(Y, X, mX, mY, G, EPS)
    ref = _mp_forces(np.c_[Y, np.zeros(5)], np.c_[X, np.zeros(7)], mX, mY, G, EPS)
    assert np.allclose(F, ref[:, :2], rtol=1e-13, atol=1e-13 * np.abs(ref).max())


def test_quadtree_theta_zero_and_huge():
    rng = np.random.default_rng(71)
    X, Y = rng.normal(size=(300, 2)), rng.normal(size=(40, 2)) * 3
    mX = rng.uniform(0.1, 1, 300)
    t = oracle.BHTree(X, mX)
    F0, c0 = t.forces(Y, None, G, EPS, 0.0, count=True)
    assert c0 == 300 * 40
    assert np.allclose(F0, oracle.direct_forces(Y, X, mX, None, G, EPS), rtol=1e-12)
    Fh, ch = t.forces(Y, None, G, EPS, 1e12, count=True)
    com = (mX[:, None] * X).sum(0) / mX.sum()
    d = Y - com
    r2 = (d ** 2).sum(1) + EPS ** 2
    assert ch == 40 and np.allclose(Fh, -G * mX.sum() * d / (r2 ** 1.5)[:, None], rtol=1e-12)


def test_quadtree_equals_octree_of_the_embedded_plane():
    """Points on the plane z = 0 split into at most 4 children per cell with
    the 2D box diagonal, so the octree of the embedded points makes the same
    decisions as the quadtree (Alg. 1 for D = 2 and D = 3)."""
    X, Y, _, _ = synth.mixture_pair(72, per_comp=64, m=200)
    X2, Y2 = X[:, :2], Y[:, :2]
    mX = np.random.default_rng(73).uniform(0.5, 1.5, len(X2))
    for th in (0.3, 0.6):
        F2, c2 = oracle.BHTree(X2, mX).forces(Y2, None, G, EPS, th, count=True)
        F3, c3 = oracle.BHTree(np.c_[X2, np.zeros(len(X2))], mX).forces(np.c_[Y2, np.zeros(len(Y2))],
                                                                         None, G, EPS, th, count=True)
        assert c2 == c3 and np.allclose(F2, F3[:, :2], rtol=1e-13) and np.all(F3[:, 2] == 0)


def test_quadtree_node_length_halves_per_level():
    """The 2D version of the node-length pin: unit masses A = (0,0) and
    B1 = (8,8), B2 = (5,5), B3 = (6.5,6.5); root diagonal 8 sqrt 2."""
    P = np.array([[0.0, 0], [8.0, 8], [5.0, 5], [6.5, 6.5]])
    y = np.array([-20.0, -20.0])
    t = oracle.BHTree(P, np.ones(4))

    def body(pts):
        d = y - pts.mean(0)
        return -G * len(pts) * d / (d @ d + EPS ** 2) ** 1.5
    pts = lambda *ix: P[list(ix)]
    c1, c2 = pts(1, 2, 3), pts(1, 3)
    th1 = 4 * np.sqrt(2) / np.linalg.norm(y - c1.mean(0))
    th2 = 2 * np.sqrt(2) / np.linalg.norm(y - c2.mean(0))
    exact = sum(body(P[k:k + 1]) for k in range(4))
    for th, ref in ((th1 * (1 + 1e-9), body(P[:1]) + body(c1)),
                    (th1 * (1 - 1e-9), body(P[:1]) + body(P[2:3]) + body(c2)),
                    (th2 * (1 - 1e-9), exact)):
        assert np.allclose(t.forces(y[None], None, G, EPS, th)[0], ref, rtol=1e-13)


def test_quadtree_leaves_match_prefix_grouping():
    rng = np.random.default_rng(74)
    X = np.vstack([rng.normal(size=(100, 2)), rng.normal(size=(4, 2)) * 1e-7])
    X = np.vstack([X, X[:2]])
    t = oracle.BHTree(X, np.ones(len(X)))
    n, ids = t.leaves()
    got = sorted(tuple(sorted(np.flatnonzero(ids == k))) for k in range(n))
    lo, ext = X.min(0), X.max(0) - X.min(0)
    q = np.minimum(np.floor((X - lo) / ext * 2.0 ** 20), 2 ** 20 - 1).astype(np.int64)
    keys = [tuple(((q[j, 0] >> b) & 1) * 2 + ((q[j, 1] >> b) & 1) for b in range(19, -1, -1))
            for j in range(len(X))]
    leaves = {}
    for j, key in enumerate(keys):
        for k in range(21):
            if sum(1 for kk in keys if kk[:k] == key[:k]) <= 1 or k == 20:
                leaves.setdefault(key[:k], []).append(j)
                break
    assert got == sorted(tuple(sorted(v)) for v in leaves.values())
    assert np.array_equal(t.quant(), q.astype(np.uint32))


def test_2d_kabsch_and_reflection():
    rng = np.random.default_rng(75)
    Y = rng.normal(size=(30, 2))
    R0 = _rot2(37.0)
    R, t = oracle.kabsch(Y, Y @ R0.T + [0.3, -0.2])
    assert np.allclose(R, R0, atol=1e-12) and np.allclose(t, [0.3, -0.2], atol=1e-12)
    M = np.diag([1.0, -1.0])
    R, _ = oracle.kabsch(Y, Y @ M.T)
    assert np.isclose(np.linalg.det(R), 1.0)


def test_2d_exact_recovery_full_overlap():
    g = (np.arange(12) + 0.5) / 12
    X = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    X = X + np.random.default_rng(76).uniform(-0.02, 0.02, X.shape)
    Ry, ty = _rot2(25.0), np.array([0.05, -0.08])
    Y = X @ Ry.T + ty
    res = oracle.register(X, Y, oracle.Params(max_iter=400, masses="uniform"))
    assert res["R"].shape == (2, 2)
    assert oracle.angular_deviation_deg(Ry.T, res["R"]) < 1e-3
    assert np.linalg.norm(res["t"] - (-Ry.T @ ty)) < 1e-4


def test_2d_niv_uses_discs_and_the_planar_lattice():
    """Two cells with 3 and 1 points: ratio 1 : 3 as in 3D; with rho = 1 and
    six points the capped case uses the disc area pi r^2 of D = 2."""
    P = np.array([[0.0, 0], [0.01, 0], [0, 0.01], [1.0, 1]])
    w = oracle.niv_masses(P)
    assert np.isclose(w[3] / w[0], 3.0, rtol=1e-14)
    P = np.vstack([np.zeros((5, 2)), np.ones((1, 2))])
    w = oracle.niv_masses(P, rho=1, a=-5, b=5, depth=20)
    vb2, vb3 = np.pi * (10.0 / 40.0) ** 2, 4.0 / 3.0 * np.pi * (10.0 / 40.0) ** 3
    assert 6 * vb2 > 1.0 > 6 * vb3  # six discs cover the unit cell, six balls would not
    assert np.allclose(w, 1.0, rtol=1e-14)


# ----------------------------------------------- Plummer energy (diagnostic)
@pytest.mark.parametrize("dims", [2, 3])
def test_bh_gpe_theta_zero_and_huge(dims):
    rng = np.random.default_rng(77 + dims)
    X, Y = rng.normal(size=(200, dims)), rng.normal(size=(30, dims)) * 3
    mX, mY = rng.uniform(0.1, 1, 200), rng.uniform(0.5, 2, 30)
    t = oracle.BHTree(X, mX)
    e0, c0 = t.gpe(Y, mY, G, EPS, 0.0, count=True)
    assert c0 == 200 * 30
    ref = -G * sum(mY[i] * (mX / np.sqrt(((Y[i] - X) ** 2).sum(1) + EPS ** 2)).sum() for i in range(30))
    assert np.isclose(e0, ref, rtol=1e-12)
    if dims == 3:
        assert np.isclose(e0, oracle.gpe(Y, X, mX, mY, G, EPS), rtol=1e-12)
    eh, ch = t.gpe(Y, mY, G, EPS, 1e12, count=True)
    com = (mX[:, None] * X).sum(0) / mX.sum()
    assert ch == 30 and np.isclose(eh, -G * (mY * mX.sum() / np.sqrt(((Y - com) ** 2).sum(1) + EPS ** 2)).sum())


def test_bh_gpe_gradient_is_bh_force():
    """With the traversal's accept/open decisions unchanged, the BH energy of
    one template point moves by -F . dy (its gradient is the BH force)."""
    X, Y, _, _ = synth.mixture_pair(79, per_comp=64, m=20)
    mX = np.full(len(X), 1.0 / len(X))
    t = oracle.BHTree(X, mX)
    y = Y[3:4].copy()
    F, c = t.forces(y, None, G, EPS, 0.5, count=True)
    for a in range(3):
        h = np.zeros((1, 3))
        h[0, a] = 1e-6
        ep, cp = t.gpe(y + h, None, G, EPS, 0.5, count=True)
        em, cm = t.gpe(y - h, None, G, EPS, 0.5, count=True)
        assert cp == cm == c
        assert np.isclose(-(ep - em) / 2e-6, F[0, a], rtol=1e-6, atol=1e-8 * np.abs(F).max())
