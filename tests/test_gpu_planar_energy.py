"""D = 2 (quadtree, planar forces, 2 x 2 Kabsch) and the Plummer-energy
diagnostic against the FP64 oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2009_14005_amd as fga  # noqa: E402
import synth  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0")


def f32(a):
    return np.ascontiguousarray(a, np.float32).astype(np.float64)


def rot2(deg):
    a = np.deg2rad(deg)
    return np.array([[np.cos(a), -np.sin(a)], [np.sin(a), np.cos(a)]])


def planar_pair(seed, per=128, m=900, deg=25.0, noise=0.005):
    """The mixture recipe in the plane: 8 Gaussian blobs, a rotated, shifted,
    noisy subset as template."""
    X, _, _, _, idx = synth.mixture_pair(seed, per_comp=per, m=m, return_index=True)
    X = X[:, :2]
    rng = np.random.default_rng(seed + 100)
    Ry, ty = rot2(deg), rng.uniform(-0.1, 0.1, 2)
    Y = X[idx] @ Ry.T + ty + noise * rng.normal(size=(m, 2))
    return X, Y, Ry.T, -Ry.T @ ty


def rel(F, ref):
    n = np.linalg.norm(ref, axis=1)
    return np.linalg.norm(F - ref, axis=1) / n


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_planar_direct_forces(dtype):
    X, Y, _, _ = planar_pair(80, per=300, m=2000)
    X, Y = f32(X), f32(Y)
    mX = np.random.default_rng(81).uniform(0.5, 1.5, len(X))
    mX = f32(mX / mX.sum())
    p = fga.default_params(precision=fga.PREC_FP64 if dtype == torch.float64 else fga.PREC_FP32_KAHAN)
    F, cnt = fga.forces_2d(dev(Y, dtype), dev(X, dtype), dev(mX, dtype), None, 0.0, p)
    ref = oracle.direct_forces(Y, X, mX)
    e = rel(F.cpu().numpy().astype(np.float64), ref)
    assert F.shape == (len(Y), 2) and cnt == len(X) * len(Y)
    assert e.max() < (1e-12 if dtype == torch.float64 else 1e-5), e.max()


@pytest.mark.parametrize("gw", [1, 64])
@pytest.mark.parametrize("theta", [0.3, 0.6])
def test_planar_quadtree_forces(gw, theta):
    X, Y, _, _ = planar_pair(82, per=500, m=3000)
    X, Y = f32(X), f32(Y)
    mX = f32(np.full(len(X), 1.0 / len(X)))
    ref, cnt_ref = oracle.BHTree(X, mX).forces(Y, None, 66.7, 0.2, theta, count=True)
    F, cnt = fga.forces_2d(dev(Y), dev(X), dev(mX), None, theta, fga.default_params(group_width=gw))
    e = rel(F.cpu().numpy().astype(np.float64), ref)
    if gw == 1:  # the per-particle walk makes Alg. 2's decisions
        assert np.median(e) < 1e-5 and abs(cnt - cnt_ref) <= 1e-3 * cnt_ref, (np.median(e), cnt, cnt_ref)
    else:
        assert np.median(e) < 1e-2


def test_planar_registration_fp64_direct_matches_oracle():
    X, Y, _, _ = planar_pair(83)
    o = oracle.register(X, Y, oracle.Params(max_iter=100))
    p = fga.default_params(theta=0.0, tol=0.0, max_iter=100, precision=fga.PREC_FP64)
    R, t, rep = fga.register_2d(dev(X, torch.float64), dev(Y, torch.float64), p)
    assert R.shape == (2, 2) and np.isclose(np.linalg.det(R), 1.0)
    assert np.abs(R - o["R"]).max() < 1e-10 and np.abs(t - o["t"]).max() < 1e-9


@pytest.mark.parametrize("masses,gw", [(fga.MASS_NIV, 1), (fga.MASS_UNIFORM, 0)])
def test_planar_registration_fp32_bh_matches_oracle(masses, gw):
    """The per-particle walk makes the quadtree decisions of Alg. 2; the group
    walk refines them (it differs from the oracle's tree by about the BH error
    itself, which on this dense planar mixture with NIV masses grows to about
    the translation gate over 80 iterations)."""
    X, Y, _, _ = planar_pair(84, per=400, m=3000)
    X, Y = f32(X), f32(Y)
    o = oracle.register(X, Y, oracle.Params(theta=0.5, max_iter=80,
                                            masses="niv" if masses == fga.MASS_NIV else "uniform"))
    R, t, _ = fga.register_2d(dev(X), dev(Y), fga.default_params(theta=0.5, tol=0.0, max_iter=80,
                                                                  mass_mode=masses, group_width=gw))
    diag = np.linalg.norm(X.max(0) - X.min(0))
    assert oracle.angular_deviation_deg(o["R"], R) < 0.05 and np.linalg.norm(t - o["t"]) / diag < 1e-4


def test_planar_exact_recovery():
    g = (np.arange(16) + 0.5) / 16
    X = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    X = X + np.random.default_rng(85).uniform(-0.02, 0.02, X.shape)
    Ry, ty = rot2(20.0), np.array([0.04, -0.03])
    Y = X @ Ry.T + ty
    p = fga.default_params(theta=0.0, tol=0.0, max_iter=400, precision=fga.PREC_FP64,
                           mass_mode=fga.MASS_UNIFORM)
    R, t, _ = fga.register_2d(dev(X, torch.float64), dev(Y, torch.float64), p)
    assert oracle.angular_deviation_deg(Ry.T, R) < 1e-3 and np.linalg.norm(t + Ry.T @ ty) < 1e-4


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_energy_direct_matches_oracle(dtype):
    X, Y, _, _ = synth.mixture_pair(86, per_comp=400, m=2000)
    X, Y = f32(X), f32(Y)
    mX = f32(np.full(len(X), 1.0 / len(X)))
    mY = f32(np.random.default_rng(87).uniform(0.5, 1.5, len(Y)))
    E, cnt = fga.energy(dev(Y, dtype), dev(X, dtype), dev(mX, dtype), dev(mY, dtype), 0.0)
    ref = oracle.gpe(Y, X, mX, mY)
    assert cnt == len(X) * len(Y)
    assert abs(E - ref) <= (1e-12 if dtype == torch.float64 else 1e-6) * abs(ref), (E, ref)


@pytest.mark.parametrize("theta", [0.3, 0.6])
def test_energy_bh_matches_oracle_tree(theta):
    X, Y, _, _ = synth.mixture_pair(88, per_comp=500, m=3000)
    X, Y = f32(X), f32(Y)
    mX = f32(np.full(len(X), 1.0 / len(X)))
    ref, cref = oracle.BHTree(X, mX).gpe(Y, None, 66.7, 0.2, theta, count=True)
    E, cnt = fga.energy(dev(Y), dev(X), dev(mX), None, theta)
    assert abs(E - ref) <= 1e-6 * abs(ref) and abs(cnt - cref) <= 1e-3 * cref, (E, ref, cnt, cref)
    direct = oracle.gpe(Y, X, mX)
    assert abs(E - direct) < 1e-2 * abs(direct)
