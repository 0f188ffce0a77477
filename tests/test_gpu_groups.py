"""Group runs of the Barnes-Hut group walk (built on the device) against the
greedy rule written out on the host: runs of at most G consecutive points,
each ending before the diagonal of its bounding box would exceed tau = f
times the median diagonal of the aligned G-runs.

The device computes the diagonals in FP32 with its own operation order, so a
diagonal within 1e-5 of tau may fall on either side; the checks below accept
either outcome there and are exact everywhere else."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2009_14005_amd as fga  # noqa: E402
import synth  # noqa: E402

pytestmark = pytest.mark.gpu
REL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)


def diag2(P):
    e = (P.max(0) - P.min(0)).astype(np.float32)
    return float(e[0] * e[0] + e[1] * e[1] + e[2] * e[2])


def tau2_of(P, G, f):
    if f == 0:
        return np.inf
    d = np.array([diag2(P[i:i + G]) for i in range(0, len(P), G)], np.float32)
    med = np.partition(d, len(d) // 2)[len(d) // 2]
    return float(np.float32(f * f) * med) if med > 0 else np.inf


def check_runs(P, runs, G, f):
    m = len(P)
    t2 = tau2_of(P, G, f)
    assert runs[0, 0] == 0 and runs[-1, 0] + runs[-1, 1] == m
    assert np.all(runs[1:, 0] == runs[:-1, 0] + runs[:-1, 1]), "runs must tile [0, m) in order"
    assert np.all((runs[:, 1] >= 1) & (runs[:, 1] <= G))
    for a, c in runs:
        if c >= 2:  # the run's box is within tau
            assert diag2(P[a:a + c]) <= t2 * (1 + REL), (a, c)
        if a + c < m and c < G:  # and the next point would have broken it
            assert diag2(P[a:a + c + 1]) > t2 * (1 - REL), (a, c)


def lidar_points():
    X, _, _, _ = synth.lidar_pair()
    return X


@pytest.mark.parametrize("G", [32, 64, 128])
@pytest.mark.parametrize("f", [0.0, 1.0, 2.0, 4.0])
def test_group_runs_follow_the_greedy_rule(G, f):
    rng = np.random.default_rng(17)
    X, _, _, _ = synth.mixture_pair(5, per_comp=600, m=100)
    P = X[np.argsort(X[:, 0] + 0.01 * rng.random(len(X)))].astype(np.float32)  # a spatially coherent order
    runs = fga.group_runs(torch.as_tensor(P, device="cuda:0"), G, f)
    check_runs(P, runs, G, f)
    if f == 0:
        assert np.array_equal(runs[:, 0], np.arange(0, len(P), G))


@pytest.mark.parametrize("m", [1, 31, 32, 33, 63, 64, 65, 127, 128, 129, 4097, 70001])
def test_group_runs_ragged_sizes(m):
    """Sizes around the block and super-block boundaries (4,096 points = 64
    blocks of 64), including a run reaching the end so the last block holds
    no run start."""
    rng = np.random.default_rng(m)
    P = np.cumsum(rng.normal(size=(m, 3)) * rng.choice([0.001, 0.05], size=(m, 1)), axis=0).astype(np.float32)
    for G, f in ((64, 1.0), (64, 4.0), (128, 2.0), (32, 1.0)):
        runs = fga.group_runs(torch.as_tensor(P, device="cuda:0"), G, f)
        check_runs(P, runs, G, f)


def test_group_runs_lidar_scan_in_morton_order():
    """The sparse LiDAR ring scan in Morton order (the groups the LiDAR
    registration walks), each tau option."""
    X = lidar_points().astype(np.float64)
    lo, hi = X.min(0), X.max(0)
    q = np.minimum(np.floor((X - lo) / (hi - lo) * 2 ** 20), 2 ** 20 - 1).astype(np.uint64)
    code = np.zeros(len(X), np.uint64)
    for b in range(20):
        for a in range(3):
            code |= ((q[:, a] >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + (2 - a))
    P = X[np.argsort(code, kind="stable")].astype(np.float32)
    for f in (1.0, 2.0, 4.0):
        runs = fga.group_runs(torch.as_tensor(P, device="cuda:0"), 64, f)
        check_runs(P, runs, 64, f)
        print(f"f {f}: {len(runs)} runs, {len(P) / len(runs):.1f} points per run")


def test_group_runs_argument_validation():
    P = torch.zeros((10, 3), device="cuda:0")
    for G, f in ((48, 1.0), (64, -1.0), (64, float("nan"))):
        with pytest.raises(fga.FGAError):
            fga.group_runs(P, G, f)
