"""The autotuner: leaf size among 1, 2, 4, 8, 16 for single registrations,
(tau option, part cap, leaf size) for the batched group walk; results against
the FP64 oracle, the cache, and a repeat in fresh processes."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2009_14005_amd as fga  # noqa: E402
import synth  # noqa: E402

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float32), device="cuda:0")


def f32(a):
    return np.ascontiguousarray(a, np.float32).astype(np.float64)


def phi_deg(Ra, Rb):
    A = Ra.T @ Rb
    s = 0.5 * np.linalg.norm([A[2, 1] - A[1, 2], A[0, 2] - A[2, 0], A[1, 0] - A[0, 1]])
    return float(np.degrees(np.arctan2(s, 0.5 * (np.trace(A) - 1.0))))


def test_leaf_autotuned_registration_matches_oracle():
    X, Y, _, _ = synth.mixture_pair(90, per_comp=1024, m=7000)
    X, Y = f32(X), f32(Y)
    o = oracle.register(X, Y, oracle.Params(theta=0.5, max_iter=60))
    R, t, rep = fga.register(dev(X), dev(Y), fga.default_params(theta=0.5, tol=0.0, max_iter=60, leaf_size=0))
    print("tuned leaf size", rep.leaf_size, "traversal", rep.traversal)
    assert rep.leaf_size in (1, 2, 4, 8, 16)
    diag = np.linalg.norm(X.max(0) - X.min(0))
    assert phi_deg(o["R"], R) < 0.05 and np.linalg.norm(t - o["t"]) / diag < 1e-4


@pytest.mark.parametrize("L", [2, 4, 8, 16])
def test_leaf_sizes_are_at_least_as_accurate_as_alg1(L):
    """Cells of up to L points summed exactly: the group walk on the leaf-L
    tree is no further from the direct sum than the oracle's Alg. 1 tree."""
    X, Y, _, _ = synth.mixture_pair(91, per_comp=800, m=3000)
    X, Y = f32(X), f32(Y)
    mX = f32(np.full(len(X), 1.0 / len(X)))
    d = oracle.direct_forces(Y, X, mX)
    nd = np.linalg.norm(d, axis=1)
    e_alg1 = np.median(np.linalg.norm(oracle.BHTree(X, mX).forces(Y, None, 66.7, 0.2, 0.5) - d, axis=1) / nd)
    F, _ = fga.forces(dev(Y), dev(X), dev(mX), None, 0.5, fga.default_params(leaf_size=L, group_width=64))
    e = np.median(np.linalg.norm(F.cpu().numpy().astype(np.float64) - d, axis=1) / nd)
    assert e <= 1.05 * e_alg1 + 1e-6, (e, e_alg1)


def test_batch_tuned_cached_and_fixed_configs():
    pairs = [synth.batch_pair(j) for j in range(12)]
    Xs, Ys = [dev(p[0]) for p in pairs], [dev(p[1]) for p in pairs]
    p = fga.default_params(theta=0.5, max_iter=40, tol=0.0, leaf_size=0)
    R1, t1, r1 = fga.register_batch(Xs, Ys, p)   # tunes (tau option, part cap, leaf size)
    R2, t2, r2 = fga.register_batch(Xs, Ys, p)   # the cached choice: the same launches
    assert np.array_equal(R1, R2) and np.array_equal(t1, t2)
    assert r1[0].leaf_size in (1, 4, 8) and all(r.iters == 40 for r in r1)
    Rf, tf, rf = fga.register_batch(Xs, Ys, fga.default_params(theta=0.5, max_iter=40, tol=0.0, tile=16))
    assert rf[0].leaf_size == 1
    for k, (X, Y, _, _) in enumerate(pairs[:4]):
        o = oracle.register(f32(X), f32(Y), oracle.Params(theta=0.5, max_iter=40))
        diag = np.linalg.norm(X.max(0) - X.min(0))
        for R, t in ((R1[k], t1[k]), (Rf[k], tf[k])):
            assert phi_deg(o["R"], R) < 0.05 and np.linalg.norm(t - o["t"]) / diag < 1e-4


def test_batch_rejects_wide_groups():
    X, Y, _, _ = synth.batch_pair(0)
    with pytest.raises(fga.FGAError) as e:
        fga.register_batch([dev(X)], [dev(Y)], fga.default_params(theta=0.5, group_width=128))
    assert e.value.name == "UNSUPPORTED"


CHILD = """
import json, sys
import numpy as np
import torch
sys.path.insert(0, {root!r})
import paper_2009_14005_amd as fga, synth
X, Y, _, _ = synth.mixture_pair(92, per_comp=1024, m=7000)
d = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device="cuda:0")
R, t, rep = fga.register(d(X), d(Y), fga.default_params(theta=0.5, tol=0.0, max_iter=60, leaf_size=0))
print(json.dumps({{"R": R.tolist(), "t": t.tolist(), "leaf": rep.leaf_size, "trav": rep.traversal}}))
"""


def test_autotuned_results_agree_across_processes():
    """The tuner chooses by timing, so fresh processes (empty caches) may pick
    different splits or leaf sizes; their results agree within the gates."""
    env = dict(os.environ)
    env.pop("FGA_TUNE_CACHE", None)
    outs = []
    for _ in range(2):
        r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT)], capture_output=True,
                           text=True, timeout=240, env=env)
        assert r.returncode == 0, r.stderr[-2000:]
        outs.append(json.loads(r.stdout.strip().splitlines()[-1]))
    X, _, _, _ = synth.mixture_pair(92, per_comp=1024, m=7000)
    diag = np.linalg.norm(X.max(0) - X.min(0))
    a, b = outs
    print("choices:", a["leaf"], a["trav"], b["leaf"], b["trav"])
    assert phi_deg(np.array(a["R"]), np.array(b["R"])) < 0.05
    assert np.linalg.norm(np.array(a["t"]) - np.array(b["t"])) / diag < 1e-4


def test_cached_choice_with_a_leaf_tree_is_reused(tmp_path):
    """A cached split that names a tree other than the first (leaf size > 1)
    is taken from the cache: no timing round runs (FGA_TUNE_LOG stays silent)
    and the registration uses that tree and walk."""
    cache = tmp_path / "tune.cache"
    env = dict(os.environ, FGA_TUNE_CACHE=str(cache))
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT)], capture_output=True, text=True,
                       timeout=240, env=env)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in cache.read_text().splitlines() if l.startswith('"bh_f32_p1_g0_')]
    assert len(lines) == 1, cache.read_text()
    key = lines[0].split('"')[1]
    # leaf index 1 (leaf size 2), group walk K = 1 with the first tau option, one part per group
    cache.write_text(f'"{key}": {(1 << 16) | (17 << 8) | 1},\n')
    env["FGA_TUNE_LOG"] = "1"
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT)], capture_output=True, text=True,
                       timeout=240, env=env)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "[fga tune]" not in r.stderr, r.stderr[-2000:]
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert (out["leaf"], out["trav"]) == (2, 64)




PLANAR_CHILD = r"""
import json, sys
sys.path.insert(0, {root!r})
import numpy as np, torch
import paper_2009_14005_amd as fga
import synth
dev = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device="cuda:0")
X2, Y2, _, _ = synth.planar_pair(per_comp=4096, m=24576)
X3, Y3, _, _ = synth.mixture_pair(7, per_comp=4096, m=24576)
p = fga.default_params(theta=0.5, max_iter=5, tol=0.0)
a = fga.register_2d(dev(X2), dev(Y2), p)
b = fga.register(dev(X3), dev(Y3), p)
c = fga.register_2d(dev(X2), dev(Y2), p)
print(json.dumps({{"t2": a[2].traversal, "t3": b[2].traversal,
                  "same": bool(np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1]))}}))
"""


def test_planar_and_3d_choices_are_cached_apart(tmp_path):
    """A planar and a 3D registration of the same sizes are tuned once each
    (their candidates differ: runs of 32 are a candidate in the plane only),
    and a repeated planar registration takes its cached choice."""
    env = dict(os.environ, FGA_TUNE_CACHE=str(tmp_path / "tune.cache"), FGA_TUNE_LOG="1")
    r = subprocess.run([sys.executable, "-c", PLANAR_CHILD.format(root=ROOT)], capture_output=True,
                       text=True, timeout=240, env=env)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stderr.count("[fga tune] initial pose") == 2, r.stderr[-3000:]
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["same"] and out["t3"] in (1, 64, 128) and out["t2"] in (1, 32, 64, 128)
