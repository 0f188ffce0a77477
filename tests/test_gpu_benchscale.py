"""Parity at the sizes and in the configurations the benchmark times.

The FP64 oracle needs minutes to hours for these registrations, so its results
are stored in tests/golden/oracle_runs.json by tests/golden/make_oracle_runs.py
(which calls only the oracle, on the FP32-rounded inputs the HIP path gets).
Each stored record carries a hash of those inputs, checked here first.
Gates: rotation within 0.05 degrees and translation within 1e-4 of the
reference's bounding-box diagonal, at equal iteration counts.
"""
import hashlib
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2009_14005_amd as fga  # noqa: E402
import synth  # noqa: E402

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_runs.json")
PHI_GATE, DT_GATE = 0.05, 1e-4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)


@pytest.fixture(scope="module")
def gold():
    return json.load(open(GOLDEN))


def f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def dev(a, dtype=torch.float32):
    return torch.as_tensor(f32(a), dtype=dtype, device="cuda:0")


def input_hash(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(f32(a).tobytes())
    return h.hexdigest()


def phi_deg(Ra, Rb):
    A = Ra.T @ Rb
    s = 0.5 * np.linalg.norm([A[2, 1] - A[1, 2], A[0, 2] - A[2, 0], A[1, 0] - A[0, 1]])
    return float(np.degrees(np.arctan2(s, 0.5 * (np.trace(A) - 1.0))))


def pose_err(rec, R, t, X):
    diag = np.linalg.norm(X.max(0) - X.min(0))
    return phi_deg(np.array(rec["R"]), R), float(np.linalg.norm(t - np.array(rec["t"])) / diag)


def record(gold, key, X, Y):
    rec = gold[key]
    assert rec["input_sha256"] == input_hash(X, Y), f"{key}: inputs differ from the stored oracle run"
    return rec


def run_state(X, Y, p, checkpoints):
    st = fga.State(dev(X), dev(Y), p)
    out, done = {}, 0
    for k in checkpoints:
        st.step(k - done)
        done = k
        R, t, rep = st.get()
        out[k] = (R, t, rep)
    st.close()
    return out


# ------------------------------------------------- LiDAR pair, 65,536 points
@pytest.mark.parametrize("gw", [0, 1])
def test_lidar_100_iterations_against_oracle(gold, gw):
    """The benchmark's LiDAR registration (theta 0.5, FP32 Kahan tiles, NIV
    masses; autotuned group walk, and the per-particle walk) for 100
    iterations, and at 6 iterations, against the oracle's."""
    X, Y, _, _ = synth.lidar_pair()
    rec = record(gold, "lidar_65536_bh0.5", X, Y)
    res = run_state(X, Y, fga.default_params(theta=0.5, tol=0.0, group_width=gw), (6, 100))
    for k, ref in ((6, rec["at"]["6"]), (100, rec)):
        R, t, rep = res[k]
        phi, dt = pose_err(ref, R, t, X)
        print(f"gw {gw} iter {k}: phi {phi:.2e} deg, dt {dt:.2e}")
        assert phi < PHI_GATE and dt < DT_GATE, (k, phi, dt)
    if gw == 1:  # the per-particle walk makes Alg. 2's decisions: same count up to FP32 flips
        c = res[100][2].interactions
        assert abs(c - rec["interactions"]) <= 2e-3 * rec["interactions"], (c, rec["interactions"])


# ----------------------------------------- weighted mesh, 1,048,576 points
@pytest.mark.parametrize("theta", [0.3, 0.5, 0.8])
def test_mesh_registration_against_oracle(gold, theta):
    """The 1,048,576 + 1,048,576 mesh registration with the autotuned group
    walk after 3 and 100 iterations against the oracle's Barnes-Hut run."""
    X, Y, _, _ = synth.mesh_pair()
    rec = record(gold, f"mesh_1048576_bh{theta}", X, Y)
    res = run_state(X, Y, fga.default_params(theta=theta, tol=0.0), (3, 100))
    for k, ref in ((3, rec["at"]["3"]), (100, rec)):
        R, t, _ = res[k]
        phi, dt = pose_err(ref, R, t, X)
        print(f"theta {theta} iter {k}: phi {phi:.2e} deg, dt {dt:.2e}")
        assert phi < PHI_GATE and dt < DT_GATE, (k, phi, dt)


def test_mesh_alg2_count_against_oracle(gold):
    """The per-particle walk's interaction count over the 100-iteration mesh
    registration equals the oracle's Alg. 2 count up to FP32 MAC flips."""
    X, Y, _, _ = synth.mesh_pair()
    rec = record(gold, "mesh_1048576_bh0.5", X, Y)
    R, t, rep = fga.register(dev(X), dev(Y), fga.default_params(theta=0.5, tol=0.0, max_iter=100,
                                                                 group_width=1, tile=1))
    assert abs(rep.interactions - rec["interactions"]) <= 2e-3 * rec["interactions"]
    phi, dt = pose_err(rec, R, t, X)
    assert phi < PHI_GATE and dt < DT_GATE, (phi, dt)


# ------------------------------------- precision study, 131,072 x 131,072
@pytest.mark.parametrize("prec", [fga.PREC_FP32_ALL, fga.PREC_FP32, fga.PREC_FP32_KAHAN])
def test_precision_modes_against_oracle(gold, prec):
    """Direct-sum registration of the precision-study pair in each precision
    mode after 10 and 100 iterations against the oracle's FP64 run."""
    X, Y, _, _ = synth.precision_pair()
    rec = record(gold, "precision_131072_direct", X, Y)
    res = run_state(X, Y, fga.default_params(theta=0.0, tol=0.0, precision=prec), (10, 100))
    for k, ref in ((10, rec["at"]["10"]), (100, rec)):
        R, t, _ = res[k]
        phi, dt = pose_err(ref, R, t, X)
        print(f"precision {prec} iter {k}: phi {phi:.2e} deg, dt {dt:.2e}")
        assert phi < PHI_GATE and dt < DT_GATE, (k, phi, dt)


# -------------------------------------------------- batched, 256 pairs
def test_batch_random_pairs_fixed_iterations_against_oracle():
    """Eight random pairs of the 256, inside a batch with the benchmark's
    parameters at a fixed iteration count, against live oracle registrations."""
    sel = sorted(np.random.default_rng(5).choice(synth.BATCH_PAIRS, 8, replace=False).tolist())
    pairs = [synth.batch_pair(j) for j in sel]
    p = fga.default_params(theta=0.5, max_iter=40, tol=0.0)
    R, t, reps = fga.register_batch([dev(x[0]) for x in pairs], [dev(x[1]) for x in pairs], p)
    for k, (X, Y, _, _) in enumerate(pairs):
        o = oracle.register(f32(X).astype(np.float64), f32(Y).astype(np.float64),
                            oracle.Params(theta=0.5, max_iter=40))
        phi, dt = pose_err(o, R[k], t[k], X)
        print(f"pair {sel[k]}: phi {phi:.2e} deg, dt {dt:.2e}")
        assert reps[k].iters == 40
        assert phi < PHI_GATE and dt < DT_GATE, (sel[k], phi, dt)


@pytest.mark.parametrize("tol", [1e-8, 1e-4])
def test_batch_256_pairs_against_oracle(gold, tol):
    """The benchmark's whole batch (per-pair stop rule, at most 200
    iterations) against the oracle's registrations of every pair: the medians
    within the gates and at least 99% of the pairs within them."""
    recs = gold[f"batch_256_bh0.5_tol{tol:g}"]
    assert len(recs) == synth.BATCH_PAIRS
    pairs = synth.batch_pairs()
    for j in (0, 17, 255):
        assert recs[j]["input_sha256"] == input_hash(pairs[j][0], pairs[j][1])
    p = fga.default_params(theta=0.5, max_iter=200, tol=tol)
    R, t, reps = fga.register_batch([dev(x[0]) for x in pairs], [dev(x[1]) for x in pairs], p)
    errs = np.array([pose_err(recs[j], R[j], t[j], pairs[j][0]) for j in range(len(pairs))])
    bad = np.flatnonzero((errs[:, 0] >= PHI_GATE) | (errs[:, 1] >= DT_GATE))
    print(f"tol {tol:g}: median phi {np.median(errs[:, 0]):.2e}, max {errs[:, 0].max():.2e}; "
          f"median dt {np.median(errs[:, 1]):.2e}; outside the gates: {bad.tolist()}")
    assert np.median(errs[:, 0]) < PHI_GATE and np.median(errs[:, 1]) < DT_GATE
    assert len(bad) <= 0.01 * len(pairs), bad


def test_batch_256_pairs_per_particle_walk_tracks_oracle(gold):
    """The whole batch with the per-particle walk (Alg. 2's own MAC for every
    particle): FP32 Kahan forces with FP64 reductions, so every pair ends
    within rounding of the oracle's registration (gates 1e-4 degrees and 1e-6
    of the diagonal, 500 and 100 times tighter than the registration gates)."""
    recs = gold["batch_256_bh0.5_tol1e-08"]
    pairs = synth.batch_pairs()
    p = fga.default_params(theta=0.5, max_iter=200, tol=1e-8, group_width=1, leaf_size=1)
    R, t, reps = fga.register_batch([dev(x[0]) for x in pairs], [dev(x[1]) for x in pairs], p)
    errs = np.array([pose_err(recs[j], R[j], t[j], pairs[j][0]) for j in range(len(pairs))])
    print(f"per-particle walk batch: max phi {errs[:, 0].max():.2e} deg, max dt {errs[:, 1].max():.2e}")
    assert all(r.traversal == 1 for r in reps)
    assert errs[:, 0].max() < 1e-4 and errs[:, 1].max() < 1e-6
    iters = np.array([r.iters for r in reps])
    ref_iters = np.array([recs[j]["iters"] for j in range(len(pairs))])
    assert np.mean(np.abs(iters - ref_iters) <= 1) >= 0.99


# ------------------------------------------- planar (D = 2) and energy
def _rot3(R2):
    R = np.eye(3)
    R[:2, :2] = np.asarray(R2)
    return R


def test_planar_registration_against_oracle(gold):
    """The planar mixture at the benchmark's size (262,144 + 196,608 points,
    quadtree, theta 0.5, FP32 Kahan, autotuned walk), after 3 and 100
    iterations, against the stored oracle registration."""
    rec = gold["planar_262144_bh0.5"]
    X, Y, _, _ = synth.planar_pair()
    assert rec["input_sha256"] == input_hash(X, Y)
    diag = np.linalg.norm(X.max(0) - X.min(0))
    for it, ref in ((3, rec["at"]["3"]), (100, rec)):
        R, t, rep = fga.register_2d(dev(X), dev(Y), fga.default_params(theta=0.5, max_iter=it, tol=0.0))
        phi = phi_deg(_rot3(ref["R"]), _rot3(R))
        dt = float(np.linalg.norm(t - np.array(ref["t"])) / diag)
        print(f"planar, {it} iterations: phi {phi:.2e} deg, dt {dt:.2e}")
        assert rep.iters == it and R.shape == (2, 2)
        assert phi < PHI_GATE and dt < DT_GATE, (it, phi, dt)


@pytest.mark.parametrize("key", ["precision_131072_direct", "mesh_1048576_bh0.5"])
def test_energy_at_benchmark_sizes_against_oracle(gold, key):
    """Plummer energy of the 131,072-point precision pair (direct) and the
    mesh pair (Alg. 2 traversal, theta 0.5) against the stored oracle values:
    relative difference under 1e-5, and the traversal's interaction count
    within 0.1% of the oracle tree's."""
    rec = gold["energy"][key]
    direct = key.startswith("precision")
    X, Y, _, _ = (synth.precision_pair if direct else synth.mesh_pair)()
    assert rec["input_sha256"] == input_hash(X, Y)
    mX = torch.full((len(X),), 1.0 / len(X), dtype=torch.float32, device="cuda:0")
    E, cnt = fga.energy(dev(Y), dev(X), mX, None, 0.0 if direct else 0.5)
    rel = abs(E - rec["E"]) / abs(rec["E"])
    print(f"{key}: E {E:.12e} oracle {rec['E']:.12e} rel {rel:.2e}, count {cnt} oracle {rec['interactions']}")
    assert rel < 1e-5
    assert abs(cnt - rec["interactions"]) <= 1e-3 * rec["interactions"]
