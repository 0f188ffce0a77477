"""The stored oracle results the benchmark reports against: each must still
be what the oracle computes on what the seeded generators produce. The
cheap records are recomputed in full, the costly ones on a few rows or from
their input hashes."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.join(os.path.dirname(__file__), "golden")
RUNS = json.load(open(os.path.join(HERE, "oracle_runs.json")))


def _hash(X, Y):
    h = hashlib.sha256()
    for a in (X, Y):
        h.update(np.ascontiguousarray(a, dtype=np.float32).tobytes())
    return h.hexdigest()


@pytest.fixture(scope="module")
def forces():
    with np.load(os.path.join(HERE, "oracle_forces.npz"), allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def test_mixture_record_is_the_oracle_registration():
    X, Y, _, _ = synth.mixture_pair()
    rec = RUNS["mixture_1024_direct_fp64"]
    assert rec["input_sha256"] == _hash(X, Y)
    o = oracle.register(np.asarray(X, np.float64), np.asarray(Y, np.float64),
                        oracle.Params(theta=0.0, max_iter=200))
    assert o["iters"] == rec["iters"] == 200
    np.testing.assert_allclose(o["R"], rec["R"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(o["t"], rec["t"], rtol=0, atol=1e-12)


def test_landmark_records_match_their_inputs_and_one_rerun():
    lm = RUNS["landmarks_misaligned90"]
    assert sorted(lm) == ["priors_0", "priors_1", "priors_3"]
    for k in (0, 1, 3):
        assert len(lm[f"priors_{k}"]) == 4
        for j, rec in enumerate(lm[f"priors_{k}"]):
            X, Y, _, _, _ = synth.misaligned_pair(j, max_deg=90.0)
            assert rec["input_sha256"] == _hash(X, Y)
    # one full rerun: three prior matches, pair 1
    X, Y, _, _, idx = synth.misaligned_pair(1, max_deg=90.0)
    pick = synth.landmark_picks(1, 3, len(Y))
    f = lambda a: np.ascontiguousarray(a, np.float32).astype(np.float64)  # noqa: E731
    o = oracle.register(f(X), f(Y), oracle.Params(theta=0.0, max_iter=300, tol=1e-8),
                        landmarks=(idx[pick], pick))
    rec = lm["priors_3"][1]
    assert o["iters"] == rec["iters"]
    np.testing.assert_allclose(o["R"], rec["R"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(o["t"], rec["t"], rtol=0, atol=1e-12)


def test_landmark_picks_are_distinct_and_seeded():
    a = synth.landmark_picks(5, 3, 1888)
    assert len(set(a.tolist())) == 3 and a.min() >= 0 and a.max() < 1888
    np.testing.assert_array_equal(a, synth.landmark_picks(5, 3, 1888))
    assert not np.array_equal(a, synth.landmark_picks(6, 3, 1888))


def test_precision_sample_forces_are_the_oracle_direct_sum(forces):
    X, Y, _, _ = synth.precision_pair()
    assert str(forces["precision_input_sha256"]) == _hash(X, Y)
    X64 = np.ascontiguousarray(X, np.float32).astype(np.float64)
    Y64 = np.ascontiguousarray(Y, np.float32).astype(np.float64)
    idx = forces["precision_idx"]
    assert len(idx) == 512 == len(set(idx.tolist()))
    F = oracle.direct_forces(np.ascontiguousarray(Y64[idx]), X64, np.full(len(X64), 1.0 / len(X64)))
    np.testing.assert_allclose(F, forces["precision_F"], rtol=1e-13, atol=0)


def test_mesh_sample_forces_on_a_few_rows(forces):
    X, Y, _, _ = synth.mesh_pair()
    assert str(forces["mesh_input_sha256"]) == _hash(X, Y)
    idx = forces["mesh_idx"]
    assert len(idx) == 4096 == len(set(idx.tolist()))
    X64 = np.ascontiguousarray(X, np.float32).astype(np.float64)
    Y64 = np.ascontiguousarray(Y, np.float32).astype(np.float64)
    rows = [0, 1, 2047, 4095]
    F = oracle.direct_forces(np.ascontiguousarray(Y64[idx[rows]]), X64, np.full(len(X64), 1.0 / len(X64)))
    np.testing.assert_allclose(F, forces["mesh_F"][rows], rtol=1e-13, atol=0)


def test_planar_record_matches_its_inputs():
    X, Y, _, _ = synth.planar_pair()
    rec = RUNS["planar_262144_bh0.5"]
    assert rec["input_sha256"] == _hash(X, Y)
    assert rec["iters"] == 100 and "3" in rec["at"]
    assert np.allclose(np.asarray(rec["R"]) @ np.asarray(rec["R"]).T, np.eye(2), atol=1e-12)


def test_energy_records_are_the_oracle_values():
    en = RUNS["energy"]
    X, Y, _, _ = synth.mesh_pair()
    assert en["mesh_1048576_bh0.5"]["input_sha256"] == _hash(X, Y)
    f = lambda a: np.ascontiguousarray(a, np.float32).astype(np.float64)  # noqa: E731
    X, Y = f(X), f(Y)
    e, cnt = oracle.BHTree(X, np.full(len(X), 1.0 / len(X))).gpe(Y, None, theta=0.5, count=True)
    assert cnt == en["mesh_1048576_bh0.5"]["interactions"]
    assert abs(e - en["mesh_1048576_bh0.5"]["E"]) <= 1e-12 * abs(e)
    Xp, Yp, _, _ = synth.precision_pair()
    assert en["precision_131072_direct"]["input_sha256"] == _hash(Xp, Yp)
    assert en["precision_131072_direct"]["interactions"] == len(Xp) * len(Yp)
