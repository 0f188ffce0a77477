"""Sequential LiDAR odometry: frame-to-frame registration of a synthetic
drive (each frame a 65,536-point ring scan) with composed poses, against
stored FP64 oracle registrations of the first frame pairs."""
import hashlib
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2009_14005_amd as fga  # noqa: E402
import synth  # noqa: E402

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_runs.json")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)


def phi_deg(Ra, Rb):
    A = Ra.T @ Rb
    s = 0.5 * np.linalg.norm([A[2, 1] - A[1, 2], A[0, 2] - A[2, 0], A[1, 0] - A[0, 1]])
    return float(np.degrees(np.arctan2(s, 0.5 * (np.trace(A) - 1.0))))


def test_sequence_pairs_match_oracle_and_compose():
    recs = json.load(open(GOLDEN))["odometry_lidar_pairs_bh0.5"]
    scans, poses = synth.lidar_sequence(len(recs) + 1)
    frames = [torch.as_tensor(np.ascontiguousarray(s, np.float32), device="cuda:0") for s in scans]
    p = fga.default_params(theta=0.5, tol=0.0, max_iter=100)
    Rr, tr, Ra, ta, reps = fga.register_sequence(frames, p)
    for k, rec in enumerate(recs):
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(scans[k], np.float32).tobytes())
        h.update(np.ascontiguousarray(scans[k + 1], np.float32).tobytes())
        assert rec["input_sha256"] == h.hexdigest()
        diag = np.linalg.norm(scans[k].max(0) - scans[k].min(0))
        phi = phi_deg(np.array(rec["R"]), Rr[k])
        dt = np.linalg.norm(tr[k] - np.array(rec["t"])) / diag
        print(f"pair {k}: phi {phi:.2e} deg, dt {dt:.2e}; iterations {reps[k].iters}")
        assert reps[k].iters == 100 and phi < 0.05 and dt < 1e-4, (k, phi, dt)
    # composition T_{k+1} = T_k T_rel(k), T_0 = I
    assert np.allclose(Ra[0], np.eye(3)) and np.allclose(ta[0], 0)
    for k in range(len(recs)):
        assert np.allclose(Ra[k + 1], Ra[k] @ Rr[k], atol=1e-12)
        assert np.allclose(ta[k + 1], Ra[k] @ tr[k] + ta[k], atol=1e-10)


def test_sequence_equals_batch_of_consecutive_pairs():
    scans, _ = synth.lidar_sequence(4)
    frames = [torch.as_tensor(np.ascontiguousarray(s, np.float32), device="cuda:0") for s in scans]
    p = fga.default_params(theta=0.5, tol=0.0, max_iter=20)
    Rr, tr, _, _, _ = fga.register_sequence(frames, p)
    Rb, tb, _ = fga.register_batch(frames[:-1], frames[1:], p)
    assert np.array_equal(Rr, Rb) and np.array_equal(tr, tb)


def test_sequence_rejects_single_frame():
    f = torch.zeros(10, 3, device="cuda:0")
    with pytest.raises(ValueError):
        fga.register_sequence([f], fga.default_params())
