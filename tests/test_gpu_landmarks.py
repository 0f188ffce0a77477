"""Landmark (RBF) masses and registration with prior correspondences against
the FP64 oracle: Eq. (RBF_function) and the SPM product of Eq. (FinalSPM)."""
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
    return torch.as_tensor(np.asarray(a), dtype=dtype, device="cuda:0")


def phi_deg(Ra, Rb):
    A = Ra.T @ Rb
    s = 0.5 * np.linalg.norm([A[2, 1] - A[1, 2], A[0, 2] - A[2, 0], A[1, 0] - A[0, 1]])
    return float(np.degrees(np.arctan2(s, 0.5 * (np.trace(A) - 1.0))))


@pytest.mark.parametrize("norm", [0, 1])
@pytest.mark.parametrize("nlm", [1, 3, 9])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_masses_landmarks_match_oracle(norm, nlm, dtype):
    X, _, _, _ = synth.mixture_pair(60, per_comp=600, m=10)
    X = np.ascontiguousarray(X, np.float32).astype(np.float64)
    idx = np.random.default_rng(61).choice(len(X), nlm, replace=False)
    p = fga.default_params(rbf_sigma=0.02, rbf_weight=40.0)
    got = fga.masses(dev(X, dtype), p, norm, landmarks=idx).cpu().numpy()
    w = oracle.niv_masses(X) * oracle.rbf_weights(X, X[idx], 0.02, 40.0)
    ref = w / w.sum() if norm == 0 else w / w.mean()
    tol = 1e-12 if dtype == torch.float64 else 2e-6
    assert np.allclose(got, ref, rtol=tol, atol=tol * np.abs(ref).max()), np.abs(got / ref - 1).max()


def test_masses_without_landmarks_equal_niv():
    X, _, _, _ = synth.mixture_pair(62, per_comp=100, m=10)
    a = fga.masses(dev(X), landmarks=np.zeros(0, np.int64)).cpu().numpy()
    b = fga.masses(dev(X)).cpu().numpy()
    assert np.array_equal(a, b)


def test_coincident_landmarks_are_degenerate():
    X, _, _, _ = synth.mixture_pair(63, per_comp=50, m=10)
    with pytest.raises(fga.FGAError) as e:
        fga.masses(dev(X), landmarks=np.array([3, 3]))
    assert e.value.name == "DEGENERATE"


def _lm_case(seed, k, min_deg=0.0, max_deg=30.0):
    X, Y, Rg, tg, sub = synth.mixture_pair(seed, return_index=True, min_deg=min_deg, max_deg=max_deg)
    pick = np.random.default_rng(seed + 1).choice(len(Y), k, replace=False)
    return X, Y, (sub[pick], pick)


@pytest.mark.parametrize("k", [1, 3])
def test_register_landmarks_fp64_direct_matches_oracle(k):
    X, Y, lm = _lm_case(64, k)
    o = oracle.register(X, Y, oracle.Params(max_iter=100), landmarks=lm)
    p = fga.default_params(theta=0.0, tol=0.0, max_iter=100, precision=fga.PREC_FP64)
    R, t, rep = fga.register(dev(X, torch.float64), dev(Y, torch.float64), p, landmarks=lm)
    assert rep.iters == 100
    assert np.abs(R - o["R"]).max() < 1e-10 and np.abs(t - o["t"]).max() < 1e-9


@pytest.mark.parametrize("damping", [fga.DAMP_FRACTION, fga.DAMP_LITERAL])
def test_register_landmarks_fp32_bh_matches_oracle(damping):
    X, Y, lm = _lm_case(65, 3)
    X32 = np.ascontiguousarray(X, np.float32).astype(np.float64)
    Y32 = np.ascontiguousarray(Y, np.float32).astype(np.float64)
    eta = 0.2 if damping == fga.DAMP_FRACTION else 2.0
    o = oracle.register(X32, Y32, oracle.Params(theta=0.5, max_iter=60, eta=eta,
                                                damping="fraction" if damping == fga.DAMP_FRACTION else "literal"),
                        landmarks=lm)
    p = fga.default_params(theta=0.5, tol=0.0, max_iter=60, damping=damping, eta=eta)
    R, t, _ = fga.register(dev(X32), dev(Y32), p, landmarks=lm)
    diag = np.linalg.norm(X.max(0) - X.min(0))
    assert phi_deg(o["R"], R) < 0.05 and np.linalg.norm(t - o["t"]) / diag < 1e-4


def test_state_with_landmarks_steps_like_register():
    X, Y, lm = _lm_case(66, 2)
    p = fga.default_params(theta=0.0, tol=0.0, max_iter=30, precision=fga.PREC_FP64)
    R, t, _ = fga.register(dev(X, torch.float64), dev(Y, torch.float64), p, landmarks=lm)
    st = fga.State(dev(X, torch.float64), dev(Y, torch.float64), p, landmarks=lm)
    st.step(30)
    R2, t2, _ = st.get()
    st.close()
    assert np.array_equal(R, R2) and np.array_equal(t, t2)
