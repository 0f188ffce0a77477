"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point declared in include/fga.h, validates arguments before any
device work, and its FP64 Kabsch solver agrees with a library SVD."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2009_14005_amd as fga
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fga.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fga_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = fga.lib()
    names = declared_functions()
    assert len(names) >= 19
    for name in names:
        assert hasattr(L, name), name


def test_default_params_are_the_papers():
    p = fga.default_params()
    assert (p.G, p.eps, p.eta, p.dt, p.theta) == (66.7, 0.2, 0.2, 0.1, 0.6)
    assert (p.a, p.b, p.rho, p.max_depth) == (-5.0, 5.0, 16, 20)
    assert (p.group_width, p.leaf_size, p.tile) == (0, 1, 0)
    assert fga.version().startswith("fga-mi355x")


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first


def call_forces(**over):
    L = fga.lib()
    p = fga.default_params()
    args = dict(Y=FAKE, m=10, X=FAKE, n=10, mX=FAKE, mY=None, dt=0, theta=0.0, p=p, F=FAKE)
    args.update(over)
    return L.fga_forces(args["Y"], args["m"], args["X"], args["n"], args["mX"], args["mY"],
                        args["dt"], args["theta"], ctypes.byref(args["p"]), args["F"], None, None)


@pytest.mark.parametrize("over,code", [
    (dict(Y=None), 1), (dict(X=None), 1), (dict(mX=None), 1), (dict(F=None), 1),
    (dict(m=0), 1), (dict(n=-3), 1), (dict(n=(1 << 27) + 1), 1), (dict(dt=7), 1),
    (dict(theta=-0.5), 1), (dict(theta=float("nan")), 1),
    (dict(p=fga.default_params(eps=0.0)), 1), (dict(p=fga.default_params(G=-1.0)), 1),
    (dict(p=fga.default_params(dt=0.0)), 1), (dict(p=fga.default_params(eta=1.5)), 1),
    (dict(p=fga.default_params(rho=0)), 1), (dict(p=fga.default_params(a=5.0, b=-5.0)), 1),
    (dict(p=fga.default_params(max_depth=12)), 6), (dict(p=fga.default_params(precision=9)), 1),
    (dict(p=fga.default_params(leaf_size=65)), 1), (dict(p=fga.default_params(leaf_size=-1)), 1),
    (dict(p=fga.default_params(group_width=48)), 1), (dict(p=fga.default_params(group_width=-1)), 1),
    (dict(p=fga.default_params(tile=256)), 1), (dict(p=fga.default_params(tile=-1)), 1),
    (dict(dt=0, p=fga.default_params(precision=2)), 1),
])
def test_forces_argument_validation(over, code):
    assert call_forces(**over) == code
    assert fga.lib().fga_last_error().decode() != ""


def test_literal_damping_allows_eta_above_one():
    # eta > 1 is only rejected for fraction damping; the call then fails later
    # on the fake pointer check, not on the parameters
    p = fga.default_params(eta=1.5, damping=fga.DAMP_LITERAL)
    st = call_forces(p=p)
    assert "eta" not in fga.lib().fga_last_error().decode()
    assert st != 0


def test_register_and_state_validation():
    L = fga.lib()
    p = fga.default_params()
    R = (ctypes.c_double * 9)()
    t = (ctypes.c_double * 3)()
    assert L.fga_register(None, 10, FAKE, 10, 0, ctypes.byref(p), R, t, None, None) == 1
    assert L.fga_register(FAKE, 10, FAKE, 0, 0, ctypes.byref(p), R, t, None, None) == 1
    assert L.fga_register(FAKE, 10, FAKE, 10, 0, ctypes.byref(p), None, t, None, None) == 1
    bad = fga.default_params(max_iter=-1)
    assert L.fga_register(FAKE, 10, FAKE, 10, 0, ctypes.byref(bad), R, t, None, None) == 1
    h = ctypes.c_void_p()
    assert L.fga_state_create(FAKE, 0, FAKE, 5, 0, ctypes.byref(p), None, ctypes.byref(h)) == 1
    assert L.fga_step(None, 1) == 1
    assert L.fga_state_get(None, R, t, None) == 1
    assert L.fga_register_batch(0, None, None, None, None, 0, ctypes.byref(p), R, t, None, None) == 1
    assert L.fga_masses(FAKE, 0, 10, ctypes.byref(p), 2, FAKE, None) == 1
    assert L.fga_masses(None, 0, 10, ctypes.byref(p), 0, FAKE, None) == 1


def numpy_kabsch(C):
    U, _, Vt = np.linalg.svd(C)
    d = np.sign(np.linalg.det(U @ Vt)) or 1.0
    return U @ np.diag([1.0, 1.0, d]) @ Vt


def test_kabsch_solver_matches_library_svd():
    rng = np.random.default_rng(3)
    for _ in range(200):
        C = rng.normal(size=(3, 3))
        assert np.allclose(fga.kabsch(C), numpy_kabsch(C), atol=1e-11)


def test_kabsch_near_identity_and_symmetric():
    """The iteration's typical input: C = R S + small perturbation."""
    rng = np.random.default_rng(4)
    for _ in range(100):
        A = rng.normal(size=(3, 3))
        S = A @ A.T + np.eye(3)
        R0 = synth.random_rotation(rng, 5.0)
        C = R0 @ S + 1e-6 * rng.normal(size=(3, 3))
        assert np.allclose(fga.kabsch(C), numpy_kabsch(C), atol=1e-11)
        assert np.allclose(fga.kabsch(R0 @ S), R0, atol=1e-12)


def test_kabsch_reflection_and_rank_two():
    rng = np.random.default_rng(5)
    C = np.diag([3.0, 2.0, -1.0])
    R = fga.kabsch(C)
    assert np.isclose(np.linalg.det(R), 1.0) and np.allclose(R, np.eye(3))
    # planar template: rank-2 C
    Y = np.c_[rng.normal(size=(20, 2)), np.zeros(20)]
    R0 = synth.random_rotation(rng, 60)
    Yc = Y - Y.mean(0)
    C = (Yc @ R0.T).T @ Yc
    assert np.allclose(fga.kabsch(C), R0, atol=1e-10)


def test_kabsch_rank_one_is_degenerate():
    v = np.array([1.0, 2.0, 3.0])
    with pytest.raises(fga.FGAError) as e:
        fga.kabsch(np.outer(v, v))
    assert e.value.name == "DEGENERATE"
    with pytest.raises(fga.FGAError) as e:
        fga.kabsch(np.full((3, 3), np.nan))
    assert e.value.name == "NONFINITE"


def test_noalloc_direct_rejects_oversized_scratch_on_the_host():
    """The size check of the static-scratch entry point runs before any
    device call (fake, never-dereferenced pointers)."""
    L = fga.lib()
    p = fga.default_params()
    fake = ctypes.c_void_p(0x1000)
    st = L.fga_forces_direct_noalloc(fake, 1 << 20, fake, 1 << 23, fake, None, fga.F32,
                                     ctypes.byref(p), fake, None)
    assert st == 1 and b"scratch" in L.fga_last_error()
    st = L.fga_forces_direct_noalloc(fake, 0, fake, 10, fake, None, fga.F32, ctypes.byref(p), fake, None)
    assert st == 1


@pytest.mark.parametrize("idx,count,over,code", [
    ([0, 1], 65, {}, 1),            # more than 64 landmarks
    ([-1], 1, {}, 1),               # index below range
    ([10], 1, {}, 1),               # index n (out of range)
    ([0], 1, {"rbf_sigma": 0.0}, 1),
    ([0], 1, {"rbf_weight": float("nan")}, 1),
])
def test_landmark_argument_validation(idx, count, over, code):
    """Landmark checks run on the host before any device call (fake pointers)."""
    L = fga.lib()
    p = fga.default_params(**over)
    fake = ctypes.c_void_p(0x1000)
    arr = (ctypes.c_int64 * max(len(idx), count))(*idx)
    st = L.fga_masses_landmarks(fake, fga.F32, 10, arr, count, ctypes.byref(p), 0, fake, None)
    assert st == code, L.fga_last_error()
    R = (ctypes.c_double * 9)()
    t = (ctypes.c_double * 3)()
    st = L.fga_register_landmarks(fake, 10, fake, 10, fga.F32, arr, arr, count, ctypes.byref(p),
                                  R, t, None, None)
    assert st == code, L.fga_last_error()


def test_energy_planar_sequence_argument_validation():
    """Host-side checks of the energy, planar and sequence entry points
    (fake, never-dereferenced pointers)."""
    L = fga.lib()
    p = fga.default_params()
    fake = ctypes.c_void_p(0x1000)
    E = ctypes.c_double(0)
    assert L.fga_energy(fake, 10, fake, 10, fake, None, fga.F32, -1.0, ctypes.byref(p),
                        ctypes.byref(E), None, None) == 1
    assert L.fga_energy(fake, 10, fake, 10, None, None, fga.F32, 0.0, ctypes.byref(p),
                        ctypes.byref(E), None, None) == 1
    assert L.fga_forces_2d(fake, 0, fake, 10, fake, None, fga.F32, 0.5, ctypes.byref(p), fake,
                           None, None) == 1
    R = (ctypes.c_double * 4)()
    t = (ctypes.c_double * 2)()
    assert L.fga_register_2d(fake, 10, None, 10, fga.F32, ctypes.byref(p), R, t, None, None) == 1
    frames = (ctypes.c_void_p * 1)(0x1000)
    sizes = (ctypes.c_int64 * 1)(10)
    R9 = (ctypes.c_double * 9)()
    t3 = (ctypes.c_double * 3)()
    assert L.fga_register_sequence(1, frames, sizes, fga.F32, ctypes.byref(p), R9, t3, None, None,
                                   None, None) == 1




def test_group_runs_argument_validation():
    L = fga.lib()
    fake = ctypes.c_void_p(0x1000)
    out = (ctypes.c_int32 * 64)()
    n = ctypes.c_int64()
    for m, G, f in ((10, 48, 1.0), (10, 64, -1.0), (10, 64, float("inf")), (0, 64, 1.0)):
        assert L.fga_group_runs(fake, m, G, f, out, 32, ctypes.byref(n), None) == 1, (m, G, f)
    assert L.fga_group_runs(None, 10, 64, 1.0, out, 32, ctypes.byref(n), None) == 1
    assert L.fga_group_runs(fake, 10, 64, 1.0, None, 32, ctypes.byref(n), None) == 1
