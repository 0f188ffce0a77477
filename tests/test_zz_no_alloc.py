"""fga_forces_direct_noalloc (static device scratch, no allocation) against
fga_forces with theta = 0, which runs the same kernels on pool memory."""
import ctypes

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


def _case(seed, per, m, dtype):
    X, Y, _, _ = synth.mixture_pair(seed, per_comp=per, m=m)
    mX = np.random.default_rng(seed).uniform(0.5, 1.5, len(X))
    mX /= mX.sum()
    d = lambda a: torch.as_tensor(a, dtype=dtype, device="cuda:0")
    return d(X), d(Y), d(mX), X, Y, mX


def _noalloc(Y, X, mX, F, p):
    L = fga.lib()
    code = fga.F64 if Y.dtype == torch.float64 else fga.F32
    st = L.fga_forces_direct_noalloc(ctypes.c_void_p(Y.data_ptr()), Y.shape[0],
                                     ctypes.c_void_p(X.data_ptr()), X.shape[0],
                                     ctypes.c_void_p(mX.data_ptr()), None, code, ctypes.byref(p),
                                     ctypes.c_void_p(F.data_ptr()),
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, L.fga_last_error().decode()


@pytest.mark.parametrize("dtype,prec", [(torch.float32, fga.PREC_FP32_KAHAN), (torch.float32, fga.PREC_FP32),
                                        (torch.float64, fga.PREC_FP64)])
def test_noalloc_matches_allocating_entry_point_twice(dtype, prec):
    p = fga.default_params(precision=prec)
    # first call: 8 x 2,000 references, 9,000 templates (several tiles, ragged
    # tail); second call smaller, on the array the first one left behind
    for seed, per, m in ((31, 2000, 9000), (32, 300, 1001)):
        Xd, Yd, mXd, X, Y, mX = _case(seed, per, m, dtype)
        F = torch.full_like(Yd, float("nan"))
        _noalloc(Yd, Xd, mXd, F, p)
        torch.cuda.synchronize()
        ref, _ = fga.forces(Yd, Xd, mXd, None, 0.0, p)
        got, want = F.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(got, want)  # same kernels, same split: identical bits
        o = oracle.direct_forces(np.asarray(Y, np.float64) if dtype == torch.float64 else
                                 Y.astype(np.float32).astype(np.float64),
                                 X if dtype == torch.float64 else X.astype(np.float32).astype(np.float64),
                                 mX if dtype == torch.float64 else mX.astype(np.float32).astype(np.float64))
        e = np.linalg.norm(got - o) / np.linalg.norm(o)
        assert e < (1e-12 if dtype == torch.float64 else 1e-5), e


def test_noalloc_rejects_oversized_before_device_work():
    Xd, Yd, mXd, _, _, _ = _case(33, 16, 64, torch.float32)
    F = torch.zeros_like(Yd)
    L = fga.lib()
    p = fga.default_params()
    st = L.fga_forces_direct_noalloc(ctypes.c_void_p(Yd.data_ptr()), 1 << 20,
                                     ctypes.c_void_p(Xd.data_ptr()), 1 << 23,
                                     ctypes.c_void_p(mXd.data_ptr()), None, fga.F32, ctypes.byref(p),
                                     ctypes.c_void_p(F.data_ptr()), None)
    assert st == 1 and b"scratch" in L.fga_last_error()
