"""Standalone building blocks on the GPU: the unfold of Sec. 4.4 (bit-exact,
it is a copy; pinned by the paper's worked example) and the FIR of Sec. 4.3
(against the FP64 oracle; impulse -> float32 taps exactly)."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_unfold_paper_example():
    from paper_2408_16551_amd.pfb import unfold
    g = json.load(open(os.path.join(GOLDEN, "unfold_example.json")))
    Y = unfold(torch.tensor(g["x"], dtype=torch.float32, device="cuda"), g["window"])
    torch.cuda.synchronize()
    assert list(Y.shape) == g["expected_shape"]
    assert np.array_equal(Y.cpu().numpy(), np.asarray(g["expected"], dtype=np.float32))


@pytest.mark.parametrize("n,width,stride", [(1000, 7, 1), (4096, 64, 16), (12345, 256, 1024), (10, 11, 1),
                                            (1 << 20, 16, 1), (777, 1, 3), (5000, 4096, 1)])
def test_unfold_matches_oracle_bitwise(oracle, n, width, stride):
    from paper_2408_16551_amd.pfb import unfold
    x = np.random.Generator(np.random.PCG64(n)).standard_normal(n).astype(np.float32)
    Y = unfold(torch.from_numpy(x).cuda(), width, stride)
    torch.cuda.synchronize()
    ref = oracle.unfold(x.astype(np.float64), width, stride)
    assert Y.shape == ref.shape
    assert np.array_equal(Y.cpu().numpy().astype(np.float64), ref)


def test_unfold_capacity_rejected():
    import ctypes
    from paper_2408_16551_amd import pfb
    x = torch.zeros(100, device="cuda")
    y = torch.full((10, 8), 3.0, device="cuda")
    rows = ctypes.c_int64()
    st = pfb.load().tina_unfold(ctypes.c_void_p(x.data_ptr()), 100, 8, 1, ctypes.c_void_p(y.data_ptr()), 10,
                                ctypes.byref(rows), None)
    torch.cuda.synchronize()
    assert st == 1 and torch.all(y == 3.0)


@pytest.mark.parametrize("K,n,cplx", [(1, 1000, False), (3, 4099, True), (64, 100000, False), (1000, 70001, True),
                                      (4097, 20000, False), (8192, 9000, True)])
def test_fir_matches_oracle(oracle, K, n, cplx):
    from paper_2408_16551_amd.pfb import Fir
    g = np.random.Generator(np.random.PCG64(K + n))
    a = g.standard_normal(K)
    x = g.standard_normal(n) + (1j * g.standard_normal(n) if cplx else 0)
    x = x.astype(np.complex64 if cplx else np.float32)
    f = Fir(a, "c64" if cplx else "r32")
    y = f(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    # Eq. (15) is the single-branch case of the oracle's polyphase FIR (P = 1,
    # taps reversed: h_0(m) = h[M-1-m] = a[m]).
    ref = oracle.fir(x, 1, K, a[::-1].copy()).reshape(-1)
    got = y.cpu().numpy().astype(np.complex128 if cplx else np.float64)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err < 1e-5, err


@pytest.mark.parametrize("cplx", [False, True])
def test_fir_impulse_gives_float32_taps(cplx):
    from paper_2408_16551_amd.pfb import Fir
    K = 300
    a = np.random.Generator(np.random.PCG64(5)).standard_normal(K)
    x = np.zeros(5000, dtype=np.complex64 if cplx else np.float32)
    x[1234] = 1.0
    y = Fir(a, "c64" if cplx else "r32")(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = np.zeros_like(x)
    ref[1234: 1234 + K] = a.astype(np.float32)
    assert np.array_equal(y, ref)
