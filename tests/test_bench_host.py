"""Host-side helpers of the benchmark: the NumPy filter bank it times beside
the oracle must compute the same thing, and the per-channel error figures must
name the right channels."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from oracle import Oracle  # noqa: E402
from paper_2408_16551_amd import workloads  # noqa: E402


def test_numpy_pfb_real_matches_oracle():
    w = workloads.small_pfb()
    o = Oracle()
    h = o.window(w.P, w.M, w.window)
    ref = o.pfb(w.x, w.P, w.M, h)
    X64 = bench.numpy_pfb(w.x, w.P, w.M, h, np.dtype(np.float64))
    assert X64.shape == ref.shape
    assert bench.rel_l2(X64, ref) < 1e-13
    X32 = bench.numpy_pfb(w.x, w.P, w.M, h, np.dtype(np.float32))
    assert X32.dtype == np.complex64
    assert bench.rel_l2(X32, ref) < 1e-5


def test_numpy_pfb_complex_matches_oracle():
    g = np.random.Generator(np.random.PCG64(5))
    P, M, n = 32, 5, 32 * 40 + 7   # ragged tail: the last 7 samples make no frame
    x = (g.standard_normal(n) + 1j * g.standard_normal(n)).astype(np.complex64)
    o = Oracle()
    h = o.window(P, M, "blackman")
    ref = o.pfb(x, P, M, h)
    X = bench.numpy_pfb(x, P, M, h, np.dtype(np.complex128))
    assert X.shape == ref.shape == (40, P)
    assert bench.rel_l2(X, ref) < 1e-13


def test_channel_errors_names_worst_channel_and_weakest_tone():
    class W:
        P, M = 8, 2
        tones = [(2 / 8, 1.0, 0.0), (5 / 8, 1e-3, 0.0), (0.3, 1e-4, 0.0)]   # the last is off-centre
    fr = np.arange(6, dtype=np.int64)
    ref = np.ones((6, 8), dtype=np.complex128)
    got = ref.copy()
    got[1:, 3] += 0.5          # channel 3 is the worst past the warm-up frame
    got[1:, 5] += 1e-3         # the weakest centre tone sits in channel 5
    got[0, :] += 100.0         # frame 0 is warm-up (M - 1 = 1) and is not counted
    e = bench.channel_errors(got, ref, W, fr)
    assert abs(e["worst_channel_rel_l2"] - 0.5) < 1e-12
    assert e["weakest_tone"]["channel"] == 5
    assert abs(e["weakest_tone"]["rel_l2"] - 1e-3) < 1e-12
