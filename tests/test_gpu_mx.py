"""Block-scaled FP8 form of the DFT (E4M3 codes, one power-of-two scale per
32 entries along the summed axis), through the C ABI.

Bars:
* With unit taps and M = 1 the FIR passes the FP32 input through exactly, so
  the GPU quantises the same values as the oracle, and the only difference
  left is the matrix unit's own sum.  Measured on MI355X with in-bounds
  probes: the scaled FP8 MFMA adds the products of one 32-K block in fixed
  point about 15 bits below the block's largest product, truncating (448 +
  31 * 2^-9 gives 448 + 24 * 2^-9; 128 + 2^-9 gives 128), and adds block
  results in FP32.  So each output must lie within two granules
  2^(floor(log2 p_b) - 14) per block b (p_b bounds the block's largest
  product) plus an FP32 accumulation term of the oracle's block-scaled DFT
  (FP64 sums of the same quantised products), and within 5e-5 relative L2
  overall (measured about 1e-5).  A wrong code, scale or lane-to-block
  assignment is orders of magnitude above both.
* With real windows, against the oracle's block-scaled DFT of the oracle's
  FIR output rounded to FP32: 2e-4 (measured about 1e-5; FP32 vs FP64 FIR
  rounding can move a value across an E4M3 rounding boundary now and then).
* Against the exact FP64 filter bank: the stated bound of the form.
* Streaming, batches and the server: bit for bit equal to one-shot execute.
"""
import numpy as np
import pytest

from test_gpu_parity import REDUCED_BOUNDS, rel_l2, _dev, _run

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _plan(P, M, cplx, window="hann", custom=None, precision="mxfp8"):
    from paper_2408_16551_amd.pfb import Plan
    return Plan(P, M, "c64" if cplx else "r32", "custom" if custom is not None else window, precision,
                custom_taps=custom)


def _ranged(N, cplx, seed, seg=16, decades=3):
    # N(0,1) samples, each run of `seg` samples scaled by 10^U(-decades, decades),
    # so that neighbouring 32-entry blocks need very different scales.
    g = np.random.Generator(np.random.PCG64(seed))
    s = np.repeat(10.0 ** g.uniform(-decades, decades, N // seg + 1), seg)[:N]
    x = g.standard_normal(N) * s
    if cplx:
        return (x + 1j * g.standard_normal(N) * s).astype(np.complex64)
    return x.astype(np.float32)


MX_SUM_BOUND = 5e-5


def _block_sum_bound(frame_re):
    # Per-frame bound on |GPU - oracle| for every output: two truncation
    # granules per 32-entry block (largest product <= 1.125 max|a| * 1.125,
    # quantised values, |coefficients| <= 1) plus an FP32 term.
    a = np.abs(frame_re).reshape(-1, 32).max(axis=1) * 1.125 * 1.125
    nz = a > 0
    gran = np.zeros_like(a)
    gran[nz] = 2.0 ** (np.floor(np.log2(a[nz])) - 14)
    return 2.0 * gran.sum() + 1e-6 * 32 * a.sum()


@pytest.mark.parametrize("P,cplx,F", [(128, False, 300), (64, True, 257), (1024, False, 131), (512, True, 200),
                                      (4096, True, 40), (8192, False, 9)])
def test_identity_fir_matches_oracle_block_scaled_dft(oracle, P, cplx, F):
    x = _ranged(P * F + P // 3, cplx, seed=P + F)
    X = _run(_plan(P, 1, cplx, custom=np.ones(P)), x)
    frames = x[: F * P].reshape(F, P).astype(np.complex128 if cplx else np.float64)
    ref = oracle.mx_dft(frames)
    err = rel_l2(X, ref)
    print(f"mxfp8 identity P={P} cplx={cplx}: rel_l2={err:.3e}")
    assert err < MX_SUM_BOUND
    re = frames.view(np.float64).reshape(F, -1) if cplx else frames
    for f in range(F):
        b = _block_sum_bound(re[f])
        d = X[f].astype(np.complex128) - ref[f]
        assert np.max(np.abs(d.real)) <= b and np.max(np.abs(d.imag)) <= b, f"frame {f}"


@pytest.mark.parametrize("P,M,cplx,F,window", [(256, 8, True, 300, "blackman"), (1024, 16, False, 200, "hann"),
                                               (128, 5, False, 129, "hamming"), (512, 12, True, 150, "hann")])
def test_pfb_matches_oracle_block_scaled_dft_of_fir(oracle, P, M, cplx, F, window):
    x = _ranged(P * F + 7, cplx, seed=3 * P + M, seg=64, decades=2)
    X = _run(_plan(P, M, cplx, window=window), x)
    h = oracle.window(P, M, window)
    y = oracle.fir(x[: F * P], P, M, h)
    y32 = y.astype(np.complex64 if cplx else np.float32).astype(np.complex128 if cplx else np.float64)
    err_q = rel_l2(X, oracle.mx_dft(y32))
    err_exact = rel_l2(X, oracle.pfb(x[: F * P], P, M, h))
    print(f"mxfp8 P={P} M={M} cplx={cplx}: vs block-scaled oracle {err_q:.3e}, vs FP64 {err_exact:.3e}")
    assert err_q < 2e-4
    assert err_exact < REDUCED_BOUNDS["mxfp8"]


@pytest.mark.parametrize("P,M,cplx", [(128, 9, False), (64, 16, True), (1024, 16, True)])
def test_streaming_chunked_equals_one_shot_bitwise(P, M, cplx):
    from paper_2408_16551_amd.pfb import State
    N = P * 70 + P // 2 + 3
    x = _ranged(N, cplx, seed=P + M)
    plan = _plan(P, M, cplx)
    one = _run(plan, x)
    st = State(plan)
    cuts = [0, 1, 1, P // 3, P * 3 + 7, P * 40 + 1, N]
    got = np.concatenate([_run(plan, np.ascontiguousarray(x[a:b]), state=st) for a, b in zip(cuts[:-1], cuts[1:])])
    assert np.array_equal(got, one)


@pytest.mark.parametrize("P,cplx", [(64, False), (32, True), (16, False), (16, True)])
def test_unsupported_channel_counts_are_rejected(P, cplx):
    from paper_2408_16551_amd.pfb import TinaError
    with pytest.raises(TinaError):
        _plan(P, 4, cplx)


def test_batch_equals_single_execute_bitwise():
    from paper_2408_16551_amd.pfb import Batch
    mix = [(256, 16, True, 256 * 37 + 5), (1024, 16, True, 1024 * 9), (512, 16, True, 0), (512, 16, True, 300),
           (128, 4, False, 128 * 500 + 3), (1024, 9, False, 1024 * 21 + 1000), (4096, 8, True, 4096 * 6 + 17),
           (64, 13, True, 64 * 333)]
    plans, xd, outs = [], [], []
    for i, (P, M, cplx, N) in enumerate(mix):
        p = _plan(P, M, cplx)
        plans.append(p)
        xd.append(_dev(_ranged(N, cplx, seed=i)))
        outs.append(p.alloc_out(max(1, p.output_frames(N))))
    b = Batch("mxfp8", max_items=16, workspace_bytes=256 << 20)
    fw = b.execute(list(zip(plans, xd, outs)))
    torch.cuda.synchronize()
    for p, x, o, f in zip(plans, xd, outs, fw):
        single = p(x)
        torch.cuda.synchronize()
        assert f == single.shape[0]
        assert torch.equal(o[:f], single)


def test_server_streams_equal_one_shot_bitwise():
    from test_gpu_server import _serve, _one_shot, _workload
    streams = [(64, 8, True), (256, 16, True), (128, 11, False), (1024, 9, True)]
    reqs = _workload(41, n_req=20, streams=streams)
    got, results, _ = _serve(reqs, "mxfp8", True, streams=streams)
    ref = _one_shot(reqs, "mxfp8", streams=streams)
    for g, r in zip(got, ref):
        if r is None:
            continue
        assert np.array_equal(g, r)
