"""The FIR fused into the FP32 DFT GEMM (TINA_DFT_FUSED): the output must be
bit for bit that of the two-kernel dense path (the tile forms the FIR output
with the FIR kernel's FMA order), including streaming with states and the
calls that fall back to two kernels, and within the FP32 bar of the oracle."""
import numpy as np
import pytest

from test_gpu_parity import FP32_BOUND, rel_l2, _dev, _run, _rand

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _plan(P, M, cplx, dft, window="hann"):
    from paper_2408_16551_amd.pfb import Plan
    return Plan(P, M, "c64" if cplx else "r32", window, "fp32", "pfb", dft=dft)


@pytest.mark.parametrize("P,M,cplx,F", [(1024, 16, False, 300), (256, 8, True, 257), (64, 5, True, 130),
                                        (4096, 8, True, 40), (32, 16, False, 1000), (512, 1, False, 129),
                                        (128, 3, False, 77)])
def test_fused_equals_dense_bitwise_and_matches_oracle(oracle, P, M, cplx, F):
    x = _rand(P * F + P // 2, cplx, seed=P + M)
    dense = _run(_plan(P, M, cplx, "dense"), x)
    fused = _run(_plan(P, M, cplx, "fused"), x)
    assert fused.shape == dense.shape
    assert np.array_equal(fused, dense)
    ref = oracle.pfb(x[: F * P], P, M, oracle.window(P, M, "hann"))
    assert rel_l2(fused, ref) < FP32_BOUND


@pytest.mark.parametrize("P,M,cplx", [(1024, 16, False), (128, 9, True)])
def test_fused_streaming_equals_one_shot_bitwise(P, M, cplx):
    # Chunk lengths that leave residues of every size: calls whose history is
    # not a whole number of float4s run the two-kernel path, the others the
    # fused tile; all must agree with one shot.
    from paper_2408_16551_amd.pfb import State
    N = P * 90 + P // 3 + 5
    x = _rand(N, cplx, seed=7 * P + M)
    plan = _plan(P, M, cplx, "fused")
    one = _run(plan, x)
    st = State(plan)
    cuts = [0, 1, 3, P // 3, P * 3 + 7, P * 40 + 4, P * 41, N]
    got = np.concatenate([_run(plan, np.ascontiguousarray(x[a:b]), state=st) for a, b in zip(cuts[:-1], cuts[1:])])
    assert np.array_equal(got, one)
    assert np.array_equal(one, _run(_plan(P, M, cplx, "dense"), x))


@pytest.mark.parametrize("P,M,cplx,precision", [(1024, 17, False, "fp32"), (1024, 16, False, "bf16"),
                                                (16, 4, False, "fp32")])
def test_fused_rejects_unsupported(P, M, cplx, precision):
    from paper_2408_16551_amd.pfb import Plan, TinaError
    with pytest.raises(TinaError):
        Plan(P, M, "c64" if cplx else "r32", "hann", precision, "pfb", dft="fused")


def test_full_size_real_stream_fused_equals_dense(oracle):
    from paper_2408_16551_amd import workloads
    w = workloads.real_stream()
    xd = _dev(w.x)
    a = _plan(w.P, w.M, False, "fused")(xd)
    b = _plan(w.P, w.M, False, "dense")(xd)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
