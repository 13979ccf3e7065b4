"""Ordering across streams: a plan's calls share its workspace, so calls on
different streams must not race on it; a device-resident server request may
be submitted while the caller's stream is still writing its input."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _x(n, seed, cplx=False):
    g = np.random.Generator(np.random.PCG64(seed))
    x = g.standard_normal(n)
    if cplx:
        x = x + 1j * g.standard_normal(n)
        return x.astype(np.complex64)
    return x.astype(np.float32)


@pytest.mark.parametrize("precision", ["fp32", "fp8", "bf16x3"])
def test_one_plan_on_two_streams_matches_single_stream_runs(precision):
    from paper_2408_16551_amd.pfb import Plan
    P, M = 1024, 16
    print(f"two streams: P={P} M={M} {precision}", flush=True)
    plan = Plan(P, M, "r32", "hann", precision)
    xa = torch.from_numpy(_x(P * 4096, 11)).cuda()
    xb = torch.from_numpy(_x(P * 4096, 12)).cuda()
    ref_a = plan(xa).clone()
    ref_b = plan(xb).clone()
    torch.cuda.synchronize()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    for _ in range(3):
        with torch.cuda.stream(sa):
            oa = plan(xa)
        with torch.cuda.stream(sb):
            ob = plan(xb)
        torch.cuda.synchronize()
        assert torch.equal(torch.view_as_real(oa), torch.view_as_real(ref_a))
        assert torch.equal(torch.view_as_real(ob), torch.view_as_real(ref_b))
    plan.close()


def test_device_request_waits_for_the_stream_writing_its_input():
    from paper_2408_16551_amd.pfb import Plan, Server
    P, M = 512, 12
    src = torch.from_numpy(_x(P * 2000 + 77, 5, cplx=True)).cuda()
    ref = Plan(P, M, "c64", "hann", "fp32")(src).cpu().numpy()
    torch.cuda.synchronize()
    sv = Server("fp32", max_streams=1, max_active=4, frames_per_step=256, use_graph=True, max_channels=512)
    sid = sv.stream(P, M, "c64")
    x = torch.empty_like(src)
    out = torch.full((src.numel() // P, P), float("nan"), dtype=torch.complex64, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        torch.cuda._sleep(20_000_000)      # hold the stream, so the copy below lands late
        x.copy_(src)
        rid = sv.submit(sid, x, out)        # no synchronize: the server orders itself after s
    r = sv.wait(rid, timeout_s=60)
    assert r["status"] == 0 and r["frames"] == out.shape[0]
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref)
    sv.close()
