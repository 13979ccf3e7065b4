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


@pytest.mark.parametrize("cplx", [False, True])
def test_state_calls_wait_for_the_plans_side_stream(cplx):
    """Export right after an execute enqueued behind a held side stream, with
    no synchronize: the state call waits for the plan's last call, so the
    history it returns is the input's last (M-1)*P + residue samples.  Import
    and the next execute then resume on another stream bit for bit."""
    from paper_2408_16551_amd.pfb import Plan, State
    P, M = 1024, 16
    n = P * 3000 + 321
    print(f"state on a side stream: P={P} M={M} complex={cplx}", flush=True)
    xh = _x(2 * n, 21, cplx)
    plan = Plan(P, M, "c64" if cplx else "r32", "hann", "fp32")
    x1 = torch.from_numpy(xh[:n]).cuda()
    x2 = torch.from_numpy(xh[n:]).cuda()
    ref_state = State(plan)
    plan(x1, state=ref_state)
    ref_tail = plan(x2, state=ref_state).cpu()
    torch.cuda.synchronize()
    st = State(plan)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        torch.cuda._sleep(20_000_000)      # hold the stream, so the call below ends late
        plan(x1, state=st, stream=s)
    hist = st.export()                      # no synchronize
    want = xh[n - ((M - 1) * P + 321):n]
    assert hist.shape == want.shape and np.array_equal(hist, want)
    st2 = State(plan)
    s2 = torch.cuda.Stream()
    with torch.cuda.stream(s2):
        torch.cuda._sleep(20_000_000)
        plan(x1[: P * 10], state=st2, stream=s2)   # overwritten by the import below
    st2.load_from(hist)                     # no synchronize: waits for s2's call first
    with torch.cuda.stream(s2):
        tail = plan(x2, state=st2, stream=s2)
    s2.synchronize()
    assert torch.equal(torch.view_as_real(tail.cpu()), torch.view_as_real(ref_tail))
    plan.close()
