"""Continuous-batching server: a stream's requests are consecutive chunks of
one signal, so the concatenated outputs must equal one filter-bank pass over
the concatenated input (bit for bit: same kernels, same arithmetic per output
element), whether the stream runs alone or mixed with others, with or without
graph replay, and under a budget that forces admission waits."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _rand(N, cplx, g):
    x = g.standard_normal(N)
    if cplx:
        return (x + 1j * g.standard_normal(N)).astype(np.complex64)
    return x.astype(np.float32)


# (P, M, cplx) per logical stream
STREAMS = [(64, 8, True), (256, 16, True), (512, 11, True), (256, 16, False), (1024, 9, True)]


def _workload(seed, n_req=24, streams=STREAMS):
    g = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    for _ in range(n_req):
        s = int(g.integers(len(streams)))
        P = streams[s][0]
        n = int(g.choice([0, P // 3, P * int(g.integers(1, 40)) + int(g.integers(P)), P * 300 + 7]))
        reqs.append((s, _rand(n, streams[s][2], g)))
    return reqs


def _serve(reqs, precision="fp32", use_graph=True, budget=1 << 30, max_active=8, fps=64, streams=STREAMS,
           only=None):
    from paper_2408_16551_amd.pfb import Server
    sv = Server(precision, max_streams=len(streams), max_active=max_active, hbm_budget_bytes=budget,
                frames_per_step=fps, use_graph=use_graph, max_channels=1024)
    sids = [sv.stream(P, M, "c64" if c else "r32") for P, M, c in streams]
    res = [0] * len(streams)
    pending = []
    for s, x in reqs:
        if only is not None and s != only:
            continue
        P = streams[s][0]
        frames = (res[s] + x.size) // P
        res[s] = (res[s] + x.size) % P
        out = np.full((frames, sv.out_rows(sids[s])), np.nan, dtype=np.complex64)
        pending.append((s, sv.submit(sids[s], x, out), out))
    outs = [[] for _ in streams]
    results = []
    for s, rid, out in pending:
        r = sv.wait(rid, timeout_s=60)
        assert r["status"] == 0
        assert r["frames"] == out.shape[0]
        outs[s].append(out)
        results.append(r)
    stats = sv.stats()
    sv.close()
    return [np.concatenate(o) if o else None for o in outs], results, stats


def _one_shot(reqs, precision, streams=STREAMS):
    from paper_2408_16551_amd.pfb import Plan
    ref = []
    for s, (P, M, c) in enumerate(streams):
        xs = [x for t, x in reqs if t == s]
        if not xs:
            ref.append(None)
            continue
        x = np.concatenate(xs)
        plan = Plan(P, M, "c64" if c else "r32", "hann", precision)
        X = plan(torch.from_numpy(x).cuda())
        torch.cuda.synchronize()
        ref.append(X.cpu().numpy())
    return ref


@pytest.mark.parametrize("precision,use_graph", [("fp32", True), ("fp32", False), ("bf16x3", True), ("fp8", True), ("fp8", False)])
def test_server_streams_equal_one_shot_bitwise(precision, use_graph):
    reqs = _workload(seed=1)
    got, results, stats = _serve(reqs, precision, use_graph)
    ref = _one_shot(reqs, precision)
    for g, r in zip(got, ref):
        if r is None:
            continue
        assert g.shape == r.shape
        assert np.array_equal(g, r)
    assert stats["completed"] == len(reqs)
    assert stats["steps"] >= 1
    for r in results:
        assert r["t_submit_us"] <= r["t_admit_us"] <= r["t_done_us"]


FRAME_STREAMS = [(512, 11, True), (1024, 16, True), (512, 8, True), (256, 16, False), (1024, 9, True)]


@pytest.mark.parametrize("precision", ["fp8", "fp16x3"])
def test_server_frame_stage_streams_equal_one_shot_bitwise(precision):
    # 512 frames per step: pieces of 256 frames or more of the 512- and
    # 1024-channel complex streams (frames of 1024 and 2048 floats) take the
    # single-pass frame stage in short units, shorter pieces and the real
    # stream the three FIR launches; every stream equals its one-shot pass.
    g = np.random.Generator(np.random.PCG64(21))
    reqs = []
    for _ in range(16):
        st = int(g.integers(len(FRAME_STREAMS)))
        P = FRAME_STREAMS[st][0]
        reqs.append((st, _rand(P * int(g.integers(200, 900)) + int(g.integers(P)), FRAME_STREAMS[st][2], g)))
    got, results, stats = _serve(reqs, precision, use_graph=False, max_active=4, fps=512, streams=FRAME_STREAMS)
    ref = _one_shot(reqs, precision, streams=FRAME_STREAMS)
    for gg, r in zip(got, ref):
        if r is None:
            continue
        assert gg.shape == r.shape
        assert np.array_equal(gg, r)
    assert stats["completed"] == len(reqs)


FACTORED_STREAMS = [(256, 16, True), (512, 11, True), (256, 16, False), (1024, 9, True), (4096, 8, True)]


@pytest.mark.parametrize("use_graph", [False, True])
def test_server_factored_streams_equal_one_shot_bitwise(use_graph):
    # FP32 server with the factored DFT (steps run as plain launches even when
    # graphs are asked for): each stream's concatenated outputs equal one
    # factored pass over its concatenated input.
    from paper_2408_16551_amd.pfb import Plan, Server
    reqs = _workload(seed=5, n_req=20, streams=FACTORED_STREAMS)
    sv = Server("fp32", max_streams=len(FACTORED_STREAMS), max_active=6, hbm_budget_bytes=1 << 30,
                frames_per_step=32, use_graph=use_graph, max_channels=4096, dft="factored")
    sids = [sv.stream(P, M, "c64" if c else "r32") for P, M, c in FACTORED_STREAMS]
    res = [0] * len(FACTORED_STREAMS)
    pending = []
    for st, x in reqs:
        P = FACTORED_STREAMS[st][0]
        frames = (res[st] + x.size) // P
        res[st] = (res[st] + x.size) % P
        out = np.full((frames, sv.out_rows(sids[st])), np.nan, dtype=np.complex64)
        pending.append((st, sv.submit(sids[st], x, out), out))
    got = [[] for _ in FACTORED_STREAMS]
    for st, rid, out in pending:
        r = sv.wait(rid, timeout_s=60)
        assert r["status"] == 0
        got[st].append(out)
    sv.close()
    for st, (P, M, c) in enumerate(FACTORED_STREAMS):
        xs = [x for t, x in reqs if t == st]
        if not xs:
            continue
        plan = Plan(P, M, "c64" if c else "r32", "hann", "fp32", "pfb", dft="factored")
        ref = plan(torch.from_numpy(np.concatenate(xs)).cuda()).cpu().numpy()
        assert np.array_equal(np.concatenate(got[st]), ref)


def test_server_factored_needs_fp32():
    from paper_2408_16551_amd.pfb import Server, TinaError
    with pytest.raises(TinaError):
        Server("bf16x3", max_streams=1, max_active=1, hbm_budget_bytes=1 << 20, frames_per_step=16,
               max_channels=256, dft="factored")


def test_server_alone_equals_in_mix():
    reqs = _workload(seed=2)
    mixed, _, _ = _serve(reqs, "bf16x3")
    for s in range(len(STREAMS)):
        alone, _, _ = _serve(reqs, "bf16x3", only=s)
        if mixed[s] is None:
            continue
        assert np.array_equal(alone[s], mixed[s])


def test_server_small_budget_forces_admission_waits():
    # Every request needs about the same arena space; the budget holds one
    # request at a time, so the others wait for memory, not for slots.
    g = np.random.Generator(np.random.PCG64(3))
    reqs = [(s, _rand(STREAMS[s][0] * 200 + 11, STREAMS[s][2], g)) for _ in range(3) for s in range(len(STREAMS))]
    need = max(x.nbytes + (x.size // STREAMS[s][0] + 1) * STREAMS[s][0] * 8 for s, x in reqs) + 1024
    got, _, stats = _serve(reqs, "fp32", budget=int(need * 1.5), max_active=8)
    ref = _one_shot(reqs, "fp32")
    for g_, r in zip(got, ref):
        if r is not None:
            assert np.array_equal(g_, r)
    assert stats["admission_waits"] > 0
    assert stats["arena_high_water"] <= int(need * 1.5)
    assert stats["completed"] == len(reqs)


def test_server_fp32_matches_oracle(oracle):
    from oracle import Stream
    streams = [(256, 16, True), (512, 8, False)]
    reqs = _workload(seed=4, n_req=10, streams=streams)
    got, _, _ = _serve(reqs, "fp32", streams=streams)
    for s, (P, M, c) in enumerate(streams):
        if got[s] is None:
            continue
        o = Stream(oracle, P, M, oracle.window(P, M, "hann"), c)
        ref = np.concatenate([o.push(x) for t, x in reqs if t == s])
        err = np.linalg.norm(got[s].astype(np.complex128) - ref) / np.linalg.norm(ref)
        assert err < 1e-5


def test_server_rejects_too_large_and_cancels():
    from paper_2408_16551_amd.pfb import Server, TinaError
    sv = Server("fp32", max_streams=2, max_active=1, hbm_budget_bytes=1 << 20, frames_per_step=16, max_channels=256)
    sid = sv.stream(256, 8, "c64")
    big = np.zeros(1 << 20, dtype=np.complex64)
    with pytest.raises(TinaError) as e:
        sv.submit(sid, big, np.zeros((4096, 256), np.complex64))
    assert e.value.status == 7
    x = np.ones(256 * 10, dtype=np.complex64)
    with pytest.raises(TinaError) as e:
        sv.submit(sid, x, np.zeros((3, 256), np.complex64))   # capacity below 10 frames
    assert e.value.status == 1
    ids = [sv.submit(sid, x, np.zeros((10, 256), np.complex64)) for _ in range(3)]
    cancelled = sv.cancel(ids[-1])
    for rid in ids[:-1]:
        assert sv.wait(rid, timeout_s=60)["status"] == 0
    if cancelled:
        assert sv.wait(ids[-1], timeout_s=60)["status"] == 9
    else:
        assert sv.wait(ids[-1], timeout_s=60)["status"] == 0
    sv.close()


def test_server_device_buffers_equal_one_shot_bitwise():
    # TINA_REQ_DEVICE_BUFFERS: CUDA tensors in and out, used in place; mixed
    # with host requests on other streams.
    from paper_2408_16551_amd.pfb import Server
    reqs = _workload(23, n_req=20)
    ref = _one_shot(reqs, "fp32")
    sv = Server("fp32", max_streams=len(STREAMS), max_active=8, hbm_budget_bytes=1 << 30, frames_per_step=64,
                use_graph=True, max_channels=1024)
    sids = [sv.stream(P, M, "c64" if c else "r32") for P, M, c in STREAMS]
    res = [0] * len(STREAMS)
    pending = []
    for s, x in reqs:
        P = STREAMS[s][0]
        frames = (res[s] + x.size) // P
        res[s] = (res[s] + x.size) % P
        if s % 2 == 0:  # device buffers
            xd = torch.from_numpy(x).cuda()
            out = torch.full((frames, sv.out_rows(sids[s])), float("nan"), dtype=torch.complex64, device="cuda")
            torch.cuda.synchronize()
            pending.append((s, sv.submit(sids[s], xd, out), out))
        else:
            out = np.full((frames, sv.out_rows(sids[s])), np.nan, dtype=np.complex64)
            pending.append((s, sv.submit(sids[s], x, out), out))
    outs = [[] for _ in STREAMS]
    for s, rid, out in pending:
        r = sv.wait(rid, timeout_s=60)
        assert r["status"] == 0 and r["frames"] == out.shape[0]
        outs[s].append(out.cpu().numpy() if hasattr(out, "is_cuda") else out)
    st = sv.stats()
    sv.close()
    for s, r in enumerate(ref):
        if r is None:
            continue
        assert np.array_equal(np.concatenate(outs[s]), r)
    assert st["completed"] == len(reqs)


def test_server_device_request_checks():
    from paper_2408_16551_amd.pfb import Server, TinaError
    sv = Server("fp32", max_streams=1, max_active=2, hbm_budget_bytes=1 << 26, frames_per_step=64,
                use_graph=False, max_channels=256)
    sid = sv.stream(256, 8, "r32")
    x = torch.zeros(256 * 4, device="cuda")
    with pytest.raises(ValueError):  # the binding refuses a host output with a device input
        sv.submit(sid, x, np.zeros((4, 129), dtype=np.complex64))
    out = torch.zeros((4 * 129 + 1,), dtype=torch.complex64, device="cuda")[1:].view(4, 129)  # offset views are fine
    rid = sv.submit(sid, x, out)
    assert sv.wait(rid, timeout_s=30)["status"] == 0
    sv.close()
