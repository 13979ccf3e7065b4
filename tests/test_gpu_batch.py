"""Batched execution (one persistent launch per stage over many ragged
stream chunks): each item equals the single-stream execute of that item bit
for bit (same arithmetic per output element), and the FP32 items match the
FP64 oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rel_l2(got, ref):
    got = np.asarray(got, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def _rand(N, cplx, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    x = g.standard_normal(N)
    if cplx:
        return (x + 1j * g.standard_normal(N)).astype(np.complex64)
    return x.astype(np.float32)


# (P, M, cplx, N): ragged lengths, an empty chunk and a chunk shorter than P.
MIX = [(256, 16, True, 256 * 37 + 5), (1024, 16, True, 1024 * 9), (512, 16, True, 0), (512, 16, True, 300),
       (16, 4, False, 16 * 500 + 3), (1024, 9, False, 1024 * 21 + 1000), (4096, 8, True, 4096 * 6 + 17),
       (64, 13, True, 64 * 333)]


def _items(mix, precision, seed=0):
    from paper_2408_16551_amd.pfb import Plan
    plans, xs, outs = [], [], []
    for i, (P, M, cplx, N) in enumerate(mix):
        plan = Plan(P, M, "c64" if cplx else "r32", "hann", precision)
        x = _rand(N, cplx, seed + i)
        plans.append(plan)
        xs.append(x)
        outs.append(plan.alloc_out(max(1, plan.output_frames(N))))
    return plans, xs, outs


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16x3", "fp8", "bf16", "fp16"])
def test_batch_equals_single_execute_bitwise(precision):
    from paper_2408_16551_amd.pfb import Batch
    plans, xs, outs = _items(MIX, precision)
    xd = [torch.from_numpy(x).cuda() for x in xs]
    b = Batch(precision, max_items=16, workspace_bytes=256 << 20)
    fw = b.execute([(p, x, o) for p, x, o in zip(plans, xd, outs)])
    torch.cuda.synchronize()
    for p, x, o, f in zip(plans, xd, outs, fw):
        single = p(x)
        torch.cuda.synchronize()
        assert f == single.shape[0]
        assert torch.equal(o[:f], single)


# Per-frame scaled forms with long items: those with 1024-, 2048- or 4096-float
# frames run the single-pass frame stage (1, 2 and 4 floats per thread), the
# 256-channel complex item the three FIR launches; all equal the single path.
LONG_MIX = [(512, 16, True, 512 * 3000 + 5), (1024, 9, False, 1024 * 2500), (2048, 8, True, 2048 * 2100 + 3),
            (256, 16, True, 256 * 2500), (1024, 13, True, 1024 * 2049)]


@pytest.mark.parametrize("precision", ["fp8", "fp16", "fp16x3"])
def test_batch_frame_stage_equals_single_execute_bitwise(precision):
    from paper_2408_16551_amd.pfb import Batch
    plans, xs, outs = _items(LONG_MIX, precision, seed=11)
    xd = [torch.from_numpy(x).cuda() for x in xs]
    b = Batch(precision, max_items=8, workspace_bytes=1 << 30)
    fw = b.execute([(p, x, o) for p, x, o in zip(plans, xd, outs)])
    torch.cuda.synchronize()
    for p, x, o, f in zip(plans, xd, outs, fw):
        single = p(x)
        torch.cuda.synchronize()
        assert f == single.shape[0]
        assert torch.equal(o[:f], single)


# Largest tap count 8 with mixed counts: every item runs the ring unrolled for
# its own M (1..8), which must give the single path's bits and the oracle's values.
SMALL_M_MIX = [(64, 3, True, 64 * 90 + 7), (128, 5, False, 128 * 70), (256, 7, True, 256 * 41 + 3),
               (32, 8, False, 32 * 200), (16, 1, True, 16 * 64), (512, 6, False, 512 * 20 + 100)]


@pytest.mark.parametrize("precision", ["fp32", "fp8", "bf16x3"])
def test_batch_small_tap_counts_bitwise_and_oracle(oracle, precision):
    from paper_2408_16551_amd.pfb import Batch
    plans, xs, outs = _items(SMALL_M_MIX, precision, seed=300)
    xd = [torch.from_numpy(x).cuda() for x in xs]
    b = Batch(precision, max_items=16, workspace_bytes=256 << 20)
    fw = b.execute([(p, x, o) for p, x, o in zip(plans, xd, outs)])
    torch.cuda.synchronize()
    for (P, M, cplx, N), p, x, xh, o, f in zip(SMALL_M_MIX, plans, xd, xs, outs, fw):
        single = p(x)
        torch.cuda.synchronize()
        assert f == single.shape[0]
        assert torch.equal(o[:f], single)
        if precision == "fp32":
            ref = oracle.pfb(xh[: (N // P) * P], P, M, oracle.window(P, M, "hann"))
            assert rel_l2(o[:f].cpu().numpy(), ref) < 1e-5


def test_batch_fp32_matches_oracle(oracle):
    from paper_2408_16551_amd.pfb import Batch
    plans, xs, outs = _items(MIX, "fp32", seed=100)
    xd = [torch.from_numpy(x).cuda() for x in xs]
    b = Batch("fp32", max_items=16)
    fw = b.execute([(p, x, o) for p, x, o in zip(plans, xd, outs)])
    torch.cuda.synchronize()
    for (P, M, cplx, N), x, o, f in zip(MIX, xs, outs, fw):
        ref = oracle.pfb(x[: (N // P) * P], P, M, oracle.window(P, M, "hann"))
        assert f == ref.shape[0]
        if f:
            assert rel_l2(o[:f].cpu().numpy(), ref) < 1e-5


def test_batch_small_workspace_runs_in_groups_bitwise():
    from paper_2408_16551_amd.pfb import Batch
    plans, xs, outs = _items(MIX, "fp32", seed=7)
    xd = [torch.from_numpy(x).cuda() for x in xs]
    big = Batch("fp32", max_items=16, workspace_bytes=256 << 20)
    small = Batch("fp32", max_items=16, workspace_bytes=1 << 20)
    outs2 = [torch.empty_like(o) for o in outs]
    fw1 = big.execute([(p, x, o) for p, x, o in zip(plans, xd, outs)])
    fw2 = small.execute([(p, x, o) for p, x, o in zip(plans, xd, outs2)])
    torch.cuda.synchronize()
    assert fw1 == fw2
    for o1, o2, f in zip(outs, outs2, fw1):
        assert torch.equal(o1[:f], o2[:f])


def test_batch_item_larger_than_workspace_is_rejected():
    from paper_2408_16551_amd.pfb import Batch, Plan, TinaError
    plan = Plan(1024, 16, "r32")
    x = torch.zeros(1024 * 1024, device="cuda")
    out = plan.alloc_out(1024)
    b = Batch("fp32", max_items=4, workspace_bytes=1 << 20)
    with pytest.raises(TinaError) as e:
        b.execute([(plan, x, out)])
    assert e.value.status == 7


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp8", "fp16x3"])
def test_batch_with_states_chunked_equals_one_shot(precision):
    # Per-frame scaled forms: items with 1024- or 2048-float frames and at
    # least 2048 frames in a call run the single-pass frame stage (here the
    # 512-channel complex and 1024-channel real items in the larger chunks),
    # the others the three FIR launches.
    from paper_2408_16551_amd.pfb import Batch, State
    mix = [(256, 16, True, 256 * 40 + 77), (512, 11, True, 512 * 6000 + 3), (1024, 16, False, 1024 * 5000 + 500),
           (1024, 13, True, 1024 * 19 + 9)]
    plans, xs, _ = _items(mix, precision, seed=3)
    b = Batch(precision, max_items=8)
    states = [State(p) for p in plans]
    cuts = [0.0, 0.13, 0.5, 0.51, 1.0]
    got = [[] for _ in mix]
    for a, c in zip(cuts[:-1], cuts[1:]):
        items = []
        for i, (p, x) in enumerate(zip(plans, xs)):
            lo, hi = int(a * x.size), int(c * x.size)
            xd = torch.from_numpy(np.ascontiguousarray(x[lo:hi])).cuda()
            out = p.alloc_out(max(1, p.output_frames(hi - lo, states[i])))
            items.append((p, xd, out, states[i]))
        fw = b.execute(items)
        torch.cuda.synchronize()
        for i, (it, f) in enumerate(zip(items, fw)):
            got[i].append(it[2][:f].cpu().numpy())
    for i, (p, x) in enumerate(zip(plans, xs)):
        one = p(torch.from_numpy(x).cuda())
        torch.cuda.synchronize()
        assert np.array_equal(np.concatenate(got[i]), one.cpu().numpy())


# FP32 batches with factored-DFT plans: every channel count the factored DFT
# takes (256..4096), real and complex input (complex 4096 runs the
# register-resident kernel), an empty chunk, a chunk shorter than P, and dense
# FP32 items in the same batch.
FACTORED_MIX = [(256, 16, True, 256 * 37 + 5, "factored"), (512, 11, False, 512 * 60 + 3, "factored"),
                (1024, 16, True, 1024 * 9, "factored"), (2048, 8, False, 2048 * 12 + 100, "factored"),
                (4096, 8, True, 4096 * 6 + 17, "factored"), (512, 16, True, 0, "factored"),
                (1024, 9, False, 300, "factored"), (1024, 16, True, 1024 * 11 + 7, "dense"),
                (256, 16, True, 256 * 20, "factored"), (4096, 4, False, 4096 * 5 + 9, "factored"),
                (4096, 8, True, 4096 * 3, "factored")]


def _factored_items(mix, seed):
    from paper_2408_16551_amd.pfb import Plan
    plans, xs = [], []
    for i, (P, M, cplx, N, dft) in enumerate(mix):
        plans.append(Plan(P, M, "c64" if cplx else "r32", "hann", "fp32", "pfb", dft=dft))
        xs.append(_rand(N, cplx, seed + i))
    return plans, xs


@pytest.mark.parametrize("workspace_mib", [256, 2])
def test_batch_factored_equals_single_execute_bitwise(workspace_mib):
    # 2 MiB of workspace: the items run in several groups, each with its own
    # factored launches.
    from paper_2408_16551_amd.pfb import Batch
    plans, xs = _factored_items(FACTORED_MIX, seed=40)
    xd = [torch.from_numpy(x).cuda() for x in xs]
    outs = [p.alloc_out(max(1, p.output_frames(x.size))) for p, x in zip(plans, xs)]
    b = Batch("fp32", max_items=16, workspace_bytes=workspace_mib << 20)
    fw = b.execute([(p, x, o) for p, x, o in zip(plans, xd, outs)])
    torch.cuda.synchronize()
    for p, x, o, f in zip(plans, xd, outs, fw):
        single = p(x)
        torch.cuda.synchronize()
        assert f == single.shape[0]
        assert torch.equal(o[:f], single)


def test_batch_factored_matches_oracle(oracle):
    from paper_2408_16551_amd.pfb import Batch
    mix = [(512, 16, True, 512 * 40 + 9, "factored"), (4096, 8, True, 4096 * 10, "factored"),
           (1024, 16, False, 1024 * 30 + 5, "factored")]
    plans, xs = _factored_items(mix, seed=50)
    xd = [torch.from_numpy(x).cuda() for x in xs]
    outs = [p.alloc_out(max(1, p.output_frames(x.size))) for p, x in zip(plans, xs)]
    fw = Batch("fp32", max_items=4).execute([(p, x, o) for p, x, o in zip(plans, xd, outs)])
    torch.cuda.synchronize()
    for (P, M, cplx, N, _), x, o, f in zip(mix, xs, outs, fw):
        h = oracle.window(P, M, "hann")
        n = (N // P) * P
        ref = oracle.pfb(x[:n], P, M, h)
        assert rel_l2(o[:f].cpu().numpy(), ref) < 1e-5


def test_batch_factored_with_states_chunked_equals_one_shot():
    from paper_2408_16551_amd.pfb import Batch, State
    mix = [(256, 16, True, 256 * 40 + 77, "factored"), (4096, 8, True, 4096 * 30 + 3, "factored"),
           (1024, 13, False, 1024 * 50 + 500, "factored"), (1024, 16, True, 1024 * 19 + 9, "dense")]
    plans, xs = _factored_items(mix, seed=60)
    b = Batch("fp32", max_items=8)
    states = [State(p) for p in plans]
    cuts = [0.0, 0.13, 0.5, 0.51, 1.0]
    got = [[] for _ in mix]
    for a, c in zip(cuts[:-1], cuts[1:]):
        items = []
        for i, (p, x) in enumerate(zip(plans, xs)):
            lo, hi = int(a * x.size), int(c * x.size)
            xdc = torch.from_numpy(np.ascontiguousarray(x[lo:hi])).cuda()
            out = p.alloc_out(max(1, p.output_frames(hi - lo, states[i])))
            items.append((p, xdc, out, states[i]))
        fw = b.execute(items)
        torch.cuda.synchronize()
        for i, (it, f) in enumerate(zip(items, fw)):
            got[i].append(it[2][:f].cpu().numpy())
    for i, (p, x) in enumerate(zip(plans, xs)):
        one = p(torch.from_numpy(x).cuda())
        torch.cuda.synchronize()
        assert np.array_equal(np.concatenate(got[i]), one.cpu().numpy())


def test_batch_rejects_compensated_plans():
    from paper_2408_16551_amd.pfb import Batch, Plan, TinaError
    p = Plan(256, 8, "c64", "hann", "fp32", "pfb", dft="compensated")
    x = torch.from_numpy(_rand(256 * 10, True, 1)).cuda()
    o = p.alloc_out(10)
    with pytest.raises(TinaError):
        Batch("fp32", max_items=2).execute([(p, x, o)])


def test_batch_tune_then_execute_bitwise():
    from paper_2408_16551_amd.pfb import Batch
    plans, xs, outs = _items(MIX[:5], "fp32", seed=11)
    xd = [torch.from_numpy(x).cuda() for x in xs]
    b = Batch("fp32", max_items=8)
    tf, tile_n = b.tune([(p, x, o) for p, x, o in zip(plans, xd, outs)])
    assert tf in (1, 2, 4) and tile_n in (128, 256)
    fw = b.execute([(p, x, o) for p, x, o in zip(plans, xd, outs)])
    torch.cuda.synchronize()
    for p, x, o, f in zip(plans, xd, outs, fw):
        assert torch.equal(o[:f], p(x))
