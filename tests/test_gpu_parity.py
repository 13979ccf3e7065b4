"""Parity of the HIP filter bank (through the C ABI) with the FP64 oracle.

Bars: FIR-only and the FP32 filter bank within 1e-5 relative L2 of the
oracle (FP64, over every real and imaginary value of every frame); each
reduced-precision form within its stated bound (REDUCED_BOUNDS, the measured
error rounded up); bit-exact where the arithmetic is exact (impulse -> taps,
chunked == one-shot on the same kernels)."""
import numpy as np
import pytest

from paper_2408_16551_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FP32_BOUND = 1e-5
# Relative-L2 bounds of the reduced forms vs the FP64 oracle: the measured error
# rounded up (the error model: unit roundoff of the operand format per operand).
# Split bf16 (hi*hi + hi*lo + lo*hi) is held to 1e-5, the bar at which it must
# beat plain FP32 on speed (measured 3.9e-6 on both workload shapes).
REDUCED_BOUNDS = {"bf16": 8e-3, "bf16x3": 1e-5, "fp16": 1e-3, "fp16x3": 1e-6, "fp8": 0.1, "mxfp8": 0.05}


def rel_l2(got, ref):
    got = np.asarray(got, dtype=np.complex128 if np.iscomplexobj(got) else np.float64)
    ref = np.asarray(ref, dtype=np.complex128 if np.iscomplexobj(ref) else np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / (den if den > 0 else 1.0))


def _plan(P, M, cplx, window="hann", precision="fp32", output="pfb", custom=None):
    from paper_2408_16551_amd.pfb import Plan
    return Plan(P, M, "c64" if cplx else "r32", window if custom is None else "custom", precision, output,
                custom_taps=custom)


def _rand(N, cplx, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    x = g.standard_normal(N)
    if cplx:
        x = x + 1j * g.standard_normal(N)
        return x.astype(np.complex64)
    return x.astype(np.float32)


def _dev(x):
    return torch.from_numpy(x).cuda()


def _run(plan, x, state=None):
    out = plan(_dev(x), state=state)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("window", ["rect", "hann", "hamming", "blackman"])
@pytest.mark.parametrize("P,M", [(16, 4), (1024, 16), (4096, 8)])
def test_taps_match_oracle(oracle, P, M, window):
    plan = _plan(P, M, False, window=window, output="fir")
    assert np.max(np.abs(plan.taps() - oracle.window(P, M, window))) < 1e-14


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("P,M,f0,p0", [(16, 4, 0, 5), (64, 7, 3, 63), (1024, 16, 20, 517)])
def test_fir_impulse_gives_fp32_taps_exactly(oracle, P, M, f0, p0, cplx):
    plan = _plan(P, M, cplx, output="fir")
    F = f0 + M + 5
    x = np.zeros(F * P, dtype=np.complex64 if cplx else np.float32)
    x[f0 * P + p0] = 1.0
    y = _run(plan, x)
    h32 = oracle.window(P, M, "hann").astype(np.float32)
    ref = np.zeros((F, P), dtype=x.dtype)
    for f in range(f0, f0 + M):
        ref[f, p0] = h32[(M - 1 - (f - f0)) * P + p0]
    assert np.array_equal(y, ref)


FIR_SHAPES = [(16, 4, 1 << 16, False), (64, 5, 64 * 37 + 11, True), (1024, 16, 1024 * 40 + 3, False),
              (256, 17, 256 * 50 + 100, True), (16, 33, 16 * 90 + 1, False), (32, 64, 32 * 140, True),
              (16, 1, 16 * 20, False), (4096, 8, 4096 * 20 + 4095, True), (128, 3, 127, False),
              (128, 12, 128 * 60 + 5, True), (512, 15, 512 * 33, False)]


@pytest.mark.parametrize("P,M,N,cplx", FIR_SHAPES)
def test_fir_only_matches_oracle(oracle, P, M, N, cplx):
    x = _rand(N, cplx, seed=P + M + N)
    h = oracle.window(P, M, "hann")
    plan = _plan(P, M, cplx, output="fir")
    y = _run(plan, x)
    ref = oracle.fir(x[: (N // P) * P], P, M, h)
    assert y.shape == ref.shape
    if ref.size:
        assert rel_l2(y, ref) < FP32_BOUND


PFB_SHAPES = [(16, 4, 1 << 16, False, "hann"), (64, 5, 64 * 300 + 11, True, "hamming"),
              (1024, 16, 1024 * 300 + 77, False, "hann"), (256, 16, 256 * 260 + 5, True, "hann"),
              (4096, 8, 4096 * 140 + 1000, True, "blackman"), (32, 33, 32 * 200, False, "blackman"),
              (16, 1, 16 * 130, True, "rect"), (8192, 2, 8192 * 20, False, "hann"),
              (2048, 64, 2048 * 70, True, "hann"), (512, 11, 512 * 90 + 7, False, "hamming")]


@pytest.mark.parametrize("P,M,N,cplx,window", PFB_SHAPES)
def test_pfb_fp32_matches_oracle(oracle, P, M, N, cplx, window):
    x = _rand(N, cplx, seed=3 * P + M)
    h = oracle.window(P, M, window)
    plan = _plan(P, M, cplx, window=window)
    X = _run(plan, x)
    ref = oracle.pfb(x[: (N // P) * P], P, M, h)
    err = rel_l2(X, ref)
    print(f"pfb fp32 P={P} M={M} N={N} cplx={cplx}: rel_l2={err:.3e}")
    assert err < FP32_BOUND
    if not cplx:
        assert np.all(X[:, 0].imag == 0) and np.all(X[:, -1].imag == 0)


def test_small_pfb_workload_fp32(oracle):
    w = workloads.small_pfb()
    plan = _plan(w.P, w.M, False)
    X = _run(plan, w.x)
    ref = oracle.pfb(w.x, w.P, w.M, oracle.window(w.P, w.M, w.window))
    assert rel_l2(X, ref) < FP32_BOUND
    # the three channel-centre tones stand out in their channels after warm-up
    ks = [int(round(f * w.P)) for f, _, _ in w.tones]
    power = np.mean(np.abs(X[w.M:]) ** 2, axis=0)
    assert set(np.argsort(power)[-3:]) == set(ks)


@pytest.mark.parametrize("precision", ["bf16", "bf16x3", "fp16", "fp16x3", "fp8"])
@pytest.mark.parametrize("P,M,N,cplx,window", [(4096, 8, 4096 * 150 + 9, True, "blackman"),
                                                (1024, 16, 1024 * 300, False, "hann")])
def test_pfb_reduced_precision_within_stated_bound(oracle, P, M, N, cplx, window, precision):
    x = _rand(N, cplx, seed=11 * P + M)
    X = _run(_plan(P, M, cplx, window=window, precision=precision), x)
    ref = _oracle_pfb(oracle, x, P, M, window, ("reduced", P, M, N, cplx))
    err = rel_l2(X, ref)
    print(f"pfb {precision} P={P} M={M} cplx={cplx}: rel_l2={err:.3e}")
    assert err < REDUCED_BOUNDS[precision]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp8", "fp16", "fp16x3"])
@pytest.mark.parametrize("P,M,cplx", [(16, 4, False), (1024, 16, True), (64, 9, False)])
def test_streaming_chunked_equals_one_shot_bitwise(oracle, P, M, cplx, precision):
    from paper_2408_16551_amd.pfb import State
    N = P * 70 + P // 2 + 3
    x = _rand(N, cplx, seed=5 * P + M)
    plan = _plan(P, M, cplx, precision=precision)
    one = _run(plan, x)
    st = State(plan)
    cuts = [0, 1, 1, P // 3, P * 3 + 7, P * 40 + 1, N]
    parts = [_run(plan, np.ascontiguousarray(x[a:b]), state=st) for a, b in zip(cuts[:-1], cuts[1:])]
    got = np.concatenate(parts)
    assert got.shape == one.shape
    assert np.array_equal(got, one)
    assert st.size()[1] == N % P
    if precision == "fp32":
        from oracle import Stream
        s = Stream(oracle, P, M, oracle.window(P, M, "hann"), cplx)
        ref = np.concatenate([s.push(x[a:b]) for a, b in zip(cuts[:-1], cuts[1:])])
        assert rel_l2(got, ref) < FP32_BOUND


@pytest.mark.parametrize("precision", ["fp8", "fp16", "fp16x3"])
@pytest.mark.parametrize("cplx", [False, True])
def test_per_frame_scale_follows_each_frame(oracle, precision, cplx):
    # Blocks of frames at scales 40 decades apart, and all-zero blocks: each
    # frame takes its own power-of-two scale, so every block keeps the form's
    # relative error, and frames whose whole window is zero come out exactly
    # zero (a zero maximum takes exponent 0).
    P, M, B = 256, 8, 24                     # channels, taps, frames per block
    scales = [1.0, 0.0, 1e-20, 1e20, 3e-5, 0.0, 7e10, 1.0]
    g = np.random.Generator(np.random.PCG64(77))
    x = np.concatenate([s * g.standard_normal(P * B) for s in scales])
    if cplx:
        x = x + 1j * np.concatenate([s * g.standard_normal(P * B) for s in scales])
        x = x.astype(np.complex64)
    else:
        x = x.astype(np.float32)
    plan = _plan(P, M, cplx, precision=precision)
    got = _run(plan, x)
    ref = oracle.pfb(x, P, M, oracle.window(P, M, "hann"))
    bound = {"fp8": 0.1, "fp16": 1e-3, "fp16x3": 2e-6}[precision]
    for b, s in enumerate(scales):
        rows = slice(b * B + M - 1, (b + 1) * B)   # frames whose window lies in block b
        if s == 0.0:
            assert np.all(got[rows] == 0)
        else:
            assert rel_l2(got[rows], ref[rows]) < bound, (b, s)


@pytest.mark.parametrize("cplx", [False, True])
def test_streaming_fir_only_matches_oracle_stream(oracle, cplx):
    from oracle import Stream
    from paper_2408_16551_amd.pfb import State
    P, M = 256, 12
    N = P * 33 + 19
    x = _rand(N, cplx, seed=77)
    plan = _plan(P, M, cplx, output="fir")
    st = State(plan)
    s = Stream(oracle, P, M, oracle.window(P, M, "hann"), cplx, fir_only=True)
    cuts = [0, 5, P * 4 + 1, P * 4 + 2, P * 20, N]
    for a, b in zip(cuts[:-1], cuts[1:]):
        got = _run(plan, np.ascontiguousarray(x[a:b]), state=st)
        ref = s.push(x[a:b])
        assert got.shape == ref.shape
        if ref.size:
            assert rel_l2(got, ref) < FP32_BOUND


def test_state_export_import_resumes_bitwise():
    from paper_2408_16551_amd.pfb import State
    P, M = 512, 10
    x = _rand(P * 60 + 100, True, seed=9)
    plan = _plan(P, M, True)
    a = State(plan)
    _run(plan, x[: P * 25 + 37], state=a)
    saved = a.export()
    assert saved.size == (M - 1) * P + 37
    tail_a = _run(plan, np.ascontiguousarray(x[P * 25 + 37:]), state=a)
    b = State(plan)
    b.load_from(saved)
    tail_b = _run(plan, np.ascontiguousarray(x[P * 25 + 37:]), state=b)
    assert np.array_equal(tail_a, tail_b)
    b.reset()
    assert b.size() == ((M - 1) * P, 0)


def test_empty_and_short_inputs():
    from paper_2408_16551_amd.pfb import State
    plan = _plan(64, 4, False)
    assert _run(plan, np.zeros(0, np.float32)).shape == (0, 33)
    assert _run(plan, np.ones(63, np.float32)).shape == (0, 33)
    st = State(plan)
    assert _run(plan, np.ones(40, np.float32), state=st).shape == (0, 33)
    assert _run(plan, np.ones(40, np.float32), state=st).shape == (1, 33)
    assert st.size()[1] == 16


def test_capacity_too_small_is_rejected_without_writes():
    import ctypes
    from paper_2408_16551_amd import pfb
    plan = _plan(64, 4, False)
    x = _dev(_rand(64 * 10, False, 1))
    out = torch.full((5, 33), 7.0 + 7.0j, dtype=torch.complex64, device="cuda")
    fw = ctypes.c_int64(-1)
    st = pfb.load().tina_pfb_execute(plan.handle, ctypes.c_void_p(x.data_ptr()), 640,
                                     ctypes.c_void_p(out.data_ptr()), 5, None, ctypes.byref(fw), None)
    torch.cuda.synchronize()
    assert st == 1 and b"capacity" in pfb.load().tina_last_error()
    assert torch.all(out == 7.0 + 7.0j)


_ORACLE_CACHE = {}


def _oracle_pfb(oracle, x, P, M, window, key):
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = oracle.pfb(x[: (x.size // P) * P], P, M, oracle.window(P, M, window))
    return _ORACLE_CACHE[key]


@pytest.fixture(scope="module")
def real_stream_wl():
    return workloads.real_stream()


@pytest.fixture(scope="module")
def wide_wl():
    return workloads.wide_dynamic_range()


def _sample_frames(F, M, n_extra, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    fr = set(range(min(F, M + 1))) | {F - 1, F - 2}
    fr |= set(g.choice(F, size=min(F, n_extra), replace=False).tolist())
    return np.array(sorted(fr), dtype=np.int64)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_full_size_real_stream_sampled(oracle, real_stream_wl, precision):
    w = real_stream_wl
    plan = _plan(w.P, w.M, False, precision=precision)
    xd = _dev(w.x)
    X = plan(xd)
    torch.cuda.synchronize()
    F = w.x.size // w.P
    assert X.shape == (F, w.P // 2 + 1)
    fr = _sample_frames(F, w.M, 48, seed=1)
    got = X[torch.from_numpy(fr).cuda()].cpu().numpy()
    key = ("real", fr.tobytes())
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = oracle.pfb(w.x, w.P, w.M, oracle.window(w.P, w.M, w.window), frames=fr)
    err = rel_l2(got, _ORACLE_CACHE[key])
    print(f"real stream {precision}: rel_l2={err:.3e}")
    assert err < (FP32_BOUND if precision == "fp32" else REDUCED_BOUNDS[precision])


# Worst channel's relative L2 error on the 60 dB workload (4096 complex
# channels, sampled frames past the warm-up).  Its noise-only channels lie
# about 120 dB (a power ratio near 1e12) below the strongest tone's channel, so
# an error floor relative to the strongest channel shows there magnified about
# 1e6: the reduced operand forms' rounding of the FIR output, and in FP32 the
# accumulation over K of a row whose partial sums carry the strong tone.
# Bounds: the measured worst channel rounded up by half.  Compensated
# accumulation (error-free two-sum per K tile) brings FP32 under 1e-2.
WORST_CHANNEL_BOUNDS = {"fp32": 0.16, "fp32/factored": 0.11, "fp32/compensated": 1e-2, "fp32/table": 0.16, "bf16": 180.0,
                        "bf16x3": 0.37, "fp16": 28.0, "fp16x3": 0.06, "fp8": 5800.0, "mxfp8": 5800.0}


def worst_channel(got, ref, fr, M):
    keep = fr >= M - 1
    g = np.asarray(got, dtype=np.complex128)[keep]
    r = np.asarray(ref, dtype=np.complex128)[keep]
    num = np.sqrt((np.abs(g - r) ** 2).sum(axis=0))
    den = np.sqrt((np.abs(r) ** 2).sum(axis=0))
    ratio = num / den
    return float(ratio.max()), int(ratio.argmax())


@pytest.mark.parametrize("entry", list(WORST_CHANNEL_BOUNDS))
def test_full_size_wide_dynamic_range_sampled(oracle, entry, wide_wl):
    from paper_2408_16551_amd.pfb import Plan
    w = wide_wl
    precision, dft = (entry.split("/") + ["dense"])[:2]
    print(f"wide dynamic range: {entry} P={w.P} M={w.M} N={w.x.size}", flush=True)
    plan = Plan(w.P, w.M, "c64", w.window, precision, dft=dft)
    X = plan(_dev(w.x))
    torch.cuda.synchronize()
    F = w.x.size // w.P
    fr = _sample_frames(F, w.M, 24, seed=2)
    got = X[torch.from_numpy(fr).cuda()].cpu().numpy()
    plan.close()
    key = ("wide", fr.tobytes())
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = oracle.pfb(w.x, w.P, w.M, oracle.window(w.P, w.M, w.window), frames=fr)
    ref = _ORACLE_CACHE[key]
    err = rel_l2(got, ref)
    wc, k = worst_channel(got, ref, fr, w.M)
    print(f"wide dynamic range {entry}: rel_l2={err:.3e} worst channel {k}: {wc:.3e}")
    assert err < (FP32_BOUND if precision == "fp32" else REDUCED_BOUNDS[precision])
    assert wc < WORST_CHANNEL_BOUNDS[entry]


# ---------------------------------------------------------------- factored DFT
@pytest.mark.parametrize("P,M,cplx,frames", [(256, 8, True, 130), (512, 11, False, 75), (1024, 16, False, 200),
                                              (1024, 16, True, 61), (2048, 5, True, 33), (4096, 8, True, 70),
                                              (4096, 3, False, 40)])
def test_factored_dft_matches_oracle(oracle, P, M, cplx, frames):
    from paper_2408_16551_amd.pfb import Plan
    N = P * frames + P // 3
    x = _rand(N, cplx, seed=17 * P + M)
    plan = Plan(P, M, "c64" if cplx else "r32", "hann", "fp32", dft="factored")
    X = _run(plan, x)
    ref = oracle.pfb(x[: (N // P) * P], P, M, oracle.window(P, M, "hann"))
    err = rel_l2(X, ref)
    print(f"factored P={P} M={M} cplx={cplx}: rel_l2={err:.3e}")
    assert err < FP32_BOUND
    if not cplx:
        assert np.all(X[:, 0].imag == 0) and np.all(X[:, -1].imag == 0)


@pytest.mark.parametrize("P,M", [(1024, 12), (4096, 8)])
def test_factored_dft_streaming_bitwise(P, M):
    from paper_2408_16551_amd.pfb import Plan, State
    N = P * 90 + 77
    x = _rand(N, True, seed=5)
    plan = Plan(P, M, "c64", "hann", "fp32", dft="factored")
    one = _run(plan, x)
    st = State(plan)
    cuts = [0, 500, P * 7, P * 50 + 3, N]
    got = np.concatenate([_run(plan, np.ascontiguousarray(x[a:b]), state=st) for a, b in zip(cuts[:-1], cuts[1:])])
    assert np.array_equal(got, one)


def test_factored_rejects_unsupported():
    from paper_2408_16551_amd.pfb import Plan, TinaError
    for kw in [dict(channels=8192, precision="fp32"), dict(channels=1024, precision="bf16x3"),
               dict(channels=128, precision="fp32")]:
        with pytest.raises(TinaError) as e:
            Plan(kw["channels"], 8, "c64", "hann", kw["precision"], dft="factored")
        assert e.value.status == 2


# ------------------------------------------------- compensated accumulation
@pytest.mark.parametrize("P,M,cplx,frames", [(64, 4, True, 300), (256, 8, True, 130), (1024, 16, False, 200),
                                              (1024, 16, True, 61), (4096, 8, True, 40), (8192, 2, False, 9)])
def test_compensated_dft_matches_oracle(oracle, P, M, cplx, frames):
    from paper_2408_16551_amd.pfb import Plan
    N = P * frames + P // 3
    x = _rand(N, cplx, seed=23 * P + M)
    print(f"compensated P={P} M={M} cplx={cplx} frames={frames}", flush=True)
    plan = Plan(P, M, "c64" if cplx else "r32", "hann", "fp32", dft="compensated")
    X = _run(plan, x)
    ref = oracle.pfb(x[: (N // P) * P], P, M, oracle.window(P, M, "hann"))
    err = rel_l2(X, ref)
    print(f"compensated P={P} M={M} cplx={cplx}: rel_l2={err:.3e}")
    assert err < FP32_BOUND / 4   # below the dense FP32 product's error
    if not cplx:
        assert np.all(X[:, 0].imag == 0) and np.all(X[:, -1].imag == 0)


def test_compensated_streaming_bitwise_and_rejects_reduced_forms():
    from paper_2408_16551_amd.pfb import Plan, State, TinaError
    P, M = 512, 12
    N = P * 300 + 77
    x = _rand(N, True, seed=9)
    plan = Plan(P, M, "c64", "hann", "fp32", dft="compensated")
    one = _run(plan, x)
    st = State(plan)
    cuts = [0, 500, P * 7, P * 150 + 3, N]
    got = np.concatenate([_run(plan, np.ascontiguousarray(x[a:b]), state=st) for a, b in zip(cuts[:-1], cuts[1:])])
    assert np.array_equal(got, one)
    with pytest.raises(TinaError) as e:
        Plan(P, M, "c64", "hann", "bf16x3", dft="compensated")
    assert e.value.status == 2


# ------------------------------------------ operand assembled from a twiddle table
# The table holds the operand's own FP32 entries (cos, sin of 2 pi r / P), so
# the product is bit for bit the dense one; covered: real and complex input,
# P from 16 to 8192 (one block per CU when the table takes 32 KiB or more),
# ragged frame counts and partial tiles.
@pytest.mark.parametrize("P,M,cplx,frames", [(16, 4, False, 700), (64, 4, True, 300), (256, 8, True, 130),
                                              (1024, 16, False, 200), (1024, 16, True, 61), (4096, 8, True, 40),
                                              (8192, 2, False, 9), (2048, 5, True, 33)])
def test_table_operand_equals_dense_bitwise_and_matches_oracle(oracle, P, M, cplx, frames):
    from paper_2408_16551_amd.pfb import Plan
    N = P * frames + P // 3
    x = _rand(N, cplx, seed=31 * P + M)
    print(f"table operand P={P} M={M} cplx={cplx} frames={frames}", flush=True)
    dense = _run(Plan(P, M, "c64" if cplx else "r32", "hann", "fp32"), x)
    X = _run(Plan(P, M, "c64" if cplx else "r32", "hann", "fp32", dft="table"), x)
    assert np.array_equal(X, dense)
    ref = oracle.pfb(x[: (N // P) * P], P, M, oracle.window(P, M, "hann"))
    assert rel_l2(X, ref) < FP32_BOUND


def test_table_operand_streaming_bitwise_and_rejects_reduced_forms():
    from paper_2408_16551_amd.pfb import Plan, State, TinaError
    P, M = 512, 12
    N = P * 300 + 77
    x = _rand(N, True, seed=10)
    plan = Plan(P, M, "c64", "hann", "fp32", dft="table")
    one = _run(plan, x)
    st = State(plan)
    cuts = [0, 500, P * 7, P * 150 + 3, N]
    got = np.concatenate([_run(plan, np.ascontiguousarray(x[a:b]), state=st) for a, b in zip(cuts[:-1], cuts[1:])])
    assert np.array_equal(got, one)
    with pytest.raises(TinaError) as e:
        Plan(P, M, "c64", "hann", "bf16", dft="table")
    assert e.value.status == 2


# ------------------------------------------------------- synthesis (inverse) bank
@pytest.mark.parametrize("P,M,F,precision", [(64, 5, 120, "fp32"), (1024, 16, 70, "fp32"), (4096, 8, 30, "fp32"),
                                             (256, 12, 200, "bf16x3"), (512, 1, 50, "fp32")])
def test_synthesis_matches_oracle(oracle, P, M, F, precision):
    from paper_2408_16551_amd.pfb import Plan
    g = np.random.Generator(np.random.PCG64(P + M))
    X = (g.standard_normal((F, P)) + 1j * g.standard_normal((F, P))).astype(np.complex64)
    plan = Plan(P, M, "c64", "hann", precision, "inverse")
    xh = plan.synthesize(torch.from_numpy(X).cuda())
    torch.cuda.synchronize()
    ref = oracle.synthesize(X, P, M, oracle.window(P, M, "hann"))
    err = rel_l2(xh.cpu().numpy(), ref)
    print(f"synthesis {precision} P={P} M={M}: rel_l2={err:.3e}")
    assert err < (FP32_BOUND if precision == "fp32" else REDUCED_BOUNDS[precision])


def test_analysis_then_synthesis_unit_bank_reconstructs():
    from paper_2408_16551_amd.pfb import Plan
    P = 256
    x = _rand(P * 100, True, seed=31)
    ana = Plan(P, 1, "c64", "custom", "fp32", custom_taps=np.ones(P))
    syn = Plan(P, 1, "c64", "custom", "fp32", "inverse", custom_taps=np.ones(P))
    X = ana(_dev(x))
    xh = syn.synthesize(X).cpu().numpy()
    assert rel_l2(xh, x) < 1e-6


def test_synthesis_streaming_and_pieces_bitwise():
    from paper_2408_16551_amd.pfb import Plan, State
    P, M, F = 128, 7, 300
    g = np.random.Generator(np.random.PCG64(8))
    X = (g.standard_normal((F, P)) + 1j * g.standard_normal((F, P))).astype(np.complex64)
    Xd = torch.from_numpy(X).cuda()
    plan = Plan(P, M, "c64", "hann", "fp32", "inverse")
    one = plan.synthesize(Xd).cpu().numpy()
    # a small workspace forces several pieces inside one call
    small = Plan(P, M, "c64", "hann", "fp32", "inverse", workspace_bytes=128 * 2 * P * 4 // 2)
    assert np.array_equal(small.synthesize(Xd).cpu().numpy(), one)
    st = State(plan)
    parts = [plan.synthesize(Xd[a:b].contiguous(), state=st).cpu().numpy()
             for a, b in [(0, 1), (1, 50), (50, 51), (51, 300)]]
    assert np.array_equal(np.concatenate(parts), one)
