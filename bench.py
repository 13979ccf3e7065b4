#!/usr/bin/env python3
"""Throughput benchmark of the MI355X filter bank.

One step = one tina_pfb_execute over the whole real stream (1024 channels,
16 taps, sinc x Hann, 2^26 float32 samples, noise + 8 tones, DFT as FP32
GEMM): the polyphase FIR kernel then the DFT-GEMM kernel, input resident in
HBM.  Prints ONE JSON line with the throughput (input GSamples/s), the
roofline of the dominant kernel (HIP events on the launch stream, inside the
timed region), the other precision forms with their error against the FP64
oracle, and the oracle itself timed on the host cores on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "bf16x3": 2500.0, "fp16": 2500.0, "fp16x3": 2500.0, "fp8": 5000.0,
               "mxfp8": 5000.0}
PEAK_HBM_GBS = 8000.0
MFMA_FLOP_MULT = {"fp32": 1, "bf16": 1, "fp16": 1, "bf16x3": 3, "fp16x3": 3, "fp8": 1, "mxfp8": 1}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_l2(got, ref):
    got = np.asarray(got, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def dft_flops_per_frame(P: int, cplx: bool) -> float:
    """Algorithmic flops of the dense DFT of one frame as the GEMM computes it:
    real frame P x P real products (the two identically-zero imaginary
    channels excluded), complex frame 2P x 2P."""
    return 2.0 * (2 * P) * (2 * P) if cplx else 2.0 * P * P


def source_digest() -> str:
    h = hashlib.sha256()
    for f in ("paper_2408_16551_amd/csrc/gemm.hip", "paper_2408_16551_amd/csrc/internal.h"):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def read_traffic(workload: str):
    """HBM bytes per DFT-GEMM launch from the committed rocprofv3 counter
    summary, or None if it is missing or was taken on other kernel source."""
    path = os.path.join(ROOT, "profiles", f"dft_gemm_fp32_{workload}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#") and "=" in line:
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_digest") != source_digest():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def timed_steps(plan, xd, out, steps, warmup, torch):
    for _ in range(warmup):
        plan(xd, out=out)
    torch.cuda.synchronize()
    plan.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan(xd, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fir_ms, nf, dft_ms, nd = plan.profile_read()
    plan.profile(False)
    return (t1 - t0) / steps, fir_ms / max(nf, 1), dft_ms / max(nd, 1)


def sampled_frames(F, M, n, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    fr = set(range(min(F, M + 1))) | {F - 1}
    fr |= set(g.choice(F, size=min(F, n), replace=False).tolist())
    return np.array(sorted(fr), dtype=np.int64)


FIR_OUT_BYTES = {"fp32": 4.0, "bf16": 2.0, "bf16x3": 4.0, "fp16": 2.0, "fp16x3": 4.0, "fp8": 1.0,
                 "mxfp8": 1.0 + 1.0 / 32}


def channel_errors(got, ref, w, fr):
    """Relative L2 error of each channel over the sampled frames past the
    warm-up: the worst channel, and the channel of the weakest tone placed at
    a channel centre (the error a strong tone leaves on a faint one)."""
    keep = fr >= w.M - 1
    g = np.asarray(got, dtype=np.complex128)[keep]
    r = np.asarray(ref, dtype=np.complex128)[keep]
    num = np.sqrt((np.abs(g - r) ** 2).sum(axis=0))
    den = np.sqrt((np.abs(r) ** 2).sum(axis=0))
    ratio = num / np.maximum(den, np.finfo(np.float64).tiny)
    res = {"worst_channel_rel_l2": float(f"{ratio.max():.3e}")}
    centre = [(f, a) for f, a, _ in w.tones if abs(f * w.P - round(f * w.P)) < 1e-9]
    if centre:
        f, a = min(centre, key=lambda t: t[1])
        k = int(round(f * w.P)) % w.P
        if k < ratio.size:
            res["weakest_tone"] = {"channel": k, "amplitude": a, "rel_l2": float(f"{ratio[k]:.3e}")}
    return res


def forms_table(w, forms, steps, warmup, torch, oracle_obj, n_frames_err):
    """Throughput and error of each precision form on workload w."""
    from paper_2408_16551_amd.pfb import Plan
    xd = torch.from_numpy(w.x).cuda()
    N = w.x.size
    F = N // w.P
    fr = sampled_frames(F, w.M, n_frames_err, seed=7)
    ref = oracle_obj.pfb(w.x, w.P, w.M, oracle_obj.window(w.P, w.M, w.window), frames=fr)
    res = {}
    for entry in forms:
        form, dft = (entry.split("/") + ["dense"])[:2]
        plan = Plan(w.P, w.M, "c64" if w.complex_input else "r32", w.window, form, "pfb", dft=dft)
        out = plan.alloc_out(F)
        sec, fir_ms, dft_ms = timed_steps(plan, xd, out, steps, warmup, torch)
        got = out[torch.from_numpy(fr).cuda()].cpu().numpy()
        flops = dft_flops_per_frame(w.P, w.complex_input) * F
        res[entry] = {
            "gsps": round(N / sec / 1e9, 3),
            "ms_per_step": round(sec * 1e3, 4),
            "rel_l2_vs_fp64_oracle": float(f"{rel_l2(got, ref):.3e}"),
            "dft_ms": round(dft_ms, 4), "fir_ms": round(fir_ms, 4),
            "dft_useful_tflops": round(flops / (dft_ms * 1e-3) / 1e12, 2),
            "dft_mfma_frac": round(flops * MFMA_FLOP_MULT[form] / (dft_ms * 1e-3) / 1e12 / PEAK_TFLOPS[form], 4),
        }
        res[entry].update(channel_errors(got, ref, w, fr))
        # FIR stage bytes: FP32 input once, and the GEMM operand it writes per
        # float (FP32 rows, or the reduced form's codes; the per-frame scaled
        # forms' second input pass is not counted: it is not algorithmic).
        fir_out_b = FIR_OUT_BYTES[form]
        fir_b = F * w.P * (2 if w.complex_input else 1) * (4.0 + fir_out_b)
        res[entry]["fir_hbm_gbs"] = round(fir_b / (fir_ms * 1e-3) / 1e9, 1)
        if dft == "factored":   # the dense-DFT flop figures do not apply
            P1 = 1 << ((int(np.log2(w.P)) + 1) // 2)
            f_fact = 8.0 * w.P * (P1 + w.P // P1) * F
            res[entry]["dft_useful_tflops"] = round(f_fact / (dft_ms * 1e-3) / 1e12, 2)
            res[entry]["dft_mfma_frac"] = round(f_fact / (dft_ms * 1e-3) / 1e12 / PEAK_TFLOPS["fp32"], 4)
            res[entry]["dft_bytes_gbs"] = round((4.0 * F * w.P * (2 if w.complex_input else 1)
                                                 + 8.0 * F * (w.P if w.complex_input else w.P // 2 + 1))
                                                / (dft_ms * 1e-3) / 1e9, 1)
        log(f"[bench] {w.name} {entry}: {res[entry]}")
        plan.close()
        del out
    return res


def cpu_baseline(w, target_s=12.0):
    """The FP64 oracle on the host cores, on a bounded sample of frames."""
    from oracle import Oracle
    o = Oracle()
    h = o.window(w.P, w.M, w.window)
    F = w.x.size // w.P
    # Double the sample until a run lasts a tenth of the target, then scale to it.
    n, dt = 16, 0.0
    while n < F:
        t = time.perf_counter()
        o.pfb(w.x, w.P, w.M, h, frames=np.arange(n, dtype=np.int64))
        dt = time.perf_counter() - t
        if dt >= target_s / 10:
            break
        n *= 2
    n = int(min(F, max(n, n * target_s / max(dt, 1e-9))))
    t = time.perf_counter()
    o.pfb(w.x, w.P, w.M, h, frames=np.arange(n, dtype=np.int64))
    dt = time.perf_counter() - t
    return {"value": round(n * w.P / dt / 1e9, 6), "unit": "GSamples/s", "cores": o.threads(), "kind": "oracle",
            "sample": f"first {n} of {F} frames ({n * w.P} input samples) of {w.name}, FP64 direct FIR + "
                      f"direct-sum DFT, {dt:.1f} s wall on {o.threads()} OpenMP threads"}


def numpy_pfb(x, P, M, h, dtype):
    """The filter bank written directly in NumPy, the kind of CPU baseline the
    paper compares against: the polyphase FIR of Eq. (20) as M shifted
    multiply-adds over the frames (tap m of branch p is h[(M-1-m)P + p]), then
    numpy.fft across the branches of each frame."""
    F = x.size // P
    X = x[: F * P].reshape(F, P).astype(dtype)
    hb = np.asarray(h).reshape(M, P).astype(np.finfo(dtype).dtype)  # real taps
    y = hb[M - 1] * X
    for m in range(1, min(M, F)):
        y[m:] += hb[M - 1 - m] * X[: F - m]
    return np.fft.fft(y, axis=1) if np.iscomplexobj(y) else np.fft.rfft(y, axis=1)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_context(w, target_s=4.0):
    """Beside the oracle on every host core: the oracle on one core, and the
    NumPy filter bank in FP32 and FP64 (one process; NumPy's loops and FFT
    run on one core), each on a bounded sample of frames."""
    from oracle import Oracle
    o = Oracle()
    h = o.window(w.P, w.M, w.window)
    F = w.x.size // w.P
    all_threads = o.threads()
    res = {"cpu_model": cpu_model(), "host_threads": all_threads}
    o.set_threads(1)
    try:
        n, dt = 8, 0.0
        while n < F:
            t = time.perf_counter()
            o.pfb(w.x, w.P, w.M, h, frames=np.arange(n, dtype=np.int64))
            dt = time.perf_counter() - t
            if dt >= target_s / 10:
                break
            n *= 2
        n = int(min(F, max(n, n * target_s / max(dt, 1e-9))))
        t = time.perf_counter()
        o.pfb(w.x, w.P, w.M, h, frames=np.arange(n, dtype=np.int64))
        dt = time.perf_counter() - t
        res["oracle_one_core"] = {"value": round(n * w.P / dt / 1e9, 6), "unit": "GSamples/s",
                                  "sample": f"first {n} of {F} frames, {dt:.1f} s"}
    finally:
        o.set_threads(all_threads)
    nf = min(F, 8192)
    xs = w.x[: nf * w.P]
    check = o.pfb(xs, w.P, w.M, h, frames=np.arange(min(nf, w.M + 2), dtype=np.int64))
    for name, dt_ in (("fp32", np.complex64 if w.complex_input else np.float32),
                      ("fp64", np.complex128 if w.complex_input else np.float64)):
        dt_ = np.dtype(dt_)
        numpy_pfb(xs[: 64 * w.P], w.P, w.M, h, dt_)  # warm up the FFT plan
        t = time.perf_counter()
        X = numpy_pfb(xs, w.P, w.M, h, dt_)
        sec = time.perf_counter() - t
        res[f"numpy_{name}"] = {"value": round(nf * w.P / sec / 1e9, 6), "unit": "GSamples/s", "cores": 1,
                                "rel_l2_vs_oracle_first_frames": float(f"{rel_l2(X[: check.shape[0]], check):.2e}"),
                                "sample": f"first {nf} of {F} frames, {sec:.2f} s"}
    return res


def cpu_context_precision(wd, frames=512, numpy_frames=4096, reps=3):
    """The CPU on the precision workload (complex input, 4096 channels,
    8 taps): the FP64 oracle on every host core over its first `frames`
    frames, and the NumPy filter bank in FP32 and FP64 over its first
    `numpy_frames` frames; each the median of `reps` runs."""
    from oracle import Oracle
    o = Oracle()
    h = o.window(wd.P, wd.M, wd.window)
    F = wd.x.size // wd.P
    n = min(F, frames)
    times = []
    for _ in range(reps):
        t = time.perf_counter()
        ref = o.pfb(wd.x, wd.P, wd.M, h, frames=np.arange(n, dtype=np.int64))
        times.append(time.perf_counter() - t)
    dt = sorted(times)[len(times) // 2]
    res = {"workload": wd.name, "oracle": {"value": round(n * wd.P / dt / 1e9, 6), "unit": "GSamples/s",
                                            "cores": o.threads(), "sample": f"first {n} of {F} frames, median of "
                                                                          f"{reps}: {dt:.2f} s"}}
    nf = min(F, numpy_frames)
    xs = wd.x[: nf * wd.P]
    for name, dt_ in (("fp32", np.complex64), ("fp64", np.complex128)):
        numpy_pfb(xs[: 64 * wd.P], wd.P, wd.M, h, np.dtype(dt_))
        times = []
        for _ in range(reps):
            t = time.perf_counter()
            X = numpy_pfb(xs, wd.P, wd.M, h, np.dtype(dt_))
            times.append(time.perf_counter() - t)
        sec = sorted(times)[len(times) // 2]
        res[f"numpy_{name}"] = {"value": round(nf * wd.P / sec / 1e9, 6), "unit": "GSamples/s", "cores": 1,
                                "rel_l2_vs_oracle": float(f"{rel_l2(X[:n], ref):.2e}"),
                                "sample": f"first {nf} of {F} frames, median of {reps}: {sec:.2f} s"}
    return res


def ops_bench(torch, steps=10):
    """The standalone building blocks: unfold (GB/s of output written, the
    bound) and the direct FIR with arbitrary taps (GSamples/s)."""
    from paper_2408_16551_amd.pfb import Fir, unfold
    res = {}
    n = 1 << 26
    x = torch.randn(n, device="cuda")
    for width, stride in ((16, 16), (64, 16)):
        rows = (n - width) // stride + 1
        out = torch.empty((rows, width), device="cuda")
        for _ in range(2):
            unfold(x, width, stride, out=out)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            unfold(x, width, stride, out=out)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t) / steps
        by = 4.0 * rows * width + 4.0 * n
        res[f"unfold_w{width}_s{stride}"] = {"ms": round(sec * 1e3, 4), "gbs": round(by / sec / 1e9, 1),
                                             "hbm_frac": round(by / sec / 1e9 / PEAK_HBM_GBS, 4)}
        del out
    g = np.random.Generator(np.random.PCG64(3))
    for K in (64, 1024):
        f = Fir(g.standard_normal(K), "r32")
        y = torch.empty_like(x)
        for _ in range(2):
            f(x, out=y)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            f(x, out=y)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t) / steps
        res[f"fir_k{K}_r32"] = {"ms": round(sec * 1e3, 4), "gsps": round(n / sec / 1e9, 2),
                                "tflops": round(2.0 * K * n / sec / 1e12, 2)}
        f.close()
    res["library_gemm"] = library_gemm(torch)
    log(f"[bench] ops: {res}")
    return res


def library_gemm(torch, reps=10):
    """Context for the DFT kernels: the ROCm library GEMM (torch.matmul, and
    torch._scaled_mm for FP8) on the DFT GEMM shapes of the two form
    workloads -- frames x K by K x N -- with random operands.  Not part of
    the filter bank; its output type is the input type (bf16) or FP32 (FP8)."""
    def t(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    res = {}
    for name, (M, K, N) in (("real_1024", (65536, 1024, 1024)), ("complex_4096", (16384, 8192, 8192))):
        a = torch.randn(M, K, device="cuda").to(torch.bfloat16)
        b = torch.randn(N, K, device="cuda").to(torch.bfloat16)
        bt = b.t().contiguous()   # K x N, row-major
        ms = t(lambda: torch.matmul(a, bt))
        res[f"bf16_{name}"] = {"ms": round(ms, 4), "tflops": round(2.0 * M * N * K / ms / 1e9, 1),
                               "frac": round(2.0 * M * N * K / ms / 1e9 / PEAK_TFLOPS["bf16"], 4)}
        try:
            a8, b8 = a.to(torch.float8_e4m3fn), b.to(torch.float8_e4m3fn)
            one = torch.ones((), device="cuda")
            b8t = b8.t()   # K x N column-major, the layout _scaled_mm takes for its second operand
            ms = t(lambda: torch._scaled_mm(a8, b8t, scale_a=one, scale_b=one, out_dtype=torch.float32))
            res[f"fp8_{name}"] = {"ms": round(ms, 4), "tflops": round(2.0 * M * N * K / ms / 1e9, 1),
                                  "frac": round(2.0 * M * N * K / ms / 1e9 / PEAK_TFLOPS["fp8"], 4)}
        except Exception as e:  # the FP8 library path is optional context
            res[f"fp8_{name}"] = {"error": repr(e)[:120]}
        del a, b, bt
    return res


def sampled_check(oracle_obj, cases, seed, n_frames=64):
    """rel-L2 vs the FP64 oracle over sampled frames of several streams:
    cases = [(x, P, M, got)], x the whole input of a stream (zero history),
    got its frames x P output (numpy).  The error is pooled over the cases
    (one norm over all sampled frames); the worst single case beside it."""
    g = np.random.Generator(np.random.PCG64(seed))
    num = den = 0.0
    worst = 0.0
    for x, P, M, got in cases:
        F = got.shape[0]
        fr = np.unique(np.concatenate([np.arange(min(F, M + 1)), [F - 1],
                                       g.choice(F, size=min(F, n_frames), replace=False)])).astype(np.int64)
        ref = oracle_obj.pfb(x, P, M, oracle_obj.window(P, M, "hann"), frames=fr)
        d = float(np.linalg.norm(got[fr].astype(np.complex128) - ref) ** 2)
        r = float(np.linalg.norm(ref) ** 2)
        num, den = num + d, den + r
        worst = max(worst, (d / r) ** 0.5)
    return {"rel_l2_vs_fp64_oracle": float(f"{(num / den) ** 0.5:.3e}"),
            "worst_stream_rel_l2": float(f"{worst:.3e}"), "streams_checked": len(cases),
            "frames_per_stream": f"first M+1, last, {n_frames} random"}


def batched_bench(torch, precisions=("fp32", "bf16x3", "fp32/factored"), steps=20, oracle_obj=None, warm=10):
    """The ragged batch: 64 complex64 streams, log-uniform lengths 2^18-2^22,
    channels from {256, 512, 1024}, 16 taps, one persistent launch per stage,
    autotuned launch shapes ("fp32/factored": FP32 with the factored DFT,
    one launch per channel count in place of the GEMM stage).  With an
    oracle: 4 seeded items of the timed batch are checked on sampled frames."""
    from paper_2408_16551_amd import workloads
    from paper_2408_16551_amd.pfb import Batch, Plan
    specs, xs = workloads.ragged_batch()
    total = int(sum(x.size for x in xs))
    xd = [torch.from_numpy(x).cuda() for x in xs]
    res = {"streams": len(specs), "samples": total,
           "channels_mix": {str(P): sum(1 for s in specs if s.P == P) for P in sorted({s.P for s in specs})}}
    for entry in precisions:
        prec, dft = (entry.split("/") + ["dense"])[:2]
        plans = {P: Plan(P, 16, "c64", "hann", prec, workspace_bytes=-1, dft=dft) for P in {s.P for s in specs}}
        outs = [torch.empty((x.size // s.P, s.P), dtype=torch.complex64, device="cuda") for s, x in zip(specs, xs)]
        items = [(plans[s.P], x, o) for s, x, o in zip(specs, xd, outs)]
        b = Batch(prec, max_items=len(items), workspace_bytes=2 << 30)
        tf, tile_n = b.tune(items)
        for _ in range(warm):  # steady state: the shader clock rises over the first milliseconds of load
            b.execute(items)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            b.execute(items)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t) / steps
        flops = sum(dft_flops_per_frame(s.P, True) * (x.size // s.P) for s, x in zip(specs, xs))
        res[entry] = {"gsps": round(total / sec / 1e9, 3), "ms_per_batch": round(sec * 1e3, 3),
                      "dft_useful_tflops_incl_fir": round(flops / sec / 1e12, 2),
                      "tuned": {"fir_frames_per_thread_mult": tf, "gemm_tile_n": tile_n}}
        if oracle_obj is not None:
            pick = np.random.Generator(np.random.PCG64(77)).choice(len(items), size=4, replace=False)
            res[entry]["check"] = sampled_check(
                oracle_obj, [(xs[i], specs[i].P, 16, outs[i].cpu().numpy()) for i in sorted(pick)], seed=78)
        log(f"[bench] batched {entry}: {res[entry]}")
        b.close()
        del outs, items
    return res


_BATCHED_CAPACITY = {}


def serving_mix_batched_capacity(torch, precision, host=False, seed=1005, reps=30, dft="dense", warm=10):
    """Capacity C of the batched path on the serving mix: one request of
    log-uniform length 2^16-2^22 on each of the 64 logical streams, run as one
    tina_pfb_batch_execute (every item with its stream's plan and state),
    closed loop, inputs and outputs in HBM.  host=True: end to end from pinned
    host buffers (each pass copies every input in, runs the batch and copies
    every output back, in order on one stream).  GSamples/s, at steady
    state: `warm` untimed passes first (the shader clock rises over the first
    few milliseconds of load; 1 warm-up pass and 5 timed ones measured the FP8
    mix at 42 GS/s, 10 and 30 at 47.5), then `reps` timed passes."""
    if (precision, host, dft) in _BATCHED_CAPACITY:
        return _BATCHED_CAPACITY[(precision, host, dft)]
    from paper_2408_16551_amd import workloads
    from paper_2408_16551_amd.pfb import Batch, Plan, State
    streams = workloads.serving_streams(seed)
    g = np.random.Generator(np.random.PCG64(seed + 11))
    lens = np.floor(2.0 ** g.uniform(16.0, 22.0, size=len(streams))).astype(np.int64)
    plans = {}
    for s in streams:
        if (s.P, s.M) not in plans:
            plans[(s.P, s.M)] = Plan(s.P, s.M, "c64", "hann", precision, workspace_bytes=-1, dft=dft)
    src = torch.from_numpy(workloads.random_tone_stream(g, int(lens.max()), 4)).cuda()
    items, states = [], []
    for s, n in zip(streams, lens):
        p = plans[(s.P, s.M)]
        st = State(p)
        states.append(st)
        out = torch.empty((int(n) // s.P + 1, s.P), dtype=torch.complex64, device="cuda")
        items.append((p, src[: int(n)], out, st))
    if host:   # each item its own device input, filled from pinned host memory
        xh = [src[: int(n)].cpu().pin_memory() for n in lens]
        oh = [torch.empty(o.shape, dtype=o.dtype).pin_memory() for _, _, o, _ in items]
        items = [(p, torch.empty_like(x, device="cuda"), o, st) for (p, _, o, st), x in zip(items, xh)]

    def one_pass():
        if host:
            for (_, xd, _, _), x in zip(items, xh):
                xd.copy_(x, non_blocking=True)
        b.execute(items)
        if host:
            for (_, _, o, _), x in zip(items, oh):
                x.copy_(o, non_blocking=True)

    b = Batch(precision, max_items=len(items), workspace_bytes=2 << 30)
    for _ in range(warm):
        one_pass()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        one_pass()
    torch.cuda.synchronize()
    cap = float(lens.sum()) * reps / (time.perf_counter() - t)
    b.close()
    for st in states:
        st.close()
    for p in plans.values():
        p.close()
    _BATCHED_CAPACITY[(precision, host, dft)] = cap
    log(f"[bench] serving mix, batched path capacity {precision}{' from host buffers' if host else ''}: "
        f"{cap / 1e9:.2f} GS/s")
    return cap


def serving_check(torch, sv, pool, device, oracle_obj, seed, n_req=16):
    """Correctness of served output: on 4 fresh logical streams (512, 1024,
    4096 channels and one more 4096; 8-16 taps), 16 requests each of
    log-uniform length 2^12-2^18 taken from the request pool; the
    concatenated outputs of each stream against the FP64 oracle on the
    concatenated input, at sampled frames."""
    g = np.random.Generator(np.random.PCG64(seed))
    cfg = [(512, 12), (1024, 16), (4096, 8), (4096, 16)]
    size = pool.numel() if device else pool.size
    reqs = []
    for P, M in cfg:
        sid = sv.stream(P, M, "c64")
        res, xs, pend = 0, [], []
        for n in np.floor(2.0 ** g.uniform(12.0, 18.0, size=n_req)).astype(np.int64):
            off = int(g.integers(0, size - n + 1))
            x = pool[off: off + int(n)]
            frames = (res + int(n)) // P
            res = (res + int(n)) % P
            if device:
                out = torch.empty((frames, P), dtype=torch.complex64, device="cuda")
            else:
                out = np.empty((frames, P), dtype=np.complex64)
            pend.append((sv.submit(sid, x, out), out))
            xs.append(x.cpu().numpy() if device else np.array(x))
        reqs.append((P, M, xs, pend))
    cases = []
    for P, M, xs, pend in reqs:
        outs = []
        for rid, out in pend:
            r = sv.wait(rid, timeout_s=120)
            if r["status"] != 0:
                raise RuntimeError(f"serving check: request failed with status {r['status']}")
            outs.append(out.cpu().numpy() if device else out)
        cases.append((np.concatenate(xs), P, M, np.concatenate(outs)))
    return sampled_check(oracle_obj, cases, seed + 1)


def serving_bench(torch, precision, budget_bytes, n_warm=200, n_meas=2000, rho=0.5, seed=1005, device=False,
                  frames_per_step=2048, oracle_obj=None, max_active=64, use_graph=False, dft="dense"):
    """Open-loop Poisson arrivals on 64 logical streams (channels from {512,
    1024, 4096}, 8-16 taps, complex64); each request is the next chunk of a
    random stream, length log-uniform 2^16-2^22.  The server runs up to
    max_active requests with samples to issue, frames_per_step frames each per
    step (64 x 2048: FP8 at 0.8 of the steady-state capacity, p99 3.3 ms against
    5.5 ms with 1024 frames; 4096 frames or 128 slots no better; at 0.5 the
    same 0.85-0.9 ms).  Steps are
    plain launches: a graph replay leaves the device idle ~8 us longer per
    step and measured no lower latency.  The rate is rho times the
    batched path's capacity C on the same mix with the same buffer placement
    (serving_mix_batched_capacity: end to end from pinned host memory, or in
    HBM); the server's own closed-burst capacity is reported beside it.  Latency =
    done - scheduled arrival, including the host-to-device and device-to-host
    copies (device=True: requests already in HBM, used in place, no copies).
    Device-busy is the summed step time over the open-loop window."""
    import threading
    from paper_2408_16551_amd import workloads
    from paper_2408_16551_amd.pfb import Server
    streams = workloads.serving_streams(seed)
    sv = Server(precision, max_streams=len(streams) + 4, max_active=max_active, hbm_budget_bytes=budget_bytes,
                frames_per_step=frames_per_step, use_graph=use_graph, max_channels=4096, dft=dft)
    sids = [sv.stream(s.P, s.M, "c64") for s in streams]
    g = np.random.Generator(np.random.PCG64(seed + 7))
    max_len = 1 << 22
    pool = torch.empty(max_len * 8, dtype=torch.complex64, pin_memory=True).numpy()
    pool[:] = workloads.random_tone_stream(g, pool.size, 4)
    n_out = 64   # output buffers in flight (frames * P <= residue + n < max_len + 4096)
    if device:
        pool = torch.from_numpy(pool).cuda()
        out_pool = [torch.empty(max_len + 4096, dtype=torch.complex64, device="cuda") for _ in range(n_out)]
        torch.cuda.synchronize()
    else:
        out_pool = [torch.empty(max_len + 4096, dtype=torch.complex64, pin_memory=True).numpy() for _ in range(n_out)]
    size = pool.numel() if device else pool.size
    free_out = list(range(n_out))
    lock = threading.Condition()
    residues = [0] * len(streams)

    def make(i, sid, n):
        P = streams[sid].P
        frames = (residues[sid] + n) // P
        residues[sid] = (residues[sid] + n) % P
        off = int(g.integers(0, size - n + 1))
        return pool[off: off + n], frames

    def lens(k):
        return np.floor(2.0 ** g.uniform(16.0, 22.0, size=k)).astype(np.int64)

    # closed-loop capacity: a burst of 256 requests (at most n_out outputs in flight)
    burst = []
    L = lens(256)
    t0 = time.perf_counter()
    for i, n in enumerate(L):
        sid = i % len(streams)
        x, frames = make(i, sid, int(n))
        if not free_out:  # recycle the oldest output buffer
            rid0, oi0 = burst.pop(0)
            sv.wait(rid0)
            free_out.append(oi0)
        oi = free_out.pop()
        out = out_pool[oi][: frames * streams[sid].P].reshape(frames, streams[sid].P)
        burst.append((sv.submit(sids[sid], x, out), oi))
    for rid, oi in burst:
        sv.wait(rid)
        free_out.append(oi)
    cap_server = float(L.sum()) / (time.perf_counter() - t0)
    cap = serving_mix_batched_capacity(torch, precision, host=not device, dft=dft)
    mean_len = float(np.mean(lens(100000)))
    lam = rho * cap / mean_len
    # open loop: every request is drawn before the clock starts (stream, input
    # slice, output rows), so the submitting loop only waits for the scheduled
    # arrival and hands the server raw pointers.  Device mode: each request
    # has its own rows of one output allocation (no recycling, the submitter
    # never waits for the collector); host mode recycles the n_out pinned
    # output buffers.
    N = n_warm + n_meas
    arrivals = np.cumsum(g.exponential(1.0 / lam, size=N))
    sid_seq = g.integers(0, len(streams), size=N)
    len_seq = lens(N)
    plan_rq = []
    out_rows = 0
    for i in range(N):
        sid = int(sid_seq[i])
        P = streams[sid].P
        n = int(len_seq[i])
        frames = (residues[sid] + n) // P
        residues[sid] = (residues[sid] + n) % P
        off = int(g.integers(0, size - n + 1))
        plan_rq.append((sid, off, n, frames, out_rows))
        out_rows += frames * P
    esz = 8   # complex64
    if device:
        out_all = torch.empty(max(out_rows, 1), dtype=torch.complex64, device="cuda")
        torch.cuda.synchronize()
        in_base, out_base = pool.data_ptr(), out_all.data_ptr()
        ready = torch.cuda.current_stream().cuda_stream
    else:
        in_base = pool.ctypes.data
        ready = 0
    lat, blocked = [None] * N, [0]
    parts = [None] * N   # (submit lag, admission wait, wait for the first step, steps until done), ms
    base = sv.stats()["now_us"] * 1e-6 - time.perf_counter()   # server clock - host clock

    def collector(q):
        for i, rid, oi in iter(q.get, None):
            r = sv.wait(rid)
            lat[i] = (r["t_done_us"] * 1e-6 - (arrivals[i] + t_start + base)) * 1e3
            parts[i] = ((r["t_submit_us"] * 1e-6 - (arrivals[i] + t_start + base)) * 1e3,
                        (r["t_admit_us"] - r["t_submit_us"]) * 1e-3, (r["t_first_step_us"] - r["t_admit_us"]) * 1e-3,
                        (r["t_done_us"] - r["t_first_step_us"]) * 1e-3, r["steps"])
            if oi is not None:
                with lock:
                    free_out.append(oi)
                    lock.notify_all()

    import queue as _q
    q = _q.Queue()
    th = threading.Thread(target=collector, args=(q,), daemon=True)
    th.start()
    import gc
    gc.collect()
    gc.disable()   # no collector pauses in the submitting loop (they would count as latency)
    st0 = sv.stats()
    t_start = time.perf_counter()
    samples_meas = 0
    clock = time.perf_counter
    for i in range(N):
        due = arrivals[i]
        while True:   # sleep to within 0.2 ms of the arrival, then spin
            d = due - (clock() - t_start)
            if d <= 0:
                break
            if d > 3e-4:
                time.sleep(d - 2e-4)
        sid, off, n, frames, orow = plan_rq[i]
        P = streams[sid].P
        if device:
            oi = None
            optr = out_base + orow * esz
        else:
            with lock:
                while not free_out:
                    blocked[0] += 1
                    lock.wait()
                oi = free_out.pop()
            optr = out_pool[oi].ctypes.data
        rid = sv.submit_ptr(sids[sid], in_base + off * esz, n, optr, frames, device, ready)
        q.put((i, rid, oi))
        if i >= n_warm:
            samples_meas += n
    q.put(None)
    th.join()
    gc.enable()
    t_total = time.perf_counter() - t_start - arrivals[n_warm - 1] if n_warm else time.perf_counter() - t_start
    st = sv.stats()
    check = serving_check(torch, sv, pool, device, oracle_obj, seed + 3) if oracle_obj is not None else None
    sv.close()
    m = np.array(lat[n_warm:], dtype=np.float64)
    pa = np.array(parts[n_warm:], dtype=np.float64)
    breakdown = {name: {"p50": round(float(np.percentile(pa[:, j], 50)), 3), "p99": round(float(np.percentile(pa[:, j], 99)), 3)}
                 for j, name in enumerate(("submit_lag_ms", "admission_ms", "to_first_step_ms", "steps_ms", "steps"))}
    return {"precision": precision if dft == "dense" else f"{precision}/{dft}", "hbm_budget_bytes": budget_bytes, "rho": rho,
            "buffers": "device (in place)" if device else "host (pinned; copied in and out)",
            "frames_per_step": frames_per_step, "max_active": max_active,
            "capacity_gsps_batched_path": round(cap / 1e9, 3), "capacity_includes_copies": not device,
            "capacity_gsps_server_closed_burst": round(cap_server / 1e9, 3), "rate_req_per_s": round(lam, 1),
            "mean_request_samples": round(mean_len), "requests_measured": n_meas, "warmup_requests": n_warm,
            "p50_ms": round(float(np.percentile(m, 50)), 3), "p99_ms": round(float(np.percentile(m, 99)), 3),
            # the same from the submit call (leaves out the client's own lag behind the schedule)
            "p50_ms_from_submit": round(float(np.percentile(m - pa[:, 0], 50)), 3),
            "p99_ms_from_submit": round(float(np.percentile(m - pa[:, 0], 99)), 3),
            "mean_ms": round(float(m.mean()), 3), "gsps_served": round(samples_meas / t_total / 1e9, 3),
            "admission_waits": st["admission_waits"], "steps": st["steps"],
            "device_busy_frac_open_loop": round((st["device_busy_ms"] - st0["device_busy_ms"]) /
                                                ((st["now_us"] - st0["now_us"]) / 1e3), 3),
            "submitter_blocked_on_output_buffers": blocked[0], "latency_parts": breakdown, "check": check}


def check_oracle():
    """The FP64 oracle, for the sampled output checks of the batched and
    serving legs (test infrastructure: it checks the GPU output, computes none
    of it)."""
    from oracle import Oracle
    return Oracle()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the precision-form tables")
    ap.add_argument("--no-batched", action="store_true", help="skip the ragged batched workload")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving workload")
    ap.add_argument("--serving-quick", action="store_true",
                    help="serving: only FP8 per-frame, device buffers, rho 0.5, 50 + 300 requests (for kernel traces)")
    ap.add_argument("--forms", default="fp32,bf16,bf16x3,fp16,fp16x3,fp8,mxfp8,fp32/factored,fp32/compensated,fp32/table",
                    help="comma-separated precision forms of the form tables (form or form/factored)")
    ap.add_argument("--form-workloads", default="real,wide",
                    help="comma-separated workloads of the form tables: real (1024-channel real stream), "
                         "wide (4096-channel complex 60 dB stream)")
    ap.add_argument("--form-steps", type=int, default=0,
                    help="timed steps per form (0: 20, after 5 warm-up steps, on both workloads)")
    ap.add_argument("--no-fir-only", action="store_true", help="skip the FIR-only run")
    ap.add_argument("--no-ops", action="store_true", help="skip the standalone building blocks")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run only a plain 1 GiB device copy (for scaling rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        sys.exit("bench.py measures one GPU only: the library has no multi-GPU path (--gpus must be 1); "
                 "independent streams would be placed whole on GPUs, one long stream split by time with a "
                 "(M-1)*P-sample halo per boundary.")

    import torch

    from paper_2408_16551_amd import workloads
    from paper_2408_16551_amd.pfb import Plan

    torch.cuda.set_device(0)
    if args.copy_probe:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        log("[bench] copy probe: 3 x (read 1 GiB + write 1 GiB)")
        return

    log("[bench] generating the real stream workload")
    w = workloads.real_stream()
    N = w.x.size
    F = N // w.P
    xd = torch.from_numpy(w.x).cuda()
    plan = Plan(w.P, w.M, "r32", w.window, "fp32", "pfb")
    out = plan.alloc_out(F)
    log(f"[bench] timing {args.steps} steps after {args.warmup} warm-up steps")
    sec, fir_ms, dft_ms = timed_steps(plan, xd, out, args.steps, args.warmup, torch)
    gsps = N / sec / 1e9
    flops = dft_flops_per_frame(w.P, False) * F
    achieved = flops / (dft_ms * 1e-3) / 1e12
    traffic = read_traffic(w.name)
    fir_bytes = 4.0 * N + 4.0 * F * w.P      # algorithmic: read input, write FIR output
    result = {
        "metric": "PFB input GSamples/s (FP32 DFT GEMM; reduced-precision forms at their rel. error in 'forms')",
        "value": round(gsps, 3),
        "unit": "GSamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded N(0,1) noise + 8 channel-centre tones)",
        "config": {"workload": w.name, "channels": w.P, "taps": w.M, "window": "sinc x hann",
                   "samples": N, "sample_type": "r32", "precision": "fp32"},
        "roofline": {"kernel": "dft_gemm_kernel<FP32>", "bound": "mfma", "achieved": round(achieved, 2),
                     "peak": PEAK_TFLOPS["fp32"], "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_TFLOPS["fp32"], 4), "traffic": traffic,
                     "flops_per_launch": flops, "avg_launch_ms": round(dft_ms, 4)},
        "stages": {"fir": {"kernel": "fir_kernel", "bound": "hbm", "avg_launch_ms": round(fir_ms, 4),
                           "achieved": round(fir_bytes / (fir_ms * 1e-3) / 1e9, 1), "peak": PEAK_HBM_GBS,
                           "unit": "GB/s", "frac": round(fir_bytes / (fir_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                           "bytes_per_launch": fir_bytes}},
    }
    del out
    plan.close()

    if not args.no_forms:
        from oracle import Oracle
        o = Oracle()
        forms = [f for f in args.forms.split(",") if f]
        fw = set(args.form_workloads.split(","))
        fs = args.form_steps
        result["forms"] = {}
        if "real" in fw:
            result["forms"][w.name] = forms_table(w, forms, fs or 20, min(5, fs or 5), torch, o, 24)
        del xd
        if "wide" in fw:
            wd = workloads.wide_dynamic_range()
            result["forms"][wd.name] = forms_table(wd, forms, fs or 20, min(5, fs or 5), torch, o, 12)
            del wd
    if not args.no_forms and not args.no_fir_only:
        # FIR-only path on the real stream (the stage the FIR roofline measures).
        fplan = Plan(w.P, w.M, "r32", w.window, "fp32", "fir")
        xd = torch.from_numpy(w.x).cuda()
        fout = fplan.alloc_out(F)
        s2, f2, _ = timed_steps(fplan, xd, fout, args.steps, 3, torch)
        result["fir_only"] = {"gsps": round(N / s2 / 1e9, 2), "kernel_ms": round(f2, 4),
                              "hbm_gbs": round(fir_bytes / (f2 * 1e-3) / 1e9, 1),
                              "hbm_frac": round(fir_bytes / (f2 * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
        del fout, xd
        fplan.close()

    if not args.no_forms and not args.no_ops:
        result["ops"] = ops_bench(torch)
    if not args.no_batched:
        log("[bench] batched ragged workload")
        result["batched"] = batched_bench(torch, oracle_obj=check_oracle())
    if not args.no_serving:
        log("[bench] serving workload")
        o = check_oracle()
        if args.serving_quick:
            result["serving"] = [serving_bench(torch, "fp8", 8 << 30, n_warm=50, n_meas=300, device=True,
                                               oracle_obj=o)]
        else:
            result["serving"] = [serving_bench(torch, prec, bud, oracle_obj=o) for prec in ("fp8", "bf16x3")
                                 for bud in (8 << 30, 256 << 20)]
            result["serving"] += [serving_bench(torch, prec, 8 << 30, device=True, rho=rho, oracle_obj=o, dft=dft)
                                  for rho in (0.5, 0.8) for prec, dft in (("fp8", "dense"), ("bf16x3", "dense"),
                                                                          ("fp32", "factored"))]

    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on the host (bounded sample)")
        result["cpu_baseline"] = cpu_baseline(w)
        result["cpu_context"] = cpu_context(w)
        wd = workloads.wide_dynamic_range()
        result["cpu_context"]["precision_workload"] = cpu_context_precision(wd)
        del wd
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
