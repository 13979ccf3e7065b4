"""Seeded synthetic inputs shaped like the filter-bank workloads.

This module draws random numbers and nothing else: it holds none of the
filter bank's arithmetic, so both the GPU tests and the CPU oracle can take
their inputs from it.  Every generator uses numpy's PCG64 with a fixed seed and
draws in a fixed order: noise, then tone frequencies, then phases, then
amplitudes.  A tone at channel centre k of a P-channel bank has frequency k/P
cycles/sample; its phase is formed from (k*n) mod P in integers so that long
streams keep full phase accuracy.

The paper's inputs are "generated randomly" (Sec. 5) with no stated
distribution; these recipes (noise plus tones) stand in for them.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    P: int                  # channels = branches
    M: int                  # taps per branch
    window: str             # prototype window
    complex_input: bool
    x: np.ndarray           # float32 or complex64 samples
    tones: list = field(default_factory=list)   # (freq cycles/sample, amplitude, phase)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _centre_phase(k: int, P: int, n: np.ndarray) -> np.ndarray:
    """2*pi*k*n/P with (k*n) mod P reduced in integers first."""
    return (2.0 * np.pi / P) * ((k * n) % P).astype(np.float64)


def channel_tone_real(N: int, P: int, k: int, amp: float, phase: float) -> np.ndarray:
    n = np.arange(N, dtype=np.int64)
    return amp * np.cos(_centre_phase(k, P, n) + phase)


def channel_tone_complex(N: int, P: int, k: int, amp: float, phase: float) -> np.ndarray:
    n = np.arange(N, dtype=np.int64)
    return amp * np.exp(1j * (_centre_phase(k, P, n) + phase))


def small_pfb(seed: int = 1001, N: int = 1 << 16) -> Workload:
    """Real float32, 16 channels, 4 taps, sinc(len 64) x Hann; N(0,1) noise plus
    3 unit cosines at distinct channel centres from {1..7}."""
    P, M = 16, 4
    g = _rng(seed)
    x = g.standard_normal(N)
    ks = g.choice(np.arange(1, 8), size=3, replace=False)
    ph = g.uniform(0.0, 2.0 * np.pi, size=3)
    tones = []
    for k, p in zip(ks, ph):
        x += channel_tone_real(N, P, int(k), 1.0, float(p))
        tones.append((int(k) / P, 1.0, float(p)))
    return Workload("small_pfb_r32_p16_m4", P, M, "hann", False, x.astype(np.float32), tones)


def real_stream(seed: int = 1002, N: int = 1 << 26, P: int = 1024, M: int = 16) -> Workload:
    """Real float32, 1024 channels, 16 taps, sinc x Hann; N(0,1) noise plus 8
    unit cosines at distinct channel centres in [1, P/2-1]."""
    g = _rng(seed)
    x = g.standard_normal(N)
    ks = g.choice(np.arange(1, P // 2), size=8, replace=False)
    ph = g.uniform(0.0, 2.0 * np.pi, size=8)
    tones = []
    for k, p in zip(ks, ph):
        x += channel_tone_real(N, P, int(k), 1.0, float(p))
        tones.append((int(k) / P, 1.0, float(p)))
    return Workload(f"real_stream_r32_p{P}_m{M}", P, M, "hann", False, x.astype(np.float32), tones)


def wide_dynamic_range(seed: int = 1003, N: int = 1 << 26, P: int = 4096, M: int = 8) -> Workload:
    """Complex64, 4096 channels, 8 taps, sinc x Blackman.  Complex noise of
    standard deviation 1e-4 plus 8 complex tones spanning 60 dB: amplitudes
    1.0 (strongest), 1e-3 (weakest) and six log-uniform in between; seven at
    channel centres, one at a random off-centre frequency."""
    g = _rng(seed)
    sigma = 1e-4
    x = (g.standard_normal(N) + 1j * g.standard_normal(N)) * (sigma / np.sqrt(2.0))
    ks = g.choice(np.arange(P), size=7, replace=False)
    f_off = g.uniform(0.0, 1.0)
    ph = g.uniform(0.0, 2.0 * np.pi, size=8)
    mid = 10.0 ** g.uniform(-3.0, 0.0, size=6)
    amps = np.concatenate([[1.0, 1e-3], mid])
    tones = []
    n = np.arange(N, dtype=np.int64)
    for i, k in enumerate(ks):
        x += channel_tone_complex(N, P, int(k), float(amps[i]), float(ph[i]))
        tones.append((int(k) / P, float(amps[i]), float(ph[i])))
    x += amps[7] * np.exp(1j * (2.0 * np.pi * ((f_off * n) % 1.0) + ph[7]))
    tones.append((float(f_off), float(amps[7]), float(ph[7])))
    return Workload(f"wide_dynamic_range_c64_p{P}_m{M}", P, M, "blackman", True,
                    x.astype(np.complex64), tones)


def random_tone_stream(g: np.random.Generator, N: int, n_tones: int) -> np.ndarray:
    """CN(0,1) noise plus n_tones complex tones, frequency U[0,1), amplitude
    U[0.1,1], phase U[0, 2 pi)."""
    x = (g.standard_normal(N) + 1j * g.standard_normal(N)) / np.sqrt(2.0)
    fr = g.uniform(0.0, 1.0, size=n_tones)
    ph = g.uniform(0.0, 2.0 * np.pi, size=n_tones)
    am = g.uniform(0.1, 1.0, size=n_tones)
    n = np.arange(N, dtype=np.int64)
    for f, p, a in zip(fr, ph, am):
        x += a * np.exp(1j * (2.0 * np.pi * ((f * n) % 1.0) + p))
    return x.astype(np.complex64)


@dataclass
class StreamSpec:
    P: int
    M: int
    window: str
    length: int


def ragged_batch_specs(seed: int = 1004, n_streams: int = 64, log2_lo: float = 18.0,
                       log2_hi: float = 22.0, channels=(256, 512, 1024), M: int = 16):
    """Shapes of the batched workload: stream lengths floor(2^U(lo,hi)),
    channels uniform from `channels`, M taps, Hann."""
    g = _rng(seed)
    lengths = np.floor(2.0 ** g.uniform(log2_lo, log2_hi, size=n_streams)).astype(np.int64)
    Ps = g.choice(np.asarray(channels), size=n_streams)
    return [StreamSpec(int(p), M, "hann", int(n)) for p, n in zip(Ps, lengths)]


def ragged_batch(seed: int = 1004, **kw):
    """The batched workload: specs plus one complex64 array per stream."""
    specs = ragged_batch_specs(seed, **kw)
    g = _rng(seed + 100000)
    xs = [random_tone_stream(g, s.length, int(g.integers(1, 9))) for s in specs]
    return specs, xs


def serving_streams(seed: int = 1005, n_streams: int = 64, channels=(512, 1024, 4096),
                    taps=(8, 16)):
    """Logical streams of the serving workload: channels uniform from
    `channels`, taps uniform in [taps[0], taps[1]], Hann."""
    g = _rng(seed)
    Ps = g.choice(np.asarray(channels), size=n_streams)
    Ms = g.integers(taps[0], taps[1] + 1, size=n_streams)
    return [StreamSpec(int(p), int(m), "hann", 0) for p, m in zip(Ps, Ms)]


def serving_requests(seed: int = 1005, n_requests: int = 2200, n_streams: int = 64,
                     log2_lo: float = 16.0, log2_hi: float = 22.0, rate_hz: float = 100.0):
    """Open-loop Poisson arrivals: (arrival_s, stream_id, n_samples) per request.
    Each request is the next chunk of a uniformly chosen stream."""
    g = _rng(seed + 1)
    gaps = g.exponential(1.0 / rate_hz, size=n_requests)
    arrivals = np.cumsum(gaps)
    sids = g.integers(0, n_streams, size=n_requests)
    lens = np.floor(2.0 ** g.uniform(log2_lo, log2_hi, size=n_requests)).astype(np.int64)
    return [(float(a), int(s), int(n)) for a, s, n in zip(arrivals, sids, lens)]


def request_payload(seed: int, request_index: int, n_samples: int) -> np.ndarray:
    """Samples of one serving request (complex64 noise plus 1-8 tones)."""
    g = _rng(seed * 1_000_003 + request_index)
    return random_tone_stream(g, n_samples, int(g.integers(1, 9)))
