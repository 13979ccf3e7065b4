"""Pins for the FP64 oracle: each test checks the oracle against something
other than itself -- a value the paper prints, a closed form, a numpy routine
for a special case, an invariant, or a brute-force computation on tiny
inputs that takes a different route (a bank of band-pass filters)."""
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# Unfolding, Sec. 4.4: the worked example printed in the paper.
# --------------------------------------------------------------------------
def test_unfold_paper_example(oracle):
    g = json.load(open(os.path.join(GOLDEN, "unfold_example.json")))
    Y = oracle.unfold(g["x"], g["window"])
    assert list(Y.shape) == g["expected_shape"]
    assert np.array_equal(Y, np.asarray(g["expected"], dtype=np.float64))


def test_unfold_shape_rule(oracle):
    # (I - J + 1) x J for stride 1 (Sec. 4.4), rows at stride s otherwise.
    x = np.arange(11.0)
    assert oracle.unfold(x, 4).shape == (8, 4)
    Y = oracle.unfold(x, 4, stride=3)
    assert Y.shape == (3, 4)
    assert np.array_equal(Y[2], [6, 7, 8, 9])


# --------------------------------------------------------------------------
# Prototype window: numpy's own sinc and window routines.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kind,npwin", [("hann", np.hanning), ("hamming", np.hamming),
                                        ("blackman", np.blackman), ("rect", np.ones)])
@pytest.mark.parametrize("P,M", [(16, 4), (1024, 16), (4096, 8), (6, 3)])
def test_window_matches_numpy(oracle, kind, npwin, P, M):
    L = P * M
    n = np.arange(L)
    ref = np.sinc((n - (L - 1) / 2.0) / P) * npwin(L)
    h = oracle.window(P, M, kind)
    assert np.max(np.abs(h - ref)) <= 2e-15


def test_window_dc_gain_close_to_P(oracle):
    # A sinc with cutoff 1/(2P) sums to about P (unit gain per branch after
    # the P-point DFT); windowing lowers it only slightly.
    h = oracle.window(1024, 16, "hann")
    assert abs(h.sum() / 1024 - 1.0) < 0.01


# --------------------------------------------------------------------------
# Twiddles and the DFT (Sec. 4.1, Eq. (12)).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("P", [16, 12, 4096])
def test_twiddle_quarter_turns_exact(oracle, P):
    if P % 4 == 0:
        assert oracle.twiddle(0, P) == complex(1, 0)
        assert oracle.twiddle(P // 4, P) == complex(0, 1)
        assert oracle.twiddle(P // 2, P) == complex(-1, 0)
        assert oracle.twiddle(3 * P // 4, P) == complex(0, -1)
    for r in range(0, P, max(1, P // 37)):
        ref = np.exp(2j * np.pi * r / P)
        assert abs(oracle.twiddle(r, P) - ref) < 1e-15
        assert oracle.twiddle(r + 5 * P, P) == oracle.twiddle(r, P)


@pytest.mark.parametrize("P", [16, 64, 12])
def test_dft_matrix_unitary(oracle, P):
    # Rows of F are the DFTs of the unit vectors; F F^H = P I.
    F = oracle.dft(np.eye(P, dtype=np.complex128))
    G = F @ F.conj().T
    assert np.max(np.abs(G - P * np.eye(P))) < 1e-12 * P


@pytest.mark.parametrize("P,p0", [(16, 3), (1024, 517), (64, 0)])
def test_dft_of_delta(oracle, P, p0):
    y = np.zeros((1, P), dtype=np.complex128)
    y[0, p0] = 1.0
    X = oracle.dft(y)[0]
    k = np.arange(P)
    ref = np.exp(-2j * np.pi * ((k * p0) % P) / P)
    assert np.max(np.abs(X - ref)) < 1e-15


@pytest.mark.parametrize("P", [16, 256, 30])
def test_dft_matches_numpy_fft(oracle, P):
    g = _rng(7)
    yc = g.standard_normal((5, P)) + 1j * g.standard_normal((5, P))
    Xc = oracle.dft(yc)
    ref = np.fft.fft(yc, axis=1)
    assert np.linalg.norm(Xc - ref) / np.linalg.norm(ref) < 1e-13
    yr = g.standard_normal((5, P))
    Xr = oracle.dft(yr)
    ref = np.fft.rfft(yr, axis=1)
    assert Xr.shape == ref.shape
    assert np.linalg.norm(Xr - ref) / np.linalg.norm(ref) < 1e-13


def test_dft_real_input_edge_channels_have_zero_imaginary(oracle):
    y = _rng(3).standard_normal((4, 64))
    X = oracle.dft(y)
    assert np.all(X[:, 0].imag == 0.0)
    assert np.all(X[:, 32].imag == 0.0)


def test_dft_parseval(oracle):
    y = _rng(11).standard_normal((3, 128)) + 1j * _rng(12).standard_normal((3, 128))
    X = oracle.dft(y)
    assert np.allclose(np.sum(np.abs(X) ** 2, axis=1), 128 * np.sum(np.abs(y) ** 2, axis=1),
                       rtol=1e-13)


# --------------------------------------------------------------------------
# Polyphase FIR (Sec. 5.2, Eq. (20)).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("P,M,f0,p0", [(16, 4, 0, 5), (16, 4, 7, 0), (32, 3, 2, 31)])
def test_fir_impulse_reproduces_taps(oracle, P, M, f0, p0):
    h = oracle.window(P, M, "hann")
    F = 12
    x = np.zeros(F * P)
    x[f0 * P + p0] = 1.0
    y = oracle.fir(x, P, M, h)
    ref = np.zeros((F, P))
    for f in range(f0, min(F, f0 + M)):
        ref[f, p0] = h[(M - 1 - (f - f0)) * P + p0]
    assert np.array_equal(y, ref)   # bit-exact: one non-zero term per output


@pytest.mark.parametrize("cplx", [False, True])
def test_fir_branch_is_causal_convolution(oracle, cplx):
    P, M, F = 8, 5, 40
    g = _rng(5)
    h = g.standard_normal(P * M)
    x = g.standard_normal(F * P) + (1j * g.standard_normal(F * P) if cplx else 0)
    y = oracle.fir(x, P, M, h)
    for p in range(P):
        taps = np.array([h[(M - 1 - m) * P + p] for m in range(M)])
        ref = np.convolve(x[p::P], taps)[:F]
        assert np.allclose(y[:, p], ref, rtol=1e-13, atol=1e-13)


def test_fir_single_unit_tap_is_identity(oracle):
    P = 16
    x = _rng(6).standard_normal(10 * P)
    y = oracle.fir(x, P, 1, np.ones(P))
    assert np.array_equal(y, x.reshape(10, P))


def test_fir_is_presum_of_stride_P_unfold(oracle):
    # The FIR of each frame equals the frame window (an unfold of width P*M
    # at stride P, Sec. 4.4) weighted by h and folded over its M blocks.
    P, M, F = 8, 3, 9
    g = _rng(8)
    h = g.standard_normal(P * M)
    x = g.standard_normal(F * P)
    ext = np.concatenate([np.zeros((M - 1) * P), x])
    U = oracle.unfold(ext, P * M, stride=P)
    assert U.shape == (F, P * M)
    ref = (U * h).reshape(F, M, P).sum(axis=1)
    assert np.allclose(oracle.fir(x, P, M, h), ref, rtol=1e-13, atol=1e-14)


# --------------------------------------------------------------------------
# The filter bank.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("cplx", [False, True])
def test_pfb_single_tap_is_framed_fft(oracle, cplx):
    P, F = 32, 17
    g = _rng(9)
    x = g.standard_normal(F * P) + (1j * g.standard_normal(F * P) if cplx else 0)
    X = oracle.pfb(x, P, 1, np.ones(P))
    ref = (np.fft.fft if cplx else np.fft.rfft)(x.reshape(F, P), axis=1)
    assert np.linalg.norm(X - ref) / np.linalg.norm(ref) < 1e-13


def _H(h, nu):
    j = np.arange(h.size)
    return np.array([np.sum(h * np.exp(-2j * np.pi * v * j)) for v in np.atleast_1d(nu)])


@pytest.mark.parametrize("P,M,k0,win", [(16, 4, 3, "hann"), (64, 8, 21, "blackman")])
def test_pfb_complex_tone_closed_form(oracle, P, M, k0, win):
    h = oracle.window(P, M, win)
    F = 3 * M
    n = np.arange(F * P)
    A, phi = 0.7, 1.3
    x = A * np.exp(1j * (2 * np.pi * ((k0 * n) % P) / P + phi))
    X = oracle.pfb(x, P, M, h)
    k = np.arange(P)
    Hk = _H(h, k / P - k0 / P)
    for f in range(M - 1, F):
        ref = A * np.exp(1j * phi) * Hk   # e^{2 pi i k0 (f-M+1)} = 1
        assert np.max(np.abs(X[f] - ref)) < 1e-12 * np.sum(np.abs(h))
        assert np.argmax(np.abs(X[f])) == k0
        assert abs(X[f, k0] - A * np.exp(1j * phi) * h.sum()) < 1e-12 * P


def test_pfb_real_cosine_off_centre_closed_form(oracle):
    P, M = 16, 4
    h = oracle.window(P, M, "hann")
    F = 20
    n = np.arange(F * P)
    f0, A, phi = 0.2137, 1.1, 0.4
    x = A * np.cos(2 * np.pi * f0 * n + phi)
    X = oracle.pfb(x, P, M, h)
    k = np.arange(P // 2 + 1)
    for f in range(M - 1, F):
        s = np.exp(2j * np.pi * f0 * (f - M + 1) * P)
        ref = 0.5 * A * (np.exp(1j * phi) * s * _H(h, k / P - f0)
                         + np.exp(-1j * phi) / s * _H(h, k / P + f0))
        assert np.max(np.abs(X[f] - ref)) < 1e-12 * P


@pytest.mark.parametrize("P,M,N,cplx", [(8, 3, 200, True), (16, 4, 512, False), (4, 2, 97, True)])
def test_pfb_equals_bank_of_bandpass_filters(oracle, P, M, N, cplx):
    # Brute force by another route: channel k is the input convolved with
    # g_k[a] = h[L-1-a] exp(+2 pi i k a / P) (a band-pass filter centred on
    # k/P) and sampled at the last sample of each frame, times exp(2 pi i k/P).
    g = _rng(10)
    L = P * M
    h = g.standard_normal(L)
    x = g.standard_normal(N) + (1j * g.standard_normal(N) if cplx else 0)
    X = oracle.pfb(x, P, M, h)
    F = N // P
    K = P if cplx else P // 2 + 1
    a = np.arange(L)
    ref = np.empty((F, K), dtype=np.complex128)
    for k in range(K):
        gk = h[::-1] * np.exp(2j * np.pi * k * a / P)
        full = np.convolve(x, gk)          # full[n] = sum_a gk[a] x[n-a], zero history
        ref[:, k] = np.exp(2j * np.pi * k / P) * full[np.arange(F) * P + P - 1]
    assert X.shape == (F, K)
    assert np.max(np.abs(X - ref)) < 1e-11 * max(1.0, np.max(np.abs(ref)))


def test_pfb_linearity(oracle):
    P, M, N = 32, 4, 32 * 25
    g = _rng(13)
    h = oracle.window(P, M, "hann")
    x, z = g.standard_normal(N), g.standard_normal(N)
    a, b = 1.7, -0.3
    lhs = oracle.pfb(a * x + b * z, P, M, h)
    rhs = a * oracle.pfb(x, P, M, h) + b * oracle.pfb(z, P, M, h)
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * np.max(np.abs(lhs))


def test_pfb_frame_shift(oracle):
    # Delaying the input by one frame delays the output by one frame, exactly.
    P, M, N = 16, 4, 16 * 30
    h = oracle.window(P, M, "hamming")
    x = _rng(14).standard_normal(N) + 1j * _rng(15).standard_normal(N)
    X = oracle.pfb(x, P, M, h)
    Xd = oracle.pfb(np.concatenate([np.zeros(P), x]), P, M, h)
    assert np.array_equal(Xd[1:], X)
    assert np.all(Xd[0] == 0)


@pytest.mark.parametrize("cplx", [False, True])
def test_stream_chunked_equals_one_shot(oracle, cplx):
    from oracle import Stream
    P, M = 16, 5
    h = oracle.window(P, M, "hann")
    g = _rng(16)
    N = 16 * 50 + 7
    x = g.standard_normal(N) + (1j * g.standard_normal(N) if cplx else 0)
    one = oracle.pfb(x, P, M, h)
    s = Stream(oracle, P, M, h, cplx)
    cuts = [0, 3, 3, 40, 41, 200, 555, N]
    outs = [s.push(x[a:b]) for a, b in zip(cuts[:-1], cuts[1:])]
    got = np.concatenate(outs)
    assert got.shape == one.shape
    assert np.array_equal(got, one)
    assert s.residue.size == N % P


def test_frame_subset_equals_full(oracle):
    P, M = 64, 8
    h = oracle.window(P, M, "blackman")
    x = _rng(17).standard_normal(64 * 40) + 0j
    full = oracle.pfb(x, P, M, h)
    fr = np.array([0, 7, 39, 12])
    assert np.array_equal(oracle.pfb(x, P, M, h, frames=fr), full[fr])


# --------------------------------------------------------------------------
# Synthesis (inverse) bank: IDFT (Sec. 4.2, Eq. (14)) then polyphase FIR.
# --------------------------------------------------------------------------
def test_idft_matches_numpy_and_inverts_dft(oracle):
    g = _rng(21)
    y = g.standard_normal((6, 64)) + 1j * g.standard_normal((6, 64))
    v = oracle.idft(y)
    assert np.linalg.norm(v - np.fft.ifft(y, axis=1)) / np.linalg.norm(v) < 1e-13
    assert np.max(np.abs(oracle.idft(oracle.dft(y)) - y)) < 1e-12


def test_synthesis_inverts_single_tap_unit_bank(oracle):
    # M = 1 with unit taps: analysis is the framed DFT, synthesis its inverse.
    P = 32
    x = _rng(22).standard_normal(P * 40) + 1j * _rng(23).standard_normal(P * 40)
    X = oracle.pfb(x, P, 1, np.ones(P))
    assert np.max(np.abs(oracle.synthesize(X, P, 1, np.ones(P)) - x)) < 1e-12


@pytest.mark.parametrize("P,M", [(8, 3), (16, 4)])
def test_analysis_then_synthesis_is_branchwise_convolution(oracle, P, M):
    # The IDFT undoes the DFT, so analysis -> synthesis filters branch p by
    # h_p then g_p: x_hat_p = g_p * h_p * x_p (brute force with np.convolve).
    g = _rng(24)
    h = g.standard_normal(P * M)
    F = 30
    x = g.standard_normal(F * P) + 1j * g.standard_normal(F * P)
    xh = oracle.synthesize(oracle.pfb(x, P, M, h), P, M, h)
    for p in range(P):
        hp = np.array([h[(M - 1 - m) * P + p] for m in range(M)])
        gp = np.array([h[m * P + p] for m in range(M)])
        ref = np.convolve(np.convolve(x[p::P], hp), gp)[:F]
        assert np.allclose(xh[p::P], ref, rtol=1e-12, atol=1e-12)


def test_synthesis_taps_are_block_reversed(oracle):
    h = np.arange(12.0)
    assert np.array_equal(oracle.synthesis_taps(h, 4, 3), [8, 9, 10, 11, 4, 5, 6, 7, 0, 1, 2, 3])


# --------------------------------------------------------------------------
# Block-scaled FP8 form of the DFT (quantisation, Sec. 1; DFT of Eq. (12)).
# Pinned to torch's float8_e4m3fn cast (a library routine, round to nearest
# even), to the format's grid, to exact cases and to a rounding-error bound.
# --------------------------------------------------------------------------
def _torch_e4m3(v):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32))
    return t.to(torch.float8_e4m3fn).to(torch.float64).numpy()


def _e4m3_grid():
    import torch
    g = torch.arange(256, dtype=torch.uint8).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    return np.unique(g[np.isfinite(g)])


def _block_exponent(amax):
    # smallest e with amax <= 448 * 2^e, from the binary exponent of amax/448
    if amax == 0.0:
        return 0
    m, E = np.frexp(amax / 448.0)
    return int(E - 1) if m == 0.5 else int(E)


def test_e4m3_matches_torch_float8(oracle):
    g = _rng(31)
    grid = _e4m3_grid()
    assert grid.max() == 448.0 and grid[grid > 0].min() == 2.0 ** -9 and grid.size == 253
    mids = (grid[1:] + grid[:-1]) / 2  # exact ties: rounding must go to the even code
    rnd = np.concatenate([g.uniform(-448, 448, 3000),
                          np.clip(g.standard_normal(3000) * 2.0 ** g.integers(-12, 8, 3000), -448, 448)])
    v = np.concatenate([grid, mids, rnd.astype(np.float32).astype(np.float64)])
    got = np.array([oracle.e4m3(x) for x in v])
    np.testing.assert_array_equal(got, _torch_e4m3(v))
    assert oracle.e4m3(1000.0) == 448.0 and oracle.e4m3(-1e30) == -448.0  # saturation


@pytest.mark.parametrize("amax", [448.0, 449.0, 1.0, 0.875, 0.8749, 3e-7, 1e-40, 6.5e4, 1e38, 0.0])
def test_mx_exponent_is_smallest_fitting_power(oracle, amax):
    e = oracle.mx_exponent(amax)
    assert e == max(-127, _block_exponent(amax))
    if amax > 0:
        assert amax <= 448.0 * 2.0 ** e
        assert e == -127 or amax > 448.0 * 2.0 ** (e - 1)


def test_mx_quantize_per_block(oracle):
    g = _rng(32)
    mags = 10.0 ** g.uniform(-4, 4, 9)
    v = np.concatenate([g.standard_normal(32) * m for m in mags])[: 32 * 8 + 11]  # ragged last block
    v = v.astype(np.float32).astype(np.float64)
    q = oracle.mx_quantize(v)
    for b in range(0, v.size, 32):
        blk = v[b:b + 32]
        e = _block_exponent(np.max(np.abs(blk)))
        np.testing.assert_array_equal(q[b:b + 32], _torch_e4m3(blk * 2.0 ** -e) * 2.0 ** e)


@pytest.mark.parametrize("P,cplx", [(4, True), (4, False), (2, False), (2, True)])
def test_mx_dft_exact_when_everything_is_representable(oracle, P, cplx):
    # Twiddles of P <= 4 are 0 and +-1 and small integers are E4M3 numbers at
    # any block scale, so the quantised DFT equals the exact one.
    g = _rng(33)
    y = g.integers(-16, 17, (7, P)).astype(np.float64)
    if cplx:
        y = y + 1j * g.integers(-16, 17, (7, P))
    ref = np.fft.fft(y, axis=1)[:, : (P if cplx else P // 2 + 1)]
    np.testing.assert_array_equal(oracle.mx_dft(y), ref)


@pytest.mark.parametrize("P,cplx,j", [(64, False, 37), (32, True, 21), (128, False, 0)])
def test_mx_dft_of_delta_is_the_quantised_coefficient(oracle, P, cplx, j):
    # y = delta at branch j: output k is coefficient j of row k, quantised with
    # the scale of the 32-entry block that holds it.
    y = np.zeros((1, P), dtype=np.complex128 if cplx else np.float64)
    y[0, j] = 1.0
    X = oracle.mx_dft(y)[0]
    for k in range(X.size):
        c, s = _exact_cos_sin(P, k)
        if cplx:
            wr = np.stack([c, s], 1).reshape(-1)
            wi = np.stack([-s, c], 1).reshape(-1)
            pos = 2 * j
        else:
            wr, wi, pos = c, -s, j
        b = (pos // 32) * 32
        for w, got in ((wr, X[k].real), (wi, X[k].imag)):
            blk = w[b:b + 32]
            e = _block_exponent(np.max(np.abs(blk)))
            assert got == _torch_e4m3(np.array([w[pos] * 2.0 ** -e]))[0] * 2.0 ** e


def _exact_cos_sin(P, k):
    # cos, sin of 2 pi pk/P for p < P, with the zeros at multiples of a
    # quarter turn exact (numpy's sin(pi) is 1.2e-16, which a block scale
    # would otherwise blow up).
    t = 2 * np.pi * ((np.arange(P) * k) % P) / P
    c, s = np.cos(t), np.sin(t)
    c[np.abs(c) < 1e-12] = 0.0
    s[np.abs(s) < 1e-12] = 0.0
    return c, s


def _mx_elem_bound(v):
    # |Q(v) - v| <= max(2^-4 |v|, 2^(e-10)) per entry (half a grid step,
    # normal or subnormal binade), e the entry's block exponent.
    out = np.empty_like(v)
    for b in range(0, v.size, 32):
        blk = v[b:b + 32]
        e = _block_exponent(np.max(np.abs(blk)))
        out[b:b + 32] = np.maximum(2.0 ** -4 * np.abs(blk), 2.0 ** (e - 10))
    return out


@pytest.mark.parametrize("P,cplx", [(128, False), (64, True)])
def test_mx_dft_within_rounding_bound(oracle, P, cplx):
    g = _rng(34)
    F = 4
    scale = np.repeat(10.0 ** g.uniform(-3, 3, (F, P * (2 if cplx else 1)) // np.array([1, 16])), 16, axis=1)
    yr = g.standard_normal(scale.shape) * scale
    y = yr[:, 0::2] + 1j * yr[:, 1::2] if cplx else yr
    X = oracle.mx_dft(y)
    ref = np.fft.fft(y, axis=1)[:, : (P if cplx else P // 2 + 1)]
    for f in range(F):
        a = yr[f]
        da = _mx_elem_bound(a)
        for k in range(X.shape[1]):
            c, s = _exact_cos_sin(P, k)
            if cplx:
                rows = (np.stack([c, s], 1).reshape(-1), np.stack([-s, c], 1).reshape(-1))
            else:
                rows = (c, -s)
            for w, got, exact in zip(rows, (X[f, k].real, X[f, k].imag), (ref[f, k].real, ref[f, k].imag)):
                dw = _mx_elem_bound(w)
                bound = np.sum(np.abs(a) * dw + da * np.abs(w) + da * dw) + 1e-9 * np.sum(np.abs(a * w))
                assert abs(got - exact) <= bound
