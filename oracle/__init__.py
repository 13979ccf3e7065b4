"""FP64 CPU oracle for the polyphase filter bank (Python side).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the product path never does.  It
shares no code with the GPU library (``paper_2408_16551_amd``) and does not
import it.

The arithmetic lives in ``pfb_oracle.c`` (plain double-precision loops, one
OpenMP loop over frames).  This module only marshals numpy arrays, builds the
extended input (history followed by the framed signal), and carries the
per-stream state between calls:

* ``window``  -- sinc x window prototype of length P*M.
* ``fir``     -- the polyphase FIR of Eq. (20) (Sec. 5.2), per branch.
* ``dft``     -- the DFT across branches, Z = X F (Sec. 4.1, Eq. (12)).
* ``pfb``     -- FIR then DFT per frame (Sec. 5.2).
* ``unfold``  -- sliding window Y(i, j) = X(i + j) (Sec. 4.4, Eq. (17)).
* ``idft`` / ``synthesize`` -- inverse DFT (Sec. 4.2, Eq. (14)) and the
  synthesis bank built on it.
* ``e4m3``, ``mx_exponent``, ``mx_quantize``, ``mx_dft`` -- the block-scaled
  FP8 form of the DFT (32-entry blocks, power-of-two scales, OCP E4M3).
* ``Stream``  -- the filter bank on a stream fed in chunks, carrying the
  (M-1)*P history samples and the partial-frame residue between calls.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pfb_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

WINDOWS = {"rect": 0, "hann": 1, "hamming": 2, "blackman": 3}

_lib = None


def build(out_path: str = _LIB, defines: tuple = ()) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", out_path, "-lm"]
    cmd[1:1] = [f"-D{d}" for d in defines]
    subprocess.run(cmd, check=True)
    return out_path


def _load(path: str | None = None):
    global _lib
    if path is None and _lib is not None:
        return _lib
    p = path or _LIB
    if not os.path.exists(p):
        build(p)
    lib = ctypes.CDLL(p)
    d, i64, i, vp = ctypes.c_double, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
    lib.oracle_threads.restype = i
    lib.oracle_set_threads.argtypes = [i]
    lib.oracle_set_threads.restype = None
    lib.oracle_twiddle.argtypes = [i64, i64, ctypes.POINTER(d), ctypes.POINTER(d)]
    lib.oracle_twiddle.restype = None
    lib.oracle_window.argtypes = [i64, i64, i, vp]
    lib.oracle_window.restype = i
    lib.oracle_unfold.argtypes = [vp, i64, i64, i64, vp]
    lib.oracle_unfold.restype = i64
    lib.oracle_fir.argtypes = [i64, i64, i, vp, vp, i64, i64, vp, vp]
    lib.oracle_fir.restype = i
    lib.oracle_dft.argtypes = [i64, i, vp, i64, vp]
    lib.oracle_dft.restype = i
    lib.oracle_pfb.argtypes = [i64, i64, i, vp, vp, i64, i64, vp, vp, vp]
    lib.oracle_pfb.restype = i
    lib.oracle_idft.argtypes = [i64, vp, i64, vp]
    lib.oracle_idft.restype = i
    lib.oracle_e4m3.argtypes = [d]
    lib.oracle_e4m3.restype = d
    lib.oracle_mx_exponent.argtypes = [d]
    lib.oracle_mx_exponent.restype = i
    lib.oracle_mx_quantize.argtypes = [vp, i64, vp]
    lib.oracle_mx_quantize.restype = i
    lib.oracle_mx_dft.argtypes = [i64, i, vp, i64, vp]
    lib.oracle_mx_dft.restype = i
    if path is None:
        _lib = lib
    return lib


class Oracle:
    """Bindings to one build of the oracle library (the default build unless
    ``path`` names another one)."""

    def __init__(self, path: str | None = None):
        self.lib = _load(path)

    @staticmethod
    def _ptr(a: np.ndarray):
        return a.ctypes.data_as(ctypes.c_void_p)

    def threads(self) -> int:
        return int(self.lib.oracle_threads())

    def set_threads(self, n: int) -> None:
        """OpenMP threads of the calls that follow (timing only)."""
        self.lib.oracle_set_threads(int(n))

    def twiddle(self, r: int, P: int) -> complex:
        """cos(2 pi r/P) + i sin(2 pi r/P)."""
        c, s = ctypes.c_double(), ctypes.c_double()
        self.lib.oracle_twiddle(int(r), int(P), ctypes.byref(c), ctypes.byref(s))
        return complex(c.value, s.value)

    def window(self, P: int, M: int, kind: str = "hann") -> np.ndarray:
        h = np.empty(P * M, dtype=np.float64)
        if self.lib.oracle_window(P, M, WINDOWS[kind], self._ptr(h)) != 0:
            raise ValueError("bad window arguments")
        return h

    def unfold(self, x, J: int, stride: int = 1) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        rows = self.lib.oracle_unfold(self._ptr(x), x.size, J, stride, None)
        Y = np.empty((rows, J), dtype=np.float64)
        if rows:
            self.lib.oracle_unfold(self._ptr(x), x.size, J, stride, self._ptr(Y))
        return Y

    @staticmethod
    def _as_ext(x, P: int, M: int, hist=None):
        """Extended input: (M-1)*P history samples (zeros unless given)
        followed by the framed signal.  Returns (flat doubles, complex?, n_ext)."""
        x = np.asarray(x)
        cplx = np.iscomplexobj(x)
        dt = np.complex128 if cplx else np.float64
        H = (M - 1) * P
        if hist is None:
            hist = np.zeros(H, dtype=dt)
        hist = np.asarray(hist, dtype=dt)
        if hist.size != H:
            raise ValueError("history must hold (M-1)*P samples")
        ext = np.concatenate([hist, x.astype(dt, copy=False)])
        flat = ext.view(np.float64) if cplx else ext
        return np.ascontiguousarray(flat), cplx, ext.size

    def fir(self, x, P: int, M: int, h, hist=None, frames=None) -> np.ndarray:
        """Polyphase FIR output y (frames x P), dtype of the promoted input."""
        h = np.ascontiguousarray(h, dtype=np.float64)
        assert h.size == P * M
        flat, cplx, n_ext = self._as_ext(x, P, M, hist)
        avail = (n_ext - (M - 1) * P) // P
        fr = None if frames is None else np.ascontiguousarray(frames, dtype=np.int64)
        nf = avail if fr is None else fr.size
        y = np.empty((nf, P * (2 if cplx else 1)), dtype=np.float64)
        rc = self.lib.oracle_fir(P, M, int(cplx), self._ptr(h), self._ptr(flat), n_ext, nf,
                                 None if fr is None else self._ptr(fr), self._ptr(y))
        if rc != 0:
            raise ValueError(f"oracle_fir failed ({rc})")
        return y.view(np.complex128) if cplx else y

    def dft(self, y) -> np.ndarray:
        """DFT across branches of each row of y (frames x P)."""
        y = np.asarray(y)
        cplx = np.iscomplexobj(y)
        P = y.shape[1]
        yy = np.ascontiguousarray(y, dtype=np.complex128 if cplx else np.float64)
        flat = yy.view(np.float64) if cplx else yy
        K = P if cplx else P // 2 + 1
        X = np.empty((y.shape[0], K), dtype=np.complex128)
        if self.lib.oracle_dft(P, int(cplx), self._ptr(flat), y.shape[0], self._ptr(X)) != 0:
            raise ValueError("oracle_dft failed")
        return X

    def idft(self, X) -> np.ndarray:
        """Inverse DFT of each row of X (frames x P complex), Sec. 4.2."""
        X = np.ascontiguousarray(X, dtype=np.complex128)
        P = X.shape[1]
        v = np.empty_like(X)
        if self.lib.oracle_idft(P, self._ptr(X.view(np.float64)), X.shape[0], self._ptr(v.view(np.float64))) != 0:
            raise ValueError("oracle_idft failed")
        return v

    def e4m3(self, v: float) -> float:
        """Nearest OCP FP8 E4M3 value (ties to even, saturating at 448)."""
        return float(self.lib.oracle_e4m3(float(v)))

    def mx_exponent(self, amax: float) -> int:
        """Smallest e in [-127, 127] with amax <= 448 * 2^e (0 for amax = 0)."""
        return int(self.lib.oracle_mx_exponent(float(amax)))

    def mx_quantize(self, v) -> np.ndarray:
        """Block-quantised copy of a real vector (blocks of 32 entries)."""
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
        out = np.empty_like(v)
        if self.lib.oracle_mx_quantize(self._ptr(v), v.size, self._ptr(out)) != 0:
            raise ValueError("oracle_mx_quantize failed")
        return out

    def mx_dft(self, y) -> np.ndarray:
        """Block-scaled FP8 DFT across branches of each row of y (frames x P,
        real or complex); frames x K complex128 like ``dft``."""
        y = np.asarray(y)
        cplx = np.iscomplexobj(y)
        P = y.shape[1]
        yy = np.ascontiguousarray(y, dtype=np.complex128 if cplx else np.float64)
        flat = yy.view(np.float64) if cplx else yy
        K = P if cplx else P // 2 + 1
        X = np.empty((y.shape[0], K), dtype=np.complex128)
        if self.lib.oracle_mx_dft(P, int(cplx), self._ptr(flat), y.shape[0], self._ptr(X)) != 0:
            raise ValueError("oracle_mx_dft failed")
        return X

    @staticmethod
    def synthesis_taps(h, P: int, M: int) -> np.ndarray:
        """Prototype g' of the synthesis FIR: branch p's taps g_p(m) = h[m P + p]
        (each analysis branch filter reversed in time), stored so that the
        polyphase FIR reads g_p(m) = g'[(M-1-m) P + p]: the M length-P blocks of
        h in reverse order."""
        return np.asarray(h, dtype=np.float64).reshape(M, P)[::-1].reshape(-1).copy()

    def synthesize(self, X, P: int, M: int, h, hist=None) -> np.ndarray:
        """Synthesis bank for complex channel frames X (frames x P): the inverse
        DFT of each frame (Sec. 4.2), then the polyphase FIR of Eq. (20) across
        frames with the synthesis taps g_p(m) = h[m P + p]; returns the
        frames * P output samples.  `hist` = the (M-1) * P IDFT samples before
        the first frame (zeros when None)."""
        v = self.idft(X)
        y = self.fir(v.reshape(-1), P, M, self.synthesis_taps(h, P, M), hist=hist)
        return y.reshape(-1)

    def pfb(self, x, P: int, M: int, h, hist=None, frames=None, return_fir: bool = False):
        """Filter-bank output X (frames x K complex128), K = P/2+1 (real x) or P."""
        h = np.ascontiguousarray(h, dtype=np.float64)
        assert h.size == P * M
        flat, cplx, n_ext = self._as_ext(x, P, M, hist)
        avail = (n_ext - (M - 1) * P) // P
        fr = None if frames is None else np.ascontiguousarray(frames, dtype=np.int64)
        nf = avail if fr is None else fr.size
        K = P if cplx else P // 2 + 1
        X = np.empty((nf, K), dtype=np.complex128)
        y = np.empty((nf, P * (2 if cplx else 1)), dtype=np.float64) if return_fir else None
        rc = self.lib.oracle_pfb(P, M, int(cplx), self._ptr(h), self._ptr(flat), n_ext, nf,
                                 None if fr is None else self._ptr(fr), self._ptr(X),
                                 None if y is None else self._ptr(y))
        if rc != 0:
            raise ValueError(f"oracle_pfb failed ({rc})")
        if return_fir:
            return X, (y.view(np.complex128) if cplx else y)
        return X


class Stream:
    """The filter bank applied to a stream delivered in chunks.

    State between calls: the last (M-1)*P samples before the next frame
    (history) and the samples that do not yet fill a frame (residue).  Each
    call returns the frames completed by that chunk; the concatenation over
    chunks equals the one-shot result on the concatenated input."""

    def __init__(self, oracle: Oracle, P: int, M: int, h, complex_input: bool, fir_only=False):
        self.o, self.P, self.M, self.h = oracle, P, M, np.asarray(h, dtype=np.float64)
        self.dt = np.complex128 if complex_input else np.float64
        self.hist = np.zeros((M - 1) * P, dtype=self.dt)
        self.residue = np.zeros(0, dtype=self.dt)
        self.fir_only = fir_only

    def push(self, chunk) -> np.ndarray:
        P, M = self.P, self.M
        framed = np.concatenate([self.residue, np.asarray(chunk, dtype=self.dt)])
        F = framed.size // P
        if self.fir_only:
            out = self.o.fir(framed[: F * P], P, M, self.h, hist=self.hist)
        else:
            out = self.o.pfb(framed[: F * P], P, M, self.h, hist=self.hist)
        ext = np.concatenate([self.hist, framed])
        self.hist = ext[F * P: F * P + (M - 1) * P].copy()
        self.residue = framed[F * P:].copy()
        return out
