"""FP64 CPU oracle for the DFT -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``oracle.c`` (plain C, built
with gcc) through ctypes and never touches the GPU library.

Conventions (the paper names the DFT and Cooley-Tukey in section III-A but
prints no formula, so the textbook definition is used):
forward ``X[k] = sum_j x[j] exp(-2 pi i j k / N)``; inverse uses ``exp(+...)``
and ``1/N``; the 2D transform is the separable product, inverse ``1/(N1 N2)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True, src: str = _SRC, out: str = _LIB) -> str:
    """Compile ``src`` (default oracle.c) to the shared library ``out`` with gcc
    (FP64, OpenMP, no fast-math)."""
    if force or not os.path.exists(out):
        tmp = out + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-fno-fast-math", "-Wall", "-I", _HERE, "-o", tmp, src, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


def _c128(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.complex128))


def _c64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.complex64))


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _check(rc):
    if rc != 0:
        raise RuntimeError("oracle call failed")


class OracleLib:
    """ctypes view of one build of oracle.c (the default build, or a copy with a
    planted mistake used to show that the pins catch it)."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        ip = ctypes.POINTER(ctypes.c_int64)
        i64, ci = ctypes.c_int64, ctypes.c_int
        lib.oracle_dft.argtypes = [dp, dp, i64, ci]
        lib.oracle_fft.argtypes = [dp, dp, i64, ci]
        lib.oracle_fft_batch_f32.argtypes = [fp, dp, i64, i64, ci, ci]
        lib.oracle_fft_ragged_f32.argtypes = [fp, dp, ip, ip, i64, ci, ci]
        lib.oracle_fft2d_f32.argtypes = [fp, dp, i64, i64, i64, ci, ci]
        lib.oracle_threads.argtypes = [ci]
        lib.oracle_rel_l2_f32.argtypes = [fp, dp, i64, i64, dp, dp, ci]
        lib.oracle_circular_conv_f32.argtypes = [fp, fp, dp, i64, i64, i64, ci]
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i32p = ctypes.POINTER(ctypes.c_int32)
        cd = ctypes.c_double
        lib.oracle_img_ycc.argtypes = [u8p, i64, i64, dp, dp, dp]
        lib.oracle_img_blocks.argtypes = [dp, i64, i64, dp, dp, dp]
        lib.oracle_img_kmeans.argtypes = [dp, dp, i64, cd, ci, ci, dp, ip]
        lib.oracle_img_encode.argtypes = [dp, dp, i64, cd, dp, ci, i32p, dp]
        for f in (lib.oracle_dft, lib.oracle_fft, lib.oracle_fft_batch_f32,
                  lib.oracle_fft_ragged_f32, lib.oracle_fft2d_f32, lib.oracle_threads,
                  lib.oracle_rel_l2_f32, lib.oracle_circular_conv_f32, lib.oracle_img_ycc,
                  lib.oracle_img_blocks, lib.oracle_img_kmeans, lib.oracle_img_encode):
            f.restype = ci
        self.lib = lib
        self.path = path

    def dft(self, x, inverse: bool = False) -> np.ndarray:
        """O(N^2) DFT of one signal from the definition (complex128 in/out)."""
        x = _c128(x).reshape(-1)
        y = np.empty_like(x)
        _check(self.lib.oracle_dft(_ptr(x, ctypes.c_double), _ptr(y, ctypes.c_double),
                                   x.size, int(inverse)))
        return y

    def fft(self, x, inverse: bool = False) -> np.ndarray:
        """Recursive mixed-radix Cooley-Tukey FFT of one signal (complex128 in/out)."""
        x = _c128(x).reshape(-1)
        y = np.empty_like(x)
        _check(self.lib.oracle_fft(_ptr(x, ctypes.c_double), _ptr(y, ctypes.c_double),
                                   x.size, int(inverse)))
        return y

    def fft_batch(self, x, inverse: bool = False, threads: int = 0) -> np.ndarray:
        """Batched FFT over the last axis of a complex64 array -> complex128."""
        x = _c64(x)
        n = x.shape[-1]
        batch = x.size // n if n else 0
        y = np.empty(x.shape, dtype=np.complex128)
        _check(self.lib.oracle_fft_batch_f32(_ptr(x, ctypes.c_float), _ptr(y, ctypes.c_double),
                                             n, batch, int(inverse), threads))
        return y

    def fft_ragged(self, flat, sizes, offsets, inverse: bool = False,
                   threads: int = 0) -> np.ndarray:
        """Ragged batch: signal i = flat[offsets[i] : offsets[i]+sizes[i]] -> complex128."""
        flat = _c64(flat).reshape(-1)
        sizes = np.ascontiguousarray(sizes, dtype=np.int64)
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        y = np.zeros(flat.shape, dtype=np.complex128)
        _check(self.lib.oracle_fft_ragged_f32(
            _ptr(flat, ctypes.c_float), _ptr(y, ctypes.c_double),
            _ptr(sizes, ctypes.c_int64), _ptr(offsets, ctypes.c_int64),
            len(sizes), int(inverse), threads))
        return y

    def fft2d(self, x, inverse: bool = False, threads: int = 0) -> np.ndarray:
        """2D FFT of images shaped (..., ny, nx) complex64 -> complex128."""
        x = _c64(x)
        ny, nx = x.shape[-2:]
        batch = x.size // (ny * nx)
        y = np.empty(x.shape, dtype=np.complex128)
        _check(self.lib.oracle_fft2d_f32(_ptr(x, ctypes.c_float), _ptr(y, ctypes.c_double),
                                         ny, nx, batch, int(inverse), threads))
        return y

    def circular_conv(self, x, h, threads: int = 0) -> np.ndarray:
        """Circular convolution over the last axis from its definition (O(N^2)
        per signal): complex64 signals ``x`` (..., n) with filters ``h`` of
        shape (n,) (one filter for all) or the shape of ``x`` (one per signal)
        -> complex128."""
        x = _c64(x)
        h = _c64(h)
        n = x.shape[-1]
        batch = x.size // n if n else 0
        if h.shape[-1] != n or h.size not in (n, x.size):
            raise ValueError(f"filter shape {h.shape} does not fit signals {x.shape}")
        h_dist = 0 if h.size == n else n
        y = np.empty(x.shape, dtype=np.complex128)
        _check(self.lib.oracle_circular_conv_f32(_ptr(x, ctypes.c_float), _ptr(h, ctypes.c_float),
                                                 _ptr(y, ctypes.c_double), n, batch, h_dist,
                                                 threads))
        return y

    # ---- image block compression (section III-B) ----
    def img_ycc(self, rgb):
        """(a)+(b): rgb uint8 (h, w, 3) -> Y (h, w), Cb, Cr (h/2, w/2), float64."""
        rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
        h, w = rgb.shape[:2]
        y = np.empty((h, w))
        cb = np.empty((h // 2, w // 2))
        cr = np.empty((h // 2, w // 2))
        _check(self.lib.oracle_img_ycc(_ptr(rgb, ctypes.c_uint8), h, w, _ptr(y, ctypes.c_double),
                                       _ptr(cb, ctypes.c_double), _ptr(cr, ctypes.c_double)))
        return y, cb, cr

    def img_blocks(self, y):
        """(c): Y (h, w) -> block means (h/4, w/4), activities (h/4, w/4),
        deviations (h/4 * w/4, 16)."""
        y = np.ascontiguousarray(y, dtype=np.float64)
        h, w = y.shape
        nb = (h // 4) * (w // 4)
        mean = np.empty((h // 4, w // 4))
        act = np.empty((h // 4, w // 4))
        dev = np.empty((nb, 16))
        _check(self.lib.oracle_img_blocks(_ptr(y, ctypes.c_double), h, w,
                                          _ptr(mean, ctypes.c_double), _ptr(act, ctypes.c_double),
                                          _ptr(dev, ctypes.c_double)))
        return mean, act, dev

    def img_kmeans(self, dev, act, tau: float, k: int, iters: int):
        """(d): codebook (k, 16) and the number of pattern blocks."""
        dev = np.ascontiguousarray(dev, dtype=np.float64).reshape(-1, 16)
        act = np.ascontiguousarray(act, dtype=np.float64).reshape(-1)
        cb = np.empty((k, 16))
        npat = ctypes.c_int64(0)
        _check(self.lib.oracle_img_kmeans(_ptr(dev, ctypes.c_double), _ptr(act, ctypes.c_double),
                                          dev.shape[0], float(tau), int(k), int(iters),
                                          _ptr(cb, ctypes.c_double), ctypes.byref(npat)))
        return cb, int(npat.value)

    def img_encode(self, dev, act, tau: float, codebook):
        """(e): codes (int32, 0 = mean only) and decision margins per block."""
        dev = np.ascontiguousarray(dev, dtype=np.float64).reshape(-1, 16)
        act = np.ascontiguousarray(act, dtype=np.float64).reshape(-1)
        cb = np.ascontiguousarray(codebook, dtype=np.float64).reshape(-1, 16)
        code = np.empty(dev.shape[0], dtype=np.int32)
        margin = np.empty(dev.shape[0])
        _check(self.lib.oracle_img_encode(_ptr(dev, ctypes.c_double), _ptr(act, ctypes.c_double),
                                          dev.shape[0], float(tau), _ptr(cb, ctypes.c_double),
                                          cb.shape[0], _ptr(code, ctypes.c_int32),
                                          _ptr(margin, ctypes.c_double)))
        return code, margin

    def threads(self, requested: int = 0) -> int:
        return self.lib.oracle_threads(requested)

    def rel_l2_f32(self, y, ref, threads: int = 0, with_norms: bool = False):
        """Per-signal relative L2 error of complex64 ``y`` against complex128
        ``ref`` over the last axis (the last two for 3D input); with
        ``with_norms`` also the reference norms (for the pooled error)."""
        y = _c64(y)
        ref = _c128(ref)
        if y.shape != ref.shape:
            raise ValueError(f"shape mismatch {y.shape} vs {ref.shape}")
        n = y.shape[-1] * (y.shape[-2] if y.ndim == 3 else 1)
        batch = y.size // n if n else 0
        err = np.empty(batch, dtype=np.float64)
        nrm = np.empty(batch, dtype=np.float64)
        _check(self.lib.oracle_rel_l2_f32(_ptr(y, ctypes.c_float), _ptr(ref, ctypes.c_double),
                                          n, batch, _ptr(err, ctypes.c_double),
                                          _ptr(nrm, ctypes.c_double), threads))
        return (err, nrm) if with_norms else err


_default = None


def default() -> OracleLib:
    """The oracle built from oracle.c (built on first use if absent)."""
    global _default
    if _default is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _default = OracleLib(_LIB)
    return _default


def dft(x, inverse: bool = False) -> np.ndarray:
    return default().dft(x, inverse)


def fft(x, inverse: bool = False) -> np.ndarray:
    return default().fft(x, inverse)


def fft_batch(x, inverse: bool = False, threads: int = 0) -> np.ndarray:
    return default().fft_batch(x, inverse, threads)


def fft_ragged(flat, sizes, offsets, inverse: bool = False, threads: int = 0) -> np.ndarray:
    return default().fft_ragged(flat, sizes, offsets, inverse, threads)


def fft2d(x, inverse: bool = False, threads: int = 0) -> np.ndarray:
    return default().fft2d(x, inverse, threads)


def img_ycc(rgb):
    return default().img_ycc(rgb)


def img_blocks(y):
    return default().img_blocks(y)


def img_kmeans(dev, act, tau, k, iters):
    return default().img_kmeans(dev, act, tau, k, iters)


def img_encode(dev, act, tau, codebook):
    return default().img_encode(dev, act, tau, codebook)


def circular_conv(x, h, threads: int = 0) -> np.ndarray:
    return default().circular_conv(x, h, threads)


def threads(requested: int = 0) -> int:
    """OpenMP thread count the batch routines use for ``requested`` (0 = default)."""
    return default().threads(requested)


def rel_l2_f32(y, ref, threads: int = 0, with_norms: bool = False):
    return default().rel_l2_f32(y, ref, threads, with_norms)


def rel_l2(y, ref) -> np.ndarray:
    """Per-signal relative L2 error ||y - ref|| / ||ref|| over the last axis
    (or the last two axes for 3D input)."""
    y = np.asarray(y)
    ref = np.asarray(ref)
    axes = tuple(range(1, ref.ndim)) if ref.ndim > 1 else None
    num = np.sqrt(np.sum(np.abs(y.astype(np.complex128) - ref) ** 2, axis=axes))
    den = np.sqrt(np.sum(np.abs(ref) ** 2, axis=axes))
    return num / np.where(den == 0, 1.0, den)
