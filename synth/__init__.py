"""Seeded synthetic inputs for the batched FFT workloads.

This module only produces input data; it contains no Fourier arithmetic.  It is
the one piece of code shared by the CPU oracle side (tests, CPU baseline) and
the GPU side (tests, bench), so that both transform bit-identical inputs.

Random numbers come from the counter-based SplitMix64 generator (Steele, Lea
and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):
value number ``c`` of the stream with seed ``s`` is ``mix64(s + (c+1)*gamma)``.
Two implementations of that one definition are given: numpy (host) and torch
(any device, uint64 arithmetic emulated on int64 with wrap-around).  A test
checks they agree bit for bit.

Layouts (all interleaved complex64 = (re, im) float32 pairs):
  * uniform batch: signal ``b``, element ``j``, part ``p`` (0 = re, 1 = im)
    uses counter ``2*(b*n + j) + p``; the value is ``(z >> 40) * 2**-23 - 1``,
    an exact float32 in [-1, 1).
  * ragged batch: signals packed in draw order; signal ``i`` starts at the
    exclusive prefix sum of the sizes, counters as above with that offset.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK64 = (1 << 64) - 1

#: Base seed of every workload; workload ``k`` (1-based) uses ``BASE_SEED + k``.
BASE_SEED = 0x12034938


# --------------------------------------------------------------------------
# SplitMix64, scalar reference (pure Python, used to pin the vector versions)
# --------------------------------------------------------------------------
def mix64_scalar(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * M1) & MASK64
    z = ((z ^ (z >> 27)) * M2) & MASK64
    return z ^ (z >> 31)


def splitmix64_scalar(seed: int, c: int) -> int:
    return mix64_scalar(seed + (c + 1) * GAMMA)


# --------------------------------------------------------------------------
# numpy implementation
# --------------------------------------------------------------------------
def splitmix64_np(seed: int, counters: np.ndarray) -> np.ndarray:
    """Value ``counters[i]`` of the stream ``seed`` (uint64 array in, uint64 out)."""
    c = counters.astype(np.uint64, copy=False)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & MASK64) + (c + np.uint64(1)) * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(M2)
        z = z ^ (z >> np.uint64(31))
    return z


def _u64_to_sym_f32(z: np.ndarray) -> np.ndarray:
    # 24 random bits -> exact float32 in [-1, 1)
    v = (z >> np.uint64(40)).astype(np.float32)
    return v * np.float32(2.0 ** -23) - np.float32(1.0)


def uniform_complex(seed: int, n: int, batch: int, first: int = 0,
                    chunk: int = 1 << 24) -> np.ndarray:
    """Signals ``first .. first+batch-1`` of the uniform batch of length-``n`` signals.

    Returns a complex64 array of shape ``(batch, n)``.
    """
    total = batch * n
    out = np.empty(2 * total, dtype=np.float32)
    base = 2 * first * n
    for s in range(0, 2 * total, chunk):
        e = min(2 * total, s + chunk)
        c = np.arange(base + s, base + e, dtype=np.uint64)
        out[s:e] = _u64_to_sym_f32(splitmix64_np(seed, c))
    return out.view(np.complex64).reshape(batch, n)


def uniform_ragged(seed: int, sizes: Sequence[int]) -> tuple[np.ndarray, np.ndarray]:
    """Packed ragged batch: returns (flat complex64 data, int64 offsets of each signal)."""
    sizes = np.asarray(sizes, dtype=np.int64)
    offsets = np.zeros(len(sizes), dtype=np.int64)
    if len(sizes) > 1:
        np.cumsum(sizes[:-1], out=offsets[1:])
    total = int(sizes.sum())
    # the packed layout uses the same counter rule as a uniform batch of one
    # long signal, so one contiguous draw covers every signal
    flat = uniform_complex(seed, total, 1).reshape(-1) if total else np.zeros(0, np.complex64)
    return flat, offsets


# --------------------------------------------------------------------------
# torch implementation (device-side generation for large batches)
# --------------------------------------------------------------------------
def _to_i64(v: int) -> int:
    v &= MASK64
    return v - (1 << 64) if v >= (1 << 63) else v


def splitmix64_torch(seed: int, counters):
    """Same stream as :func:`splitmix64_np`, on int64 torch tensors (bit pattern of uint64)."""
    import torch

    def lsr(x, k):  # logical right shift on the uint64 bit pattern
        return (x >> k) & ((1 << (64 - k)) - 1)

    z = (counters + 1) * _to_i64(GAMMA) + _to_i64(seed)
    z = (z ^ lsr(z, 30)) * _to_i64(M1)
    z = (z ^ lsr(z, 27)) * _to_i64(M2)
    z = z ^ lsr(z, 31)
    return z


def uniform_complex_torch(seed: int, n: int, batch: int, device, first: int = 0,
                          chunk: int = 1 << 26):
    """Torch twin of :func:`uniform_complex`: complex64 tensor ``(batch, n)`` on ``device``."""
    import torch

    total = batch * n
    out = torch.empty(2 * total, dtype=torch.float32, device=device)
    base = 2 * first * n
    for s in range(0, 2 * total, chunk):
        e = min(2 * total, s + chunk)
        c = torch.arange(base + s, base + e, dtype=torch.int64, device=device)
        z = splitmix64_torch(seed, c)
        v = ((z >> 40) & ((1 << 24) - 1)).to(torch.float32)
        out[s:e] = v * (2.0 ** -23) - 1.0
    return torch.view_as_complex(out.view(total, 2)).view(batch, n)


# --------------------------------------------------------------------------
# Ragged size sampler: 7-smooth sizes drawn log-uniform
# --------------------------------------------------------------------------
def smooth_sizes(lo: int = 64, hi: int = 65536, primes=(2, 3, 5, 7)) -> list[int]:
    """Sorted integers in [lo, hi] whose prime factors are all in ``primes``."""
    vals = {1}
    for p in primes:
        grown = set()
        for v in vals:
            while v <= hi:
                grown.add(v)
                v *= p
        vals = grown
    return sorted(v for v in vals if lo <= v <= hi)


def ragged_sizes(seed: int, count: int, lo: int = 64, hi: int = 65536) -> np.ndarray:
    """``count`` sizes: u ~ U[ln lo, ln hi), then the 7-smooth size nearest to e^u in
    log distance (ties go to the smaller size)."""
    table = np.asarray(smooth_sizes(lo, hi), dtype=np.int64)
    logs = np.log(table.astype(np.float64))
    z = splitmix64_np(seed, np.arange(count, dtype=np.uint64))
    frac = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    u = math.log(lo) + frac * (math.log(hi) - math.log(lo))
    idx = np.searchsorted(logs, u)  # logs[idx-1] < u <= logs[idx]
    idx = np.clip(idx, 1, len(table) - 1)
    below = u - logs[idx - 1]
    above = logs[idx] - u
    pick = np.where(above < below, idx, idx - 1)
    return table[pick]


# --------------------------------------------------------------------------
# Synthetic greyscale images: smooth noise field plus uniform noise
# --------------------------------------------------------------------------
IMG_CELL = 64


def smooth_noise_image(seed: int, index: int, h: int = 2048, w: int = 2048,
                       cell: int = IMG_CELL) -> np.ndarray:
    """uint8 image ``index`` of the stream ``seed``.

    A lattice of uniform[0,1) values every ``cell`` pixels is interpolated with
    smoothstep-weighted bilinear interpolation (C1-continuous) to ``s``; each
    pixel is ``clamp(floor(40 + 160*s + U[-24,24) + 0.5), 0, 255)``.
    Counters: lattice point (a, b) uses ``index*2**40 + a*(gw) + b``; the noise
    of pixel (y, x) uses ``index*2**40 + 2**32 + y*w + x``.
    """
    gh, gw = (h + cell - 1) // cell + 1, (w + cell - 1) // cell + 1
    base = np.uint64(index) << np.uint64(40)
    lat_c = base + np.arange(gh * gw, dtype=np.uint64)
    lat = (splitmix64_np(seed, lat_c) >> np.uint64(40)).astype(np.float64) * 2.0 ** -24
    lat = lat.reshape(gh, gw)

    def axis(n):
        pos = np.arange(n, dtype=np.float64) / cell
        i0 = np.floor(pos).astype(np.int64)
        f = pos - i0
        return i0, f * f * (3.0 - 2.0 * f)

    iy, sy = axis(h)
    ix, sx = axis(w)
    top = lat[iy][:, ix] * (1 - sx) + lat[iy][:, ix + 1] * sx
    bot = lat[iy + 1][:, ix] * (1 - sx) + lat[iy + 1][:, ix + 1] * sx
    s = top * (1 - sy)[:, None] + bot * sy[:, None]
    noise_c = base + np.uint64(1 << 32) + np.arange(h * w, dtype=np.uint64)
    u = (splitmix64_np(seed, noise_c) >> np.uint64(40)).astype(np.float64) * 2.0 ** -24
    v = 40.0 + 160.0 * s + (-24.0 + 48.0 * u.reshape(h, w))
    return np.ascontiguousarray(np.clip(np.floor(v + 0.5), 0, 255).astype(np.uint8))


def images_complex(seed: int, count: int, h: int = 2048, w: int = 2048,
                   first: int = 0) -> np.ndarray:
    """Images ``first..first+count-1`` as complex64 (imag = 0), shape ``(count, h, w)``."""
    out = np.zeros((count, h, w), dtype=np.complex64)
    for i in range(count):
        out[i].real = smooth_noise_image(seed, first + i, h, w)
    return out


def images_rgb(seed: int, count: int, h: int = 2048, w: int = 2048, first: int = 0) -> np.ndarray:
    """Colour images ``first..first+count-1``: three smooth-noise channels per
    image (channel ch of image i is the greyscale image 3 i + ch of the stream),
    uint8 of shape ``(count, h, w, 3)``."""
    out = np.empty((count, h, w, 3), dtype=np.uint8)
    for i in range(count):
        for ch in range(3):
            out[i, :, :, ch] = smooth_noise_image(seed, 3 * (first + i) + ch, h, w)
    return out


def pattern_set(seed: int, k: int) -> np.ndarray:
    """``k`` random 4x4 integer patterns, values uniform in [28, 228), uint8
    of shape ``(k, 4, 4)``."""
    z = splitmix64_np(seed, np.arange(k * 16, dtype=np.uint64))
    return (28 + (z >> np.uint64(40)) % np.uint64(200)).astype(np.uint8).reshape(k, 4, 4)


def pattern_picks(seed: int, n: int, k: int) -> np.ndarray:
    """``n`` uniform draws from ``range(k)`` (int64)."""
    z = splitmix64_np(seed, np.arange(n, dtype=np.uint64))
    return ((z >> np.uint64(40)) % np.uint64(k)).astype(np.int64)


def blocks_to_grey_rgb(pats: np.ndarray, pick: np.ndarray) -> np.ndarray:
    """Grey RGB images (R = G = B) whose 4x4 block (r, c) of image i is
    ``pats[pick[i, r, c]]``; ``pick`` has shape ``(count, h/4, w/4)``."""
    count, bh, bw = pick.shape
    grey = pats[pick].transpose(0, 1, 3, 2, 4).reshape(count, 4 * bh, 4 * bw)
    return np.ascontiguousarray(np.repeat(grey[..., None], 3, axis=3))


# --------------------------------------------------------------------------
# The workloads (shapes, sizes and seeds only)
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Workload:
    name: str
    seed: int
    kind: str            # "uniform" | "image2d" | "ragged"
    n: int = 0           # 1D length (uniform)
    batch: int = 0       # signals / images
    shape2d: tuple = ()  # (ny, nx) for image2d
    count: int = 0       # ragged signals
    precision: str = "fp32"


def workloads() -> dict[str, Workload]:
    w = {}
    w["c1_n4096_b64"] = Workload("c1_n4096_b64", BASE_SEED + 1, "uniform", 4096, 64)
    for lg, b in ((10, 131072), (14, 8192), (18, 512), (22, 32)):
        nm = f"c2_n2^{lg}_b{b}"
        w[nm] = Workload(nm, BASE_SEED + 2, "uniform", 1 << lg, b)
    w["c3_img2048_b16"] = Workload("c3_img2048_b16", BASE_SEED + 3, "image2d",
                                   batch=16, shape2d=(2048, 2048))
    for prec in ("fp32", "fp16", "bf16", "fp16_split", "bf16_split", "bf16_split3"):
        nm = f"c4_n2^16_b4096_{prec}"
        w[nm] = Workload(nm, BASE_SEED + 4, "uniform", 1 << 16, 4096, precision=prec)
    w["c5_ragged_10000"] = Workload("c5_ragged_10000", BASE_SEED + 5, "ragged", count=10000)
    return w
