"""Checks that pin the FP64 oracle to facts fixed by mathematics, not by itself.

Every check takes an :class:`oracle.OracleLib` and returns ``(ok, detail)``.
They are run against the real oracle (``test_oracle.py``) and against copies of
the oracle with a planted mistake (``test_oracle_mutants.py``), which must each
fail at least one check.

The pins (the paper names the DFT and the Cooley-Tukey recursion in section
III-A without printing a formula or a value, so all of them come from the
textbook definition X[k] = sum_j x[j] exp(-2 pi i j k / N)):
  * hand-derived golden values (tests/golden/dft_small.txt);
  * the recursive FFT against the brute-force O(N^2) sum, for every 7-smooth
    N <= 1024 and lengths with a prime factor above 7;
  * closed forms: impulse, constant, pure tone, geometric sequence;
  * invariants: linearity, Parseval, shift theorem, round trip, Hermitian
    symmetry of real input (1D and 2D), exact integer DC bin of an image;
  * an independent library, numpy.fft (pocketfft), for batched, ragged and 2D
    shapes;
  * circular convolution: delta and shifted delta, polynomial products with
    exact binomial coefficients, numpy's linear convolution, and the
    convolution theorem with the oracle's FFT;
  * image block compression (section III-B): grey levels and primaries of
    the colour transform and the published JFIF inverse, 2x2 chroma squares
    and sums, the gradient of a luminance ramp, block means and deviations,
    exact recovery of well-separated clusters, the monotone k-means
    objective, and brute-force nearest codewords.
"""
from __future__ import annotations

import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "dft_small.txt")

TOL = 1e-13  # FP64 recursive FFT vs exact: ~log2(N) * 1e-16, far below this


def smooth7(limit: int) -> list[int]:
    out = []
    for n in range(1, limit + 1):
        m = n
        for p in (2, 3, 5, 7):
            while m % p == 0:
                m //= p
        if m == 1:
            out.append(n)
    return out


def _rng(seed):
    return np.random.default_rng(seed)


def _crand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _rel(a, b):
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    den = np.linalg.norm(b.ravel())
    num = np.linalg.norm((a - b).ravel())
    return num / den if den > 0 else num


def _omega(n, t, sign=-1.0):
    """exp(sign * 2 pi i t / n) with t reduced exactly mod n first."""
    t = np.mod(np.asarray(t, dtype=np.int64), n)
    return np.exp(sign * 2j * np.pi * (t.astype(np.float64) / n))


def load_golden(path: str = GOLDEN):
    cases = []
    cur = None
    with open(path) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            tag, *rest = line.split()
            if tag == "case":
                cur = {"name": rest[0], "x": [], "X": []}
                cases.append(cur)
            elif tag == "n":
                cur["n"] = int(rest[0])
            elif tag in ("x", "X"):
                cur[tag].append(complex(float(rest[0]), float(rest[1])))
    for c in cases:
        assert len(c["x"]) == c["n"] == len(c["X"]), c["name"]
    return cases


# ----------------------------------------------------------------------------
def pin_golden(o):
    bad = []
    for c in load_golden():
        x, X = np.array(c["x"]), np.array(c["X"])
        scale = max(1.0, np.abs(X).max())
        for nm, got in (("fft", o.fft(x)), ("dft", o.dft(x))):
            if np.abs(got - X).max() > 1e-14 * scale:
                bad.append(f"{c['name']}:{nm}")
        for nm, got in (("ifft", o.fft(X, True)), ("idft", o.dft(X, True))):
            if np.abs(got - x).max() > 1e-14 * max(1.0, np.abs(x).max()):
                bad.append(f"{c['name']}:{nm}")
    return not bad, ",".join(bad)


def pin_fft_vs_dft(o, quick=False):
    sizes = [1, 2, 3, 4, 5, 6, 7, 8, 9, 12, 16, 22, 25, 30, 49, 60, 64, 105, 121, 210, 256] if quick \
        else smooth7(1024) + [11, 13, 22, 26, 121, 143, 187, 2 * 11 * 13, 17 * 8]
    rng = _rng(1)
    worst = (0.0, None)
    for n in sizes:
        x = _crand(rng, n)
        for inv in (False, True):
            e = _rel(o.fft(x, inv), o.dft(x, inv))
            if e > worst[0]:
                worst = (e, (n, inv))
    return worst[0] <= TOL, f"max rel {worst[0]:.2e} at {worst[1]}"


CF_SIZES = [1, 2, 3, 8, 12, 60, 343, 1024, 4096, 6561, 3 * 5 * 7 * 16]


def pin_impulse(o, quick=False):
    worst = 0.0
    for n in CF_SIZES:
        for j0 in sorted({0, 1 % n, n // 3, n - 1}):
            x = np.zeros(n, complex)
            x[j0] = 1.0
            ref = _omega(n, j0 * np.arange(n))
            worst = max(worst, _rel(o.fft(x), ref))
            # inverse of delta[k-j0] is exp(+2 pi i j0 j / N) / N
            worst = max(worst, _rel(o.fft(x, True), _omega(n, j0 * np.arange(n), +1.0) / n))
    return worst <= TOL, f"max rel {worst:.2e}"


def pin_constant(o, quick=False):
    worst = 0.0
    c = 0.75 - 0.5j
    for n in CF_SIZES:
        ref = np.zeros(n, complex)
        ref[0] = c * n
        worst = max(worst, _rel(o.fft(np.full(n, c)), ref))
    return worst <= TOL, f"max rel {worst:.2e}"


def pin_tone(o, quick=False):
    worst = 0.0
    for n in CF_SIZES[1:]:
        for f in sorted({1, n // 2, n - 1}):
            x = _omega(n, f * np.arange(n), +1.0)
            ref = np.zeros(n, complex)
            ref[f % n] = n
            worst = max(worst, _rel(o.fft(x), ref))
    return worst <= TOL, f"max rel {worst:.2e}"


def pin_geometric(o, quick=False):
    """x[j] = a^j  ->  X[k] = (1 - a^N) / (1 - a w_N^k); every bin is non-zero."""
    a = 0.9 * np.exp(0.3j)
    worst = 0.0
    for n in CF_SIZES[1:]:
        j = np.arange(n)
        x = np.exp(j * np.log(a))
        k = np.arange(n)
        ref = (1 - a ** n) / (1 - a * _omega(n, k))
        worst = max(worst, _rel(o.fft(x), ref))
    return worst <= 1e-12, f"max rel {worst:.2e}"


def pin_linearity(o, quick=False):
    rng = _rng(2)
    worst = 0.0
    for n in (30, 256, 360, 1000):
        x, y = _crand(rng, n), _crand(rng, n)
        al, be = 0.3 - 1.1j, -2.0 + 0.25j
        worst = max(worst, _rel(o.fft(al * x + be * y), al * o.fft(x) + be * o.fft(y)))
    return worst <= TOL, f"max rel {worst:.2e}"


def pin_parseval(o, quick=False):
    rng = _rng(3)
    worst = 0.0
    for n in (7, 64, 210, 1024, 4096):
        x = _crand(rng, n)
        X = o.fft(x)
        lhs = np.sum(np.abs(x) ** 2)
        rhs = np.sum(np.abs(X) ** 2) / n
        worst = max(worst, abs(lhs - rhs) / lhs)
    return worst <= TOL, f"max rel {worst:.2e}"


def pin_shift(o, quick=False):
    """fft(x[j - s]) = w_N^{s k} X[k]."""
    rng = _rng(4)
    worst = 0.0
    for n, s in ((12, 5), (256, 3), (1050, 17)):
        x = _crand(rng, n)
        ref = _omega(n, s * np.arange(n)) * o.fft(x)
        worst = max(worst, _rel(o.fft(np.roll(x, s)), ref))
    return worst <= TOL, f"max rel {worst:.2e}"


def pin_round_trip(o, quick=False):
    rng = _rng(5)
    worst = 0.0
    for n in (1, 2, 5, 96, 343, 4096):
        x = _crand(rng, n)
        worst = max(worst, _rel(o.fft(o.fft(x), True), x))
    return worst <= TOL, f"max rel {worst:.2e}"


def pin_hermitian(o, quick=False):
    rng = _rng(6)
    worst = 0.0
    for n in (8, 15, 98, 1024):
        X = o.fft(rng.standard_normal(n))
        worst = max(worst, _rel(X, np.conj(X[(-np.arange(n)) % n])))
    return worst <= TOL, f"max rel {worst:.2e}"


def pin_numpy_batch(o, quick=False):
    rng = _rng(7)
    worst = (0.0, None)
    shapes = [(4, 4096), (3, 64), (5, 1000)] if quick else \
        [(4, 4096), (3, 64), (5, 1000), (2, 1 << 14), (1, 1 << 16), (2, 3 * 5 * 7 * 64)]
    for b, n in shapes:
        x = _crand(rng, b, n).astype(np.complex64)
        xd = x.astype(np.complex128)
        for inv, ref in ((False, np.fft.fft(xd, axis=-1)), (True, np.fft.ifft(xd, axis=-1))):
            got = o.fft_batch(x, inv)
            e = max(_rel(got[i], ref[i]) for i in range(b))
            if e > worst[0]:
                worst = (e, (b, n, inv))
    return worst[0] <= TOL, f"max rel {worst[0]:.2e} at {worst[1]}"


def pin_numpy_ragged(o, quick=False):
    rng = _rng(8)
    sizes = np.array([64, 7, 1000, 81, 4096, 1, 625, 343, 2 * 3 * 5 * 7], np.int64)
    gaps = np.array([0, 3, 0, 1, 5, 0, 2, 0, 4], np.int64)
    offsets = np.cumsum(np.concatenate([[0], sizes[:-1] + gaps[1:]]))
    total = int(offsets[-1] + sizes[-1] + 2)
    flat = _crand(rng, total).astype(np.complex64)
    worst = 0.0
    for inv in (False, True):
        got = o.fft_ragged(flat, sizes, offsets, inv)
        for n, off in zip(sizes, offsets):
            seg = flat[off:off + n].astype(np.complex128)
            ref = np.fft.ifft(seg) if inv else np.fft.fft(seg)
            worst = max(worst, _rel(got[off:off + n], ref))
    return worst <= TOL, f"max rel {worst:.2e}"


def pin_numpy_2d(o, quick=False):
    rng = _rng(9)
    worst = 0.0
    for b, ny, nx in ((2, 12, 20), (1, 64, 48), (2, 128, 128)):
        x = _crand(rng, b, ny, nx).astype(np.complex64)
        xd = x.astype(np.complex128)
        for inv in (False, True):
            ref = np.fft.ifft2(xd) if inv else np.fft.fft2(xd)
            got = o.fft2d(x, inv)
            worst = max(worst, max(_rel(got[i], ref[i]) for i in range(b)))
    return worst <= TOL, f"max rel {worst:.2e}"


def pin_image_2d(o, quick=False):
    """Real uint8 image: exact integer DC bin and Hermitian symmetry
    X[k1, k2] = conj(X[-k1, -k2])."""
    rng = _rng(10)
    img = rng.integers(0, 256, size=(96, 160)).astype(np.float32)
    X = o.fft2d(img.astype(np.complex64))
    dc_ok = X[0, 0].real == float(img.sum()) and X[0, 0].imag == 0.0
    ky = (-np.arange(96)) % 96
    kx = (-np.arange(160)) % 160
    herm = _rel(X, np.conj(X[ky][:, kx]))
    return dc_ok and herm <= TOL, f"dc={X[0, 0]} vs {img.sum()}, hermitian rel {herm:.2e}"


# ---------------------------------------------------------------------------
# circular convolution (section III-A names convolution and polynomial
# multiplication among the uses of the DFT): y[j] = sum_m x[m] h[(j - m) mod n]
# ---------------------------------------------------------------------------
def pin_conv_delta_and_shift(o, quick=False):
    """h = delta[j - s] moves x by s places, exactly (s = 0: y = x)."""
    rng = _rng(21)
    ok = True
    for n in (1, 2, 7, 16, 60):
        x = _crand(rng, 3, n).astype(np.complex64)
        for s in sorted({0, 1 % n, n - 1, n // 2}):
            h = np.zeros(n, np.complex64)
            h[s] = 1.0
            y = o.circular_conv(x, h)
            ok &= bool(np.array_equal(y, np.roll(x.astype(np.complex128), s, axis=-1)))
    return ok, "delta and shifted delta"


def pin_conv_polynomial(o, quick=False):
    """Polynomial multiplication: (1 + z)^p (1 + z)^q = (1 + z)^(p+q), whose
    coefficients are binomial numbers, exact in double; zero padding to
    n > p + q makes the circular product the ordinary one.  Also (1 + i z)^p
    times (1 - i z)^p = (1 + z^2)^p."""
    from math import comb
    ok = True
    for p_, q_, n in ((3, 4, 8), (7, 9, 32), (12, 5, 18)):
        a = np.zeros(n, np.complex64)
        b = np.zeros(n, np.complex64)
        a[: p_ + 1] = [comb(p_, k) for k in range(p_ + 1)]
        b[: q_ + 1] = [comb(q_, k) for k in range(q_ + 1)]
        want = np.zeros(n)
        want[: p_ + q_ + 1] = [comb(p_ + q_, k) for k in range(p_ + q_ + 1)]
        ok &= bool(np.array_equal(o.circular_conv(a, b), want.astype(np.complex128)))
    p_, n = 6, 16
    a = np.array([comb(p_, k) * (1j ** k) for k in range(p_ + 1)] + [0] * (n - p_ - 1), np.complex64)
    b = np.array([comb(p_, k) * ((-1j) ** k) for k in range(p_ + 1)] + [0] * (n - p_ - 1),
                 np.complex64)
    want = np.zeros(n, np.complex128)
    want[0: 2 * p_ + 1: 2] = [comb(p_, k) for k in range(p_ + 1)]
    ok &= bool(np.array_equal(o.circular_conv(a, b), want))
    return ok, "binomial products"


def pin_conv_numpy(o, quick=False):
    """Independent library: the circular convolution is the middle of numpy's
    linear convolution of x with two periods of h (per-signal filters and one
    shared filter)."""
    rng = _rng(22)
    worst = 0.0
    for n in (5, 64, 210):
        x = _crand(rng, 4, n).astype(np.complex64)
        hs = _crand(rng, 4, n).astype(np.complex64)
        y1 = o.circular_conv(x, hs)
        y2 = o.circular_conv(x, hs[1])
        for b in range(4):
            xd = x[b].astype(np.complex128)
            for y, h in ((y1[b], hs[b]), (y2[b], hs[1])):
                hh = np.concatenate([h, h]).astype(np.complex128)
                ref = np.convolve(xd, hh)[n:2 * n]
                worst = max(worst, _rel(y, ref))
    return worst <= TOL, f"max rel {worst:.2e}"


def pin_conv_theorem(o, quick=False):
    """Convolution theorem: DFT(x conv h) = DFT(x) DFT(h), with the oracle's
    own recursive FFT on both sides."""
    rng = _rng(23)
    worst = 0.0
    for n in (8, 45, 256):
        x = _crand(rng, n).astype(np.complex64)
        h = _crand(rng, n).astype(np.complex64)
        lhs = o.fft(o.circular_conv(x, h))
        rhs = o.fft(x.astype(np.complex128)) * o.fft(h.astype(np.complex128))
        worst = max(worst, _rel(lhs, rhs))
    return worst <= TOL, f"max rel {worst:.2e}"


# ---------------------------------------------------------------------------
# image block compression (section III-B, steps a-e)
# ---------------------------------------------------------------------------
def pin_img_ycc_values(o, quick=False):
    """(a) White, black and every grey map to Y = the grey level and Cb = Cr =
    128 exactly (each row of the transform sums to 1, 0, 0); the published
    JFIF inverse, R = Y + 1.402 (Cr - 128), G = Y - 0.344136 (Cb - 128) -
    0.714136 (Cr - 128), B = Y + 1.772 (Cb - 128), written independently,
    recovers random colours; the pure primaries give the standard values."""
    ok = True
    for v in (0, 1, 128, 254, 255):
        rgb = np.full((2, 2, 3), v, np.uint8)
        y, cb, cr = o.img_ycc(rgb)
        ok &= bool(np.allclose(y, v, rtol=0, atol=1e-12) and np.allclose(cb, 128, atol=1e-12)
                   and np.allclose(cr, 128, atol=1e-12))
    rng = _rng(31)
    rgb = rng.integers(0, 256, (2, 200, 3)).astype(np.uint8)
    # per-pixel values: undo the 2x2 averaging by using 2x2 constant squares
    rgb4 = np.repeat(np.repeat(rgb[:1], 2, axis=0), 2, axis=1)
    y, cb, cr = o.img_ycc(rgb4)
    Y = y[0, ::2]
    R = Y + 1.402 * (cr[0] - 128)
    G = Y - 0.344136 * (cb[0] - 128) - 0.714136 * (cr[0] - 128)
    B = Y + 1.772 * (cb[0] - 128)
    err = np.max(np.abs(np.stack([R, G, B], -1) - rgb[0].astype(np.float64)))
    ok &= bool(err < 2e-3)
    red = np.zeros((2, 2, 3), np.uint8)
    red[..., 0] = 255
    y, cb, cr = o.img_ycc(red)
    ok &= bool(abs(y[0, 0] - 76.245) < 1e-9 and abs(cb[0, 0] - (128 - 43.02768)) < 1e-9
               and abs(cr[0, 0] - 255.5) < 1e-9)
    return ok, f"inverse max err {err:.2e}"


def pin_img_downscale(o, quick=False):
    """(b) A chroma plane constant on each 2x2 square comes out as those
    constants; any image keeps the chroma sum (4 x the downscaled sum)."""
    rng = _rng(32)
    small = rng.integers(0, 256, (5, 7, 3)).astype(np.uint8)
    big = np.repeat(np.repeat(small, 2, axis=0), 2, axis=1)
    _, cb, cr = o.img_ycc(big)
    r, g, b = (small[..., i].astype(np.float64) for i in range(3))
    want_cb = 128 - 0.168736 * r - 0.331264 * g + 0.5 * b
    ok = bool(np.allclose(cb, want_cb, rtol=0, atol=1e-9))
    img = rng.integers(0, 256, (12, 20, 3)).astype(np.uint8)
    _, cb2, cr2 = o.img_ycc(img)
    r, g, b = (img[..., i].astype(np.float64) for i in range(3))
    full_cr = 128 + 0.5 * r - 0.418688 * g - 0.081312 * b
    ok &= bool(abs(4 * cr2.sum() - full_cr.sum()) < 1e-7)
    ok &= bool(np.allclose(cr2, full_cr.reshape(6, 2, 10, 2).mean(axis=(1, 3)), atol=1e-9))
    return ok, "square constants and chroma sums"


def pin_img_blocks(o, quick=False):
    """(c) A luminance ramp Y = a x + b y has |grad Y| = sqrt(a^2 + b^2) at
    every pixel off the edges (half that along an axis at the edges, where the
    difference is one-sided over one pixel); a block's mean is the ramp at its
    centre and its deviations sum to zero; a flat image has zero activity and
    deviations."""
    h, w = 16, 24
    a, b = 3.0, -1.5
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    Y = a * xx + b * yy
    mean, act, dev = o.img_blocks(Y)
    inner = act[1:-1, 1:-1]
    ok = bool(np.allclose(inner, np.hypot(a, b), rtol=0, atol=1e-12))
    centres = a * (4 * np.arange(w // 4) + 1.5)[None, :] + b * (4 * np.arange(h // 4) + 1.5)[:, None]
    ok &= bool(np.allclose(mean, centres, atol=1e-12))
    ok &= bool(np.allclose(dev.sum(axis=1), 0, atol=1e-11))
    ok &= bool(np.allclose(dev[0].reshape(4, 4), Y[:4, :4] - Y[:4, :4].mean(), atol=1e-12))
    # corner block: edge pixels see one-sided differences
    g = np.zeros((4, 4))
    for i in range(4):
        for j in range(4):
            gx = 0.5 * (Y[i, min(j + 1, w - 1)] - Y[i, max(j - 1, 0)])
            gy = 0.5 * (Y[min(i + 1, h - 1), j] - Y[max(i - 1, 0), j])
            g[i, j] = np.hypot(gx, gy)
    ok &= bool(abs(act[0, 0] - g.mean()) < 1e-12)
    m2, a2, d2 = o.img_blocks(np.full((8, 8), 77.0))
    ok &= bool(np.all(a2 == 0) and np.all(d2 == 0) and np.all(m2 == 77.0))
    return ok, "ramp, corner and flat image"


def pin_img_kmeans_clusters(o, quick=False):
    """(d) K well-separated clusters of equal size, stored one cluster after
    the other: the initial codewords (ranks floor(c P / K)) fall one in each
    cluster, and one Lloyd iteration gives exactly the cluster means (numpy);
    more iterations leave them there.  Blocks below tau take no part."""
    rng = _rng(33)
    K, per = 6, 40
    centres = rng.normal(0, 50, (K, 16))
    dev = np.concatenate([centres[c] + rng.normal(0, 0.5, (per, 16)) for c in range(K)])
    act = np.full(K * per, 10.0)
    extra = rng.normal(0, 50, (7, 16))       # uniform blocks, never clustered
    dev_all = np.concatenate([dev[:100], extra, dev[100:]])
    act_all = np.concatenate([act[:100], np.full(7, 0.5), act[100:]])
    want = np.stack([dev[c * per:(c + 1) * per].mean(axis=0) for c in range(K)])
    ok = True
    for iters in (1, 4):
        cb, P = o.img_kmeans(dev_all, act_all, 1.0, K, iters)
        ok &= bool(P == K * per and np.allclose(cb, want, rtol=0, atol=1e-10))
    cb0, _ = o.img_kmeans(dev_all, act_all, 1.0, K, 0)
    ok &= bool(np.array_equal(cb0, dev[[c * per for c in range(K)]]))
    return ok, "cluster means"


def pin_img_kmeans_monotone(o, quick=False):
    """(d) Lloyd's iteration never increases the within-cluster sum of
    squares (each step is a minimisation), here on unclustered data."""
    rng = _rng(34)
    dev = rng.normal(0, 10, (500, 16))
    act = np.full(500, 5.0)
    prev = np.inf
    ok = True
    for it in range(6):
        cb, _ = o.img_kmeans(dev, act, 1.0, 12, it)
        d = ((dev[:, None, :] - cb[None]) ** 2).sum(-1).min(axis=1).sum()
        ok &= bool(d <= prev * (1 + 1e-12))
        prev = d
    return ok, f"final sse {prev:.4g}"


def pin_img_encode(o, quick=False):
    """(e) Brute force with numpy: code 0 below tau, else 1 + the argmin of
    the squared distances (first index on ties); margins are the gap to the
    second-nearest."""
    rng = _rng(35)
    dev = rng.normal(0, 10, (300, 16))
    act = rng.uniform(0, 10, 300)
    cb = rng.normal(0, 10, (9, 16))
    cb[4] = cb[2]                      # a tie: the lower index must win
    dev[7] = cb[2]
    act[7] = 6.0
    act[5] = 4.0                       # activity exactly tau: a pattern block
    code, margin = o.img_encode(dev, act, 4.0, cb)
    d = ((dev[:, None, :] - cb[None]) ** 2).sum(-1)
    want = np.where(act < 4.0, 0, 1 + np.argmin(d, axis=1))
    srt = np.sort(d, axis=1)
    ok = bool(np.array_equal(code, want))
    pat = act >= 4.0
    ok &= bool(np.allclose(margin[pat], (srt[:, 1] - srt[:, 0])[pat], rtol=1e-12, atol=1e-9))
    ok &= bool(code[7] == 3 and code[5] != 0)
    return ok, "brute-force codes"


ALL_PINS = [pin_golden, pin_fft_vs_dft, pin_impulse, pin_constant, pin_tone, pin_geometric,
            pin_linearity, pin_parseval, pin_shift, pin_round_trip, pin_hermitian,
            pin_numpy_batch, pin_numpy_ragged, pin_numpy_2d, pin_image_2d,
            pin_conv_delta_and_shift, pin_conv_polynomial, pin_conv_numpy, pin_conv_theorem,
            pin_img_ycc_values, pin_img_downscale, pin_img_blocks, pin_img_kmeans_clusters,
            pin_img_kmeans_monotone, pin_img_encode]


def run_all(o, quick=True):
    res = {}
    for p in ALL_PINS:
        try:
            ok, detail = p(o) if p is pin_golden else p(o, quick=quick)
        except Exception as e:  # a crash counts as a failed pin
            ok, detail = False, f"raised {type(e).__name__}: {e}"
        res[p.__name__] = (ok, detail)
    return res
