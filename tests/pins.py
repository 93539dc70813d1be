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
    convolution theorem with the oracle's FFT.
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


ALL_PINS = [pin_golden, pin_fft_vs_dft, pin_impulse, pin_constant, pin_tone, pin_geometric,
            pin_linearity, pin_parseval, pin_shift, pin_round_trip, pin_hermitian,
            pin_numpy_batch, pin_numpy_ragged, pin_numpy_2d, pin_image_2d,
            pin_conv_delta_and_shift, pin_conv_polynomial, pin_conv_numpy, pin_conv_theorem]


def run_all(o, quick=True):
    res = {}
    for p in ALL_PINS:
        try:
            ok, detail = p(o) if p is pin_golden else p(o, quick=quick)
        except Exception as e:  # a crash counts as a failed pin
            ok, detail = False, f"raised {type(e).__name__}: {e}"
        res[p.__name__] = (ok, detail)
    return res
