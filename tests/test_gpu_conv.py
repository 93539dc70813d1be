"""GPU parity of the fused circular convolution (FFT_F_CONV plans, fft_conv_exec).

Section III-A of the paper names convolution and polynomial multiplication
among the uses of the DFT.  The library computes out_b = IDFT(DFT(x_b) H_b),
with H_b = DFT(h_b) taken by the library's own forward transform (tested
elsewhere), in one launch for N <= 16384 and three for longer N.  The
reference is the oracle's O(N^2) circular convolution from its definition
(lengths up to 2^15), or, for longer lengths and the full benchmark batch,
the oracle's FFT of x times the oracle's FFT of h, rounded to complex64 and
taken back by the oracle's inverse (the convolution theorem, which the oracle
pins against its direct sum; the complex64 rounding adds about 6e-8).
Tolerance: relative L2 <= 1e-5 per signal, gated on the max over the batch.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL_FP32, say, to_dev

pytestmark = pytest.mark.gpu


def _dp():
    import paper_1203_4938_amd as dp
    return dp


def _theorem_ref(x: np.ndarray, h: np.ndarray) -> np.ndarray:
    """Oracle convolution through its FFT: x (batch, n), h (n,) or (batch, n)."""
    X = oracle.fft_batch(x)
    H = oracle.fft_batch(h.reshape(-1, x.shape[-1]))
    prod = (X * H).astype(np.complex64)
    return oracle.fft_batch(prod, inverse=True)


def _check(y, ref, what):
    e = oracle.rel_l2(y, ref)
    say(f"   {what}: max rel L2 {float(np.max(e)):.3e} over {len(e)} signals")
    assert float(np.max(e)) <= TOL_FP32, (what, float(np.max(e)))


def _run(n, batch, shared, seed, direct=True, inplace=False, dist=0, fdist=0):
    import torch
    dp = _dp()
    x = synth.uniform_complex(seed, n, batch)
    hb = 1 if shared else batch
    h = synth.uniform_complex(seed + 7777, n, hb)
    p = dp.Plan(n, batch, conv=True, inplace=inplace, dist=dist)
    hp = dp.Plan(n, hb)
    H = hp.exec(to_dev(h))  # the filter spectrum, natural order
    if dist:
        xd = torch.zeros((batch - 1) * dist + n, dtype=torch.complex64, device="cuda")
        for b in range(batch):
            xd[b * dist:b * dist + n].copy_(torch.from_numpy(x[b]))
    else:
        xd = to_dev(x)
    if fdist and not shared:
        Hs = torch.zeros((batch - 1) * fdist + n, dtype=torch.complex64, device="cuda")
        for b in range(batch):
            Hs[b * fdist:b * fdist + n].copy_(H[b])
        ws = p.workspace(xd.device)
        out = xd if inplace else torch.empty_like(xd)
        st = dp.fft_conv_exec(p.handle, xd.data_ptr(), Hs.data_ptr(), fdist, out.data_ptr(),
                              ws.data_ptr() if ws is not None else 0,
                              torch.cuda.current_stream().cuda_stream)
        assert st == dp.FFT_OK, dp.fft_last_error()
        y = out
    else:
        y = p.conv(xd, H.reshape(-1) if shared else H, out=xd if inplace else None)
    torch.cuda.synchronize()
    yh = y.cpu().numpy()
    if dist:
        yh = np.stack([yh[b * dist:b * dist + n] for b in range(batch)])
    ref = oracle.circular_conv(x, h[0] if shared else h) if direct else \
        _theorem_ref(x, h[0] if shared else h)
    return yh.reshape(batch, n), ref


@pytest.mark.parametrize("shared", [True, False], ids=["shared", "per_signal"])
@pytest.mark.parametrize("lg", list(range(0, 15)))
def test_single_pass_conv(lg, shared):
    """Every power of two 1..2^14, one launch; batches with a partly empty last
    workgroup."""
    n = 1 << lg
    batch = 2 * max(1, 256 // max(1, n // 16)) + 3 if n <= 2048 else 5
    say(f"[conv] n={n} batch={batch} shared={shared}")
    y, ref = _run(n, batch, shared, synth.BASE_SEED + 300 + lg)
    _check(y, ref, f"n={n}")


@pytest.mark.parametrize("lg,batch", [(15, 2), (16, 2), (18, 2), (20, 1), (22, 1), (24, 1)])
def test_four_step_conv(lg, batch):
    """Three launches: forward column pass, fused rows, inverse column pass.
    2^15 against the direct sum, longer lengths through the oracle's FFT."""
    n = 1 << lg
    say(f"[conv four-step] n=2^{lg} batch={batch}")
    for shared in (True, False):
        y, ref = _run(n, batch, shared, synth.BASE_SEED + 330 + lg, direct=(lg <= 15))
        _check(y, ref, f"n=2^{lg} shared={shared}")


@pytest.mark.parametrize("n", [64, 4096, 1 << 16])
def test_conv_in_place_and_strided(n):
    say(f"[conv layouts] n={n}")
    y, ref = _run(n, 3, False, synth.BASE_SEED + 350, direct=(n <= 4096), inplace=True)
    _check(y, ref, "in place")
    y, ref = _run(n, 3, False, synth.BASE_SEED + 351, direct=(n <= 4096), dist=n + 40,
                  fdist=n + 24)
    _check(y, ref, "dist and filter_dist above N")


def test_polynomial_product_exact():
    """Integer polynomials of degree < n/2, zero-padded to n: the circular
    convolution is their product, and rounding the FP32 result gives every
    coefficient exactly (the oracle's sums are exact in FP64 here)."""
    import torch
    dp = _dp()
    n, batch = 2048, 16
    rng = np.random.default_rng(12034938)
    a = np.zeros((batch, n), np.complex64)
    b = np.zeros((batch, n), np.complex64)
    a[:, :n // 2] = rng.integers(-9, 10, (batch, n // 2))
    b[:, :n // 2] = rng.integers(-9, 10, (batch, n // 2))
    p = dp.Plan(n, batch, conv=True)
    B = p.exec(to_dev(b))
    y = p.conv(to_dev(a), B)
    torch.cuda.synchronize()
    got = np.rint(y.cpu().numpy().real).astype(np.int64)
    want = oracle.circular_conv(a, b)
    assert np.array_equal(want.imag, np.zeros_like(want.imag))
    assert np.array_equal(got, want.real.astype(np.int64))
    err = float(np.max(np.abs(y.cpu().numpy() - want)))
    say(f"[conv polynomial] n={n}: all coefficients exact after rounding (max abs err {err:.2e})")


def test_conv_batch_zero_and_errors():
    import torch
    dp = _dp()
    p = dp.Plan(64, 0, conv=True)
    assert dp.fft_conv_exec(p.handle, 0, 0, 0, 0) == dp.FFT_OK
    q = dp.Plan(64, 4)  # made without FFT_F_CONV
    x = torch.zeros(4 * 64, dtype=torch.complex64, device="cuda")
    assert dp.fft_conv_exec(q.handle, x.data_ptr(), x.data_ptr(), 0, x.data_ptr() + 0) == \
        dp.FFT_E_INVALID
    r = dp.Plan(64, 4, conv=True)
    y = torch.empty_like(x)
    assert dp.fft_conv_exec(r.handle, x.data_ptr(), 0, 0, y.data_ptr()) == dp.FFT_E_INVALID
    assert dp.fft_conv_exec(r.handle, x.data_ptr(), x.data_ptr(), 10, y.data_ptr()) == \
        dp.FFT_E_INVALID
    assert dp.fft_conv_exec(r.handle, x.data_ptr(), x.data_ptr() + 4, 0, y.data_ptr()) == \
        dp.FFT_E_INVALID
    assert dp.fft_conv_exec(r.handle, x.data_ptr(), x.data_ptr(), 0, x.data_ptr()) == \
        dp.FFT_E_INVALID  # in place without FFT_F_INPLACE
    big = dp.Plan(1 << 16, 2, conv=True)
    xb = torch.zeros(2 << 16, dtype=torch.complex64, device="cuda")
    assert dp.fft_conv_exec(big.handle, xb.data_ptr(), xb.data_ptr(), 0,
                            torch.empty_like(xb).data_ptr(), 0) == dp.FFT_E_INVALID  # no workspace


def test_conv_full_benchmark_batch_every_signal():
    """The benchmark's convolution workload: N = 4096, batch 32768 (1 GiB),
    one shared filter, in the plan the benchmark times; every signal against
    the oracle (through its FFT), streamed in chunks."""
    import torch
    dp = _dp()
    n, batch = 4096, 32768
    seed = synth.BASE_SEED + 6
    x = synth.uniform_complex_torch(seed, n, batch, "cuda")
    h = synth.uniform_complex(seed + 7777, n, 1)
    p = dp.Plan(n, batch, conv=True)
    say("[conv full]", p.describe().replace("\n", " | "))
    H = dp.Plan(n, 1).exec(to_dev(h))
    y = p.conv(x, H.reshape(-1))
    torch.cuda.synchronize()
    Hd = oracle.fft_batch(h)
    worst = 0.0
    k = 2048
    for s0 in range(0, batch, k):
        xs = x[s0:s0 + k].cpu().numpy()
        prod = (oracle.fft_batch(xs) * Hd).astype(np.complex64)
        ref = oracle.fft_batch(prod, inverse=True)
        e = oracle.rel_l2(y[s0:s0 + k].cpu().numpy(), ref)
        worst = max(worst, float(np.max(e)))
    say(f"   every signal: max rel L2 {worst:.3e} over {batch} signals")
    assert worst <= TOL_FP32
