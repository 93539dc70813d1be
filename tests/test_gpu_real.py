"""Parity of the real-input transforms (FFT_F_REAL) with the FP64 oracle.

A real signal's spectrum is the complex DFT of the signal with zero imaginary
parts, of which the library returns bins 0..N/2 (rank 2: columns 0..nx/2).  The
oracle therefore checks the forward transform with its own complex transform
of the same samples, cut to those bins, and the inverse with its complex
inverse of the Hermitian extension of the half spectrum the library was
given (the real part; the imaginary part of that inverse is zero up to FP64
rounding).  Tolerance: relative L2 <= 1e-5 per signal (image), gated on the
max over the batch, as for the complex FP32 path."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL_FP32, say

pytestmark = pytest.mark.gpu


def herm_extend_1d(half: np.ndarray, n: int) -> np.ndarray:
    """Full length-n spectra from bins 0..n/2 (last axis): X[n-k] = conj X[k]."""
    full = np.empty(half.shape[:-1] + (n,), dtype=np.complex128)
    w = n // 2 + 1
    full[..., :w] = half
    k = np.arange(w, n)
    full[..., w:] = np.conj(half[..., n - k])
    return full


def herm_extend_2d(half: np.ndarray, nx: int) -> np.ndarray:
    """Full (ny, nx) spectra from columns 0..nx/2: X[ky, kx] = conj X[-ky, -kx]."""
    ny = half.shape[-2]
    w = nx // 2 + 1
    full = np.empty(half.shape[:-1] + (nx,), dtype=np.complex128)
    full[..., :w] = half
    ky = (-np.arange(ny)) % ny
    kx = np.arange(w, nx)
    full[..., w:] = np.conj(half[..., ky[:, None], (nx - kx)[None, :]])
    return full


def _as_c64(real: np.ndarray) -> np.ndarray:
    return real.astype(np.complex64)


def _real_batch(seed: int, n: int, batch: int) -> np.ndarray:
    """Real samples: the real parts of the seeded uniform stream."""
    return np.ascontiguousarray(synth.uniform_complex(seed, n, batch).real)


SIZES_1D = [2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384, 32768,
            1 << 16, 1 << 18, 1 << 20, 1 << 22,
            # even 7-smooth lengths: the runtime-radix core (single pass up to
            # N/2 = 16384, then the four-step pair) and the pairing launch
            6, 10, 14, 30, 96, 1000, 6000, 30000, 100000, 118098, 2 * 5 ** 7]


@pytest.mark.parametrize("n", SIZES_1D)
def test_real_1d_forward_inverse(n):
    import torch

    import paper_1203_4938_amd as dp
    # several workgroups and a ragged last tile; above 32768 (the four-step
    # core and the pairing launch) a few signals
    batch = 521 if n <= 1024 else 37 if n <= 32768 else 3
    x = _real_batch(synth.BASE_SEED + 31, n, batch)
    p = dp.Plan(n, batch, real=True)
    say(f"[real 1d] n={n} batch={batch}:", p.describe().replace("\n", " | "))
    xd = torch.from_numpy(x).cuda()
    spec = p.exec(xd)
    torch.cuda.synchronize()
    assert spec.shape == (batch, n // 2 + 1) and spec.dtype == torch.complex64
    ref = oracle.fft_batch(_as_c64(x))[:, : n // 2 + 1]
    ef = oracle.rel_l2_f32(spec.cpu().numpy(), ref)
    # inverse of the oracle's half spectrum (complex64) vs the oracle's inverse
    half = ref.astype(np.complex64)
    back = p.exec(torch.from_numpy(half).cuda(), inverse=True)
    rt = p.exec(spec, inverse=True)
    torch.cuda.synchronize()
    assert back.shape == (batch, n) and back.dtype == torch.float32
    iref = oracle.fft_batch(herm_extend_1d(half, n).astype(np.complex64), inverse=True)
    ei = oracle.rel_l2_f32(_as_c64(back.cpu().numpy()), iref)
    er = oracle.rel_l2_f32(_as_c64(rt.cpu().numpy()), x.astype(np.complex128))
    say(f"   forward max {ef.max():.3e}  inverse max {ei.max():.3e}  round trip max {er.max():.3e}")
    assert ef.max() <= TOL_FP32
    assert ei.max() <= TOL_FP32
    assert er.max() <= TOL_FP32


def test_real_1d_closed_forms():
    """A cosine of frequency f has exactly two nonzero bins: X[f] = N/2
    (and X[N-f], which the half spectrum does not hold); a constant puts N*c
    in bin 0; alternating signs put N in bin N/2."""
    import torch

    import paper_1203_4938_amd as dp
    for n in (4096, 1 << 20):  # one launch; the four-step core and the pairing launch
        j = np.arange(n)
        f = 37
        rows = np.stack([np.cos(2 * np.pi * f * j / n), np.full(n, 0.75), (-1.0) ** j]).astype(np.float32)
        p = dp.Plan(n, 3, real=True)
        y = p.exec(torch.from_numpy(rows).cuda()).cpu().numpy()
        expect = np.zeros((3, n // 2 + 1), dtype=np.complex128)
        expect[0, f] = n / 2
        expect[1, 0] = 0.75 * n
        expect[2, n // 2] = n
        err = np.abs(y - expect).max(axis=1) / np.abs(expect).max(axis=1)
        say(f"[real closed forms] n={n} max abs error / peak: {err}")
        assert np.all(err <= 1e-5)


def test_real_2d_small_images():
    """Rank-2 real plans on small images, several shapes, against the
    oracle's 2D transforms."""
    import torch

    import paper_1203_4938_amd as dp
    for ny, nx, b in ((1, 8, 3), (16, 2, 5), (64, 128, 7), (256, 64, 3), (32, 4096, 2)):
        x = _real_batch(synth.BASE_SEED + 33, ny * nx, b).reshape(b, ny, nx)
        p = dp.Plan(shape=(ny, nx), batch=b, rank=2, real=True)
        xd = torch.from_numpy(x).cuda()
        spec = p.exec(xd)
        torch.cuda.synchronize()
        ref = oracle.fft2d(_as_c64(x))[:, :, : nx // 2 + 1]
        ef = oracle.rel_l2_f32(spec.cpu().numpy(), ref)
        half = ref.astype(np.complex64)
        back = p.exec(torch.from_numpy(half).cuda(), inverse=True)
        torch.cuda.synchronize()
        iref = oracle.fft2d(herm_extend_2d(half, nx).astype(np.complex64), inverse=True)
        ei = oracle.rel_l2_f32(_as_c64(back.cpu().numpy()), iref)
        say(f"[real 2d] {b} x {ny}x{nx}: forward max {ef.max():.3e} inverse max {ei.max():.3e}")
        assert ef.max() <= TOL_FP32 and ei.max() <= TOL_FP32


@pytest.mark.parametrize("ny,nx,b", [(100, 128, 3), (96, 90, 2), (3, 6, 4), (1, 10, 3), (30, 2, 3),
                                     (243, 1000, 2), (2048, 2000, 1), (64, 30000, 1)])
def test_real_2d_mixed_images(ny, nx, b):
    """Real images whose sides are not both powers of two (runtime-radix rows,
    the pairing launch, runtime-radix columns), both directions against the
    oracle's 2D transforms, and the round trip."""
    import torch

    import paper_1203_4938_amd as dp
    x = _real_batch(synth.BASE_SEED + 34, ny * nx, b).reshape(b, ny, nx)
    p = dp.Plan(shape=(ny, nx), batch=b, rank=2, real=True)
    say(f"[real 2d mixed] {b} x {ny}x{nx}:", p.describe().replace("\n", " | "))
    xd = torch.from_numpy(x).cuda()
    spec = p.exec(xd)
    torch.cuda.synchronize()
    assert spec.shape == (b, ny, nx // 2 + 1)
    ref = oracle.fft2d(_as_c64(x))[:, :, : nx // 2 + 1]
    ef = oracle.rel_l2_f32(spec.cpu().numpy(), ref)
    half = ref.astype(np.complex64)
    back = p.exec(torch.from_numpy(half).cuda(), inverse=True)
    rt = p.exec(spec, inverse=True)
    torch.cuda.synchronize()
    iref = oracle.fft2d(herm_extend_2d(half, nx).astype(np.complex64), inverse=True)
    ei = oracle.rel_l2_f32(_as_c64(back.cpu().numpy()), iref)
    er = oracle.rel_l2_f32(_as_c64(rt.cpu().numpy()), x.astype(np.complex128))
    say(f"   forward max {ef.max():.3e} inverse max {ei.max():.3e} round trip max {er.max():.3e}")
    assert ef.max() <= TOL_FP32 and ei.max() <= TOL_FP32 and er.max() <= TOL_FP32


def test_real_2d_c3_every_image():
    """The 16 greyscale images of 2048 x 2048 (the image workload), every
    image, both directions, plus the round trip and the exact DC bins."""
    import torch

    import paper_1203_4938_amd as dp
    seed = synth.BASE_SEED + 3
    ny = nx = 2048
    b = 16
    w = nx // 2 + 1
    imgs = np.ascontiguousarray(
        np.stack([synth.smooth_noise_image(seed, i) for i in range(b)]).astype(np.float32))
    p = dp.Plan(shape=(ny, nx), batch=b, rank=2, real=True)
    say("[real c3]", p.describe().replace("\n", " | "))
    xd = torch.from_numpy(imgs).cuda()
    spec = p.exec(xd)
    rt = p.exec(spec, inverse=True)
    torch.cuda.synchronize()
    ef, ei, er = np.empty(b), np.empty(b), np.empty(b)
    half_all = np.empty((b, ny, w), dtype=np.complex64)
    for i0 in range(0, b, 2):
        sl = slice(i0, i0 + 2)
        ref = oracle.fft2d(_as_c64(imgs[sl]))[:, :, :w]
        ef[sl] = oracle.rel_l2_f32(spec[sl].cpu().numpy(), ref)
        half_all[sl] = ref.astype(np.complex64)
        er[sl] = oracle.rel_l2_f32(_as_c64(rt[sl].cpu().numpy()), imgs[sl].astype(np.complex128))
    dc = spec[:, 0, 0].real.double().cpu().numpy()
    sums = imgs.astype(np.float64).reshape(b, -1).sum(axis=1)
    del spec, rt
    back = p.exec(torch.from_numpy(half_all).cuda(), inverse=True)
    torch.cuda.synchronize()
    for i0 in range(0, b, 2):
        sl = slice(i0, i0 + 2)
        iref = oracle.fft2d(herm_extend_2d(half_all[sl], nx).astype(np.complex64), inverse=True)
        ei[sl] = oracle.rel_l2_f32(_as_c64(back[sl].cpu().numpy()), iref)
    say(f"   forward max {ef.max():.3e} mean {ef.mean():.3e}; inverse max {ei.max():.3e}; "
        f"round trip max {er.max():.3e}; DC max rel dev {np.max(np.abs(dc - sums) / sums):.2e}")
    assert ef.max() <= TOL_FP32 and ei.max() <= TOL_FP32 and er.max() <= TOL_FP32
    assert np.all(np.abs(dc - sums) <= 1e-5 * sums)
    del back
    torch.cuda.empty_cache()


def test_real_plan_edges():
    """Empty batch is a no-op; the real plans reject what they do not support
    before any launch."""
    import torch

    import paper_1203_4938_amd as dp
    p = dp.Plan(64, 0, real=True)
    x = torch.zeros(0, device="cuda")
    st = dp.fft_exec(p.handle, 0, 0, dp.FFT_FORWARD)
    assert st == dp.FFT_OK
    del x
    for kw, code in ((dict(n=64, batch=2, real=True, inplace=True), dp.FFT_E_UNSUPPORTED),
                     (dict(n=22, batch=2, real=True), dp.FFT_E_UNSUPPORTED),
                     (dict(n=1 << 25, batch=2, real=True), dp.FFT_E_UNSUPPORTED),
                     (dict(n=64, batch=2, real=True, dist=80), dp.FFT_E_INVALID),
                     (dict(n=64, batch=2, real=True, precision="fp16"), dp.FFT_E_UNSUPPORTED)):
        with pytest.raises(dp.FftError) as e:
            dp.Plan(**kw)
        assert e.value.status == code, (kw, e.value)
