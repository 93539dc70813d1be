"""GPU parity of the power-of-two FP32 path against the FP64 oracle.

Single-pass lengths 1..2^14, the four-step lengths 2^15..2^22 and 2D images,
forward and inverse, each signal's relative L2 error against the oracle
gated at 1e-5.  Batches are chosen so the last workgroup is partly empty
(ragged tail) and grids span several tiles.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL_FP32, max_rel, run_plan, say, to_dev

pytestmark = pytest.mark.gpu


def _dp():
    import paper_1203_4938_amd as dp
    return dp


@pytest.mark.parametrize("lg", list(range(0, 15)))
def test_single_pass_lengths(lg):
    dp = _dp()
    n = 1 << lg
    batch = 37 if n <= 4096 else 5
    say(f"[single-pass] n={n} batch={batch}")
    x = synth.uniform_complex(synth.BASE_SEED + 100 + lg, n, batch)
    p = dp.Plan(n, batch)
    xd = to_dev(x)
    for inv in (False, True):
        y = run_plan(p, xd, inverse=inv).cpu().numpy()
        ref = oracle.fft_batch(x, inverse=inv)
        e = max_rel(y, ref)
        say(f"   inverse={inv} max rel L2 = {e:.3e}")
        assert e <= TOL_FP32, (n, inv, e)


def test_c1_n4096_b64_forward_inverse_roundtrip():
    dp = _dp()
    w = synth.workloads()["c1_n4096_b64"]
    x = synth.uniform_complex(w.seed, w.n, w.batch)
    p = dp.Plan(w.n, w.batch)
    say("[c1] plan:", p.describe())
    xd = to_dev(x)
    yf = run_plan(p, xd)
    yi = run_plan(p, xd, inverse=True)
    rt = run_plan(p, yf, inverse=True)
    ef = max_rel(yf.cpu().numpy(), oracle.fft_batch(x))
    ei = max_rel(yi.cpu().numpy(), oracle.fft_batch(x, inverse=True))
    er = max_rel(rt.cpu().numpy(), x.astype(np.complex128))
    say(f"[c1] fwd {ef:.3e} inv {ei:.3e} roundtrip {er:.3e}")
    assert ef <= TOL_FP32 and ei <= TOL_FP32 and er <= TOL_FP32


@pytest.mark.parametrize("lg,batch", [(15, 3), (16, 2), (17, 2), (18, 2), (19, 1), (20, 1),
                                      (21, 1), (22, 1)])
def test_four_step_lengths(lg, batch):
    dp = _dp()
    n = 1 << lg
    say(f"[four-step] n=2^{lg} batch={batch}")
    x = synth.uniform_complex(synth.BASE_SEED + 200 + lg, n, batch)
    p = dp.Plan(n, batch)
    say("   plan:", p.describe().splitlines()[0])
    assert p.workspace_bytes == n * batch * 8
    xd = to_dev(x)
    for inv in (False, True):
        y = run_plan(p, xd, inverse=inv).cpu().numpy()
        ref = oracle.fft_batch(x, inverse=inv)
        e = max_rel(y, ref)
        say(f"   inverse={inv} max rel L2 = {e:.3e}")
        assert e <= TOL_FP32, (n, inv, e)


@pytest.mark.parametrize("ny,nx,batch", [(16, 32, 3), (64, 128, 2), (256, 256, 2),
                                         (2048, 2048, 1), (128, 4096, 1)])
def test_2d_images(ny, nx, batch):
    dp = _dp()
    say(f"[2d] {batch} x {ny}x{nx}")
    x = synth.images_complex(synth.BASE_SEED + 3, batch, ny, nx) if ny >= 64 and nx >= 64 else \
        synth.uniform_complex(synth.BASE_SEED + 300, ny * nx, batch).reshape(batch, ny, nx)
    p = dp.Plan(shape=(ny, nx), batch=batch, rank=2)
    xd = to_dev(x)
    for inv in (False, True):
        y = run_plan(p, xd, inverse=inv).cpu().numpy()
        ref = oracle.fft2d(x, inverse=inv)
        e = max_rel(y, ref)
        say(f"   inverse={inv} max rel L2 = {e:.3e}")
        assert e <= TOL_FP32, (ny, nx, inv, e)


def test_2d_image_dc_bin_and_roundtrip():
    dp = _dp()
    x = synth.images_complex(synth.BASE_SEED + 3, 2, 512, 512)
    p = dp.Plan(shape=(512, 512), batch=2, rank=2)
    xd = to_dev(x)
    y = run_plan(p, xd)
    rt = run_plan(p, y, inverse=True).cpu().numpy()
    yh = y.cpu().numpy()
    for i in range(2):
        dc = float(x[i].real.astype(np.float64).sum())
        assert abs(yh[i, 0, 0].real - dc) <= 1e-6 * dc
    assert max_rel(rt, x.astype(np.complex128)) <= TOL_FP32


def test_batch_zero_is_noop_and_n1_identity():
    dp = _dp()
    import torch
    p = dp.Plan(1024, 0)
    x = torch.zeros(0, dtype=torch.complex64, device="cuda")
    p.exec(x)  # no launch, no error
    p1 = dp.Plan(1, 5)
    x1 = to_dev(synth.uniform_complex(1, 1, 5))
    y1 = run_plan(p1, x1)
    assert torch.equal(y1, x1)
    yi = run_plan(p1, x1, inverse=True)
    assert torch.equal(yi, x1)


def test_inplace_and_strided_dist():
    dp = _dp()
    import torch
    n, b, dist = 2048, 6, 2048 + 40
    x = synth.uniform_complex(5, dist, b)  # each row: signal in the first n entries
    p = dp.Plan(n, b, dist=dist, inplace=True)
    xd = to_dev(x)
    ref = oracle.fft_batch(x[:, :n])
    y = run_plan(p, xd, out=xd)  # in place
    yh = y.cpu().numpy()
    assert max_rel(yh[:, :n], ref) <= TOL_FP32
    # the gap between signals is untouched
    assert np.array_equal(yh[:, n:], x[:, n:])


@pytest.mark.parametrize("force", ["", "p0=1 t0=512"])
def test_signals_more_than_4gib_apart(force, monkeypatch):
    """Rows of one tile lie 2 GiB apart (dist = 2^28 complex64): every line is
    addressed from its own 64-bit base (plain 4-row tiles, and the persistent
    16-row tiles, whose 13 idle lanes repeat the last row)."""
    import torch
    dp = _dp()
    monkeypatch.setenv("DPFFT_FORCE_PLAN", force)
    n, b, dist = 1024, 3, 1 << 28
    x = synth.uniform_complex(synth.BASE_SEED + 31, n, b)
    xd = torch.zeros((b - 1) * dist + n, dtype=torch.complex64, device="cuda")
    for i in range(b):
        xd[i * dist:i * dist + n] = torch.from_numpy(x[i]).to("cuda")
    p = dp.Plan(n, b, dist=dist)
    say("[far apart]", p.describe().replace("\n", " | "))
    for inv in (False, True):
        y = run_plan(p, xd, inverse=inv)
        got = np.stack([y[i * dist:i * dist + n].cpu().numpy() for i in range(b)])
        e = max_rel(got, oracle.fft_batch(x, inverse=inv))
        say(f"   inverse={inv} max rel L2 = {e:.3e}")
        assert e <= TOL_FP32
    del xd, y
    torch.cuda.empty_cache()


def test_exec_rejects_bad_arguments():
    dp = _dp()
    import torch
    p = dp.Plan(256, 4)
    x = to_dev(synth.uniform_complex(1, 256, 4))
    st = dp.fft_exec(p.handle, x.data_ptr(), x.data_ptr(), dp.FFT_FORWARD, 0, 0)
    assert st == dp.FFT_E_INVALID  # in == out without the in-place flag
    st = dp.fft_exec(p.handle, x.data_ptr(), x.data_ptr() + 4, dp.FFT_FORWARD, 0, 0)
    assert st == dp.FFT_E_INVALID  # misaligned
    st = dp.fft_exec(p.handle, x.data_ptr(), 0, dp.FFT_FORWARD, 0, 0)
    assert st == dp.FFT_E_INVALID
    st = dp.fft_exec(p.handle, x.data_ptr(), x.data_ptr(), 3, 0, 0)
    assert st == dp.FFT_E_INVALID
    p4 = dp.Plan(1 << 16, 1)
    y = torch.empty(1 << 16, dtype=torch.complex64, device="cuda")
    z = torch.empty_like(y)
    st = dp.fft_exec(p4.handle, y.data_ptr(), z.data_ptr(), dp.FFT_FORWARD, 0, 0)
    assert st == dp.FFT_E_INVALID  # workspace required


VARIANTS = [
    (4096, 10, "p0=1"), (8192, 6, "p0=1"), (1024, 37, "c0=8"), (2048, 9, "c0=4"),
    (4096, 7, "c0=2"), (1 << 22, 1, "s=11 c0=4 c1=4"), (1 << 20, 2, "c0=8 c1=8"),
    (1 << 18, 3, "c0=16 c1=16"), (1 << 22, 1, "s=11 c0=8 c1=8"),
    # chunked four-step: the batch in groups of k signals, with a short last group
    (1 << 18, 5, "k=2"), (1 << 15, 7, "k=3"), (1 << 20, 3, "k=1"),
    # persistent 1024-thread instances
    (16384, 300, "p0=1 t0=1024"), (16384, 7, "p0=0"), (4096, 9, "c0=2 p0=0"),
    (1 << 20, 3, "p0=1 t0=1024"), (1 << 20, 3, "p0=0"),
    # other four-step splits of 2^22 (4096 x 1024, 1024 x 4096)
    (1 << 22, 1, "s=12"), (1 << 22, 1, "s=10"),
    # 32 elements per thread, radix-32 passes
    (16384, 11, "p0=1 t0=512"), (8192, 7, "p0=1 t0=256"), (8192, 5, "p0=0"),
    # persistent column and transposed-row tiles with 32 elements per thread
    (1 << 22, 1, "s=11 p0=1 t0=512 p1=1 t1=512"), (1 << 20, 3, "p0=1 t0=512 p1=1 t1=512"),
    (1 << 22, 2, "s=10 p0=1 t0=1024"),
    (1024, 37, "c0=8 t0=256"), (1024, 37, "c0=16 t0=512 p0=0"), (1024, 37, "p0=1 t0=512"),
    (1 << 18, 3, "c0=16 t0=256 p0=0 c1=16 t1=256 p1=0"), (1 << 18, 3, "t0=512"),
    (1024, 37, "c0=4 p0=0"), (4096, 9, "c0=1"), (1 << 22, 2, "s=10 p1=1 t1=512"), (1 << 20, 3, "p1=0"),
    (1 << 18, 3, "p0=0 p1=0"), (1 << 22, 2, "s=12 p0=1 t0=512"),
    (1 << 18, 3, "c0=32 t0=512 p0=0 c1=32 t1=512 p1=0"),
    (1 << 18, 3, "p0=1 c0=32 t0=512 p1=1 c1=32 t1=512"), (1 << 18, 3, "p0=1 c0=16 t0=256 p1=1 c1=16 t1=256"),
    # split-first transposed rows (two sub-lines through half the LDS)
    (1 << 20, 3, "c1=16 t1=512 p1=0"), (1 << 21, 2, "s=11 c1=16 t1=512 p1=0"),
    (1 << 20, 2, "h1=2"), (1 << 20, 2, "h1=1 p1=0 t1=1024"),
]


@pytest.mark.parametrize("n,batch,force", VARIANTS, ids=[f"{v[0]}-{v[2]}" for v in VARIANTS])
def test_forced_variants(n, batch, force, monkeypatch):
    """Every kernel variant the planner or the tuner may pick matches the oracle."""
    dp = _dp()
    monkeypatch.setenv("DPFFT_FORCE_PLAN", force)
    say(f"[variant] n={n} batch={batch} force={force}")
    x = synth.uniform_complex(synth.BASE_SEED + 400, n, batch)
    p = dp.Plan(n, batch)
    say("   plan:", p.describe().replace("\n", " | "))
    xd = to_dev(x)
    for inv in (False, True):
        y = run_plan(p, xd, inverse=inv).cpu().numpy()
        e = max_rel(y, oracle.fft_batch(x, inverse=inv))
        say(f"   inverse={inv} max rel L2 = {e:.3e}")
        assert e <= TOL_FP32, (n, force, inv, e)


@pytest.mark.parametrize("n,force", [(2048, "c1=8"), (2048, "c1=4"), (2048, "k=1"), (1024, "p1=1"), (1024, "p1=0"),
                                     (2048, "p1=1 t1=512"), (1024, "p1=1 t1=512"), (512, "c1=16 t1=256"), (512, "c1=16 t1=512"),
                                     (2048, "p1=0"), (1024, "c1=16 t1=1024 p1=0"), (1024, "c1=16 t1=512 p1=0")])
def test_forced_2d_variants(n, force, monkeypatch):
    dp = _dp()
    monkeypatch.setenv("DPFFT_FORCE_PLAN", force)
    x = synth.images_complex(synth.BASE_SEED + 3, 2, n, n)
    p = dp.Plan(shape=(n, n), batch=2, rank=2)
    xd = to_dev(x)
    for inv in (False, True):
        y = run_plan(p, xd, inverse=inv).cpu().numpy()
        assert max_rel(y, oracle.fft2d(x, inverse=inv)) <= TOL_FP32
