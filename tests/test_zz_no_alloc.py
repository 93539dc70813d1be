"""fft_exec_noalloc: the plan's workspace comes from the library's own device
array instead of a caller buffer.  Its output must equal fft_exec's (same
kernels, same launch shapes) and stay within the oracle's FP32 bound, on two
calls in a row with the second on a smaller input, for a four-step plan, a
ragged graph plan and a two-launch real-input image plan; a plan whose
workspace exceeds the array is rejected before any launch."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL_FP32, say, to_dev

pytestmark = pytest.mark.gpu


def _dp():
    import paper_1203_4938_amd as dp
    return dp


def _both(p, xd, inverse, out_shape=None, out_dtype=None):
    """(fft_exec output, fft_exec_noalloc output) for the same input."""
    import torch
    dp = _dp()
    shape = out_shape if out_shape is not None else xd.shape
    dtype = out_dtype if out_dtype is not None else xd.dtype
    ya = torch.empty(shape, dtype=dtype, device="cuda")
    yb = torch.full(shape, float("nan"), dtype=dtype, device="cuda") if dtype.is_floating_point \
        else torch.full(shape, complex(float("nan"), float("nan")), dtype=dtype, device="cuda")
    ws = p.workspace(xd.device)
    s = torch.cuda.current_stream().cuda_stream
    d = dp.FFT_INVERSE if inverse else dp.FFT_FORWARD
    assert dp.fft_exec(p.handle, xd.data_ptr(), ya.data_ptr(), d,
                       ws.data_ptr() if ws is not None else 0, s) == dp.FFT_OK
    st = dp.fft_exec_noalloc(p.handle, xd.data_ptr(), yb.data_ptr(), d, s)
    assert st == dp.FFT_OK, dp.fft_last_error()
    torch.cuda.synchronize()
    return ya.cpu().numpy(), yb.cpu().numpy()


def test_noalloc_four_step_two_calls():
    dp = _dp()
    # first call: a workspace of exactly 64 MiB; second: a smaller plan
    for n, b in ((1 << 18, 32), (1 << 15, 3)):
        say(f"[noalloc] four-step n={n} batch={b} workspace={b * n * 8} B")
        x = synth.uniform_complex(synth.BASE_SEED + 400, n, b)
        p = dp.Plan(n, b)
        assert p.workspace_bytes == b * n * 8
        for inv in (False, True):
            ya, yb = _both(p, to_dev(x), inv)
            assert np.array_equal(ya, yb), (n, inv)
            k = min(b, 4)
            e = float(np.max(oracle.rel_l2(yb[:k], oracle.fft_batch(x[:k], inverse=inv))))
            say(f"   inverse={inv}: equal to fft_exec, max rel L2 (first {k}) {e:.2e}")
            assert e <= TOL_FP32


def test_noalloc_ragged_graph_plan():
    dp = _dp()
    sizes = [40000, 64, 18000, 65536, 1000, 30870]
    flat, offs = synth.uniform_ragged(synth.BASE_SEED + 401, sizes)
    p = dp.Plan(ragged_sizes=sizes, graph=True)
    say(f"[noalloc] ragged graph plan, workspace {p.workspace_bytes} B")
    for inv in (False, True):
        ya, yb = _both(p, to_dev(flat), inv)
        assert np.array_equal(ya, yb)
        ref = oracle.fft_ragged(flat, sizes, offs, inverse=inv)
        for n, o in zip(sizes, offs):
            e = float(oracle.rel_l2(yb[o:o + n][None], ref[o:o + n][None])[0])
            assert e <= TOL_FP32, (n, inv, e)


def test_noalloc_real_images_inverse():
    import torch
    dp = _dp()
    b, ny, nx = 3, 256, 512
    imgs = np.ascontiguousarray(np.stack([synth.smooth_noise_image(synth.BASE_SEED + 3, i, ny, nx)
                                          for i in range(b)]).astype(np.float32))
    p = dp.Plan(shape=(ny, nx), batch=b, rank=2, real=True)
    spec = p.exec(torch.from_numpy(imgs).cuda())
    torch.cuda.synchronize()
    ya, yb = _both(p, spec, True, out_shape=(b, ny, nx), out_dtype=torch.float32)
    assert np.array_equal(ya, yb)
    e = float(np.max(np.abs(yb - imgs)) / 255.0)
    say(f"[noalloc] real images inverse: equal to fft_exec, max abs round-trip err/255 {e:.2e}")
    assert e <= 1e-5


def test_noalloc_real_1d_four_step_core():
    """Real signals of 2^17 samples: the four-step core runs in the library's
    array (the forward also uses the output as scratch), both directions equal
    to fft_exec, the forward within the oracle's bound."""
    import torch
    dp = _dp()
    n, b = 1 << 17, 3
    x = np.ascontiguousarray(synth.uniform_complex(synth.BASE_SEED + 402, n, b).real)
    p = dp.Plan(n, b, real=True)
    assert p.workspace_bytes == b * (n // 2) * 8
    xd = torch.from_numpy(x).cuda()
    ya, yb = _both(p, xd, False, out_shape=(b, n // 2 + 1), out_dtype=torch.complex64)
    assert np.array_equal(ya, yb)
    ref = oracle.fft_batch(x.astype(np.complex64))[:, : n // 2 + 1]
    e = float(np.max(oracle.rel_l2_f32(yb, ref)))
    say(f"[noalloc] real 1d n={n}: forward equal to fft_exec, max rel L2 {e:.2e}")
    assert e <= TOL_FP32
    za, zb = _both(p, torch.from_numpy(ya).cuda(), True, out_shape=(b, n), out_dtype=torch.float32)
    assert np.array_equal(za, zb)
    er = float(np.max(np.abs(zb - x)))
    say(f"   inverse equal to fft_exec, max abs round-trip error {er:.2e}")
    assert er <= 1e-5


def test_noalloc_rejects_large_workspace():
    import torch
    dp = _dp()
    n, b = 1 << 18, 33  # 66 MiB of workspace
    p = dp.Plan(n, b)
    x = torch.zeros(n * b, dtype=torch.complex64, device="cuda")
    st = dp.fft_exec_noalloc(p.handle, x.data_ptr(), torch.empty_like(x).data_ptr(),
                             dp.FFT_FORWARD, 0)
    assert st == dp.FFT_E_UNSUPPORTED
    assert "workspace" in dp.fft_last_error()
