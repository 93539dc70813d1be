"""GPU parity of the runtime-radix (2/3/4/5/7/8/16) path against the FP64 oracle:
every prime radix alone and combined, lengths with ragged last workgroups,
the largest single-pass lengths and the two-pass four-step for lengths above
16384, forward and inverse, rel L2 <= 1e-5 per signal."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL_FP32, max_rel, run_plan, say, to_dev

pytestmark = pytest.mark.gpu

SINGLE = [3, 5, 6, 7, 9, 12, 15, 25, 27, 49, 60, 100, 125, 192, 343, 360, 1000, 1680, 2187,
          2401, 6561, 9600, 12005, 15552, 15625, 16000]


@pytest.mark.parametrize("n", SINGLE)
def test_mixed_single_pass(n):
    import paper_1203_4938_amd as dp
    batch = 11
    say(f"[mixed] n={n} batch={batch}")
    x = synth.uniform_complex(synth.BASE_SEED + 500 + n % 97, n, batch)
    p = dp.Plan(n, batch)
    say("   plan:", p.describe().replace("\n", " | "))
    xd = to_dev(x)
    for inv in (False, True):
        y = run_plan(p, xd, inverse=inv).cpu().numpy()
        e = max_rel(y, oracle.fft_batch(x, inverse=inv))
        say(f"   inverse={inv} max rel L2 = {e:.3e}")
        assert e <= TOL_FP32, (n, inv, e)


@pytest.mark.parametrize("n,batch", [(49152, 2), (78125, 1), (59049, 1), (26880, 2),
                                     (117649, 1), (39366, 1)])
def test_mixed_four_step(n, batch):
    import paper_1203_4938_amd as dp
    say(f"[mixed four-step] n={n} batch={batch}")
    x = synth.uniform_complex(synth.BASE_SEED + 600, n, batch)
    p = dp.Plan(n, batch)
    say("   plan:", p.describe().replace("\n", " | "))
    xd = to_dev(x)
    for inv in (False, True):
        y = run_plan(p, xd, inverse=inv).cpu().numpy()
        e = max_rel(y, oracle.fft_batch(x, inverse=inv))
        say(f"   inverse={inv} max rel L2 = {e:.3e}")
        assert e <= TOL_FP32, (n, inv, e)


def test_mixed_closed_forms_on_device():
    """Impulse -> constant, constant -> scaled delta, tone -> delta at its bin."""
    import paper_1203_4938_amd as dp
    n = 3 * 5 * 7 * 9
    x = np.zeros((3, n), np.complex64)
    x[0, 0] = 1.0
    x[1, :] = 0.5
    j = np.arange(n)
    x[2] = np.exp(2j * np.pi * 17 * j / n).astype(np.complex64)
    y = run_plan(dp.Plan(n, 3), to_dev(x)).cpu().numpy().astype(np.complex128)
    assert np.max(np.abs(y[0] - 1.0)) < 1e-6
    ref1 = np.zeros(n)
    ref1[0] = 0.5 * n
    assert np.max(np.abs(y[1] - ref1)) < 1e-4
    ref2 = np.zeros(n)
    ref2[17] = n
    assert np.linalg.norm(y[2] - ref2) / n < 1e-5


@pytest.mark.parametrize("ny,nx,batch", [(100, 128, 3), (96, 81, 2), (1000, 7, 2), (243, 250, 2),
                                         (6, 3000, 2), (16384, 3, 1), (3, 16384, 1), (1, 30, 4),
                                         (30, 1, 4), (125, 2048, 1)])
def test_mixed_2d_images(ny, nx, batch):
    """Images whose sides are 7-smooth but not both powers of two: the row and
    column passes on the runtime-radix kernels, both directions against the
    oracle's separable 2D transforms (sides of 1 included: the identity pass
    still takes the inverse's swap)."""
    import paper_1203_4938_amd as dp
    x = synth.uniform_complex(synth.BASE_SEED + 310, ny * nx, batch).reshape(batch, ny, nx)
    p = dp.Plan(shape=(ny, nx), batch=batch, rank=2)
    say(f"[mixed 2d] {batch} x {ny}x{nx}:", p.describe().replace("\n", " | "))
    xd = to_dev(x)
    for inv in (False, True):
        y = run_plan(p, xd, inverse=inv).cpu().numpy()
        e = max_rel(y, oracle.fft2d(x, inverse=inv))
        say(f"   inverse={inv} max rel L2 = {e:.3e}")
        assert e <= TOL_FP32, (ny, nx, inv, e)

