"""Parity of every signal of the benchmark's full-size batches, in the plans the
benchmark times.

The c2 batches (N = 2^10 ... 2^22, batch*N = 2^27), the FP32 c4 batch
(N = 2^16 x 4096) and the c3 image batch (16 x 2048^2) are generated and
planned exactly as the benchmark does.  Every signal (every image) is then
compared with the FP64 oracle, streamed through it chunk by chunk: the forward
transform of the input, the inverse transform of the oracle's spectrum
(rounded to complex64) against the oracle's inverse of that same input, and
the round trip.  Tolerance: relative L2 <= 1e-5 per signal, gated on the max
over the batch (the FP32 bound)."""
import numpy as np
import pytest

import synth
from gpu_util import TOL_FP32, assert_generator_rows, full_parity, oracle_2d, say

pytestmark = pytest.mark.gpu

C2 = [(1 << 10, 131072), (1 << 14, 8192), (1 << 18, 512), (1 << 22, 32)]


def _check_all(stats, tol, what):
    for k, st in stats.items():
        assert st.max <= tol, (what, k, st.line())


@pytest.mark.parametrize("n,b", C2, ids=[f"n2^{int(np.log2(n))}" for n, _ in C2])
def test_c2_full_batch_every_signal(n, b):
    import torch

    import paper_1203_4938_amd as dp
    seed = synth.BASE_SEED + 2  # the c2 workload's stream
    say(f"[full c2] n={n} batch={b}: every signal, both directions")
    x = synth.uniform_complex_torch(seed, n, b, "cuda")
    assert_generator_rows(x, seed, n, (0, b - 1))
    p = dp.Plan(n, b)
    say("   plan:", p.describe().replace("\n", " | "))
    st = full_parity(p, x, label=f"c2 n=2^{int(np.log2(n))}")
    _check_all(st, TOL_FP32, f"c2 n={n}")
    del x
    torch.cuda.empty_cache()


def test_c4_fp32_full_batch_every_signal():
    """C4 shape (N = 2^16, batch 4096, 2 GiB) in FP32, in the launch
    configuration the benchmark times (65536 tiles per pass, the round-based
    tile order)."""
    import torch

    import paper_1203_4938_amd as dp
    n, b = 1 << 16, 4096
    seed = synth.BASE_SEED + 4
    say(f"[full c4 fp32] n={n} batch={b}: every signal, both directions")
    x = synth.uniform_complex_torch(seed, n, b, "cuda")
    assert_generator_rows(x, seed, n, (0, b - 1))
    p = dp.Plan(n, b)
    say("   plan:", p.describe().replace("\n", " | "))
    st = full_parity(p, x, label="c4 fp32")
    _check_all(st, TOL_FP32, "c4 fp32")
    del x
    torch.cuda.empty_cache()


def test_c3_full_batch_every_image():
    import torch

    import paper_1203_4938_amd as dp
    seed = synth.BASE_SEED + 3  # the c3 workload's stream
    imgs = synth.images_complex(seed, 16, 2048, 2048)
    x = torch.from_numpy(imgs).to("cuda")
    p = dp.Plan(shape=(2048, 2048), batch=16, rank=2)
    say("[full c3]", p.describe().replace("\n", " | "))
    st = full_parity(p, x, ref=oracle_2d, label="c3 16x2048^2")
    _check_all(st, TOL_FP32, "c3")
    # the DC bin of an integer image is an exact integer sum, for every image
    y = p.exec(x)
    torch.cuda.synchronize()
    dc = y[:, 0, 0].real.double().cpu().numpy()
    sums = imgs.real.astype(np.float64).reshape(16, -1).sum(axis=1)
    say(f"   DC bins: max relative deviation {np.max(np.abs(dc - sums) / sums):.2e}")
    assert np.all(np.abs(dc - sums) <= 1e-5 * sums)
    del x, y
    torch.cuda.empty_cache()
