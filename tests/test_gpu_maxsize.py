"""The largest lengths the library accepts (N up to 2^24): a power of two and
a 7-smooth length near the top of the range, one signal checked against the
oracle, the other by the round trip and a closed form (a pure tone must land
in its bin)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL_FP32, max_rel, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1 << 24, 3 ** 15, 7 ** 8])
def test_largest_lengths(n):
    import torch

    import paper_1203_4938_amd as dp
    x = synth.uniform_complex(synth.BASE_SEED + 70, n, 2)
    j = np.arange(n, dtype=np.float64)
    f = 12345 % n
    x[1] = np.exp(2j * np.pi * f * j / n).astype(np.complex64)  # tone in bin f
    p = dp.Plan(n, 2)
    say(f"[max size] n={n}:", p.describe().splitlines()[0])
    xd = to_dev(x)
    y = p.exec(xd)
    z = p.exec(y, inverse=True)
    torch.cuda.synchronize()
    e = max_rel(y[:1].cpu().numpy(), oracle.fft_batch(x[:1]))
    r = max_rel(z.cpu().numpy(), x.astype(np.complex128))
    tone = y[1].cpu().numpy().astype(np.complex128)
    peak = abs(tone[f] - n) / n
    rest = np.sqrt(np.sum(np.abs(np.delete(tone, f)) ** 2)) / n
    say(f"   forward rel L2 {e:.3e}, round trip {r:.3e}, tone peak {peak:.2e}, leakage {rest:.2e}")
    assert e <= TOL_FP32 and r <= TOL_FP32
    assert peak <= 1e-5 and rest <= 1e-5
