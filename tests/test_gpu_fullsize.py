"""Parity at the benchmark's full sizes, in the plans the benchmark times.

The c2 batches (N = 2^10 ... 2^22, batch*N = 2^27), the FP32 c4 batch
(N = 2^16 x 4096) and the c3 image batch (16 x 2048^2) are generated and
transformed exactly as the benchmark does;
the oracle then recomputes a seeded sample of whole signals (first, last and
random ones) one by one, and the inverse of the full output must return the
input on those signals."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL_FP32, max_rel, say

pytestmark = pytest.mark.gpu

C2 = [(1 << 10, 131072, 8), (1 << 14, 8192, 6), (1 << 18, 512, 4), (1 << 22, 32, 2)]


def _sample(b, k, seed):
    rng = np.random.default_rng(seed)
    picks = {0, b - 1}
    while len(picks) < min(k, b):
        picks.add(int(rng.integers(0, b)))
    return sorted(picks)


@pytest.mark.parametrize("n,b,k", C2, ids=[f"n2^{int(np.log2(n))}" for n, _, _ in C2])
def test_c2_full_batch_sampled(n, b, k):
    import torch

    import paper_1203_4938_amd as dp
    seed = synth.BASE_SEED + 2  # the c2 workload's stream
    say(f"[full c2] n={n} batch={b} sampled={k}")
    x = synth.uniform_complex_torch(seed, n, b, "cuda")
    p = dp.Plan(n, b)
    say("   plan:", p.describe().splitlines()[0])
    y = p.exec(x)
    z = p.exec(y, inverse=True)
    torch.cuda.synchronize()
    for s in _sample(b, k, 1000 + n):
        xs = synth.uniform_complex(seed, n, 1, first=s)
        ref = oracle.fft_batch(xs)
        e = max_rel(y[s:s + 1].cpu().numpy(), ref)
        r = max_rel(z[s:s + 1].cpu().numpy(), xs.astype(np.complex128))
        say(f"   signal {s}: forward rel L2 {e:.3e}, round trip {r:.3e}")
        assert e <= TOL_FP32 and r <= TOL_FP32, (n, s, e, r)


def test_c4_fp32_full_batch_sampled():
    """C4 shape (N = 2^16, batch 4096, 2 GiB) in FP32, in the launch
    configuration the benchmark times (65536 tiles per pass, the round-based
    tile order); a seeded sample of whole signals against the oracle."""
    import torch

    import paper_1203_4938_amd as dp
    n, b = 1 << 16, 4096
    seed = synth.BASE_SEED + 4
    say(f"[full c4 fp32] n={n} batch={b}")
    x = synth.uniform_complex_torch(seed, n, b, "cuda")
    p = dp.Plan(n, b)
    say("   plan:", p.describe().replace("\n", " | "))
    y = p.exec(x)
    z = p.exec(y, inverse=True)
    torch.cuda.synchronize()
    for s in _sample(b, 5, 4242):
        xs = synth.uniform_complex(seed, n, 1, first=s)
        e = max_rel(y[s:s + 1].cpu().numpy(), oracle.fft_batch(xs))
        r = max_rel(z[s:s + 1].cpu().numpy(), xs.astype(np.complex128))
        say(f"   signal {s}: forward rel L2 {e:.3e}, round trip {r:.3e}")
        assert e <= TOL_FP32 and r <= TOL_FP32, (s, e, r)
    del x, y, z
    torch.cuda.empty_cache()


def test_c3_full_batch_sampled():
    import torch

    import paper_1203_4938_amd as dp
    seed = synth.BASE_SEED + 3  # the c3 workload's stream
    imgs = synth.images_complex(seed, 16, 2048, 2048)
    x = torch.from_numpy(imgs).to("cuda")
    p = dp.Plan(shape=(2048, 2048), batch=16, rank=2)
    say("[full c3]", p.describe().splitlines()[0])
    y = p.exec(x)
    z = p.exec(y, inverse=True)
    torch.cuda.synchronize()
    for i in _sample(16, 3, 77):
        ref = oracle.fft2d(imgs[i:i + 1])
        e = max_rel(y[i:i + 1].cpu().numpy().reshape(1, -1), ref.reshape(1, -1))
        r = max_rel(z[i:i + 1].cpu().numpy().reshape(1, -1),
                    imgs[i:i + 1].astype(np.complex128).reshape(1, -1))
        # the DC bin of an integer image is an exact integer sum
        dc = float(y[i, 0, 0].real.item())
        say(f"   image {i}: forward rel L2 {e:.3e}, round trip {r:.3e}, DC {dc:.1f}")
        assert e <= TOL_FP32 and r <= TOL_FP32, (i, e, r)
        assert abs(dc - float(imgs[i].real.astype(np.float64).sum())) <= 1e-5 * abs(dc)
