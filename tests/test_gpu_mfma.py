"""GPU parity of the matrix-core (MFMA) precision forms against the FP64 oracle.

Tolerances (relative L2 per signal, gated on the max): 1e-5 for the split
forms (FP16 hi/lo, BF16 hi/lo, BF16 hi/mid/lo), 2e-3 for plain FP16.  Plain
BF16 keeps only 8 significant bits per operand; its error is recorded and
checked against 2e-3 as an expected failure, and against a sanity bound."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL_FP32, max_rel, run_plan, say, to_dev

pytestmark = pytest.mark.gpu

TOL = {"fp16": 2e-3, "bf16": 2e-3, "fp16_split": 1e-5, "bf16_split": 1e-5, "bf16_split3": 1e-5}
SANITY = {"bf16": 2e-2}


def _check(prec, n, batch, seed):
    import paper_1203_4938_amd as dp
    x = synth.uniform_complex(seed, n, batch)
    p = dp.Plan(n, batch, precision=prec)
    say(f"[mfma {prec}] n={n} batch={batch} plan: " + p.describe().replace("\n", " | "))
    xd = to_dev(x)
    errs = []
    for inv in (False, True):
        y = run_plan(p, xd, inverse=inv).cpu().numpy()
        e = max_rel(y, oracle.fft_batch(x, inverse=inv))
        say(f"   inverse={inv} max rel L2 = {e:.3e}")
        errs.append(e)
    return max(errs)


@pytest.mark.parametrize("prec", ["fp16", "fp16_split", "bf16_split", "bf16_split3"])
@pytest.mark.parametrize("n,batch", [(256, 37), (65536, 3)])
def test_mfma_forms(prec, n, batch):
    e = _check(prec, n, batch, synth.BASE_SEED + 700)
    assert e <= TOL[prec], (prec, n, e)


@pytest.mark.parametrize("n,batch", [(256, 37), (65536, 3)])
def test_mfma_bf16_plain(n, batch):
    e = _check("bf16", n, batch, synth.BASE_SEED + 701)
    assert e <= SANITY["bf16"], e
    if e > TOL["bf16"]:
        pytest.xfail(f"plain BF16 rel L2 {e:.2e} exceeds the 2e-3 bound (8-bit significands)")


@pytest.mark.parametrize("prec", ["fp16", "bf16", "fp16_split", "bf16_split", "bf16_split3"])
def test_mfma_c4_sampled_full_size(prec):
    """C4 shape (N=2^16, batch 4096) in the launch configuration the benchmark
    times: sampled signals against the oracle, for each matrix-core form.  Plain
    BF16 is held to its sanity bound (its 2e-3 miss is recorded above)."""
    import torch

    import paper_1203_4938_amd as dp
    n, batch = 1 << 16, 4096
    w = synth.workloads()[f"c4_n2^16_b4096_{prec}"]
    x = synth.uniform_complex_torch(w.seed, n, batch, "cuda")
    p = dp.Plan(n, batch, precision=prec)
    y = run_plan(p, x)
    tol = SANITY.get(prec, TOL[prec])
    for b in (0, 1, 2047, 4095):
        xs = synth.uniform_complex(w.seed, n, 1, first=b)
        ref = oracle.fft_batch(xs)
        e = max_rel(y[b:b + 1].cpu().numpy(), ref)
        say(f"   [{prec}] signal {b}: rel L2 {e:.3e}")
        assert e <= tol, (prec, b, e)
    del x, y
    torch.cuda.empty_cache()


def test_mfma_unsupported_length_is_reported():
    import paper_1203_4938_amd as dp
    with pytest.raises(dp.FftError) as ei:
        dp.Plan(4096, 4, precision="fp16_split")
    assert ei.value.status == dp.FFT_E_UNSUPPORTED
