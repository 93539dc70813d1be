"""GPU parity of the matrix-core (MFMA) precision forms against the FP64 oracle.

Tolerances (relative L2 per signal, gated on the max): 1e-5 for the split
forms (FP16 hi/lo, BF16 hi/lo, BF16 hi/mid/lo), 2e-3 for plain FP16.  Plain
BF16 keeps only 8 significant bits per operand; it is held to the same 2e-3
and marked as an expected failure when it misses, with the measured error in
the reason (it is never passed at a looser bound).

The input-range cases (amplitudes 1e3 and 1e-6, signals of very different
amplitudes in one batch, a constant of 16, and the inverse of a
full-amplitude spectrum) pin the FP16 forms' per-line power-of-two scaling:
without it the FP16 pieces overflow or lose their low bits."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import (TOL_FP32, assert_generator_rows, full_parity, max_rel, run_plan, say,
                      to_dev)

pytestmark = pytest.mark.gpu

TOL = {"fp16": 2e-3, "bf16": 2e-3, "fp16_split": 1e-5, "bf16_split": 1e-5, "bf16_split3": 1e-5}
FORMS = ["fp16", "bf16", "fp16_split", "bf16_split", "bf16_split3"]
#: plain BF16 above this is a defect, not the known 8-bit-significand miss
BF16_DEFECT = 2e-2


def _gate(prec, e, what):
    """Hold `e` to the form's tolerance; plain BF16 misses are recorded xfails."""
    if prec == "bf16":
        assert e <= BF16_DEFECT, (what, e)
        if e > TOL["bf16"]:
            pytest.xfail(f"plain BF16 {what}: measured max rel L2 {e:.3e} > 2e-3 "
                         "(8-bit significands)")
    else:
        assert e <= TOL[prec], (prec, what, e)


def _check(prec, x, inverse_input=None):
    """Forward of x and inverse of `inverse_input` (default x) against the oracle."""
    import paper_1203_4938_amd as dp
    batch, n = x.shape
    p = dp.Plan(n, batch, precision=prec)
    xi = x if inverse_input is None else inverse_input
    errs = []
    for inv, inp in ((False, x), (True, xi)):
        y = run_plan(p, to_dev(inp), inverse=inv).cpu().numpy()
        e = max_rel(y, oracle.fft_batch(inp, inverse=inv))
        say(f"   [{prec}] n={n} inverse={inv} max rel L2 = {e:.3e}")
        errs.append(e)
    return max(errs)


@pytest.mark.parametrize("prec", FORMS)
@pytest.mark.parametrize("n,batch", [(256, 37), (65536, 3), (1 << 14, 5), (1 << 15, 3), (1 << 18, 2),
                                     (1 << 20, 1)])
def test_mfma_forms(prec, n, batch):
    """N = 256 and 65536 on the matrix cores throughout; N = 256 N2 for other
    N2 (the 256-point column pass on the matrix cores, the rows in FP32)."""
    x = synth.uniform_complex(synth.BASE_SEED + 700, n, batch)
    _gate(prec, _check(prec, x), f"n={n} uniform")


def _spectrum64(x):
    return oracle.fft_batch(x).astype(np.complex64)


RANGES = {
    # amplitude 1e3 and 1e-6: FP16 overflow after a few stages, FP16 subnormals
    "amp1e3": lambda x: (x * np.float32(1e3)).astype(np.complex64),
    "amp1e-6": lambda x: (x * np.float32(1e-6)).astype(np.complex64),
    # a constant 16: the whole energy lands in one bin, 16 * N at DC
    "const16": lambda x: np.full_like(x, 16.0 + 0.0j),
    # one batch, four amplitudes: each line is scaled on its own
    "mixed": lambda x: (x * np.array([1e-6, 1.0, 1e3, 1e-3], np.float32)[:, None]).astype(np.complex64),
}


@pytest.mark.parametrize("prec", FORMS)
@pytest.mark.parametrize("case", sorted(RANGES))
@pytest.mark.parametrize("n", [256, 65536, 1 << 18])
def test_mfma_input_range(prec, case, n):
    base = synth.uniform_complex(synth.BASE_SEED + 702, n, 4)
    x = RANGES[case](base)
    _gate(prec, _check(prec, x), f"n={n} {case}")


@pytest.mark.parametrize("prec", FORMS)
@pytest.mark.parametrize("n", [256, 65536])
def test_mfma_inverse_of_spectrum(prec, n):
    """Inverse of the oracle's spectrum of a uniform batch (values up to about
    N in magnitude), against the oracle's inverse of the same complex64 input."""
    x = synth.uniform_complex(synth.BASE_SEED + 703, n, 4)
    _gate(prec, _check(prec, x, inverse_input=_spectrum64(x)), f"n={n} inverse of spectrum")


@pytest.mark.parametrize("prec", FORMS)
def test_mfma_c4_full_batch_every_signal(prec):
    """C4 shape (N=2^16, batch 4096) in the launch configuration the benchmark
    times: every signal against the oracle, the forward transform of the
    input and the inverse of the oracle's spectrum (the amplitude range the
    benchmark's inverse sees), plus the round trip."""
    import torch

    import paper_1203_4938_amd as dp
    n, batch = 1 << 16, 4096
    w = synth.workloads()[f"c4_n2^16_b4096_{prec}"]
    say(f"[full c4 {prec}] n={n} batch={batch}: every signal, both directions")
    x = synth.uniform_complex_torch(w.seed, n, batch, "cuda")
    assert_generator_rows(x, w.seed, n, (0, batch - 1))
    p = dp.Plan(n, batch, precision=prec)
    say("   plan:", p.describe().replace("\n", " | "))
    st = full_parity(p, x, label=f"c4 {prec}")
    del x
    torch.cuda.empty_cache()
    # the round trip goes through two transforms of this form
    rt_tol = 2 * TOL[prec]
    assert st["round_trip"].max <= (BF16_DEFECT if prec == "bf16" else rt_tol), \
        st["round_trip"].line()
    _gate(prec, max(st["forward"].max, st["inverse"].max), "c4 full batch")


def test_mfma_unsupported_length_is_reported():
    import paper_1203_4938_amd as dp
    with pytest.raises(dp.FftError) as ei:
        dp.Plan(4096, 4, precision="fp16_split")
    assert ei.value.status == dp.FFT_E_UNSUPPORTED


def test_fp32_reference_at_the_same_ranges():
    """The FP32 path on the same range cases, for comparison (bound 1e-5)."""
    import paper_1203_4938_amd as dp
    for case, f in sorted(RANGES.items()):
        x = f(synth.uniform_complex(synth.BASE_SEED + 702, 65536, 4))
        p = dp.Plan(65536, 4)
        for inv in (False, True):
            y = run_plan(p, to_dev(x), inverse=inv).cpu().numpy()
            e = max_rel(y, oracle.fft_batch(x, inverse=inv))
            say(f"   [fp32] {case} inverse={inv} max rel L2 {e:.3e}")
            assert e <= TOL_FP32, (case, inv, e)
