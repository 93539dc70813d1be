"""Streams and in-place execution.

fft_exec only enqueues work on the caller's stream: plans running on two
streams at once (each with its own workspace) must not interfere, and a plan
made with FFT_F_INPLACE must give the same result in place (four-step and 2D
plans read their input through a workspace or column tiles)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL_FP32, max_rel, say, to_dev

pytestmark = pytest.mark.gpu


def test_two_streams_concurrently():
    import torch

    import paper_1203_4938_amd as dp
    cases = [(1 << 18, 6), (20480, 5), (4096, 33)]
    plans, xs, outs, streams = [], [], [], []
    for i, (n, b) in enumerate(cases):
        x = synth.uniform_complex(synth.BASE_SEED + 50 + i, n, b)
        xs.append(x)
        plans.append(dp.Plan(n, b))
        streams.append(torch.cuda.Stream())
    xd = [to_dev(x) for x in xs]
    torch.cuda.synchronize()
    for rep in range(3):
        outs = []
        for p, x, s in zip(plans, xd, streams):
            with torch.cuda.stream(s):
                y = p.exec(x, stream=s)
                z = p.exec(y, inverse=True, stream=s)
                outs.append((y, z))
        torch.cuda.synchronize()
        for (n, b), x, (y, z) in zip(cases, xs, outs):
            e = max_rel(y.cpu().numpy(), oracle.fft_batch(x))
            r = max_rel(z.cpu().numpy(), x.astype(np.complex128))
            say(f"[streams] rep {rep} n={n} b={b}: forward {e:.3e}, round trip {r:.3e}")
            assert e <= TOL_FP32 and r <= TOL_FP32


@pytest.mark.parametrize("kind", ["fourstep", "mixed_fourstep", "2d"])
def test_inplace_multi_pass(kind):
    import paper_1203_4938_amd as dp
    if kind == "2d":
        x = synth.images_complex(synth.BASE_SEED + 60, 2, 1024, 1024)
        p = dp.Plan(shape=(1024, 1024), batch=2, rank=2, inplace=True)
        ref = oracle.fft2d(x)
    else:
        n = (1 << 18) if kind == "fourstep" else 20480
        x = synth.uniform_complex(synth.BASE_SEED + 61, n, 3)
        p = dp.Plan(n, 3, inplace=True)
        ref = oracle.fft_batch(x)
    xd = to_dev(x)
    y = p.exec(xd, out=xd)
    import torch
    torch.cuda.synchronize()
    e = max_rel(y.cpu().numpy().reshape(ref.shape[0], -1), ref.reshape(ref.shape[0], -1))
    say(f"[in place] {kind}: {e:.3e}")
    assert e <= TOL_FP32
    z = p.exec(xd, out=xd, inverse=True)
    torch.cuda.synchronize()
    r = max_rel(z.cpu().numpy().reshape(x.shape[0], -1),
                x.astype(np.complex128).reshape(x.shape[0], -1))
    assert r <= TOL_FP32
