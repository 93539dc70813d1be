"""Helpers shared by the GPU parity tests: move seeded inputs to the device,
run a dpfft plan through the C ABI, compare with the FP64 oracle."""
from __future__ import annotations

import sys

import numpy as np

import oracle

#: relative L2 bound for the FP32 path (per signal, gated on the max)
TOL_FP32 = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(x: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def run_plan(plan, x_dev, inverse=False, out=None):
    import torch
    y = plan.exec(x_dev, out=out, inverse=inverse)
    torch.cuda.synchronize()
    return y


def max_rel(y, ref) -> float:
    e = oracle.rel_l2(y, ref)
    return float(np.max(e)) if np.size(e) else 0.0
