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


# ---------------------------------------------------------------------------
# full-batch parity: every signal (or image) of a planned batch, streamed
# through the oracle chunk by chunk
# ---------------------------------------------------------------------------
#: complex points the oracle handles per chunk (its output: 16 B per point)
CHUNK_POINTS = 1 << 23


class ErrStats:
    """Per-item relative L2 errors of one direction over a whole batch."""

    def __init__(self, items: int):
        self.err = np.full(items, np.nan)
        self.nrm = np.full(items, np.nan)

    def put(self, s0: int, err, nrm):
        self.err[s0:s0 + len(err)] = err
        self.nrm[s0:s0 + len(nrm)] = nrm

    @property
    def max(self) -> float:
        assert not np.isnan(self.err).any(), "items left unchecked"
        return float(np.max(self.err))

    @property
    def mean(self) -> float:
        return float(np.mean(self.err))

    @property
    def pooled(self) -> float:
        """||Y - R|| / ||R|| over the whole batch."""
        num = np.sqrt(np.sum((self.err * self.nrm) ** 2))
        den = np.sqrt(np.sum(self.nrm ** 2))
        return float(num / den) if den > 0 else float(num)

    def line(self) -> str:
        return (f"max {self.max:.3e} mean {self.mean:.3e} pooled {self.pooled:.3e} "
                f"over {len(self.err)} items (worst item {int(np.argmax(self.err))})")


def _host(t) -> np.ndarray:
    return t.detach().cpu().numpy()


def oracle_1d(x: np.ndarray, inverse: bool) -> np.ndarray:
    return oracle.fft_batch(x, inverse=inverse)


def oracle_2d(x: np.ndarray, inverse: bool) -> np.ndarray:
    return oracle.fft2d(x, inverse=inverse)


def full_parity(plan, x_dev, ref=oracle_1d, label: str = "") -> dict:
    """Compare every item of a batch with the oracle, in both directions.

    forward: the plan's forward transform of x against the oracle's forward
             transform of the same input;
    inverse: the plan's inverse transform of the oracle's spectrum, rounded to
             complex64 (the amplitude range an inverse sees in practice),
             against the oracle's inverse of that same complex64 input;
    round trip: the plan's inverse of its own forward output against x.
    Items are the first axis of x_dev (signals, or images for 2D plans).
    Returns ErrStats for "forward", "inverse" and "round_trip"."""
    import torch
    items = x_dev.shape[0]
    per = x_dev[0].numel()
    k = max(1, CHUNK_POINTS // per)
    y = plan.exec(x_dev)
    torch.cuda.synchronize()
    spec = torch.empty_like(x_dev)
    fwd, inv, rt = ErrStats(items), ErrStats(items), ErrStats(items)
    for s0 in range(0, items, k):
        xs = _host(x_dev[s0:s0 + k])
        r = ref(xs, False)
        fwd.put(s0, *oracle.rel_l2_f32(_host(y[s0:s0 + k]), r, with_norms=True))
        spec[s0:s0 + k].copy_(torch.from_numpy(r.astype(np.complex64)))
        del r
    say(f"   [{label}] forward    {fwd.line()}")
    z = plan.exec(spec, inverse=True)
    w = plan.exec(y, inverse=True)
    torch.cuda.synchronize()
    del y
    for s0 in range(0, items, k):
        r = ref(_host(spec[s0:s0 + k]), True)
        inv.put(s0, *oracle.rel_l2_f32(_host(z[s0:s0 + k]), r, with_norms=True))
        del r
        xs = _host(x_dev[s0:s0 + k]).astype(np.complex128)
        rt.put(s0, *oracle.rel_l2_f32(_host(w[s0:s0 + k]), xs, with_norms=True))
    say(f"   [{label}] inverse    {inv.line()}")
    say(f"   [{label}] round trip {rt.line()}")
    del z, w, spec
    torch.cuda.empty_cache()
    return {"forward": fwd, "inverse": inv, "round_trip": rt}


def assert_generator_rows(x_dev, seed: int, n: int, rows) -> None:
    """Rows of a device-generated uniform batch equal the numpy generator's
    (the inputs the oracle reads back are the generator's, bit for bit)."""
    import synth
    for r in rows:
        ref = synth.uniform_complex(seed, n, 1, first=r)
        assert np.array_equal(_host(x_dev[r:r + 1]), ref), f"generator row {r} differs"
