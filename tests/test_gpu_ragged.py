"""GPU parity of ragged batches (packed signals of mixed 7-smooth lengths)
against the FP64 oracle: the launches (one workgroup per item, or resident
workgroups walking the item lists), the same launches replayed
from a HIP graph (several replays with eager work between them, each checked),
and the one-launch-per-length baseline; forward and inverse; lengths from 1 to
65536 including four-step lengths above 16384; every per-length choice the
autotuner can make; and the full 10,000-signal workload, tuned, checked
signal by signal."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import TOL_FP32, say, to_dev

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 3, 5, 7, 64, 100, 343, 1000, 4096, 6561, 16384, 15625, 20480, 65536, 49152,
         3 ** 10, 2 * 3 * 5 * 7 * 11 // 11 * 8, 17640, 64, 64, 1000, 81, 20480, 2]


def _ragged_errors(got, flat, sizes, offsets, inverse):
    ref = oracle.fft_ragged(flat, sizes, offsets, inverse=inverse)
    errs = []
    for n, o in zip(sizes, offsets):
        r = ref[o:o + n]
        d = np.linalg.norm(r)
        errs.append(np.linalg.norm(got[o:o + n].astype(np.complex128) - r) / (d if d else 1.0))
    return np.array(errs)


@pytest.mark.parametrize("mode", ["queue", "graph", "per_size"])
def test_ragged_modes(mode):
    import paper_1203_4938_amd as dp
    rng = np.random.default_rng(3)
    sizes = list(SIZES) + [int(v) for v in rng.choice(synth.smooth_sizes(2, 30000), 60)]
    flat, offs = synth.uniform_ragged(synth.BASE_SEED + 800, sizes)
    p = dp.Plan(ragged_sizes=sizes, graph=(mode == "graph"), per_size=(mode == "per_size"))
    say(f"[ragged {mode}] {p.describe()}")
    x = to_dev(flat)
    for inv in (False, True):
        y = p.exec(x, inverse=inv)
        e = _ragged_errors(y.cpu().numpy(), flat, sizes, offs, inv)
        say(f"   inverse={inv} max rel L2 = {e.max():.3e} over {len(sizes)} signals")
        assert e.max() <= TOL_FP32


def test_ragged_graph_replays_with_eager_work_between():
    import torch

    import paper_1203_4938_amd as dp
    sizes = [64, 20480, 343, 65536, 1000, 7, 49152, 4096]
    flat, offs = synth.uniform_ragged(synth.BASE_SEED + 801, sizes)
    p = dp.Plan(ragged_sizes=sizes, graph=True)
    x = to_dev(flat)
    ref = oracle.fft_ragged(flat, sizes, offs)
    out = torch.empty_like(x)
    for rep in range(4):
        out.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        p.exec(x, out=out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        e = max(np.linalg.norm(got[o:o + n] - ref[o:o + n]) / np.linalg.norm(ref[o:o + n])
                for n, o in zip(sizes, offs))
        say(f"   replay {rep}: max rel L2 {e:.3e} (junk {float(junk):.1f})")
        assert e <= TOL_FP32


def test_graph_cache_beyond_its_capacity():
    """A graph plan run on 10 output buffers (more than the 8 graphs a plan
    keeps), then on the first one again (its graph was evicted and is built
    anew): every result matches the oracle."""
    import torch

    import paper_1203_4938_amd as dp
    sizes = [64, 20480, 343, 1000, 49152, 7]
    flat, offs = synth.uniform_ragged(synth.BASE_SEED + 805, sizes)
    p = dp.Plan(ragged_sizes=sizes, graph=True)
    x = to_dev(flat)
    outs = [torch.empty_like(x) for _ in range(10)]
    for i in list(range(10)) + [0, 1]:
        outs[i].fill_(3)
        y = p.exec(x, out=outs[i]).cpu().numpy()
        assert _ragged_errors(y, flat, sizes, offs, False).max() <= TOL_FP32, i
    say("[ragged graph cache] 10 buffer sets and two revisits match the oracle")


def test_plans_with_different_lds_needs_coexist():
    """A plan whose 1024-thread items need less LDS, built after one that
    needs more, leaves the first plan runnable (the kernels' LDS limit is set
    to the class budget, not to the last plan's need)."""
    import paper_1203_4938_amd as dp
    big, small = [16384, 15625, 16000, 16384], [5000, 5120, 6000, 5103]
    fa, oa = synth.uniform_ragged(synth.BASE_SEED + 803, big)
    fb, ob = synth.uniform_ragged(synth.BASE_SEED + 804, small)
    pa = dp.Plan(ragged_sizes=big)
    pb = dp.Plan(ragged_sizes=small)
    say(f"[lds coexist] {pa.describe()} | {pb.describe()}")
    for p, f, sz, of in ((pb, fb, small, ob), (pa, fa, big, oa)):
        y = p.exec(to_dev(f)).cpu().numpy()
        assert _ragged_errors(y, f, sz, of, False).max() <= TOL_FP32


def test_ragged_with_gaps_and_explicit_offsets():
    import paper_1203_4938_amd as dp
    sizes = [100, 7, 20480, 64]
    offs = [5, 200, 300, 300 + 20480 + 11]
    total = offs[-1] + sizes[-1] + 3
    flat = synth.uniform_complex(synth.BASE_SEED + 802, total, 1).reshape(-1)
    p = dp.Plan(ragged_sizes=sizes, ragged_offsets=offs)
    x = to_dev(flat)
    y = p.exec(x, out=x.clone()).cpu().numpy()
    e = _ragged_errors(y, flat, sizes, offs, False)
    assert e.max() <= TOL_FP32
    # untouched gaps keep the original values
    assert np.array_equal(y[:5], flat[:5]) and np.array_equal(y[107:200], flat[107:200])


FORMS = ["f=0", "f=2", "f=1", "b=0", "o=1", "o=1 f=1", "f=1 c0=2 c1=2", "f=2 c0=1", "x=0", "x=0 f=1",
         "p0=1", "p0=1 x=0"]


@pytest.mark.parametrize("force", FORMS)
def test_ragged_forced_choices(force, monkeypatch):
    """Every form a per-length choice can name (single pass in 256 or 1024
    threads, four-step, no 1024-thread class, odd radices first, narrower
    tiles), forced on every length where it fits, forward and inverse."""
    import paper_1203_4938_amd as dp
    sizes = [64, 1000, 4096, 4800, 6000, 7776, 10080, 16384, 15625, 17640, 65536, 2, 49152]
    flat, offs = synth.uniform_ragged(synth.BASE_SEED + 803, sizes)
    monkeypatch.setenv("DPFFT_FORCE_PLAN", force)
    p = dp.Plan(ragged_sizes=sizes)
    say(f"[ragged {force}] {p.describe()}")
    x = to_dev(flat)
    for inv in (False, True):
        y = p.exec(x, inverse=inv)
        e = _ragged_errors(y.cpu().numpy(), flat, sizes, offs, inv)
        assert e.max() <= TOL_FP32, (force, inv, e.max())


def _tune_c5(dp, sizes):
    d, keep = dp.make_desc(ragged_sizes=sizes.tolist())
    st, rep = dp.fft_autotune(d, reps=3)
    assert st == dp.FFT_OK, rep
    say(f"[c5 tune] {rep.strip()}")


def test_c5_full_workload_every_signal():
    """The 10,000-signal workload in the launch configuration the benchmark
    times (per-length choices from the autotuner, the launches in a HIP graph),
    every signal against the oracle."""
    import paper_1203_4938_amd as dp
    w = synth.workloads()["c5_ragged_10000"]
    sizes = synth.ragged_sizes(w.seed, w.count)
    flat, offs = synth.uniform_ragged(w.seed, sizes)
    _tune_c5(dp, sizes)
    p = dp.Plan(ragged_sizes=sizes.tolist(), graph=True)
    assert "578 lengths with tuned choices" in p.describe()
    say(f"[c5] {p.describe()}")
    x = to_dev(flat)
    for inv in (False, True):
        y = p.exec(x, inverse=inv)
        e = _ragged_errors(y.cpu().numpy(), flat, sizes, offs, inv)
        say(f"   inverse={inv} max rel L2 {e.max():.3e}, mean {e.mean():.3e}")
        assert e.max() <= TOL_FP32
