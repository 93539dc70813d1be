#!/usr/bin/env python3
"""Throughput of the batched C2C FFT on one MI355X.

Default workload (one "step"): plain FP32 batched 1D complex-to-complex FFTs,
N in {2^10, 2^14, 2^18, 2^22} with batch*N = 2^27 (1 GiB of complex64 per
size), each transformed forward and then inverse, inputs resident in HBM.
Metric: GFLOP/s in the 5 N log2 N convention per transform and direction.

Prints one JSON line.  Per-kernel durations come from HIP events recorded on
the launch stream around every kernel inside the timed region; the roofline
entry is for the kernel with the largest share of the step.

Other workloads (not part of the default line): --config c1|c3|c4|c5.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "batched C2C FFT GFLOP/s (5N·log2N) + % HBM BW; FP32 vs split-FP16 at ≤1e-5"
HBM_PEAK_GBPS = 8000.0
C2_SIZES = [(1 << 10, 131072), (1 << 14, 8192), (1 << 18, 512), (1 << 22, 32)]


def flops(n: int, batch: int) -> float:
    return 5.0 * n * math.log2(n) * batch if n > 1 else 0.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of CPU oracle work for the baseline sample")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also time a plain 1 GiB device copy (bandwidth reference)")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# Sources of the power-of-two line kernels and of the planner that picks them:
# the kernels of the c2 workload.  A change to any of them voids the stored
# counter profile.
TRAFFIC_SOURCES = ("line_kernels.hip", "kernels.h", "fft_common.h", "api.cpp", "plan.h",
                   "internal.h", "twiddle.cpp", "twiddle.h")


def src_digest() -> str:
    """Hash of the line-kernel and planner sources; a stored counter profile is
    valid only for it."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1203_4938_amd", "csrc")
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_key: str):
    """HBM traffic per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    if data.get("src_digest") != src_digest():
        return None
    ent = data.get("kernels", {}).get(kernel_key)
    return None if ent is None else ent.get("hbm_bytes_per_launch")


# ---------------------------------------------------------------------------
class Item:
    """One planned transform of the workload: a plan and its device buffers."""

    def __init__(self, dp, torch, name, plan, x, y, flop, alg_bytes_per_transform, compare=False):
        self.name, self.plan, self.x, self.y = name, plan, x, y
        self.compare = compare  # timed after the step, for comparison only
        self.flop = flop
        self.alg_bytes = alg_bytes_per_transform
        self.nsteps = plan.num_steps()
        self.torch = torch

    def run(self, events=None):
        """forward x -> y, inverse y -> x; one launch at a time when timing."""
        for inv, (src, dst) in ((False, (self.x, self.y)), (True, (self.y, self.x))):
            if events is None:
                self.plan.exec(src, out=dst, inverse=inv)
                continue
            for s in range(self.nsteps):
                e0 = self.torch.cuda.Event(enable_timing=True)
                e1 = self.torch.cuda.Event(enable_timing=True)
                e0.record()
                self.plan.exec_steps(src, dst, s, 1, inverse=inv)
                e1.record()
                events.append((self.name, s, e0, e1))


def build_c2(dp, torch, synth, dev):
    items = []
    seed = synth.BASE_SEED + 2
    for n, b in C2_SIZES:
        x = synth.uniform_complex_torch(seed, n, b, dev)
        y = torch.empty_like(x)
        p = dp.Plan(n, b)
        items.append(Item(dp, torch, f"n2^{int(math.log2(n))}", p, x, y, flops(n, b), 16.0 * n * b))
    cfg = {"workload": "c2: FP32 batched 1D C2C FFT, N in {2^10,2^14,2^18,2^22}, "
                       "batch*N = 2^27 complex64 per size, forward then inverse",
           "sizes": [[n, b] for n, b in C2_SIZES], "layout": "interleaved complex64, dense",
           "four_step_from": 1 << 15}
    return items, cfg


def build_c1(dp, torch, synth, dev):
    x = synth.uniform_complex_torch(synth.BASE_SEED + 1, 4096, 64, dev)
    p = dp.Plan(4096, 64)
    return [Item(dp, torch, "n4096_b64", p, x, torch.empty_like(x), flops(4096, 64),
                 16.0 * 4096 * 64)], {"workload": "c1: N=4096 batch 64 FP32, forward then inverse"}


def build_c3(dp, torch, synth, dev):
    import numpy as np
    imgs = synth.images_complex(synth.BASE_SEED + 3, 16, 2048, 2048)
    x = torch.from_numpy(imgs).to(dev)
    p = dp.Plan(shape=(2048, 2048), batch=16, rank=2)
    n = 2048 * 2048
    return [Item(dp, torch, "img2048_b16", p, x, torch.empty_like(x), flops(n, 16), 16.0 * n * 16)], \
        {"workload": "c3: 16 synthetic 2048x2048 uint8 images as complex64, 2D FFT forward then inverse"}


def build_c4(dp, torch, synth, dev):
    items = []
    x = synth.uniform_complex_torch(synth.BASE_SEED + 4, 1 << 16, 4096, dev)
    for prec in ("fp32", "fp16", "bf16", "fp16_split", "bf16_split", "bf16_split3"):
        try:
            p = dp.Plan(1 << 16, 4096, precision=prec)
        except dp.FftError as e:
            print(f"# c4 {prec}: {e}", file=sys.stderr)
            continue
        items.append(Item(dp, torch, f"c4_{prec}", p, x.clone(), torch.empty_like(x),
                          flops(1 << 16, 4096), 16.0 * (1 << 16) * 4096))
    return items, {"workload": "c4: N=2^16 batch 4096, precision forms"}


def build_c5(dp, torch, synth, dev):
    import numpy as np
    sizes = synth.ragged_sizes(synth.BASE_SEED + 5, 10000)
    flat, offs = synth.uniform_ragged(synth.BASE_SEED + 5, sizes)
    x = torch.from_numpy(flat).to(dev)
    fl = float(sum(flops(int(n), 1) for n in sizes))
    items = []
    for name, kw, cmp in (("ragged10000_persistent_graph", dict(graph=True), False),
                          ("ragged10000_persistent", dict(), True),
                          ("ragged10000_per_length_launches", dict(per_size=True), True)):
        p = dp.Plan(ragged_sizes=sizes.tolist(), **kw)
        items.append(Item(dp, torch, name, p, x.clone(), torch.empty_like(x), fl,
                          16.0 * float(sizes.sum()), compare=cmp))
    return items, {"workload": "c5: ragged batch of 10000 7-smooth sizes in [64, 65536], "
                               "log-uniform; the step is the two persistent launches in a HIP "
                               "graph; the same launches without the graph and one launch per "
                               "distinct length are timed after it for comparison"}


# ---------------------------------------------------------------------------
def cpu_baseline(budget_s: float):
    """The FP64 oracle on the host cores, on a bounded prefix of the C2 batches."""
    import numpy as np

    import oracle
    import synth
    thr = oracle.threads(0)
    seed = synth.BASE_SEED + 2
    total_t, total_f = 0.0, 0.0
    per = {}
    share = budget_s / len(C2_SIZES)
    sample = []
    for n, b in C2_SIZES:
        # one chunk of `threads` signals, then one more sized to fill this
        # size's share of the budget
        spent, done_f, done_sig = 0.0, 0.0, 0
        k = max(1, min(b, thr))
        for _ in range(2):
            kk = min(k, b - done_sig)
            if kk <= 0:
                break
            x = synth.uniform_complex(seed, n, kk, first=done_sig)
            t0 = time.perf_counter()
            oracle.fft_batch(x, inverse=False)
            oracle.fft_batch(x, inverse=True)
            spent += time.perf_counter() - t0
            done_f += 2 * flops(n, kk)
            done_sig += kk
            per_sig = spent / done_sig
            k = int((share - spent) / per_sig) // thr * thr
            if k < thr:
                break
        rate = done_f / spent
        per[n] = rate
        sample.append(f"N=2^{int(math.log2(n))}: {done_sig}/{b} signals")
        total_t += 2 * flops(n, b) / rate
        total_f += 2 * flops(n, b)
    return {"value": round(total_f / total_t / 1e9, 4), "unit": "GFLOP/s", "cores": thr,
            "kind": "oracle",
            "sample": "forward+inverse of a prefix of each c2 batch (" + "; ".join(sample) +
                      "), each size's rate scaled to its full batch",
            "per_size_gflops": {f"2^{int(math.log2(n))}": round(r / 1e9, 4) for n, r in per.items()}}


def copy_probe(torch, dev, reps=10):
    a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return 2 * a.numel() * 4 / (ms * 1e-3) / 1e9


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only; --gpus {args.gpus} is not "
              "supported (batched transforms would shard by signal with no communication)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1203_4938_amd as dp
    import synth
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    builder = {"c1": build_c1, "c2": build_c2, "c3": build_c3, "c4": build_c4, "c5": build_c5}
    items, cfg = builder[args.config](dp, torch, synth, dev)
    print(f"# {cfg['workload']}", file=sys.stderr, flush=True)

    probe = copy_probe(torch, dev) if args.copy_probe else None

    step_items = [it for it in items if not it.compare]
    for _ in range(args.warmup):
        for it in items:
            it.run()
    torch.cuda.synchronize()

    events = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for it in step_items:
            it.run(events)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    # comparison items: same number of steps, outside the timed step
    for _ in range(args.steps):
        for it in items:
            if it.compare:
                it.run(events)
    torch.cuda.synchronize()

    # per-kernel durations from the events of the timed region
    kern = {}
    for name, s, e0, e1 in events:
        kern.setdefault((name, s), []).append(e0.elapsed_time(e1))
    step_flop = sum(2 * it.flop for it in step_items)
    value = step_flop / (ms_step * 1e-3) / 1e9
    breakdown = {}
    for it in items:
        tot_ms = sum(sum(kern[(it.name, s)]) for s in range(it.nsteps)) / args.steps / 2
        breakdown[it.name] = {
            "ms_per_transform": round(tot_ms, 4),
            "gflops": round(it.flop / (tot_ms * 1e-3) / 1e9, 1),
            "hbm_frac_alg": round(it.alg_bytes / (tot_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
            "kernels": [{"launch": s, "avg_ms": round(sum(kern[(it.name, s)]) / len(kern[(it.name, s)]), 4)}
                        for s in range(it.nsteps)],
            "plan": it.plan.describe().splitlines()[0],
        }
        if it.compare:
            breakdown[it.name]["comparison_only"] = True
    # dominant kernel: largest total time over the step
    step_names = {it.name for it in step_items}
    (dn, ds), dur = max(((k, v) for k, v in kern.items() if k[0] in step_names),
                        key=lambda kv: sum(kv[1]))
    dit = next(it for it in items if it.name == dn)
    avg_ms = sum(dur) / len(dur)
    alg_per_launch = dit.alg_bytes / dit.nsteps  # the transform's 16 B/pt split over its launches
    achieved = alg_per_launch / (avg_ms * 1e-3) / 1e9
    key = f"{dn}/launch{ds}"
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": load_traffic(key),
            "kernel": key, "kernel_desc": dit.plan.describe().splitlines()[1 + ds].strip(),
            "avg_launch_ms": round(avg_ms, 4), "alg_bytes_per_launch": alg_per_launch}

    out = {"metric": METRIC, "value": round(value, 1), "unit": "GFLOP/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (seeded SplitMix64 uniform[-1,1) complex64)",
           "config": cfg, "roofline": roof, "breakdown": breakdown}
    if probe is not None:
        out["copy_probe_GBps"] = round(probe, 1)
    if not args.no_cpu and args.config == "c2":
        out["cpu_baseline"] = cpu_baseline(args.cpu_budget)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
