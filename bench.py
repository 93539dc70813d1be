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
    ap.add_argument("--no-extras", action="store_true",
                    help="c2: skip the comparison entries timed after the step")
    ap.add_argument("--no-tune", action="store_true",
                    help="c5: skip the ragged autotuning (plans read DPFFT_TUNE_CACHE if set)")
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
        """forward x -> y, inverse y -> x; one launch at a time when timing a
        step item, each direction as a whole for a comparison item."""
        for inv, (src, dst) in ((False, (self.x, self.y)), (True, (self.y, self.x))):
            if events is None:
                self.plan.exec(src, out=dst, inverse=inv)
            elif self.compare:
                timed(self.torch, events, self.name, -1, lambda: self.plan.exec(src, out=dst, inverse=inv))
            else:
                for s in range(self.nsteps):
                    timed(self.torch, events, self.name, s,
                          lambda: self.plan.exec_steps(src, dst, s, 1, inverse=inv))


def timed(torch, events, name, s, fn):
    """Run fn between two HIP events recorded on the current stream (the
    stream every launch of this benchmark goes to)."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    fn()
    e1.record()
    events.append((name, s, e0, e1))


class MultiItem:
    """A comparison entry made of several callables per direction (one plan per
    distinct length, or forward + product + inverse); timed per direction as a
    whole."""

    def __init__(self, torch, name, fwd, inv, flop, alg_bytes, desc):
        self.torch, self.name, self.fwd, self.inv = torch, name, fwd, inv
        self.flop, self.alg_bytes, self.desc = flop, alg_bytes, desc
        self.compare = True
        self.nsteps = 1

    def run(self, events=None):
        for fn in (self.fwd, self.inv):
            if events is None:
                fn()
            else:
                timed(self.torch, events, self.name, -1, fn)


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


def build_c5(dp, torch, synth, dev, tune=True):
    sizes = synth.ragged_sizes(synth.BASE_SEED + 5, 10000)
    flat, offs = synth.uniform_ragged(synth.BASE_SEED + 5, sizes)
    x = torch.from_numpy(flat).to(dev)
    fl = float(sum(flops(int(n), 1) for n in sizes))
    # per-length choices from the autotuner (plan time, outside any timing)
    d, keep = dp.make_desc(ragged_sizes=sizes.tolist())
    t0 = time.perf_counter()
    st, rep = dp.fft_autotune(d, reps=3) if tune else (dp.FFT_OK, "skipped (--no-tune)")
    tune_s = time.perf_counter() - t0
    if st != dp.FFT_OK:
        raise RuntimeError(f"ragged autotune failed: {rep}")
    print(f"# c5 autotune ({tune_s:.1f} s): {rep.strip()}", file=sys.stderr, flush=True)
    items = []
    for name, kw, cmp in (("ragged10000_graph", dict(graph=True), False),
                          ("ragged10000_no_graph", dict(), True),
                          ("ragged10000_heuristic_graph", dict(graph=True, autotune=False), True),
                          ("ragged10000_one_launch_per_length_runtime_radix", dict(per_size=True),
                           True)):
        p = dp.Plan(ragged_sizes=sizes.tolist(), **kw)
        items.append(Item(dp, torch, name, p, x.clone(), torch.empty_like(x), fl,
                          16.0 * float(sizes.sum()), compare=cmp))
    return items, {"workload": "c5: ragged batch of 10000 7-smooth sizes in [64, 65536], "
                               "log-uniform; the step is the ragged launches in a HIP graph "
                               "with autotuned per-length choices; the same launches without the "
                               "graph, the untuned heuristic plan and one launch per distinct "
                               "length are timed after it for comparison",
                   "autotune_s": round(tune_s, 1), "autotune": rep.strip()}


def build_c5_fair(dp, torch, synth, dev):
    """Per-length baseline: the c5 signals grouped by length (the gather into
    that order is not timed) and one batched plan per distinct length, each on
    the library's compile-time kernels where the length is a power of two."""
    import numpy as np
    sizes = synth.ragged_sizes(synth.BASE_SEED + 5, 10000)
    order = np.argsort(sizes, kind="stable")
    flat, offs = synth.uniform_ragged(synth.BASE_SEED + 5, sizes)
    parts = [flat[offs[i]:offs[i] + sizes[i]] for i in order]
    x = torch.from_numpy(np.concatenate(parts)).to(dev)
    y = torch.empty_like(x)
    plans, o = [], 0
    for n in np.unique(sizes):
        cnt = int((sizes == n).sum())
        plans.append((dp.Plan(int(n), cnt), o, int(n) * cnt))
        o += int(n) * cnt

    def go(src, dst, inv):
        for p, o0, m in plans:
            p.exec(src[o0:o0 + m], out=dst[o0:o0 + m], inverse=inv)

    fl = float(sum(flops(int(n), 1) for n in sizes))
    return MultiItem(torch, "ragged10000_one_plan_per_length", lambda: go(x, y, False),
                     lambda: go(y, x, True), fl, 16.0 * float(sizes.sum()),
                     f"{len(plans)} batched plans, one per distinct length, signals grouped by length")


def build_conv(dp, torch, synth, dev):
    """Fused circular convolution against forward + product + inverse: N = 4096,
    batch 32768 (1 GiB), one shared filter."""
    n, b = 4096, 32768
    x = synth.uniform_complex_torch(synth.BASE_SEED + 6, n, b, dev)
    h = synth.uniform_complex_torch(synth.BASE_SEED + 6 + 7777, n, 1, dev)
    p = dp.Plan(n, b, conv=True)
    H = dp.Plan(n, 1).exec(h).reshape(-1)
    y = torch.empty_like(x)
    fl = b * (2 * 5.0 * n * math.log2(n) + 6.0 * n)
    fused = MultiItem(torch, "conv4096_b32768_fused", lambda: p.conv(x, H, out=y),
                      lambda: p.conv(y, H, out=x), fl, 16.0 * n * b,
                      p.describe().splitlines()[-1].strip())
    z = torch.empty_like(x)

    def unfused_fwd():
        p.exec(x, out=z)
        z.mul_(H)
        p.exec(z, out=y, inverse=True)

    def unfused_inv():
        p.exec(y, out=z)
        z.mul_(H)
        p.exec(z, out=x, inverse=True)

    three = MultiItem(torch, "conv4096_b32768_unfused", unfused_fwd, unfused_inv, fl,
                      16.0 * n * b, "fft_exec forward, torch mul_ by H, fft_exec inverse "
                                    "(three HBM round trips)")
    return [fused, three]


def build_real(dp, torch, synth, dev):
    """The c3 images as real input: 16 x 2048^2 float32 -> 16 x 2048 x 1025 bins."""
    import numpy as np
    imgs = np.stack([synth.smooth_noise_image(synth.BASE_SEED + 3, i) for i in range(16)])
    x = torch.from_numpy(np.ascontiguousarray(imgs.astype(np.float32))).to(dev)
    p = dp.Plan(shape=(2048, 2048), batch=16, rank=2, real=True)
    spec = torch.empty((16, 2048, 1025), dtype=torch.complex64, device=dev)
    n = 2048 * 2048
    # real transforms: half the conventional complex flop count; bytes: 4 B per
    # sample read plus 8 B per bin written (the inverse: the reverse)
    alg = 16 * (4.0 * n + 8.0 * 2048 * 1025)
    return MultiItem(torch, "img2048_b16_real", lambda: p.exec(x, out=spec),
                     lambda: p.exec(spec, out=x, inverse=True), 0.5 * flops(n, 16), alg,
                     p.describe().splitlines()[0])


def build_real_1d(dp, torch, synth, dev):
    """The c2 signals of 2^22 points as real input (their real parts): 32 x 2^22
    float32 -> 32 x (2^21 + 1) bins, through the 2^21-point four-step core and
    the pairing launch."""
    n, b = 1 << 22, 32
    x = synth.uniform_complex_torch(synth.BASE_SEED + 2, n, b, dev).real.contiguous()
    p = dp.Plan(n, b, real=True)
    spec = torch.empty((b, n // 2 + 1), dtype=torch.complex64, device=dev)
    alg = b * (4.0 * n + 8.0 * (n // 2 + 1))
    return MultiItem(torch, "real2^22_b32", lambda: p.exec(x, out=spec),
                     lambda: p.exec(spec, out=x, inverse=True), 0.5 * flops(n, b), alg,
                     p.describe().splitlines()[0])


def build_img(dp, torch, synth, dev):
    """Image block compression (section III-B): 16 colour photographs of
    2048 x 2048, k = 64 codewords, 8 Lloyd iterations, tau = 8.  Algorithmic
    bytes per pixel: 3 read and 10.5 written by steps a-c, 0.5 for the pattern
    counts, 4.25 per iteration and 4.5 for the codes (18.5 + 4.25 iters)."""
    B, h, w, k, iters, tau = 16, 2048, 2048, 64, 8, 8.0
    rgb = torch.from_numpy(synth.images_rgb(synth.BASE_SEED + 7, B, h, w)).to(dev)
    first = dp.img_compress(rgb, k, iters, tau)
    d = dp.ImgDesc(height=h, width=w, batch=B, k=k, iters=iters, tau=tau, flags=dp.IMG_F_GRAPH)
    o = dp.ImgOut(*(first[n].data_ptr() for n in ("y", "cb", "cr", "mean", "act", "dev",
                                                   "codebook", "code")))
    ws = first["_workspace"]

    def run():
        st = dp._lib.img_compress(d, rgb.data_ptr(), o, ws.data_ptr(),
                                  torch.cuda.current_stream().cuda_stream)
        if st != dp.FFT_OK:
            raise dp.FftError(st, "img_compress", dp.fft_last_error())

    npx = B * h * w
    nb = npx // 16
    item = MultiItem(torch, "img2048_b16_block_compress", run, run,
                     float(nb * k * 48 * (iters + 1)), (18.5 + 4.25 * iters) * npx,
                     f"img_compress: {B} RGB images {h}x{w}, k={k}, {iters} Lloyd iterations, "
                     f"tau={tau}, replayed as a HIP graph (IMG_F_GRAPH); GFLOP/s counts the "
                     f"codeword distances of every block")
    item.keep = (rgb, first)
    return item


def build_extras(dp, torch, synth, dev):
    """Comparison entries timed after the c2 step: the c4 precision forms, the
    c5 ragged batch (graph, no graph, one plan per length, one launch per
    length), the c3 images as complex and as real input, the c2 signals of 2^22
    points as real input, the fused
    convolution against its unfused chain, and the image block compression."""
    out = []
    c4, _ = build_c4(dp, torch, synth, dev)
    c5, _ = build_c5(dp, torch, synth, dev)
    c3, _ = build_c3(dp, torch, synth, dev)
    for it in c4 + c5 + c3:
        it.compare = True
        out.append(it)
    out.append(build_c5_fair(dp, torch, synth, dev))
    out.append(build_real(dp, torch, synth, dev))
    out.append(build_real_1d(dp, torch, synth, dev))
    out.extend(build_conv(dp, torch, synth, dev))
    out.append(build_img(dp, torch, synth, dev))
    return out


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
    # one thread, one size (N = 2^14), about two seconds of work
    n1, k1, t1s, f1 = 1 << 14, 0, 0.0, 0.0
    while t1s < 2.0 and k1 < 4096:
        x = synth.uniform_complex(seed, n1, 8, first=k1)
        t0 = time.perf_counter()
        oracle.fft_batch(x, inverse=False, threads=1)
        t1s += time.perf_counter() - t0
        f1 += flops(n1, 8)
        k1 += 8
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": round(total_f / total_t / 1e9, 4), "unit": "GFLOP/s", "cores": thr,
            "kind": "oracle", "cpu_model": model, "host_cpus_visible": os.cpu_count(),
            "one_thread": {"value": round(f1 / t1s / 1e9, 4), "unit": "GFLOP/s",
                           "sample": f"forward transforms of {k1} signals of N=2^14, 1 thread"},
            "sample": "forward+inverse of a prefix of each c2 batch (" + "; ".join(sample) +
                      "), each size's rate scaled to its full batch",
            "per_size_gflops": {f"2^{int(math.log2(n))}": round(r / 1e9, 4) for n, r in per.items()}}


def copy_probe(torch, dev, reps=10):
    """Two plain 1 GiB device-to-device passes of known traffic (1 GiB read,
    1 GiB written each): torch's copy (a blit kernel) and an elementwise
    float64 negation (8-byte loads and stores over the whole buffer).  Their
    rates are a practical bandwidth reference; their FETCH_SIZE / WRITE_SIZE
    readings calibrate the counters (two points)."""
    a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    a64, b64 = a.view(torch.float64), b.view(torch.float64)
    res = {}
    for name, fn in (("copy", lambda: b.copy_(a)), ("neg_f64", lambda: torch.neg(a64, out=b64))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[name] = round(2 * a.numel() * 4 / (ms * 1e-3) / 1e9, 1)
    return res


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
    if args.config == "c5":
        items, cfg = build_c5(dp, torch, synth, dev, tune=not args.no_tune)
    else:
        items, cfg = builder[args.config](dp, torch, synth, dev)
    print(f"# {cfg['workload']}", file=sys.stderr, flush=True)
    if args.config == "c2" and not args.no_extras:
        items += build_extras(dp, torch, synth, dev)
        print(f"# {len(items)} entries planned", file=sys.stderr, flush=True)

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
        if it.compare:
            tot_ms = sum(kern[(it.name, -1)]) / args.steps / 2
        else:
            tot_ms = sum(sum(kern[(it.name, s)]) for s in range(it.nsteps)) / args.steps / 2
        ent = {
            "ms_per_transform": round(tot_ms, 4),
            "gflops": round(it.flop / (tot_ms * 1e-3) / 1e9, 1),
            "hbm_frac_alg": round(it.alg_bytes / (tot_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        }
        if it.compare:
            ent["comparison_only"] = True
        else:
            ent["kernels"] = [{"launch": s, "avg_ms": round(sum(kern[(it.name, s)]) /
                                                            len(kern[(it.name, s)]), 4)}
                              for s in range(it.nsteps)]
        ent["plan"] = it.desc if isinstance(it, MultiItem) else it.plan.describe().splitlines()[0]
        breakdown[it.name] = ent
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
        out["copy_probe_GBps"] = probe
    if not args.no_cpu and args.config == "c2":
        out["cpu_baseline"] = cpu_baseline(args.cpu_budget)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
