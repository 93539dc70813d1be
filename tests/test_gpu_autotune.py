"""The autotuner on the GPU: it times every candidate kernel variant of a
descriptor, stores the fastest in the tuning-cache file, and a plan built
afterwards in a fresh process picks that variant up and still matches the
oracle.  Each case runs in child processes so the cache file is read anew."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu

TUNE = """
import sys
import paper_1203_4938_amd as dp
d, keep = dp.make_desc(**{kw})
st, rep = dp.fft_autotune(d, reps=3)
print(rep)
sys.exit(0 if st == dp.FFT_OK else 1)
"""

CHECK = """
import sys
import numpy as np
import torch
sys.path.insert(0, {tests!r})
import oracle, synth
import paper_1203_4938_amd as dp
from gpu_util import max_rel, to_dev
kw = {kw}
p = dp.Plan(**kw)
print(p.describe())
if kw.get("rank", 1) == 2:
    x = synth.images_complex(synth.BASE_SEED + 9, kw["batch"], *kw["shape"])
    ref = oracle.fft2d(x)
else:
    x = synth.uniform_complex(synth.BASE_SEED + 9, kw["n"], kw["batch"])
    ref = oracle.fft_batch(x)
y = p.exec(to_dev(x)).cpu().numpy()
torch.cuda.synchronize()
print("err", max_rel(y, ref))
"""


def _child(code, env):
    r = subprocess.run([sys.executable, "-u", "-c", code], capture_output=True, text=True,
                       cwd=ROOT, env=env, timeout=300)
    print(r.stdout[-3000:], r.stderr[-2000:], flush=True)
    return r


@pytest.mark.parametrize("kw", [
    dict(n=4096, batch=64),
    dict(n=1 << 18, batch=8),
    dict(rank=2, shape=(1024, 1024), batch=2),
], ids=["n4096", "n2^18", "2d1024"])
def test_autotune_then_plan(kw, tmp_path):
    env = dict(os.environ)
    env["DPFFT_TUNE_CACHE"] = str(tmp_path / "tune.json")
    env.pop("DPFFT_FORCE_PLAN", None)
    desc_kw = dict(kw)
    if "shape" in desc_kw:
        desc_kw["shape"] = tuple(desc_kw["shape"])
    r = _child(TUNE.format(kw=repr(desc_kw)), env)
    assert r.returncode == 0, r.stderr
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    timed = [l for l in lines if l.endswith(" ms")]
    assert len(timed) >= 2, "expected several timed candidates"
    best = [l for l in lines if l.startswith("best: ")]
    assert len(best) == 1
    choice = best[0][len("best: "):].split(" (")[0]
    cache = json.loads((tmp_path / "tune.json").read_text())
    assert choice in cache["entries"].values()

    r = _child(CHECK.format(kw=repr(desc_kw), tests=os.path.join(ROOT, "tests")), env)
    assert r.returncode == 0, r.stderr
    assert f'override="{choice}"' in r.stdout
    err = float([l for l in r.stdout.splitlines() if l.startswith("err ")][0].split()[1])
    assert err <= 1e-5
