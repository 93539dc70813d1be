"""Host-side planning (no GPU): factorization and variant choice seen through
fft_plan_dry, the override hook, and the tuning-cache file (valid entry used,
corrupt file ignored, FFT_F_NO_AUTOTUNE honoured)."""
import json
import re
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _dp():
    import paper_1203_4938_amd as dp
    return dp


def _dry(**kw):
    dp = _dp()
    d, keep = dp.make_desc(**kw)
    st, text = dp.fft_plan_dry(d)
    assert st == dp.FFT_OK, text
    return text


@pytest.mark.parametrize("n,variant,launches", [
    (1, "single-pass", 1), (4096, "single-pass", 1), (16384, "single-pass", 1),
    (1 << 15, "four-step 128x256", 2), (1 << 18, "four-step 512x512", 2),
    (1 << 22, "four-step 2048x2048", 2), (1 << 24, "four-step 4096x4096", 2),
    (1000, "mixed single-pass", 1), (15625, "mixed single-pass", 1),
    (78125, "mixed four-step 125x625", 2), (3 ** 15, "mixed four-step 2187x6561", 2),
])
def test_variant_by_length(n, variant, launches):
    t = _dry(n=n, batch=3)
    assert f"variant={variant} " in t, t
    assert f"launches={launches}" in t


def test_radix_plans_of_mixed_lengths():
    assert "radices=8x5x5x5" in _dry(n=1000, batch=1)
    assert "radices=16x7x3" in _dry(n=336, batch=1)
    assert "radices=7x7x7x7" in _dry(n=2401, batch=1)
    # pairs of 3s become radix-9 passes, a lone 3 stays
    assert "radices=9x9x9x9" in _dry(n=6561, batch=1)
    assert "radices=16x7x5x9x3" in _dry(n=15120, batch=1)
    assert "mixed four-step 49x343" in _dry(n=16807, batch=1)


def test_workspace_sizes():
    dp = _dp()
    for n, b, ws in ((4096, 64, 0), (1 << 18, 4, (1 << 18) * 4 * 8)):
        t = _dry(n=n, batch=b)
        assert f"workspace={ws}B" in t


def test_mfma_forms_plan():
    t = _dry(n=65536, batch=4096, precision="bf16_split3")
    assert "mfma four-step 256x256" in t and "bf16_split3" in t
    # N = 256 N2: matrix-core columns, FP32 transposed rows of N2
    t = _dry(n=1 << 18, batch=2, precision="fp16_split")
    assert "mfma four-step 256x1024 (matrix-core columns, FP32 rows)" in t
    assert "fourstep_rows_transposed: L=1024" in t, t
    dp = _dp()
    for n in (4096, 1 << 21, 3 * 256):
        d, keep = dp.make_desc(n=n, batch=2, precision="fp16")
        st, text = dp.fft_plan_dry(d)
        assert st == dp.FFT_E_UNSUPPORTED, (n, text)


def test_ragged_plan_counts():
    import synth
    sizes = synth.ragged_sizes(synth.BASE_SEED + 5, 10000)
    t = _dry(ragged_sizes=sizes.tolist(), flags=4)
    assert "10000 signals" in t and "HIP graph" in t and "3 launches" in t
    assert "one workgroup per item" in t
    m = re.search(r"(\d+) single-pass lengths, (\d+) single-pass lengths of 1024 threads, "
                  r"(\d+) four-step lengths", t)
    assert m and sum(int(v) for v in m.groups()) == len(set(sizes.tolist())), t
    assert int(m.group(2)) > 0
    t2 = _dry(ragged_sizes=sizes.tolist(), flags=8)
    assert "one launch per length" in t2


def test_ragged_override_without_the_1024_thread_class():
    import synth
    sizes = synth.ragged_sizes(synth.BASE_SEED + 5, 10000).tolist()
    code = ("import paper_1203_4938_amd as dp\n"
            f"d, k = dp.make_desc(ragged_sizes={sizes!r}, flags=2)\n"
            "print(dp.fft_plan_dry(d)[1])\n")
    out = _run(code, {"DPFFT_FORCE_PLAN": "b=0"})
    assert " 0 single-pass lengths of 1024 threads" in out and "2 launches" in out, out
    out = _run(code, {"DPFFT_FORCE_PLAN": "p0=1"})
    assert "3 persistent launches" in out and "grid=" in out, out


def _run(code, env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT,
                       env=env, timeout=120)
    assert r.returncode == 0, r.stderr
    return r.stdout


CODE = """
import paper_1203_4938_amd as dp
d, k = dp.make_desc(4096, 64, flags={flags})
print(dp.fft_plan_dry(d)[1])
"""


def test_override_env_changes_the_kernel():
    out = _run(CODE.format(flags=0), {"DPFFT_FORCE_PLAN": "c0=2"})
    assert "C=2" in out and 'override="c0=2"' in out


SPLIT_FIRST = """
import paper_1203_4938_amd as dp
d, k = dp.make_desc(shape=(1024, 1024), rank=2, batch=8)
print(dp.fft_plan_dry(d)[1])
d, k = dp.make_desc(1 << 20, 4)
print(dp.fft_plan_dry(d)[1])
"""


def test_split_first_tiles_and_the_h_override():
    """The 2D 1024-point column pass defaults to the split-first tiles (two
    sub-lines through half the LDS: 512 threads, 73600 B); h1=1 forces the
    plain tiles; h1=2 puts the 2^20 transposed rows on the split-first tiles."""
    def line(out, name):
        return next(l for l in out.splitlines() if l.strip().startswith(name))

    out = _run(SPLIT_FIRST, {})
    col = line(out, "columns:")
    assert "L=1024 C=16 threads=512 grid=" in col and "lds=73600B" in col, out
    assert "lds=73600B" not in line(out, "fourstep_rows_transposed:"), out
    out = _run(SPLIT_FIRST, {"DPFFT_FORCE_PLAN": "h1=1"})
    assert "lds=73600B" not in line(out, "columns:"), out
    out = _run(SPLIT_FIRST, {"DPFFT_FORCE_PLAN": "h1=2"})
    rows = line(out, "fourstep_rows_transposed:")
    assert "threads=512 grid=" in rows and "lds=73600B" in rows, out


def _tune_key() -> str:
    out = _run(CODE.format(flags=0), {})
    key = re.search(r"tune_key=(\S+)", out).group(1)
    # the key names the architecture and a digest of the compiled kernel registry
    assert key.startswith("gfx950|k=") and "|n=4096|b=2^6|fp32" in key
    return key


def test_tune_cache_file_is_used(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"dpfft_tune_cache": 1, "entries": {_tune_key(): "c0=2 p0=0"}}))
    out = _run(CODE.format(flags=0), {"DPFFT_TUNE_CACHE": str(path)})
    assert "C=2" in out
    # FFT_F_NO_AUTOTUNE ignores the cache
    out = _run(CODE.format(flags=2), {"DPFFT_TUNE_CACHE": str(path)})
    assert "C=1" in out and "override" not in out


def test_tune_cache_entry_of_another_build_is_ignored(tmp_path):
    """An entry keyed without the current registry digest (written by a build
    with other kernels) is not applied."""
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"dpfft_tune_cache": 1,
                                "entries": {"gfx950|r1|n=4096|b=2^6|fp32": "c0=2 p0=0"}}))
    out = _run(CODE.format(flags=0), {"DPFFT_TUNE_CACHE": str(path)})
    assert "C=1" in out and "override" not in out


def test_tune_cache_entry_naming_a_missing_kernel_falls_back(tmp_path):
    """A cached choice that no compiled instance satisfies (here 3 lines per
    tile) does not make a supported size fail: the plan is built again with
    the heuristic choices."""
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"dpfft_tune_cache": 1, "entries": {_tune_key(): "c0=3"}}))
    out = _run(CODE.format(flags=0), {"DPFFT_TUNE_CACHE": str(path)})
    assert "variant=single-pass" in out and "C=1" in out and "override" not in out


@pytest.mark.parametrize("content", ["not json at all", '{"dpfft_tune_cache": 1, "entries": {"k": ',
                                     "", '{"other": 2}'])
def test_corrupt_tune_cache_falls_back_to_heuristic(tmp_path, content):
    path = tmp_path / "tune.json"
    path.write_text(content)
    out = _run(CODE.format(flags=0), {"DPFFT_TUNE_CACHE": str(path)})
    assert "C=1" in out and "override" not in out


def test_autotune_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("checks the no-device path")
    dp = _dp()
    d, k = dp.make_desc(4096, 64)
    st, msg = dp.fft_autotune(d)
    assert st in (dp.FFT_E_DEVICE, dp.FFT_E_INTERNAL)
    d, k = dp.make_desc(65536, 8, precision="fp16")
    st, msg = dp.fft_autotune(d)
    assert st == dp.FFT_OK and "nothing to tune" in msg
    d, k = dp.make_desc(ragged_sizes=[64, 6000, 40000])
    st, msg = dp.fft_autotune(d)
    assert st == dp.FFT_E_DEVICE


def test_plans_with_signals_far_apart():
    """Signals 2 GiB apart keep the multi-line row kernels (each line has its
    own base address); only column tiles need a span below 4 GiB."""
    t = _dry(n=1024, batch=3, dist=1 << 28)
    assert "variant=single-pass" in t and "C=4" in t
    t = _dry(n=1024, batch=5000, dist=1 << 28)
    assert "variant=single-pass" in t and "C=16" in t and "persistent" in t
    t = _dry(n=1 << 16, batch=2, dist=1 << 28)
    assert "four-step" in t


@pytest.mark.parametrize("n", [2, 4, 64, 2048, 32768])
def test_real_1d_plans(n):
    dp = _dp()
    t = _dry(n=n, batch=5, flags=dp.FFT_F_REAL)
    assert "variant=real single-pass" in t and "launches=1" in t and "workspace=0B" in t
    assert f"real_forward: N={n} ({n // 2}-point complex core)" in t
    assert f"real_inverse: N={n}" in t


@pytest.mark.parametrize("n", [1 << 16, 1 << 20, 1 << 24])
def test_real_1d_four_step_plans(n):
    """Real lengths above 32768: the N/2-point core as the four-step pair of
    launches and the pairing of k with N/2 - k as a third, after the pair
    (forward) or before it (inverse); workspace batch * N/2 complex64."""
    dp = _dp()
    b = 3
    t = _dry(n=n, batch=b, flags=dp.FFT_F_REAL)
    assert "variant=real four-step" in t and "launches=3" in t, t
    assert f"workspace={b * (n // 2) * 8}B" in t, t
    fwd, inv = t.split("\n  inverse:")
    assert fwd.index("real_core_columns:") < fwd.index("real_core_rows_transposed:") < fwd.index("real_pairs:")
    assert inv.index("real_pairs_inverse:") < inv.index("real_core_columns_inverse:") \
        < inv.index("real_core_rows_transposed_inverse:")
    assert f"L={n // 2} (N={n}) batch={b}" in t


@pytest.mark.parametrize("n,core,launches", [(6, "runtime-radix single-pass", 2),
                                              (1000, "runtime-radix single-pass", 2),
                                              (30000, "runtime-radix single-pass", 2),
                                              (100000, "four-step 200x250", 3),
                                              (118098, "four-step 243x243", 3)])
def test_real_1d_mixed_plans(n, core, launches):
    """Even 7-smooth lengths that are not powers of two: the N/2-point core on
    the runtime-radix kernels (single pass, or the four-step pair), then the
    pairing launch; the inverse pairs first."""
    dp = _dp()
    t = _dry(n=n, batch=3, flags=dp.FFT_F_REAL)
    assert f"variant=real {core} + pairing" in t and f"launches={launches}" in t, t
    assert f"workspace={3 * (n // 2) * 8}B" in t, t
    fwd, inv = t.split("\n  inverse:")
    assert fwd.index("real_core") < fwd.index("real_pairs:")
    assert inv.index("real_pairs_inverse:") < inv.index("real_core")


@pytest.mark.parametrize("shape", [(100, 128), (96, 81), (1, 30), (16384, 3)])
def test_mixed_2d_plans(shape):
    """Images with 7-smooth sides that are not both powers of two: the
    runtime-radix row pass, then the column tiles in place; no workspace."""
    t = _dry(rank=2, shape=shape, batch=2)
    assert "variant=mixed 2d rows+columns" in t and "launches=2" in t and "workspace=0B" in t, t
    assert t.index("mixed_rows:") < t.index("mixed_columns:")


def test_real_2d_plan_layout():
    """Forward: real rows then in-place columns over nx/2 + 1 columns; inverse:
    columns into a workspace of batch * ny * (nx/2 + 1) complex64, then the
    complex-to-real rows."""
    dp = _dp()
    t = _dry(rank=2, shape=(2048, 2048), batch=16, flags=dp.FFT_F_REAL)
    assert "variant=real 2d rows+columns" in t and "launches=2" in t
    assert f"workspace={16 * 2048 * 1025 * 8}B" in t
    fwd, inv = t.split("\n  inverse:")
    assert fwd.index("real_rows:") < fwd.index("columns:")
    assert inv.index("columns_inverse:") < inv.index("real_rows_inverse:")
    # 1025 columns in tiles of 8: 129 tiles per image
    assert "grid=2064" in inv


@pytest.mark.parametrize("kw,status", [
    (dict(n=64, batch=2, flags=16 | 1), "FFT_E_UNSUPPORTED"),      # in place
    (dict(n=22, batch=2, flags=16), "FFT_E_UNSUPPORTED"),          # prime factor 11
    (dict(n=15, batch=2, flags=16), "FFT_E_UNSUPPORTED"),          # odd
    (dict(n=1, batch=2, flags=16), "FFT_E_UNSUPPORTED"),           # N = 1 has no pairs
    (dict(n=1 << 25, batch=2, flags=16), "FFT_E_UNSUPPORTED"),     # above 2^24
    (dict(n=64, batch=2, dist=64, flags=16), "FFT_E_INVALID"),     # dense only
    (dict(n=64, batch=2, flags=16, precision="bf16"), "FFT_E_UNSUPPORTED"),
    (dict(rank=2, shape=(22, 64), batch=1, flags=16), "FFT_E_UNSUPPORTED"),  # prime factor 11
    (dict(rank=2, shape=(64, 15), batch=1, flags=16), "FFT_E_UNSUPPORTED"),  # odd rows
    (dict(rank=2, shape=(32768, 64), batch=1, flags=16), "FFT_E_UNSUPPORTED"),
    (dict(ragged_sizes=[64, 128], flags=16), "FFT_E_UNSUPPORTED"),
])
def test_real_plans_rejected(kw, status):
    dp = _dp()
    d, keep = dp.make_desc(**kw)
    st, msg = dp.fft_plan_dry(d)
    assert dp.fft_status_str(st) == status, msg


@pytest.mark.parametrize("n,launches", [(1, 1), (64, 1), (4096, 1), (16384, 1), (1 << 15, 3),
                                        (1 << 18, 3), (1 << 22, 3), (1 << 24, 3)])
def test_conv_plans(n, launches):
    """FFT_F_CONV: one fused launch up to 16384 points, else the forward column
    pass, the fused row launch and the inverse column pass (workspace of one
    complex64 per point of the batch)."""
    dp = _dp()
    t = _dry(n=n, batch=3, flags=dp.FFT_F_CONV)
    fwd, conv = t.split("\n  convolution:")
    steps = [ln for ln in conv.splitlines() if ln.strip()]
    assert len(steps) == launches, t
    if launches == 1:
        assert "conv_single_pass: L=%d " % n in conv
    else:
        lg = n.bit_length() - 1
        n1, n2 = 1 << (lg // 2), 1 << (lg - lg // 2)
        assert "conv_fourstep_columns: L=%d " % n1 in steps[0]
        assert "conv_fourstep_rows: L=%d " % n2 in steps[1]
        assert "conv_columns_inverse: L=%d " % n1 in steps[2]
        assert "workspace=%dB" % (3 * n * 8) in t


@pytest.mark.parametrize("kw,status", [
    (dict(n=96, batch=2, flags=32), "FFT_E_UNSUPPORTED"),                # not a power of two
    (dict(n=64, batch=2, flags=32, precision="fp16"), "FFT_E_UNSUPPORTED"),
    (dict(n=64, batch=2, flags=32 | 16), "FFT_E_UNSUPPORTED"),           # real
    (dict(rank=2, shape=(64, 64), batch=1, flags=32), "FFT_E_UNSUPPORTED"),
    (dict(ragged_sizes=[64, 128], flags=32), "FFT_E_UNSUPPORTED"),
    (dict(n=1 << 25, batch=1, flags=32), "FFT_E_UNSUPPORTED"),
])
def test_conv_plans_rejected(kw, status):
    dp = _dp()
    d, keep = dp.make_desc(**kw)
    st, msg = dp.fft_plan_dry(d)
    assert dp.fft_status_str(st) == status, msg
