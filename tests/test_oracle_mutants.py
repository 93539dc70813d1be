"""Planted mistakes in copies of the oracle must each fail at least one pin.

Each mutant is a plausible slip (a dropped term, a wrong sign, index or
stride, a missing scale, lost precision) applied as a text edit to a copy of
oracle/oracle.c, compiled with gcc into a temporary library and run through
the quick pin suite.  The unmodified copy is the control and must pass.
"""
import os
import shutil

import pytest

import oracle
import pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

# (name, old text, new text, which occurrence (0-based))
MUTANTS = [
    ("fft_twiddle_sign", "double ang = -TWO_PI * ((double)t / (double)n);",
     "double ang = TWO_PI * ((double)t / (double)n);", 0),
    ("fft_twiddle_fp32", "tab[t].re = cos(ang);", "tab[t].re = (float)cos(ang);", 0),
    ("combine_twiddle_index", "tab[((r * k) % n) * tstride]", "tab[((r * (k % m)) % n) * tstride]", 0),
    ("combine_drops_last_term", "for (int64_t r = 0; r < p; ++r) {\n            cplx t",
     "for (int64_t r = 0; r < p - 1; ++r) {\n            cplx t", 0),
    ("combine_child_slot", "tmp[r * m + (k % m)]", "tmp[r * m + ((k / p) % m)]", 0),
    ("subsequence_offset", "fft_rec(x + r * stride, stride * p, m,", "fft_rec(x + r, stride * p, m,", 0),
    ("fallback_table_stride", "tab[((j * k) % n) * tstride]", "tab[((j * k) % n)]", 0),
    ("inverse_no_scale", "double s = 1.0 / (double)n;\n    for (int64_t k = 0; k < n; ++k) {",
     "double s = 1.0;\n    for (int64_t k = 0; k < n; ++k) {", 0),
    ("inverse_output_not_conjugated", "y[k].im = -y[k].im * s;", "y[k].im = y[k].im * s;", 0),
    ("dft_sign", "double sign = inverse ? 1.0 : -1.0;", "double sign = inverse ? -1.0 : 1.0;", 0),
    ("dft_inverse_unscaled", "sr /= (double)n;", "sr /= 1.0;", 0),
    ("batch_signal_stride", "const float *src = x + 2 * b * n;", "const float *src = x + b * n;", 0),
    ("batch_drops_imag", "xin[j].im = (double)src[2 * j + 1];", "xin[j].im = 0.0;", 0),
    ("ragged_offset_units", "const float *src = x + 2 * offsets[i];", "const float *src = x + offsets[i];", 0),
    ("ragged_drops_imag", "xin[j].im = (double)src[2 * j + 1];", "xin[j].im = 0.0;", 1),
    ("fft2d_column_gather_transposed", "col[r] = out[r * nx + c];", "col[r] = out[c * ny + r];", 0),
    ("fft2d_inverse_scale", "double s = 1.0 / ((double)nx * (double)ny);", "double s = 1.0 / (double)nx;", 0),
    ("fft2d_inverse_input_not_conjugated", "double sg = inverse ? -1.0 : 1.0;", "double sg = 1.0;", 0),
    ("conv_index_sign", "const int64_t t = ((j - m) % n + n) % n;",
     "const int64_t t = ((j + m) % n + n) % n;", 0),
    ("conv_drops_cross_term", "sr += xr * hr - xi * hi;", "sr += xr * hr;", 0),
    ("conv_imag_sign", "si += xr * hi + xi * hr;", "si += xr * hi - xi * hr;", 0),
    ("conv_filter_dist_ignored", "const float *hb = h + 2 * b * h_dist;", "const float *hb = h;", 0),
    ("conv_signal_stride", "const float *xb = x + 2 * b * n;", "const float *xb = x + b * n;", 0),
    ("img_cb_sign", "- 0.331264 * g + 0.5 * b;", "+ 0.331264 * g + 0.5 * b;", 0),
    ("img_downscale_offset", "fcb[p + w] + fcb[p + w + 1]", "fcb[p + w] + fcb[p + w - 1]", 0),
    ("img_gradient_unhalved", "const double gx = 0.5 * (", "const double gx = (", 0),
    ("img_gradient_edge", "ru = r > 0 ? r - 1 : 0", "ru = r > 0 ? r - 1 : 1", 0),
    ("img_kmeans_init_rank", "pat[(int64_t)c * P / k]", "pat[(int64_t)c * P / k / 2]", 0),
    ("img_kmeans_mean", "sum[16 * c + t] / (double)cnt[c]", "sum[16 * c + t] / (double)(cnt[c] + 1)", 0),
    ("img_encode_tie", "        if (d < d1) {", "        if (d <= d1) {", 0),
    ("img_encode_threshold", "        if (act[b] < tau) {", "        if (act[b] <= tau) {", 0),
]


def _apply(text, old, new, occ):
    pos = -1
    for _ in range(occ + 1):
        pos = text.find(old, pos + 1)
        assert pos >= 0, f"mutation site not found: {old!r}"
    return text[:pos] + new + text[pos + len(old):]


@pytest.fixture(scope="module")
def workdir(tmp_path_factory):
    d = tmp_path_factory.mktemp("mutants")
    shutil.copy(os.path.join(os.path.dirname(SRC), "oracle.h"), d / "oracle.h")
    return d


def _build(workdir, name, text):
    src = workdir / f"{name}.c"
    src.write_text(text)
    out = str(workdir / f"lib{name}.so")
    oracle.build(force=True, src=str(src), out=out)
    return oracle.OracleLib(out)


def test_control_copy_passes(workdir):
    lib = _build(workdir, "control", open(SRC).read())
    res = pins.run_all(lib, quick=True)
    failed = {k: v for k, v in res.items() if not v[0]}
    assert not failed, failed


@pytest.mark.parametrize("name,old,new,occ", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(workdir, name, old, new, occ):
    text = _apply(open(SRC).read(), old, new, occ)
    lib = _build(workdir, name, text)
    res = pins.run_all(lib, quick=True)
    caught = [k for k, v in res.items() if not v[0]]
    assert caught, f"mutant {name} passed every pin"
