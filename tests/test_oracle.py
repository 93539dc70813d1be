"""The FP64 oracle against facts fixed by mathematics (CPU only)."""
import numpy as np
import pytest

import oracle
import pins


@pytest.fixture(scope="module")
def o():
    oracle.build(force=False)
    return oracle.default()


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(o, pin):
    ok, detail = pin(o) if pin is pins.pin_golden else pin(o, quick=False)
    assert ok, detail


def test_golden_file_parses():
    cases = pins.load_golden()
    assert len(cases) >= 8
    assert {c["n"] for c in cases} >= {1, 2, 3, 4, 8}


def test_batch_matches_single_signal_calls(o):
    """The batch entry point is the single-signal transform applied per signal."""
    rng = np.random.default_rng(11)
    x = (rng.standard_normal((3, 360)) + 1j * rng.standard_normal((3, 360))).astype(np.complex64)
    got = o.fft_batch(x)
    for i in range(3):
        ref = o.fft(x[i].astype(np.complex128))
        assert np.array_equal(got[i], ref)


def test_threads_reported(o):
    assert o.threads(3) == 3
    assert o.threads(0) >= 1


def test_bad_arguments_rejected(o):
    with pytest.raises(RuntimeError):
        o.fft(np.zeros(0, complex))
    with pytest.raises(RuntimeError):
        o.fft_ragged(np.zeros(4, np.complex64), [0], [0])


def test_rel_l2_metric():
    ref = np.array([[3 + 4j, 0], [1, 1]], np.complex128)
    y = ref.copy()
    y[0, 1] += 0.5
    e = oracle.rel_l2(y, ref)
    assert e[0] == pytest.approx(0.1)
    assert e[1] == 0.0


def test_rel_l2_f32_metric():
    """The C metric of the full-size parity tests: hand-computed values (3-4-5
    triangle, an all-zero reference) and agreement with the numpy metric."""
    ref = np.array([[3 + 4j, 0], [1, 1], [0, 0]], np.complex128)
    y = ref.astype(np.complex64)
    y[0, 1] += 0.5
    y[2, 0] = 2.0
    e = oracle.rel_l2_f32(y, ref)
    assert e[0] == pytest.approx(0.1, rel=1e-15)
    assert e[1] == 0.0
    assert e[2] == 2.0  # ||ref|| = 0: the absolute distance
    rng = np.random.default_rng(5)
    ref = rng.standard_normal((4, 7, 9)) + 1j * rng.standard_normal((4, 7, 9))
    y = (ref * (1 + 1e-3 * rng.standard_normal(ref.shape))).astype(np.complex64)
    np.testing.assert_allclose(oracle.rel_l2_f32(y, ref), oracle.rel_l2(y, ref), rtol=1e-12)
