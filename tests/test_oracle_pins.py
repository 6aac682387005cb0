"""CPU tests: the oracle against the pins in tests/pins.py."""
import pytest

import oracle
import pins
import golden_io


@pytest.fixture(scope="module")
def o():
    oracle.build(force=False)
    return oracle.get()


@pytest.mark.parametrize("path", golden_io.golden_files(),
                         ids=lambda p: p.rsplit("/", 1)[-1])
def test_golden(o, path):
    pins.check_golden(o, path)


def test_isqrt(o):
    pins.check_isqrt(o)


def test_alpha0_is_box_rms(o):
    pins.check_alpha0_box(o)


def test_scatter_equals_gather(o):
    pins.check_scatter_gather(o)


def test_gate_free_closed_form(o):
    pins.check_closed_form_random(o)


def test_exhaustive_3x3(o):
    pins.check_exhaustive_3x3(o)


def test_invariants(o):
    pins.check_invariants(o)


def test_window_crop(o):
    pins.check_window_crop(o)


def test_invalid_arguments(o):
    import numpy as np
    img = np.zeros((5, 5), np.uint8)
    for args in [(-1, 1, 1), (256, 1, 1), (20, 0, 1), (20, 1, -1), (20, 1, 1025)]:
        with pytest.raises(ValueError):
            o.denoise(img, *args)


def test_splitmix64_reference_outputs(o):
    pins.check_splitmix64(o)


def test_salt_pepper_rule(o):
    pins.check_salt_pepper(o)


def test_sq_diff_sum(o):
    pins.check_sq_diff_sum(o)


def test_cycle_stop(o):
    pins.check_cycle_stop(o)
