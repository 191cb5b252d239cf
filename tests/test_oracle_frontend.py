"""Pins of the oracle's front end (real series -> normalised spectrum), CPU only.

Checked against hand-computed spectra of tiny series, the defining DFT sum,
the statistics of white noise (unit mean power after scaling), a closed-form
tone, and a planted mistake (the zeroed DC bin counted in the median).
"""

import math

import numpy as np
import pytest

import oracle


def test_impulse_by_hand():
    # x = delta_0: every bin is 1; bins 1..3 have power 1, median 1
    x = np.zeros(8)
    x[0] = 1.0
    a, med = oracle.spectrum64(x)
    assert med == 1.0
    s = math.sqrt(math.log(2.0))
    assert a[0] == 0 and np.allclose(a[1:], s, atol=1e-15)


def test_two_sample_pulse_by_hand():
    # x = [1, 1, 0, ...]: A_k = 1 + exp(-i pi k / 4), |A_k|^2 = 2 + 2 cos(pi k / 4)
    x = np.zeros(8)
    x[:2] = 1.0
    a, med = oracle.spectrum64(x)
    assert abs(med - 2.0) < 1e-14          # bins 1..3: 3.414, 2, 0.586
    k = np.arange(1, 4)
    raw = 1 + np.exp(-1j * np.pi * k / 4)
    assert np.max(np.abs(a[1:] - raw * math.sqrt(math.log(2.0) / 2.0))) < 1e-14


def test_planted_median_mistake_is_caught():
    """Counting the zeroed DC bin in the median changes the pulse's scale."""
    x = np.zeros(8)
    x[:2] = 1.0
    raw = np.fft.rfft(x)[:4]
    raw[0] = 0
    wrong = float(np.median(np.abs(raw) ** 2))        # includes DC
    assert abs(wrong - 2.0) > 0.1                      # (0.586 + 2) / 2


@pytest.mark.parametrize("n", [4, 16, 64, 256])
def test_library_rfft_equals_the_defining_sum(n):
    x = np.random.default_rng(n).standard_normal(n)
    a1, m1 = oracle.spectrum64(x)
    a2, m2 = oracle.spectrum64(x, naive=True)
    assert abs(m1 - m2) < 1e-10 * m2
    assert np.max(np.abs(a1 - a2)) < 1e-12 * np.max(np.abs(a2))


def test_white_noise_has_unit_mean_power():
    n = 1 << 18
    x = np.random.default_rng(4).standard_normal(n)
    a, med = oracle.spectrum64(x)
    # unnormalised |A_k|^2 of unit-variance noise has mean n; median n ln 2
    assert abs(med / (n * math.log(2.0)) - 1) < 0.02
    p = np.abs(a[1:]) ** 2
    assert abs(p.mean() - 1.0) < 0.02


def test_tone_closed_form_and_zero_median():
    # cos(2 pi f j / n): bin f of the transform holds n/2, every other bin 0
    n, f = 256, 37
    x = np.cos(2 * np.pi * f * np.arange(n) / n)
    raw = oracle.rfft_naive(x)
    assert abs(raw[f] - n / 2) < 1e-9
    assert np.max(np.abs(np.delete(raw, f))) < 1e-9
    # a series without noise has median 0: the spectrum is left unscaled
    a, med = oracle.spectrum64(np.zeros(n))
    assert med == 0.0 and not np.any(a)
