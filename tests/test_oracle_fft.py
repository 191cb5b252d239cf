"""Pins of the oracle's DFT (eq. 3, both directions, unnormalised), CPU only.

``dft64`` (numpy's FFT in complex128) is checked against the defining sum
written out with exact phase reduction, and both against properties the
transform must have whatever its implementation: a shifted unit impulse maps
to a pure phase ramp, the two directions invert each other up to n, and
Parseval's relation holds.
"""

import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("n", [2, 8, 16, 64, 256, 1024])
def test_library_transform_equals_the_defining_sum(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    for sign in (-1, 1):
        a = oracle.dft64(x, sign)
        b = oracle.dft_naive(x, sign)
        assert np.max(np.abs(a - b)) < 1e-11 * np.sqrt(n) * np.max(np.abs(b))


@pytest.mark.parametrize("sign", [-1, 1])
def test_shifted_impulse_is_a_phase_ramp(sign):
    n, j0 = 64, 5
    x = np.zeros(n, complex)
    x[j0] = 1.0
    k = np.arange(n)
    ref = np.cos(2 * np.pi * j0 * k / n) + 1j * sign * np.sin(2 * np.pi * j0 * k / n)
    assert np.max(np.abs(oracle.dft_naive(x, sign) - ref)) < 1e-13
    assert np.max(np.abs(oracle.dft64(x, sign) - ref)) < 1e-13


def test_forward_sign_is_that_of_eq3():
    """A tone exp(+2 pi i f j / n) lands in bin f of the forward transform."""
    n, f = 256, 37
    x = np.exp(2j * np.pi * f * np.arange(n) / n)
    X = oracle.dft64(x, -1)
    assert abs(X[f] - n) < 1e-9 and np.max(np.abs(np.delete(X, f))) < 1e-9


def test_round_trip_and_parseval():
    rng = np.random.default_rng(9)
    n = 512
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    X = oracle.dft64(x, -1)
    assert np.max(np.abs(oracle.dft64(X, 1) / n - x)) < 1e-12
    assert abs(np.sum(np.abs(X) ** 2) - n * np.sum(np.abs(x) ** 2)) < 1e-9 * n * n


def test_planted_sign_mistake_is_caught():
    """The conjugate transform fails the eq. 3 tone pin."""
    n, f = 256, 37
    x = np.exp(2j * np.pi * f * np.arange(n) / n)
    wrong = oracle.dft64(x, +1)
    assert abs(wrong[f]) < 1e-6
