"""Pins of the oracle's interbinned (half-bin) plane, CPU only.

The corrected response of Section 1 is defined at any r; the interbinned plane
adds r + 1/2 for every integer r (row 2i + 1 of a plane with 2 nz rows,
template z_i at offsets q - 1/2 over the same m + 1 bins as row 2i). These
tests pin it against computations that do not go through ``templates64``'s
half-bin rows: quadrature of the defining integral at half-integer offsets,
the textbook scalloping loss of a tone half-way between bins, the real-r
response ``correlate_at``, and the overlap-and-save form.
"""

import math

import numpy as np
import pytest

import oracle
from oracle import templates as T
from paper_1711_10855_amd import synth


def test_half_bin_rows_follow_the_defining_integral():
    m = 16
    z, h = oracle.templates64(6.0, 2.0, m, interbin=True)
    assert h.shape == (2 * 7, m + 1)
    assert np.array_equal(z[::2], z[1::2])
    q = np.arange(-m // 2, m // 2 + 1) - 0.5
    for i, zi in enumerate(z[::2]):
        g = T.response_g_quadrature(zi, q)
        ref = np.exp(-1j * np.pi * q) * g
        assert np.max(np.abs(h[2 * i + 1] - ref)) < 1e-12
    # one point against 30-digit quadrature
    ref = np.exp(-1j * np.pi * -1.5) * T.response_g_mpmath(4.0, -1.5)
    assert abs(h[2 * 5 + 1][m // 2 - 1] - ref) < 1e-13


def test_even_rows_are_the_integer_plane():
    a = synth.small_random_spectrum(700, seed=3)
    p2 = oracle.plane_direct(a, 6.0, 2.0, 16, interbin=True)
    p1 = oracle.plane_direct(a, 6.0, 2.0, 16)
    assert p2.shape == (2 * p1.shape[0], p1.shape[1])
    assert np.array_equal(p2[0::2], p1)


def test_half_bin_rows_equal_the_real_r_response():
    a = synth.small_random_spectrum(600, seed=4)
    m = 16
    p = oracle.plane_direct(a, 6.0, 2.0, m, interbin=True)
    z = oracle.z_grid(6.0, 2.0)
    for i in (0, 3, 6):
        for r in (0, 2, 100, 314, 598):   # round(r + 1/2) == r for even r
            b = oracle.correlate_at(a, z[i], r + 0.5, m)
            assert abs(p[2 * i + 1, r] - abs(b) ** 2) < 1e-12 * max(1.0, abs(b) ** 2)


def test_interbinned_overlap_save_matches_direct():
    a = synth.small_random_spectrum(333, seed=5)
    pd = oracle.plane_direct(a, 4.0, 2.0, 8, interbin=True)
    po = oracle.plane_ols_naive(a, 4.0, 2.0, 8, 32, interbin=True)
    assert np.max(np.abs(pd - po)) < 1e-12 * pd.max()


def test_scalloping_loss_is_recovered_half_way_between_bins():
    """A steady tone half-way between bins: the integer bins see |sinc(1/2)|^2
    = 4/pi^2 of its matched power, the half-bin response sees all of it."""
    n = 1 << 14
    r0, snr = 3000.5, 10.0
    a = synth.noise_free_chirp_spectrum(n, synth.Chirp(r0, 0.0, snr, 0.4))
    m = 64
    p = oracle.plane_direct(a, 2.0, 2.0, m, interbin=True)   # z in {-2, 0, 2}
    full = p[2 * 1 + 1, 3000]            # z = 0 row at r + 1/2 = r0
    near = max(p[2 * 1, 3000], p[2 * 1, 3001])
    q = np.arange(-m // 2, m // 2 + 1) - 0.5
    ew = float(np.sum(np.sinc(q) ** 2))  # window's share of |H_0|^2
    assert abs(full - snr ** 2 * ew * ew) < 2e-3 * snr ** 2
    assert abs(near / full - 4.0 / math.pi ** 2) < 0.01
    iz, ir = np.unravel_index(np.argmax(p), p.shape)
    assert (iz, ir) == (3, 3000)


@pytest.mark.parametrize("shift", [+0.5, -0.25])
def test_planted_half_bin_mistakes_are_caught(shift):
    """A half-bin bank built at the wrong offset fails the scalloping pin."""
    n = 1 << 14
    a = synth.noise_free_chirp_spectrum(n, synth.Chirp(3000.5, 0.0, 10.0, 0.4))
    m = 64
    q = np.arange(-m // 2, m // 2 + 1, dtype=np.float64)
    wrong = T.template_h(0.0, q + shift)[None, :]   # should be q - 1/2
    b = oracle.correlate_direct(a, wrong, m)[0, 3000]
    right = oracle.plane_direct(a, 0.0, 2.0, m, interbin=True)[1, 3000]
    assert abs(abs(b) ** 2 - right) > 0.05 * right


def test_candidates_are_the_thresholded_plane():
    """Candidates of unit-power complex Gaussian noise: P at each point is
    exponential with mean E_w (the window's share of sum |H|^2), so the
    expected count above t is N exp(-t / E_w); and a strong injected tone
    is among them at its bin."""
    n = 1 << 15
    a = synth.small_random_spectrum(n, seed=77).astype(np.complex128)
    m, t = 64, 7.0
    row, r, p = oracle.candidates_direct(a, 16.0, 2.0, m, t)
    assert np.all(p >= t) and np.all(np.diff(row * n + r) > 0)
    _, h = oracle.templates64(16.0, 2.0, m)
    ew = np.sum(np.abs(h) ** 2, axis=1)            # per row, <= 1
    expect = float(np.sum(n * np.exp(-t / ew)))
    assert 0.7 * expect < row.size < 1.3 * expect
    tone = synth.noise_free_chirp_spectrum(1 << 16, synth.Chirp(3000.0, 0.0, 8.0, 0.2))
    row2, r2, _ = oracle.candidates_direct(tone[:n], 16.0, 2.0, m, 30.0)
    assert (8, 3000) in set(zip(row2.tolist(), r2.tolist()))   # z = 0 row
