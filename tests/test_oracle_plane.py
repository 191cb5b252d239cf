"""Pins for the oracle's correlation (eq. 2) and overlap-and-save (CPU only).

Checks: explicit loops on tiny inputs, direct sum vs naive-DFT overlap-save
(two independent computations), the z = 0 identity, the conjugate / -z
symmetry, the dechirp identity (fixes conj and the index direction against a
time-domain computation), point sampling, and recovery of an injected chirp at
its known (r0, z0) with the closed-form peak power. The ``mutant`` tests plant
mistakes in copies of the oracle's sum and show the checks reject them.
"""

import math

import numpy as np
import pytest

import oracle
from oracle import correlate as C
from oracle import templates as T
from paper_1711_10855_amd import synth


def rand_spec(n, seed):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / math.sqrt(2)


def test_bruteforce_equals_vectorised():
    a = rand_spec(32, 1)
    _, h = T.templates64(2.0, 2.0, 8)  # nz = 3
    b = np.array(C.correlate_bruteforce(list(a), [list(r) for r in h], 8))
    assert np.max(np.abs(b - C.correlate_direct(a, h, 8))) < 1e-13


@pytest.mark.parametrize("n,m,L", [(1000, 16, 32), (1000, 16, 48), (777, 16, 64),
                                   (300, 8, 100), (513, 32, 128), (20, 16, 32),
                                   (5, 8, 16)])
def test_direct_equals_naive_ols(n, m, L):
    a = rand_spec(n, n + L)
    zmax = 6.0
    p1 = oracle.plane_direct(a, zmax, 2.0, m)
    p2 = oracle.plane_ols_naive(a, zmax, 2.0, m, L)
    assert np.max(np.abs(p1 - p2)) <= 1e-12 * np.max(p1)


def test_z0_row_is_power_spectrum():
    a = rand_spec(4096, 7)
    p = oracle.plane_direct(a, 8.0, 2.0, 32)
    assert np.max(np.abs(p[4] - np.abs(a) ** 2)) < 1e-13


def test_conjugate_minus_z_symmetry():
    a = rand_spec(2048, 9)
    p = oracle.plane_direct(a, 10.0, 2.0, 32)
    pc = oracle.plane_direct(np.conj(a), 10.0, 2.0, 32)
    assert np.max(np.abs(p - pc[::-1])) <= 1e-13 * np.max(p)


def dechirp_error(correlate, n=64, z=5.0, seed=3):
    """eq. 2 with the discrete template and full circular width must equal the
    time-domain dechirped DFT  sum_n x_n exp(-i pi z s_n^2) exp(-2 pi i r n/N)."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    a = np.fft.fft(x)
    s = np.arange(n) / n - 0.5
    c = np.fft.fft(np.exp(1j * np.pi * z * s * s)) / n
    taps = np.array([c[q % n] for q in range(-n // 2, n // 2 + 1)])
    taps[0] *= 0.5   # q = -N/2 and q = +N/2 alias; split the tap between them
    taps[-1] *= 0.5
    b = correlate(np.concatenate([a, a, a]), taps[None, :], n)[0][n:2 * n]
    nn = np.arange(n)
    ref = np.array([np.sum(x * np.exp(-1j * np.pi * z * s * s - 2j * np.pi * r * nn / n))
                    for r in range(n)])
    return float(np.max(np.abs(b - ref)) / np.max(np.abs(ref)))


def test_dechirp_identity():
    assert dechirp_error(C.correlate_direct) < 1e-12


def test_index_direction_does_not_change_power():
    # eq. 2 writes H*_{r0-k}; the oracle defines H on q = k - r. G_z is even in
    # q and exp(-i pi q) vs exp(+i pi q) differ by a phase that is constant for
    # a given output bin, so both readings give the same power, at integer and
    # at fractional r.
    a = rand_spec(512, 4)
    _, h = T.templates64(14.0, 2.0, 32)
    b1 = C.correlate_direct(a, h, 32)
    b2 = C.correlate_direct(a, h[:, ::-1], 32)
    assert np.max(np.abs(np.abs(b1) - np.abs(b2))) < 1e-12
    for r in (100.3, 250.75):
        k = np.arange(int(round(r)) - 16, int(round(r)) + 17)
        v1 = np.sum(a[k] * np.conj(T.template_h(9.0, k - r)))
        v2 = np.sum(a[k] * np.conj(T.template_h(9.0, r - k)))
        assert abs(abs(v1) - abs(v2)) < 1e-12


def test_plane_points_match_plane():
    a = rand_spec(3000, 11)
    p = oracle.plane_direct(a, 12.0, 2.0, 64)
    rng = np.random.default_rng(0)
    iz = rng.integers(0, p.shape[0], 500)
    r = np.concatenate([rng.integers(0, 3000, 490), [0, 1, 2, 31, 32, 2999, 2998, 2968, 2967, 1500]])
    v = oracle.plane_points(a, 12.0, 2.0, 64, iz, r)
    assert np.max(np.abs(v - p[iz, r])) <= 1e-13 * np.max(p)


def test_bank_natural_reproduces_segment_correlation():
    # The Fourier-domain bank times a segment spectrum, inverse-transformed
    # without 1/L, equals the segment's circular correlation with H.
    m, L = 16, 64
    _, h = T.templates64(4.0, 2.0, m)
    bank = C.bank_natural(h, m, L)
    x = rand_spec(L, 5)
    y = np.fft.ifft(np.fft.fft(x)[None, :] * bank, axis=1) * L
    for i in range(h.shape[0]):
        for j in range(m // 2, L - m // 2):
            ref = sum(x[j + q] * np.conj(h[i, q + m // 2]) for q in range(-m // 2, m // 2 + 1))
            assert abs(y[i, j] - ref) < 1e-12


def test_injection_recovery_noise_free():
    n = 1 << 16
    chirp = synth.Chirp(5000.3, 7.0, 20.0, 1.1)
    a = synth.noise_free_chirp_spectrum(n, chirp)
    m = 64
    from scipy.optimize import minimize

    def negp(v):
        return -abs(oracle.correlate_at(a, v[1], v[0], m)) ** 2

    res = minimize(negp, x0=[5000.0, 6.0], method="Nelder-Mead",
                   options={"xatol": 1e-6, "fatol": 1e-9, "maxiter": 4000})
    r_hat, z_hat = res.x
    assert abs(r_hat - 5000.3) < 0.005 and abs(z_hat - 7.0) < 0.01
    # closed form: P = SNR^2 * E_w^2 with E_w the window's share of |H|^2
    q = np.arange(5000 - 32, 5000 + 33) - 5000.3
    ew = float(np.sum(np.abs(T.template_h(7.0, q)) ** 2))
    p_hat = abs(oracle.correlate_at(a, 7.0, 5000.3, m)) ** 2
    assert abs(p_hat - 400.0 * ew * ew) < 2e-3 * 400.0
    # on the grid (dz = 2) the peak sits on rows z = 6 and z = 8 at bin 5000
    p = oracle.plane_direct(a, 16.0, 2.0, m)
    iz, ir = np.unravel_index(np.argmax(p), p.shape)
    assert ir == 5000 and iz in (11, 12)
    assert abs(p[11, 5000] - p[12, 5000]) < 0.02 * p[11, 5000]


def test_workload1_detects_injection():
    a, chirps = synth.single_series("fp32-small")
    p = oracle.plane_direct(a, 16.0, 2.0, 64)
    iz, ir = np.unravel_index(np.argmax(p), p.shape)
    assert abs(ir - 5000.3) <= 1 and iz in (11, 12)
    assert p.max() > 150.0


def test_noise_normalisation_unit_mean():
    a, _ = synth.single_series("fp32-small")
    pw = np.abs(a.astype(np.complex128)) ** 2
    assert abs(np.mean(pw[100:]) - 1.0) < 0.03


# ---- planted mistakes ----------------------------------------------------

def _mut_no_conj(a, h, m):
    return C.correlate_direct(a, np.conj(h), m)


def _mut_off_by_one(a, h, m):
    b = C.correlate_direct(a, h, m)
    return np.roll(b, 1, axis=1)


@pytest.mark.parametrize("mutant", [_mut_no_conj, _mut_off_by_one])
def test_planted_correlation_mistakes_are_caught(mutant):
    assert dechirp_error(mutant) > 1e-3


def test_planted_ols_mistake_is_caught(monkeypatch):
    a = rand_spec(700, 2)
    p1 = oracle.plane_direct(a, 6.0, 2.0, 16)
    orig = C._dft_matrix
    # inverse transform built with the forward sign (flipping both signs is
    # not a mistake: the correlation theorem holds in either convention)
    monkeypatch.setattr(C, "_dft_matrix", lambda n, sign: orig(n, -1))
    p2 = C.plane_ols_naive(a, 6.0, 2.0, 16, 48)
    assert np.max(np.abs(p1 - p2)) > 1e-3 * np.max(p1)
