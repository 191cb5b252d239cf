"""Pins for the oracle's response templates (CPU only).

Each check compares the oracle with something other than itself: numerical
quadrature of the defining integral, stored high-precision values, Parseval's
identity, the z = 0 special case, and the discrete dechirp template. The
``mutant`` tests plant plausible mistakes in copies of the oracle's formula and
show that the same checks reject them.
"""

import math
import os

import numpy as np
import pytest

from oracle import templates as T

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "templates_mpmath.txt")


def quad_error(g_func, zs=(2.0, 7.0, 16.0, 100.0, -7.0, -100.0, 0.5)):
    q = np.concatenate([np.arange(-260.0, 261.0, 13.0), [0.3, -0.3, 12.5, -99.7, 0.0]])
    err = 0.0
    for z in zs:
        err = max(err, float(np.max(np.abs(g_func(z, q) - T.response_g_quadrature(z, q)))))
    return err


def parseval_defect(g_func, z):
    q = np.arange(-20000, 20001, dtype=np.float64)
    return abs(1.0 - float(np.sum(np.abs(g_func(z, q)) ** 2)))


def test_closed_form_matches_quadrature():
    assert quad_error(T.response_g) < 1e-13


def test_closed_form_matches_golden_mpmath():
    rows = np.loadtxt(GOLDEN)
    for z, q, re, im in rows:
        g = complex(T.response_g(z, np.array([q]))[0])
        assert abs(g - complex(re, im)) < 5e-15, (z, q)


@pytest.mark.parametrize("z", [2.0, 16.0, 100.0, 200.0])
def test_parseval_integer_offsets(z):
    # G_z(q) are the Fourier-series coefficients of exp(i pi z s^2) on a unit
    # interval, so their squared moduli sum to 1 at integer q.
    assert parseval_defect(T.response_g, z) < 1e-9


def test_symmetries():
    q = np.arange(-200.0, 201.0) + 0.25
    for z in (3.0, 16.0, 90.0):
        g = T.response_g(z, q)
        assert np.max(np.abs(g - T.response_g(z, -q))) < 1e-14      # even in q
        assert np.max(np.abs(T.response_g(-z, q) - np.conj(g))) < 1e-15


def test_z0_is_kronecker_delta_and_sinc():
    q = np.arange(-50.0, 51.0)
    h = T.template_h(0.0, q)
    ref = (q == 0).astype(np.complex128)
    assert np.max(np.abs(h - ref)) < 1e-15
    qf = q + 0.5
    g = T.response_g(0.0, qf)
    assert np.max(np.abs(g - np.sin(np.pi * qf) / (np.pi * qf))) < 1e-15


def test_small_z_tends_to_z0():
    q = np.arange(-20.0, 21.0)
    d = np.max(np.abs(T.response_g(1e-7, q) - T.response_g(0.0, q)))
    assert d < 1e-6


@pytest.mark.parametrize("n", [256, 1024, 4096])
def test_continuous_template_vs_discrete_dechirp(n):
    # H_z(q) = int_0^1 exp(i pi z (u - 1/2)^2) exp(-2 pi i q u) du; the N-point
    # rectangle rule of that integral is DFT_N(exp(i pi z s_n^2))[q] / N.
    # The two differ by O((z/N)^2) -- this fixes the sign of z, the direction
    # of q and the centring against an independent computation.
    z = 7.0
    s = np.arange(n) / n - 0.5
    c = np.fft.fft(np.exp(1j * np.pi * z * s * s)) / n
    q = np.arange(-n // 2, n // 2)
    h = T.template_h(z, q.astype(np.float64))
    assert np.max(np.abs(h - c[q % n])) < (z / n) ** 2


def test_templates64_layout():
    z, h = T.templates64(16.0, 2.0, 64)
    assert z.shape == (17,) and h.shape == (17, 65)
    assert z[0] == -16.0 and z[-1] == 16.0
    q = np.arange(-32.0, 33.0)
    assert np.array_equal(h[3], T.template_h(z[3], q))


def test_z_grid_validation():
    assert T.z_grid(100, 2).size == 101
    assert T.z_grid(0, 2).size == 1
    assert np.array_equal(T.z_grid(3, 2), [-3.0, -1.0, 1.0, 3.0])
    with pytest.raises(ValueError):
        T.z_grid(3, 4)
    with pytest.raises(ValueError):
        T.z_grid(-1, 2)


# ---- planted mistakes: the same checks must reject them -------------------

def _mutant_no_sqrt(z, q):
    q = np.asarray(q, dtype=np.float64)
    if z == 0:
        return np.sinc(q).astype(np.complex128)
    az = abs(z)
    rt = math.sqrt(2 * az)
    t1, t2 = rt * (-0.5 - q / az), rt * (0.5 - q / az)
    f = T._fresnel_f(t2) - T._fresnel_f(t1)
    g = np.exp(-1j * np.pi * np.fmod(q * q, 2 * az) / az) * f   # dropped 1/sqrt(2z)
    return np.conj(g) if z < 0 else g


def _mutant_wrong_phase_sign(z, q):
    g = T.response_g(z, q)
    q = np.asarray(q, dtype=np.float64)
    az = abs(z) if z else 1.0
    ph = np.exp(-2j * np.pi * np.fmod(q * q, 2 * az) / az)  # flips the sign of pi q^2/z
    return g * ph if z else g


def _mutant_z_sign(z, q):
    return T.response_g(-z, q)


def _mutant_fresnel_scale(z, q):
    q = np.asarray(q, dtype=np.float64)
    if z == 0:
        return np.sinc(q).astype(np.complex128)
    az = abs(z)
    rt = math.sqrt(2 * az)
    rz = math.sqrt(az)                                       # sqrt(z) for sqrt(2z)
    t1, t2 = rz * (-0.5 - q / az), rz * (0.5 - q / az)
    f = T._fresnel_f(t2) - T._fresnel_f(t1)
    g = np.exp(-1j * np.pi * np.fmod(q * q, 2 * az) / az) * f / rt
    return np.conj(g) if z < 0 else g


@pytest.mark.parametrize("mutant", [_mutant_no_sqrt, _mutant_wrong_phase_sign,
                                    _mutant_z_sign, _mutant_fresnel_scale])
def test_planted_template_mistakes_are_caught(mutant):
    caught = quad_error(mutant) > 1e-6 or parseval_defect(mutant, 16.0) > 1e-6
    assert caught
