"""Oracle: FP64 response templates for constant frequency derivative.

Test infrastructure only (see ``oracle/__init__.py``); the product path never
imports this module.

Paper reference: Section 1 (Introduction) names the quantity this module
computes -- the predicted, normalised Fourier response H of a signal whose
frequency drifts by z bins over the observation (eq. 1 gives the meaning of
z). The paper does not print a formula for H; it defers to the correlation
technique of Ransom, Eikenberry & Middleditch (2002). The readings fixed here
(listed again in the design notes) are:

* A unit complex signal with mid-observation frequency r and drift z is
  ``exp(2 pi i (r s + z s^2 / 2))`` with ``s = u - 1/2`` and u the time over
  the observation in [0, 1].
* Its DFT-normalised response at bin ``r + q`` is, up to a phase that does not
  depend on q,

      H_z(q) = exp(-i pi q) G_z(q),
      G_z(q) = integral_{-1/2}^{1/2} exp(i pi (z s^2 - 2 q s)) ds.

* Completing the square gives, for z > 0,

      G_z(q) = exp(-i pi q^2 / z) / sqrt(2 z) * [F(t2) - F(t1)],
      t1 = sqrt(2 z) (-1/2 - q/z),  t2 = sqrt(2 z) (1/2 - q/z),

  with F(x) = C(x) + i S(x) the Fresnel integrals
  ``C(x) = int_0^x cos(pi t^2 / 2) dt`` and ``S(x) = int_0^x sin(pi t^2/2) dt``.
  For z < 0, G_z = conj(G_|z|) (G is even in q); for z = 0, G_0(q) = sinc(q).
* No renormalisation after truncating to the window: the untruncated response
  already satisfies sum_q |G_z(q)|^2 = 1 at integer q (Parseval), which the
  tests check.

``response_g`` takes the Fresnel integrals from ``scipy.special.fresnel`` (a
library primitive) and reduces the large phase ``pi q^2 / z`` exactly with
``fmod``. ``response_g_quadrature`` and ``response_g_mpmath`` evaluate the
defining integral numerically instead; they exist to pin ``response_g``.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import fresnel


def z_grid(zmax: float, dz: float) -> np.ndarray:
    """Trial drifts z_i = -zmax + i*dz, i in [0, nz), nz = 2*zmax/dz + 1.

    Both ends are included. ``2*zmax/dz`` must be an integer (to 1e-9).
    """
    if not (zmax >= 0 and dz > 0):
        raise ValueError("need zmax >= 0 and dz > 0")
    span = 2.0 * zmax / dz
    n = int(round(span))
    if abs(span - n) > 1e-9:
        raise ValueError("2*zmax/dz must be an integer")
    return -zmax + dz * np.arange(n + 1, dtype=np.float64)


def _fresnel_f(x: np.ndarray) -> np.ndarray:
    """F(x) = C(x) + i S(x), Fresnel integrals with the pi t^2 / 2 kernel."""
    s, c = fresnel(x)
    return c + 1j * s


def response_g(z: float, q) -> np.ndarray:
    """G_z(q) = int_{-1/2}^{1/2} exp(i pi (z s^2 - 2 q s)) ds, closed form.

    ``z`` is a scalar; ``q`` may be any real array (integer or fractional
    offsets in bins). Returns complex128 with the shape of ``q``.
    """
    q = np.asarray(q, dtype=np.float64)
    z = float(z)
    if z == 0.0:
        return np.sinc(q).astype(np.complex128)  # sin(pi q) / (pi q)
    az = abs(z)
    rt = math.sqrt(2.0 * az)
    t1 = rt * (-0.5 - q / az)
    t2 = rt * (0.5 - q / az)
    fdiff = _fresnel_f(t2) - _fresnel_f(t1)
    # exp(-i pi q^2 / z) with q^2 reduced modulo 2|z| exactly (fmod is exact).
    red = np.fmod(q * q, 2.0 * az)
    g = np.exp(-1j * np.pi * red / az) * fdiff / rt
    if z < 0:
        g = np.conj(g)
    return g


def template_h(z: float, q) -> np.ndarray:
    """H_z(q) = exp(-i pi q) G_z(q): the response at bin offset q = k - r."""
    q = np.asarray(q, dtype=np.float64)
    ph = np.exp(-1j * np.pi * np.fmod(q, 2.0))  # exact reduction of pi*q
    return ph * response_g(z, q)


def templates64(zmax: float, dz: float, m: int, interbin: bool = False):
    """The template bank in the time (bin-offset) domain, FP64.

    Returns ``(z, H)`` with ``z`` the nz trial drifts and ``H[i, j] =
    H_{z_i}(j - m/2)`` for j in [0, m] (m + 1 taps, offsets -m/2..m/2, the
    bounds of the eq. 2 sum).

    ``interbin``: the response is also wanted half-way between bins (the
    corrected response of Section 1 at a non-integer r). Row 2i is then
    template z_i at integer r and row 2i + 1 the same template at r + 1/2,
    over the same m + 1 bins [r - m/2, r + m/2]: offsets k - (r + 1/2) =
    q - 1/2, so H[2i + 1, j] = H_{z_i}(j - m/2 - 1/2). ``z`` then lists each
    drift twice.
    """
    if m < 2 or m % 2:
        raise ValueError("m must be even and >= 2")
    z = z_grid(zmax, dz)
    q = np.arange(-(m // 2), m // 2 + 1, dtype=np.float64)
    shifts = (0.0, 0.5) if interbin else (0.0,)
    h = np.empty((z.size * len(shifts), m + 1), dtype=np.complex128)
    for i, zi in enumerate(z):
        for p, sh in enumerate(shifts):
            h[len(shifts) * i + p] = template_h(zi, q - sh)
    return np.repeat(z, len(shifts)), h


def response_g_quadrature(z: float, q, order: int = 32) -> np.ndarray:
    """G_z(q) by composite Gauss-Legendre quadrature of its defining integral.

    Independent of the Fresnel closed form; used to pin ``response_g``. The
    panel count keeps the integrand's phase change per panel below ~8 rad, so
    a 32-point rule is exact to rounding.
    """
    q = np.atleast_1d(np.asarray(q, dtype=np.float64))
    x, w = np.polynomial.legendre.leggauss(order)
    out = np.empty(q.shape, dtype=np.complex128)
    for idx, qi in np.ndenumerate(q):
        rate = math.pi * (abs(z) + 2.0 * abs(qi)) + 1.0
        panels = int(math.ceil(rate / 8.0)) + 2
        edges = np.linspace(-0.5, 0.5, panels + 1)
        a = edges[:-1, None]
        b = edges[1:, None]
        s = 0.5 * (b - a) * x[None, :] + 0.5 * (a + b)
        ph = math.pi * (z * s * s - 2.0 * qi * s)
        out[idx] = np.sum(0.5 * (b - a) * w[None, :] * np.exp(1j * ph))
    return out


def response_g_mpmath(z: float, q: float, dps: int = 30) -> complex:
    """G_z(q) to ``dps`` digits by mpmath quadrature of the defining integral.

    Splits [-1/2, 1/2] into panels by phase so tanh-sinh converges; used only
    to write the stored golden values.
    """
    import mpmath as mp

    with mp.workdps(dps):
        zz = mp.mpf(z)
        qq = mp.mpf(q)
        f = lambda s: mp.expj(mp.pi * (zz * s * s - 2 * qq * s))  # noqa: E731
        rate = float(abs(z) + 2 * abs(q)) * math.pi + 1.0
        panels = int(math.ceil(rate / 4.0)) + 2
        pts = [mp.mpf(-0.5) + mp.mpf(k) / panels for k in range(panels + 1)]
        val = mp.quad(f, pts)
        return complex(val)
