"""Front end of the search: real time series -> normalised complex spectrum
(test infrastructure only).

The correlation of eq. 2 runs on the Fourier spectrum of the observation
(Section 1). Before it the series is Fourier transformed with a real FFT,
the Nyquist bin is dropped, the zero-frequency bin is set to zero, and the
spectrum is scaled so that the noise has unit mean power: for white noise
|A_k|^2 is exponentially distributed, its median is ln 2 times its mean, so
the scale is sqrt(ln 2 / median |A_k|^2) over bins 1 .. n/2 - 1. A zero
median (a series with no noise) leaves the spectrum unscaled. The paper
names this step only as part of the FDAS pipeline; the normalisation used
here is the reading the synthetic workloads are built with.
"""

import math

import numpy as np

from .correlate import _dft_matrix


def rfft_naive(x: np.ndarray) -> np.ndarray:
    """Bins 0 .. n/2 - 1 of the forward DFT (eq. 3 sign) of a real series,
    by the defining sum (small n)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    return (x @ _dft_matrix(n, -1))[: n // 2]


def spectrum64(x: np.ndarray, naive: bool = False):
    """(A, median): the normalised spectrum A (complex128, n // 2 bins, A_0 = 0)
    of a real series of even length n, and the median of |A_k|^2 over bins
    1 .. n/2 - 1 before scaling."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    if n < 4 or n % 2:
        raise ValueError("need an even length >= 4")
    a = rfft_naive(x) if naive else np.fft.rfft(x)[: n // 2]
    a = a.astype(np.complex128, copy=True)
    a[0] = 0.0
    p = a[1:].real ** 2 + a[1:].imag ** 2
    med = float(np.median(p))
    if med > 0.0:
        a *= math.sqrt(math.log(2.0) / med)
    return a, med
