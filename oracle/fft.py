"""Discrete Fourier transform of eq. 3 (test infrastructure only).

The oracle of the standalone batched FFT: the transform that Section 2 uses
for every overlap-and-save segment (eq. 3 sign convention for the forward
direction), with no normalisation in either direction:

    X[k] = sum_j x[j] exp(sign * 2 pi i j k / n),  sign = -1 forward, +1 inverse.

``dft_naive`` is that sum written out as a matrix product with exact integer
phase reduction (small n); ``dft64`` evaluates it with numpy's FFT in
complex128 (a library primitive standing for the same sum).
"""

import numpy as np

from .correlate import _dft_matrix


def dft_naive(x: np.ndarray, sign: int) -> np.ndarray:
    """Rows of x transformed by the defining sum (O(n^2); n up to ~1024)."""
    if sign not in (-1, 1):
        raise ValueError("sign must be -1 or +1")
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[-1]
    return x @ _dft_matrix(n, sign)


def dft64(x: np.ndarray, sign: int) -> np.ndarray:
    """Rows of x transformed in complex128 through numpy's FFT."""
    if sign not in (-1, 1):
        raise ValueError("sign must be -1 or +1")
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[-1]
    return np.fft.fft(x, axis=-1) if sign < 0 else np.fft.ifft(x, axis=-1) * n
