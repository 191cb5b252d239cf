"""FP64 CPU oracle for the FDAS correlation step (test infrastructure only).

This package is the checker, not the product. Only ``tests/``, the smoke
check in ``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py``
may import it. It shares no code with the HIP path: nothing here imports the
package ``paper_1711_10855_amd`` and nothing there imports this package.

What it computes (paper: Adamek, Dimoudi, Giles & Armour, "Improved
Acceleration of the GPU Fourier Domain Acceleration Search Algorithm"):

* ``templates``  -- the predicted, normalised Fourier response H of a signal
  with constant frequency derivative (Section 1, the response named before
  eq. 2), in the closed form derived from its defining integral.
* ``correlate``  -- the matched-filter sum of eq. 2 (Section 1) evaluated
  directly, and, independently, the same result by overlap-and-save
  (Section 2) with naive DFT matrices built from eq. 3.
* ``fft``        -- the unnormalised DFT of eq. 3 in both directions, for the
  standalone batched FFT.
* ``frontend``   -- real series -> spectrum: real DFT, Nyquist dropped, DC
  zeroed, median normalisation to unit mean noise power.
* ``peaks``      -- the candidate search after the plane (Section 3 names
  it): points at or above a threshold that are local maxima of their 3 x 3
  (z, r) neighbourhood, ties going to the lowest (z, r).
"""

from .templates import (  # noqa: F401
    z_grid,
    response_g,
    template_h,
    templates64,
    response_g_quadrature,
    response_g_mpmath,
)
from .correlate import (  # noqa: F401
    correlate_direct,
    plane_direct,
    plane_points,
    plane_ols_naive,
    correlate_bruteforce,
    correlate_at,
    bank_natural,
    candidates_direct,
)
from .fft import dft_naive, dft64  # noqa: F401
from .frontend import rfft_naive, spectrum64  # noqa: F401
from .peaks import peak_mask, peaks_from_plane, peaks_direct  # noqa: F401
