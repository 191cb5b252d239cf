"""Oracle: peak picking over the thresholded z-r plane.

Test infrastructure only (see ``oracle/__init__.py``); the product path never
imports this module.

Section 3 of the paper names the candidate search that follows the plane in
the FDAS pipeline but does not define it. The reading used here, and by the
library's detection epilogue:

* The plane is a grid over (z, r). Without interbinning it is the plane
  itself, grid[iz][c] = P[iz][c]. With interbinning (2 nz rows, row 2i + h
  holding z_i at r + h/2) the grid has nz rows and 2 nbins half-bin columns,
  grid[i][2r + h] = P[2i + h][r], so that neighbouring columns are half a
  bin apart at the same z.
* A candidate is a grid point with value >= threshold (inclusive).
* Points are totally ordered by (value, then lower iz first, then lower
  column first): p outranks q when P_p > P_q, or P_p == P_q and
  (iz_p, c_p) < (iz_q, c_q) lexicographically.
* A peak is a candidate that outranks every other grid point of its 3 x 3
  neighbourhood (one row and one column either side, diagonals included);
  neighbours outside the grid do not exist. Among equal values the point
  with the lowest (iz, c) wins, so a plateau yields exactly one peak.

A neighbour below the threshold is below every candidate, so the peaks of
the plane are exactly the peaks among its candidates; the library uses this
to pick peaks from the candidate list without the plane.

Everything is float64 on the plane it is given.
"""

from __future__ import annotations

import numpy as np

from .correlate import plane_direct


def _grid(p: np.ndarray, interbin: bool) -> np.ndarray:
    """The (z, r) grid of a plane: the plane itself, or with interbinning the
    rows 2i and 2i + 1 interleaved column by column into row i."""
    p = np.asarray(p, dtype=np.float64)
    if not interbin:
        return p
    if p.shape[0] % 2:
        raise ValueError("an interbinned plane has an even number of rows")
    nz, n = p.shape[0] // 2, p.shape[1]
    g = np.empty((nz, 2 * n), dtype=np.float64)
    g[:, 0::2] = p[0::2]
    g[:, 1::2] = p[1::2]
    return g


def peak_mask(g: np.ndarray, threshold: float) -> np.ndarray:
    """Boolean mask of the peaks of a grid (definition in the module doc).

    Each of the 8 neighbour offsets (dz, dc) is compared in turn: the point
    is outranked by that neighbour if the neighbour's value is larger, or
    equal and the neighbour comes first in (iz, c) order, which for an
    offset means dz < 0, or dz == 0 and dc < 0."""
    g = np.asarray(g, dtype=np.float64)
    nz, nc = g.shape
    pad = np.full((nz + 2, nc + 2), -np.inf)
    pad[1:-1, 1:-1] = g
    mask = g >= threshold
    for dz in (-1, 0, 1):
        for dc in (-1, 0, 1):
            if dz == 0 and dc == 0:
                continue
            w = pad[1 + dz:1 + dz + nz, 1 + dc:1 + dc + nc]
            first = dz < 0 or (dz == 0 and dc < 0)
            beaten = (w > g) | ((w == g) if first else np.zeros_like(mask))
            mask &= ~beaten
    return mask


def peaks_from_plane(p: np.ndarray, threshold: float, interbin: bool = False):
    """Peaks of a power plane as (row, r, P) arrays, in (iz, c) order; row
    and r index the plane as stored (row 2i + h with interbinning)."""
    g = _grid(p, interbin)
    iz, c = np.nonzero(peak_mask(g, threshold))
    vals = g[iz, c]
    if interbin:
        return 2 * iz + (c & 1), c >> 1, vals
    return iz, c, vals


def peaks_direct(a: np.ndarray, zmax: float, dz: float, m: int, threshold: float,
                 interbin: bool = False):
    """Peaks of the direct eq. 2 plane of spectrum ``a``."""
    return peaks_from_plane(plane_direct(a, zmax, dz, m, interbin), threshold, interbin)
