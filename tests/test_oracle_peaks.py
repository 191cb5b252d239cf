"""Pins of the oracle's peak picking (the candidate search after the plane),
CPU only.

The paper names the search but does not define it; the reading (3 x 3 local
maxima in (z, r) at or above a threshold, ties to the lowest (z, r), the
interbinned plane as a half-bin grid) is pinned here by hand-built planes
whose peaks are known, by a library routine on planes without ties, by the
density of local maxima in i.i.d. noise (1/9 for a 3 x 3 window), and by
noise-free tones and a chirp whose location is known.
"""

import numpy as np
import pytest
import scipy.ndimage

import oracle
from paper_1711_10855_amd import synth


def as_set(row, r):
    return set(zip(np.asarray(row).tolist(), np.asarray(r).tolist()))


def test_hand_built_plane():
    p = np.zeros((8, 14))
    p[1, 1] = 5.0                       # isolated
    p[4, 4], p[5, 5] = 6.0, 7.0         # diagonal neighbours: only the larger
    p[1, 5], p[1, 7] = 4.0, 4.5         # two columns apart: both
    p[3, 9] = p[3, 10] = 3.0            # tie in r: the lower r
    p[4, 1] = p[5, 1] = 2.5             # tie in z: the lower z
    p[5, 9] = p[6, 8] = 2.2             # diagonal tie: the lower z
    p[0, 13] = 1.0                      # corner, exactly at the threshold
    p[7, 0], p[7, 13] = 2.0, 3.0        # other corners (no wrap-around)
    p[7, 6] = 0.99                      # below the threshold
    row, r, v = oracle.peaks_from_plane(p, 1.0)
    want = {(1, 1), (5, 5), (1, 5), (1, 7), (3, 9), (4, 1), (5, 9), (0, 13), (7, 0), (7, 13)}
    assert as_set(row, r) == want
    assert np.array_equal(v, p[row, r])
    assert np.all(np.diff(row * 14 + r) > 0)     # (iz, r) order


def test_hand_built_interbinned_plane():
    # rows 2i + h hold z_i at r + h/2: the grid interleaves them by column
    p = np.zeros((4, 4))
    p[0, 1], p[1, 1] = 5.0, 6.0         # z0 at r = 1 and r = 1.5: neighbours
    p[3, 2], p[0, 3] = 4.0, 4.5         # z1 at r = 2.5, z0 at r = 3: diagonal
    row, r, _ = oracle.peaks_from_plane(p, 1.0, interbin=True)
    assert as_set(row, r) == {(1, 1), (0, 3)}
    # read as a plain plane the same values give other peaks
    row, r, _ = oracle.peaks_from_plane(p, 1.0)
    assert as_set(row, r) == {(1, 1), (0, 3), (3, 2)}


@pytest.mark.parametrize("interbin", [False, True])
def test_a_plateau_has_one_peak(interbin):
    p = np.full((6 if interbin else 5, 9), 2.0)
    row, r, _ = oracle.peaks_from_plane(p, 1.0, interbin)
    assert as_set(row, r) == {(0, 0)}
    row, r, _ = oracle.peaks_from_plane(p, 2.5, interbin)
    assert row.size == 0


def test_equals_a_maximum_filter_without_ties():
    rng = np.random.default_rng(5)
    p = rng.exponential(size=(40, 300))
    for thr in (0.0, 2.0):
        mx = scipy.ndimage.maximum_filter(p, size=3, mode="constant", cval=-np.inf)
        want = np.nonzero((p == mx) & (p >= thr))
        row, r, _ = oracle.peaks_from_plane(p, thr)
        assert as_set(row, r) == as_set(*want)
    # interbinned: the same on the half-bin grid built here column by column
    q = rng.exponential(size=(2 * 20, 150))
    grid = np.zeros((20, 300))
    for i in range(20):
        for c in range(300):
            grid[i, c] = q[2 * i + c % 2, c // 2]
    mx = scipy.ndimage.maximum_filter(grid, size=3, mode="constant", cval=-np.inf)
    gi, gc = np.nonzero((grid == mx) & (grid >= 1.0))
    row, r, _ = oracle.peaks_from_plane(q, 1.0, interbin=True)
    assert as_set(row, r) == as_set(2 * gi + gc % 2, gc // 2)


def test_density_of_peaks_in_iid_noise_is_one_ninth():
    # an interior point of i.i.d. continuous values is the largest of its
    # 3 x 3 window with probability 1/9 (1/5 without diagonals, 1/25 at 5 x 5)
    p = np.random.default_rng(11).standard_normal((402, 402))
    row, r, _ = oracle.peaks_from_plane(p, -np.inf)
    inner = (row > 0) & (row < 401) & (r > 0) & (r < 401)
    frac = inner.sum() / 400.0 ** 2
    assert abs(frac - 1.0 / 9.0) < 0.004


@pytest.mark.parametrize("r0,row_want", [(3000.5, 2 * 2 + 1), (3000.0, 2 * 2)])
def test_tone_peaks_on_its_half_bin(r0, row_want):
    # noise-free tone (z0 = 0): on the half-bin grid its one peak above half
    # the maximum is at the row of z = 0 and the half bin of r0
    a = synth.noise_free_chirp_spectrum(1 << 14, synth.Chirp(r0, 0.0, 10.0, 0.3))
    row, r, v = oracle.peaks_direct(a, 4.0, 2.0, 32, 0.0, interbin=True)
    top = v >= 0.5 * v.max()
    assert as_set(row[top], r[top]) == {(row_want, 3000)}


def test_chirp_peaks_at_its_drift_and_frequency():
    c = synth.Chirp(5000.3, 6.6, 20.0, 0.0)
    a = synth.noise_free_chirp_spectrum(1 << 16, c)[:8192]
    row, r, v = oracle.peaks_direct(a, 16.0, 2.0, 64, 0.0)
    k = int(np.argmax(v))
    assert (row[k], r[k]) == ((6 + 16) // 2, 5000)   # z = 6 is the nearest trial drift
    # the strongest point of the plane is a peak and carries the matched power
    p = oracle.plane_direct(a, 16.0, 2.0, 64)
    assert v[k] == p.max()


# ---- planted mistakes ------------------------------------------------------
# Copies of the peak rule with one plausible mistake each; the hand-built
# plane, the plateau and the noise density reject every one of them.

def _mutant_mask(g, thr, reach=1, diagonals=True, tie="first", wrap=False, inclusive=True):
    nz, nc = g.shape
    mask = (g >= thr) if inclusive else (g > thr)
    for dz in range(-reach, reach + 1):
        for dc in range(-reach, reach + 1):
            if (dz, dc) == (0, 0) or (not diagonals and dz and dc):
                continue
            if wrap:
                w = np.roll(np.roll(g, -dz, axis=0), -dc, axis=1)
            else:
                pad = np.full((nz + 2 * reach, nc + 2 * reach), -np.inf)
                pad[reach:-reach, reach:-reach] = g
                w = pad[reach + dz:reach + dz + nz, reach + dc:reach + dc + nc]
            before = dz < 0 or (dz == 0 and dc < 0)
            wins = {"first": before, "last": not before, "none": False, "all": True}[tie]
            mask &= ~((w > g) | ((w == g) & wins))
    return mask


def _pins_hold(mask_fn):
    p = np.zeros((8, 14))
    p[1, 1] = 5.0
    p[4, 4], p[5, 5] = 6.0, 7.0
    p[1, 5], p[1, 7] = 4.0, 4.5
    p[3, 9] = p[3, 10] = 3.0
    p[4, 1] = p[5, 1] = 2.5
    p[5, 9] = p[6, 8] = 2.2
    p[0, 13] = 1.0
    p[7, 0], p[7, 13] = 2.0, 3.0
    want = {(1, 1), (5, 5), (1, 5), (1, 7), (3, 9), (4, 1), (5, 9), (0, 13), (7, 0), (7, 13)}
    if as_set(*np.nonzero(mask_fn(p, 1.0))) != want:
        return False
    if as_set(*np.nonzero(mask_fn(np.full((5, 9), 2.0), 1.0))) != {(0, 0)}:
        return False
    noise = np.random.default_rng(11).standard_normal((402, 402))
    inner = mask_fn(noise, -np.inf)[1:-1, 1:-1]
    return abs(inner.mean() - 1.0 / 9.0) < 0.004


def test_pins_accept_the_oracle_rule():
    assert _pins_hold(oracle.peak_mask)
    assert _pins_hold(_mutant_mask)   # the unmutated copy


@pytest.mark.parametrize("mistake", [dict(diagonals=False), dict(reach=2), dict(tie="last"),
                                     dict(tie="none"), dict(tie="all"), dict(wrap=True),
                                     dict(inclusive=False)])
def test_planted_peak_mistakes_are_caught(mistake):
    assert not _pins_hold(lambda g, thr: _mutant_mask(g, thr, **mistake))
