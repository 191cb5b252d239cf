"""Oracle: the matched-filter correlation of eq. 2 and its overlap-and-save form.

Test infrastructure only (see ``oracle/__init__.py``); the product path never
imports this module.

Paper reference:

* eq. 2 (Section 1): the corrected response at bin r is the sum over the
  m + 1 bins k in [r - m/2, r + m/2] of A_k times the conjugated template.
  The printed lower bound is garbled; the reading here is r - m/2 with both
  bounds inclusive. Writing the offset as q = k - r, with H defined on q:

      B_z(r) = sum_{q=-m/2}^{m/2} A_{r+q} conj(H_z(q)),   P_z(r) = |B_z(r)|^2,

  with A_k = 0 outside [0, nbins) (zero padding at the edges).
* Section 2: overlap-and-save splits the input into segments, convolves each
  in the Fourier domain and keeps only the part that equals the linear
  result. ``plane_ols_naive`` follows that description with DFT matrices
  written from eq. 3 (forward kernel exp(-i 2 pi n m / N)), so it shares no
  arithmetic with ``correlate_direct`` beyond the template values.

Everything is complex128 / float64.
"""

from __future__ import annotations

import numpy as np

from .templates import templates64, template_h


def _check_m(m: int) -> int:
    if m < 2 or m % 2:
        raise ValueError("m must be even and >= 2")
    return m // 2


def correlate_direct(a: np.ndarray, h: np.ndarray, m: int) -> np.ndarray:
    """B[i, r] = sum_{q=-m/2}^{m/2} A[r+q] conj(h[i, q+m/2])  (eq. 2).

    ``a``: complex spectrum, length nbins. ``h``: templates, shape (nz, m+1),
    column j holding offset q = j - m/2. Returns complex128 (nz, nbins).
    """
    half = _check_m(m)
    a = np.asarray(a, dtype=np.complex128)
    h = np.atleast_2d(np.asarray(h, dtype=np.complex128))
    if h.shape[1] != m + 1:
        raise ValueError("h must have m + 1 columns")
    n = a.size
    apad = np.zeros(n + m, dtype=np.complex128)
    apad[half:half + n] = a
    hc = np.conj(h)
    out = np.zeros((h.shape[0], n), dtype=np.complex128)
    for i in range(h.shape[0]):
        acc = out[i]
        for j in range(m + 1):  # q = j - half; A[r + q] = apad[r + j]
            acc += apad[j:j + n] * hc[i, j]
    return out


def plane_direct(a: np.ndarray, zmax: float, dz: float, m: int,
                 interbin: bool = False) -> np.ndarray:
    """The z-r power plane P[i, r] = |B_{z_i}(r)|^2 by the direct eq. 2 sum.

    ``interbin``: 2 nz rows, row 2i + 1 holding the power at r + 1/2 (see
    ``templates64``)."""
    _, h = templates64(zmax, dz, m, interbin)
    b = correlate_direct(a, h, m)
    return (b.real ** 2 + b.imag ** 2)


def plane_points(a: np.ndarray, zmax: float, dz: float, m: int,
                 iz: np.ndarray, r: np.ndarray, chunk: int = 4096,
                 interbin: bool = False) -> np.ndarray:
    """P at selected plane points (iz[k], r[k]) by the direct eq. 2 sum.

    Used for spot checks at sizes where the full plane is too large.
    """
    half = _check_m(m)
    _, h = templates64(zmax, dz, m, interbin)
    hc = np.conj(h)
    a = np.asarray(a, dtype=np.complex128)
    n = a.size
    apad = np.zeros(n + m, dtype=np.complex128)
    apad[half:half + n] = a
    iz = np.asarray(iz, dtype=np.int64).ravel()
    r = np.asarray(r, dtype=np.int64).ravel()
    if iz.shape != r.shape:
        raise ValueError("iz and r must have equal length")
    out = np.empty(iz.size, dtype=np.float64)
    taps = np.arange(m + 1)
    for s in range(0, iz.size, chunk):
        rr = r[s:s + chunk]
        win = apad[rr[:, None] + taps[None, :]]  # A[r + q], q = j - half
        b = np.sum(win * hc[iz[s:s + chunk]], axis=1)
        out[s:s + chunk] = b.real ** 2 + b.imag ** 2
    return out


def _dft_matrix(n: int, sign: int) -> np.ndarray:
    """D[j, k] = exp(sign * i 2 pi ((j k) mod n) / n), exact integer reduction."""
    jk = np.outer(np.arange(n), np.arange(n)) % n
    return np.exp(sign * 2j * np.pi * jk / n)


def plane_ols_naive(a: np.ndarray, zmax: float, dz: float, m: int,
                    seg_len: int, interbin: bool = False) -> np.ndarray:
    """The same plane by overlap-and-save with naive O(L^2) DFTs (Section 2).

    Segment s reads x_j = A[s U - m/2 + j], j in [0, L), U = L - m, zero
    outside [0, nbins). Each template is wrapped circularly,
    h[q mod L] = H(q), and the segment's circular correlation with it is
    y = conj(D) (X * conj(D h)) / L with X = D x (D the forward DFT of
    eq. 3). Outputs y[m/2 + t], t in [0, U), are the linear result at
    r = s U + t. Small sizes only.
    """
    half = _check_m(m)
    L = int(seg_len)
    if L <= m:
        raise ValueError("seg_len must exceed m")
    _, h = templates64(zmax, dz, m, interbin)
    a = np.asarray(a, dtype=np.complex128)
    n = a.size
    U = L - m
    nseg = -(-n // U)
    dft = _dft_matrix(L, -1)
    idft = _dft_matrix(L, +1)
    hw = np.zeros((h.shape[0], L), dtype=np.complex128)
    for j in range(m + 1):
        hw[:, (j - half) % L] += h[:, j]
    hf = hw @ dft.T  # row i: D h_i
    out = np.zeros((h.shape[0], n), dtype=np.float64)
    for s in range(nseg):
        start = s * U - half
        x = np.zeros(L, dtype=np.complex128)
        lo = max(start, 0)
        hi = min(start + L, n)
        if hi > lo:
            x[lo - start:hi - start] = a[lo:hi]
        xf = dft @ x
        y = (xf[None, :] * np.conj(hf)) @ idft.T / L
        t_end = min(U, n - s * U)
        seg = y[:, half:half + t_end]
        out[:, s * U:s * U + t_end] = seg.real ** 2 + seg.imag ** 2
    return out


def correlate_bruteforce(a, h, m: int):
    """eq. 2 as explicit Python loops over (i, r, q); tiny inputs only."""
    half = _check_m(m)
    n = len(a)
    nz = len(h)
    out = [[0j] * n for _ in range(nz)]
    for i in range(nz):
        for r in range(n):
            acc = 0j
            for q in range(-half, half + 1):
                k = r + q
                if 0 <= k < n:
                    acc += complex(a[k]) * complex(h[i][q + half]).conjugate()
            out[i][r] = acc
    return out


def correlate_at(a: np.ndarray, z: float, r: float, m: int) -> complex:
    """B_z(r) at a real-valued bin r: sum over k in [c - m/2, c + m/2], c =
    round(r), of A_k conj(H_z(k - r)). Equals eq. 2 at integer r; used for
    the continuous (r, z) location of an injected signal.
    """
    half = _check_m(m)
    a = np.asarray(a, dtype=np.complex128)
    c = int(round(r))
    k = np.arange(c - half, c + half + 1)
    ok = (k >= 0) & (k < a.size)
    hv = template_h(z, k[ok] - r)
    return complex(np.sum(a[k[ok]] * np.conj(hv)))


def bank_natural(h: np.ndarray, m: int, seg_len: int) -> np.ndarray:
    """Fourier-domain bank T_i[k] = conj(FFT_L(h_i))[k] / L, natural k order.

    h_i is wrapped circularly (h[q mod L] = H_i(q)). This is what the
    overlap-and-save product multiplies each segment spectrum by; the
    library's planner produces the same values (in its own storage order).
    """
    half = _check_m(m)
    L = int(seg_len)
    h = np.atleast_2d(np.asarray(h, dtype=np.complex128))
    hw = np.zeros((h.shape[0], L), dtype=np.complex128)
    for j in range(m + 1):
        hw[:, (j - half) % L] += h[:, j]
    return np.conj(np.fft.fft(hw, axis=1)) / L


def candidates_direct(a: np.ndarray, zmax: float, dz: float, m: int, threshold: float,
                      interbin: bool = False):
    """Detection step after the plane (Section 3 names it; only its threshold
    part): every plane point with P >= threshold, as (row, r, P) arrays in
    row-major order, from the direct eq. 2 plane."""
    p = plane_direct(a, zmax, dz, m, interbin)
    row, r = np.nonzero(p >= threshold)
    return row, r, p[row, r]
