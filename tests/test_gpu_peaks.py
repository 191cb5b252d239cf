"""Detection epilogue with peak picking (fdas_convolve_peaks), through the C
ABI. The peak decision is taken on FP32 powers on the device, so it is
compared exactly with the oracle's peak rule applied to the same kernel's
FP32 plane; against the FP64 oracle's own peaks it is compared within the
form's tolerance band (peaks that are clear by more than the band must be
found, and every peak found must be one within the band)."""

import numpy as np
import pytest

import oracle
from paper_1711_10855_amd import synth

pytestmark = pytest.mark.gpu


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).cuda()


def as_set(row, r):
    return set(zip(np.asarray(row).tolist(), np.asarray(r).tolist()))


def grid_of(p, interbin):
    """The (z, r) grid of a plane as the peak rule reads it."""
    if not interbin:
        return p
    g = np.empty((p.shape[0] // 2, 2 * p.shape[1]))
    g[:, 0::2], g[:, 1::2] = p[0::2], p[1::2]
    return g


def neighbour_max(g):
    pad = np.full((g.shape[0] + 2, g.shape[1] + 2), -np.inf)
    pad[1:-1, 1:-1] = g
    out = np.full(g.shape, -np.inf)
    for dz in (-1, 0, 1):
        for dc in (-1, 0, 1):
            if dz or dc:
                out = np.maximum(out, pad[1 + dz:1 + dz + g.shape[0], 1 + dc:1 + dc + g.shape[1]])
    return out


def to_grid_index(row, r, interbin):
    row, r = np.asarray(row), np.asarray(r)
    return (row >> 1, 2 * r + (row & 1)) if interbin else (row, r)


@pytest.mark.parametrize("prec,L,m,flags,tol", [("fp32", 256, 64, 0, 1e-4),
                                                ("fp32", 1024, 64, 4, 1e-4),
                                                ("fp16", 4096, 64, 0, 1e-3),
                                                ("bf16", 4096, 64, 1, 1e-3),
                                                ("fp16", 4096, 128, 4, 1e-3),
                                                ("fp16", 2048, 64, 0, 1e-3),
                                                ("fp16", 2048, 128, 4, 1e-3)])
def test_peaks_match_oracle(gpu, prec, L, m, flags, tol):
    a = synth.small_random_spectrum(20000, seed=90)
    a[7000:7010] *= 6.0                       # strong bins among the noise
    a[15000] *= 9.0
    thr = 5.0
    interbin = bool(flags & gpu.FLAG_INTERBIN)
    print(f"peaks {prec} L={L} m={m} flags={flags}", flush=True)
    with gpu.Plan(16.0, 2.0, m, L, prec, flags) as p:
        out = p.peaks(to_dev(a), thr, cand_capacity=1 << 17, peak_capacity=1 << 15)
        row, r, pw, n_cand, n_peak = gpu.decode_peaks(out[0], out[1])
        plane = p.convolve(to_dev(a)).cpu().numpy()
        again = p.peaks(to_dev(a), thr, buf=out)          # the table is cleared per call
        row2, r2, _, n_cand2, n_peak2 = gpu.decode_peaks(again[0], again[1])
    print(f"  {n_cand} candidates, {n_peak} peaks", flush=True)
    assert n_cand <= 1 << 17 and 0 < n_peak == row.size <= 1 << 15
    got = as_set(row, r)
    assert len(got) == n_peak                   # no duplicates
    assert (n_cand2, n_peak2) == (n_cand, n_peak) and as_set(row2, r2) == got
    # exactly: the oracle's rule on the same FP32 plane
    assert n_cand == int(np.count_nonzero(plane >= thr))
    want_row, want_r, want_v = oracle.peaks_from_plane(plane.astype(np.float64), thr, interbin)
    assert got == as_set(want_row, want_r)
    assert np.array_equal(pw, plane[row, r])
    # against the FP64 oracle, within the band
    ref = oracle.plane_direct(a, 16.0, 2.0, m, interbin)
    band = tol * ref.max()
    g = grid_of(ref, interbin)
    nb = neighbour_max(g)
    o_row, o_r, _ = oracle.peaks_from_plane(ref, thr, interbin)
    gi, gc = to_grid_index(o_row, o_r, interbin)
    clear = (g[gi, gc] >= thr + band) & (g[gi, gc] > nb[gi, gc] + 2 * band)
    assert clear.sum() > 10
    assert as_set(o_row[clear], o_r[clear]) <= got
    gi, gc = to_grid_index(row, r, interbin)
    assert np.all(g[gi, gc] >= thr - band)
    assert np.all(g[gi, gc] >= nb[gi, gc] - 2 * band)


@pytest.mark.parametrize("flags", [0, 4])
def test_a_flat_plane_has_one_peak(gpu, flags):
    """A zero spectrum gives a plane of equal zeros: with threshold 0 every
    point is a candidate and the tie rule leaves exactly the first one."""
    import torch
    a = torch.zeros(700, dtype=torch.complex64, device="cuda")
    with gpu.Plan(16.0, 2.0, 64, 256, "fp32", flags) as p:
        rows = p.info.nz
        row, r, pw, n_cand, n_peak = gpu.decode_peaks(*p.peaks(a, 0.0, 1 << 16, 64)[:2])
    assert n_cand == rows * 700
    assert (n_peak, row.tolist(), r.tolist(), pw.tolist()) == (1, [0], [0], [0.0])


def test_capacities_are_reported(gpu):
    a = synth.small_random_spectrum(30000, seed=91)
    with gpu.Plan(16.0, 2.0, 64, 512) as p:
        full = p.peaks(to_dev(a), 3.0, 1 << 18, 1 << 16)
        _, _, _, n_cand, n_peak = gpu.decode_peaks(full[0], full[1])
        # too few peak slots: all are counted, the first ones stored are peaks
        few = p.peaks(to_dev(a), 3.0, 1 << 18, 7)
        row, r, _, n_cand2, n_peak2 = gpu.decode_peaks(few[0], few[1])
        # too few candidate slots: the count says so
        short = p.peaks(to_dev(a), 3.0, 1000, 1 << 16)
        n_cand3 = int(short[1].cpu()[0])
        want = as_set(*gpu.decode_peaks(full[0], full[1])[:2])
    assert n_cand > 1000 and n_peak > 7
    assert (n_cand2, n_peak2) == (n_cand, n_peak) and row.size == 7
    assert as_set(row, r) <= want
    assert n_cand3 == n_cand


def test_convolve_rejects_a_plane_over_the_spectrum(gpu):
    """fdas_convolve refuses a power buffer that overlaps its input (the
    plane of 17 rows at stride 1000 ends 16 * 1000 + 500 values in)."""
    import ctypes as C

    import torch
    buf = torch.zeros(17 * 1000 + 2000, dtype=torch.float32, device="cuda")
    with gpu.Plan(16.0, 2.0, 64, 256) as p:
        base = buf.data_ptr()
        st = gpu.load().fdas_convolve(p._h, C.c_void_p(base + 4 * 16500 - 8), 500,
                                      C.c_void_p(base), 1000, None)
        assert st == gpu.ERR_INVALID and "overlaps" in gpu.last_error()
        st = gpu.load().fdas_convolve(p._h, C.c_void_p(base + 4 * 16500), 500,
                                      C.c_void_p(base), 1000, None)
        assert st == gpu.OK
        torch.cuda.synchronize()
