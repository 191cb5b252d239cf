"""Context measurements that mirror the paper's Tables 1 and 2 on this GPU.

Table 1 (Section 3): many transforms of 1024 points with the shared-memory
FFT at 2, 4 and 8 elements per thread, against the vendor FFT library.
Here: ``fdas_fft_exec`` (the correlation kernel's FFT stages on their own,
natural order in and out) at 2, 4, 8 and 16 elements per thread, against
``torch.fft.fft`` (rocFFT) on the same device buffers, both as one launch of
100,000 transforms and as 1000 launches of 100 (the paper's count).

Table 2 (Section 3): the whole convolution with the custom FFT against one
built from the library FFT, for filter lengths 64 .. 512. Here:
``fdas_convolve`` (plain FP32, and the FP16 matrix-core form) against an
overlap-and-save made of library calls on the same bank: ``torch.fft.fft``
of every segment, a broadcast product with the bank, ``torch.fft.ifft`` and
the discard/|.|^2 as torch element-wise kernels, the way a library-based
convolution is assembled. The library pipeline is a comparator only; its
plane is checked against the fused kernel's. Each row also gives the fused
kernels' plane points/s and their fraction of the HBM roofline, at
4 + 8/nz algorithmic bytes per point (one FP32 power written, each input bin
read once).

Front end: ``fdas_frontend_exec`` (real series -> normalised spectrum on the
device) for series of 2^16 .. 2^24 samples, against the same steps as torch
library calls (``torch.fft.rfft``, ``torch.median``, scaling).

Usage: python -m paper_1711_10855_amd.microbench [--table1] [--table2]
       [--frontend] [--out FILE]   (one JSON object per line)
"""

from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if os.path.dirname(HERE) not in sys.path:
    sys.path.insert(0, os.path.dirname(HERE))

from paper_1711_10855_amd import fdas  # noqa: E402

HBM_PEAK = 8.0e12    # MI355X HBM3E peak, bytes/s


def _time(fn, reps, warm):
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def table1(emit, n=1024, batch=100_000):
    import torch
    rng = np.random.default_rng(1711)
    x = torch.from_numpy(rng.standard_normal((batch, 2 * n), dtype=np.float32)).view(
        torch.complex64).cuda()
    out = torch.empty_like(x)
    small = x[:100].contiguous()
    small_out = torch.empty_like(small)
    bytes_moved = 2 * 8 * n * batch
    rows = []
    for e in (2, 4, 8, 16):
        with fdas.FFT(n, e) as f:
            ms = _time(lambda: f(x, out=out), reps=50, warm=50)
            ms_small = _time(lambda: [f(small, out=small_out) for _ in range(1000)], reps=3, warm=1)
            ref = torch.fft.fft(x[:64])
            err = float((out[:64] - ref).abs().max() / ref.abs().max())
            rows.append({"table": 1, "impl": f.kernel, "elems_per_thread": e, "n": n,
                         "ms_100k": ms, "ms_1000x100": ms_small, "GB_s": bytes_moved / ms / 1e6,
                         "max_rel_diff_vs_library": err})
    # no out= argument: torch would then add a copy kernel after rocFFT's
    ms = _time(lambda: torch.fft.fft(x), reps=50, warm=50)
    ms_small = _time(lambda: [torch.fft.fft(small) for _ in range(1000)], reps=3, warm=1)
    rows.append({"table": 1, "impl": "torch.fft.fft (rocFFT)", "elems_per_thread": None, "n": n,
                 "ms_100k": ms, "ms_1000x100": ms_small, "GB_s": bytes_moved / ms / 1e6})
    lib = rows[-1]
    for r in rows[:-1]:
        r["speedup_vs_library_100k"] = lib["ms_100k"] / r["ms_100k"]
        r["speedup_vs_library_1000x100"] = lib["ms_1000x100"] / r["ms_1000x100"]
    for r in rows:
        emit(r)


class LibraryOLS:
    """Overlap-and-save from library FFT calls and element-wise kernels."""

    def __init__(self, bank, m, nbins, chunk=16):
        import torch
        self.bank = bank                      # complex64 [nz, L], natural order, /L folded
        self.nz, self.L = bank.shape
        self.m, self.half, self.U = m, m // 2, self.L - m
        self.nbins = nbins
        self.S = -(-nbins // self.U)
        self.padded = torch.zeros(self.S * self.U + m, dtype=torch.complex64, device=bank.device)
        self.chunk = chunk

    def __call__(self, spec, power):
        import torch
        h, U, S, L = self.half, self.U, self.S, self.L
        self.padded[h:h + self.nbins].copy_(spec)
        X = torch.fft.fft(self.padded.unfold(0, L, U))          # [S, L]
        for z0 in range(0, self.nz, self.chunk):
            z1 = min(self.nz, z0 + self.chunk)
            Y = X.unsqueeze(1) * self.bank[z0:z1].unsqueeze(0)   # [S, c, L]
            y = torch.fft.ifft(Y, norm="forward")                # no 1/L (in the bank)
            p = y[:, :, h:h + U].abs().square()                  # discard, |.|^2
            p = p.permute(1, 0, 2).reshape(z1 - z0, S * U)
            power[z0:z1].copy_(p[:, :self.nbins])


def table2(emit, filters=(64, 128, 256, 384, 512), nbins=1 << 21, zmax=100.0, dz=2.0):
    import torch
    rng = np.random.default_rng(1711)
    a = (rng.standard_normal(nbins) + 1j * rng.standard_normal(nbins)).astype(np.complex64)
    spec = torch.from_numpy(a).cuda()
    for m in filters:
        with fdas.Plan(zmax, dz, m, 0, "fp32") as p:
            nz, L = p.nz, p.info.seg_len
            plane = torch.empty((nz, nbins), dtype=torch.float32, device="cuda")
            ms = _time(lambda: p.convolve(spec, out=plane), reps=100, warm=200)
            lib = LibraryOLS(p.bank(), m, nbins)
            ref = torch.empty_like(plane)
            ms_lib = _time(lambda: lib(spec, ref), reps=5, warm=2)
            diff = float((plane - ref).abs().max() / ref.max())
            kern = p.info.kernel
        pts = nz * nbins
        bpp = 4.0 + 8.0 / nz    # one FP32 power written per point, each input bin read once
        row = {"table": 2, "m": m, "nz": nz, "nbins": nbins, "seg_len": L, "kernel": kern,
               "ms": ms, "points_per_s": pts / ms * 1e3,
               "hbm_roofline_frac": pts / ms * 1e3 * bpp / HBM_PEAK,
               "ms_library_ols": ms_lib, "speedup_vs_library": ms_lib / ms,
               "max_rel_diff_vs_library": diff}
        with fdas.Plan(zmax, dz, m, 0, "fp16") as q:
            plane16 = torch.empty((q.nz, nbins), dtype=torch.float32, device="cuda")
            ms16 = _time(lambda: q.convolve(spec, out=plane16), reps=100, warm=200)
            row.update({"kernel_fp16": q.info.kernel, "seg_len_fp16": q.info.seg_len,
                        "ms_fp16": ms16, "points_per_s_fp16": pts / ms16 * 1e3,
                        "hbm_roofline_frac_fp16": pts / ms16 * 1e3 * bpp / HBM_PEAK,
                        "speedup_fp16_vs_library": ms_lib / ms16})
        emit(row)


def frontend(emit, sizes=(1 << 16, 1 << 20, 1 << 22, 1 << 24)):
    import math
    import torch
    for n in sizes:
        rng = np.random.default_rng(n)
        x = torch.from_numpy(rng.standard_normal(n, dtype=np.float32)).cuda()
        out = torch.empty(n // 2, dtype=torch.complex64, device="cuda")
        with fdas.FrontEnd(n) as fe:
            ms = _time(lambda: fe(x, out=out), reps=50, warm=20)

        def library():
            a = torch.fft.rfft(x)[: n // 2]
            a[0] = 0
            med = torch.median(a[1:].abs().square())
            return a * torch.sqrt(math.log(2.0) / med)

        ref = library()
        diff = float((out - ref).abs().max() / ref.abs().max())
        ms_lib = _time(library, reps=20, warm=5)
        emit({"table": "frontend", "n": n, "ms": ms, "ms_library": ms_lib,
              "speedup_vs_library": ms_lib / ms, "max_rel_diff_vs_library": diff,
              "GB_s_series_plus_spectrum": 8.0 * n / ms / 1e6})


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--table1", action="store_true")
    ap.add_argument("--table2", action="store_true")
    ap.add_argument("--frontend", action="store_true")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    if not (a.table1 or a.table2 or a.frontend):
        a.table1 = a.table2 = a.frontend = True
    fdas.load()
    fh = open(a.out, "w") if a.out else None

    def emit(row):
        line = json.dumps(row)
        print(line, flush=True)
        if fh:
            fh.write(line + "\n")
            fh.flush()

    if a.table1:
        table1(emit)
    if a.table2:
        table2(emit)
    if a.frontend:
        frontend(emit)
    if fh:
        fh.close()


if __name__ == "__main__":
    main()
