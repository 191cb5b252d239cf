"""Thin ctypes binding of the C ABI in include/fdas.h.

Argument marshalling only: every step of the correlation runs in the HIP
library ``libfdas.so`` built next to this file. PyTorch is used for device
memory and streams; the functions take and return torch tensors and pass
their device pointers and the current HIP stream through the ABI. If the
library is missing, ``load()`` raises -- there is no fallback path.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdas.so")

OK = 0
ERR_INVALID = -1
ERR_UNSUPPORTED = -2
ERR_NOMEM = -3
ERR_DEVICE = -4

FP32 = 0
MIXED_FP16 = 1
MIXED_BF16 = 2
PRECISIONS = {"fp32": FP32, "fp16": MIXED_FP16, "bf16": MIXED_BF16}

FLAG_SPLIT = 1
FLAG_AUTOTUNE = 2
FLAG_INTERBIN = 4
FLAG_BANK = 8

EXPORTS = (
    "fdas_plane_rows", "fdas_resolve_params", "fdas_make_templates", "fdas_plan",
    "fdas_plan_get_info", "fdas_plan_bank", "fdas_convolve", "fdas_convolve_batch",
    "fdas_destroy", "fdas_status_string", "fdas_last_error", "fdas_kernel_variants",
    "fdas_convolve_candidates", "fdas_fft_plan", "fdas_fft_get_info", "fdas_fft_exec",
    "fdas_fft_destroy", "fdas_fft_variants", "fdas_frontend_plan", "fdas_frontend_exec",
    "fdas_frontend_destroy", "fdas_convolve_batch_noalloc", "fdas_peaks_workspace_bytes",
    "fdas_convolve_peaks",
)


class Params(C.Structure):
    _fields_ = [("zmax", C.c_double), ("dz", C.c_double), ("m", C.c_int),
                ("seg_len", C.c_int), ("precision", C.c_int), ("flags", C.c_uint)]


class Series(C.Structure):
    _fields_ = [("spectrum", C.c_void_p), ("nbins", C.c_int64), ("zmax", C.c_double),
                ("power", C.c_void_p), ("ld", C.c_int64)]


class PlanInfo(C.Structure):
    _fields_ = [("nz", C.c_int), ("m", C.c_int), ("seg_len", C.c_int), ("valid", C.c_int),
                ("precision", C.c_int), ("flags", C.c_uint), ("threads", C.c_int),
                ("templates_per_block", C.c_int), ("segments_per_block", C.c_int),
                ("bank_bytes", C.c_size_t), ("plan_ms", C.c_double), ("kernel", C.c_char * 64)]


class FftInfoC(C.Structure):
    _fields_ = [("n", C.c_int), ("elems_per_thread", C.c_int), ("threads", C.c_int),
                ("transforms_per_block", C.c_int), ("kernel", C.c_char * 64)]


class FdasError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str):
        super().__init__(f"{what}: {status} ({detail})")
        self.status = status


_lib = None


def load():
    """Load libfdas.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing; run paper_1711_10855_amd.build first")
    # torch ships its own HIP runtime under the same soname; it must be the one
    # in the process before libfdas.so resolves its HIP dependency, so that the
    # library and torch's allocator and streams share one runtime instance.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER
    lib.fdas_plane_rows.argtypes = [P(Params)]
    lib.fdas_plane_rows.restype = C.c_int
    lib.fdas_resolve_params.argtypes = [P(Params), P(Params)]
    lib.fdas_resolve_params.restype = C.c_int
    lib.fdas_make_templates.argtypes = [P(Params), C.c_void_p, P(C.c_size_t), C.c_void_p]
    lib.fdas_make_templates.restype = C.c_int
    lib.fdas_plan.argtypes = [P(C.c_void_p), P(Params), C.c_int, C.c_void_p]
    lib.fdas_plan.restype = C.c_int
    lib.fdas_plan_get_info.argtypes = [C.c_void_p, P(PlanInfo)]
    lib.fdas_plan_get_info.restype = C.c_int
    lib.fdas_plan_bank.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
    lib.fdas_plan_bank.restype = C.c_int
    lib.fdas_convolve.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                  C.c_void_p]
    lib.fdas_convolve.restype = C.c_int
    lib.fdas_convolve_batch.argtypes = [C.c_void_p, P(Series), C.c_int, C.c_void_p]
    lib.fdas_convolve_batch.restype = C.c_int
    lib.fdas_convolve_batch_noalloc.argtypes = [C.c_void_p, P(Series), C.c_int, C.c_void_p]
    lib.fdas_convolve_batch_noalloc.restype = C.c_int
    lib.fdas_convolve_candidates.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_float,
                                             C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
    lib.fdas_convolve_candidates.restype = C.c_int
    lib.fdas_peaks_workspace_bytes.argtypes = [C.c_int64]
    lib.fdas_peaks_workspace_bytes.restype = C.c_size_t
    lib.fdas_convolve_peaks.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_float,
                                        C.c_void_p, C.c_size_t, C.c_int64, C.c_void_p,
                                        C.c_int64, C.c_void_p, C.c_void_p]
    lib.fdas_convolve_peaks.restype = C.c_int
    lib.fdas_destroy.argtypes = [C.c_void_p]
    lib.fdas_destroy.restype = C.c_int
    lib.fdas_status_string.argtypes = [C.c_int]
    lib.fdas_status_string.restype = C.c_char_p
    lib.fdas_kernel_variants.argtypes = [C.c_int, C.c_int, C.c_char_p, C.c_size_t]
    lib.fdas_kernel_variants.restype = C.c_int
    lib.fdas_fft_plan.argtypes = [P(C.c_void_p), C.c_int, C.c_int, C.c_int, C.c_void_p]
    lib.fdas_fft_plan.restype = C.c_int
    lib.fdas_fft_get_info.argtypes = [C.c_void_p, P(FftInfoC)]
    lib.fdas_fft_get_info.restype = C.c_int
    lib.fdas_fft_exec.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int,
                                  C.c_void_p]
    lib.fdas_fft_exec.restype = C.c_int
    lib.fdas_fft_destroy.argtypes = [C.c_void_p]
    lib.fdas_fft_destroy.restype = C.c_int
    lib.fdas_fft_variants.argtypes = [C.c_int, C.c_char_p, C.c_size_t]
    lib.fdas_fft_variants.restype = C.c_int
    lib.fdas_frontend_plan.argtypes = [P(C.c_void_p), C.c_int64, C.c_int, C.c_void_p]
    lib.fdas_frontend_plan.restype = C.c_int
    lib.fdas_frontend_exec.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.fdas_frontend_exec.restype = C.c_int
    lib.fdas_frontend_destroy.argtypes = [C.c_void_p]
    lib.fdas_frontend_destroy.restype = C.c_int
    lib.fdas_last_error.argtypes = []
    lib.fdas_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def last_error() -> str:
    return load().fdas_last_error().decode()


def _check(status: int, what: str):
    if status != OK:
        raise FdasError(status, what, last_error())


def params(zmax, dz, m=0, seg_len=0, precision="fp32", flags=0) -> Params:
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    return Params(float(zmax), float(dz), int(m or 0), int(seg_len or 0), prec, int(flags))


def plane_rows(zmax, dz, flags=0) -> int:
    n = load().fdas_plane_rows(C.byref(params(zmax, dz, 0, 0, "fp32", flags)))
    if n < 0:
        _check(n, "fdas_plane_rows")
    return n


def resolve(zmax, dz, m=0, seg_len=0, precision="fp32", flags=0) -> Params:
    out = Params()
    _check(load().fdas_resolve_params(C.byref(params(zmax, dz, m, seg_len, precision, flags)),
                                      C.byref(out)), "fdas_resolve_params")
    return out


def kernel_variants(seg_len=0, precision=-1):
    """Names of the compiled hot-kernel variants (host-only query)."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    n = load().fdas_kernel_variants(int(seg_len), prec, None, 0)
    if n < 0:
        _check(n, "fdas_kernel_variants")
    buf = C.create_string_buffer(64 * (n + 1))
    load().fdas_kernel_variants(int(seg_len), prec, buf, len(buf))
    return [x for x in buf.value.decode().split("\n") if x]


def _plane_ok(out, rows, nbins, ld, device):
    """Raise unless `out` can hold rows x nbins float32 values at row stride ld
    on `device` (the kernels write through the pointer; a short or mistyped
    buffer must never reach them)."""
    import torch
    if (not isinstance(out, torch.Tensor) or out.dtype != torch.float32 or out.device != device
            or out.dim() != 2 or out.shape[0] != rows or out.stride(1) != 1):
        raise TypeError(f"output must be a float32 tensor [{rows}, >= {nbins}] with unit column "
                        f"stride on {device}")
    if ld < nbins or out.shape[1] < nbins or (rows > 1 and out.stride(0) != ld):
        raise ValueError(f"output rows hold {out.shape[1]} values at stride {out.stride(0)}; "
                         f"need >= {nbins} at stride ld = {ld}")


def _stream(device=None):
    import torch
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def make_templates(zmax, dz, m=0, flags=0):
    """FP64 templates H_{z_i}(q), complex128 tensor [rows, m+1] on the current
    device (rows = nz, or 2 nz with FLAG_INTERBIN)."""
    import torch
    p = params(zmax, dz, m, 0, "fp32", flags)
    nbytes = C.c_size_t(0)
    _check(load().fdas_make_templates(C.byref(p), None, C.byref(nbytes), None),
           "fdas_make_templates(size)")
    r = resolve(zmax, dz, m, 0, "fp32", flags)
    nz = plane_rows(zmax, dz, flags)
    out = torch.empty((nz, r.m + 1), dtype=torch.complex128, device="cuda")
    _check(load().fdas_make_templates(C.byref(p), C.c_void_p(out.data_ptr()), C.byref(nbytes),
                                      _stream()), "fdas_make_templates")
    return out


def make_bank(zmax, dz, m=0, seg_len=0, flags=0):
    """The Fourier-domain template bank T_i[k], complex64 tensor [rows, L] in
    natural frequency order on the current device (FP64 direct sums rounded
    to FP32; fdas_make_templates with FLAG_BANK)."""
    import torch
    p = params(zmax, dz, m, seg_len, "fp32", flags | FLAG_BANK)
    nbytes = C.c_size_t(0)
    _check(load().fdas_make_templates(C.byref(p), None, C.byref(nbytes), None),
           "fdas_make_templates(bank size)")
    r = resolve(zmax, dz, m, seg_len, "fp32", flags)
    nz = plane_rows(zmax, dz, flags)
    out = torch.empty((nz, r.seg_len), dtype=torch.complex64, device="cuda")
    _check(load().fdas_make_templates(C.byref(p), C.c_void_p(out.data_ptr()), C.byref(nbytes),
                                      _stream()), "fdas_make_templates(bank)")
    return out


@dataclass
class Info:
    nz: int
    m: int
    seg_len: int
    valid: int
    precision: int
    flags: int
    threads: int
    templates_per_block: int
    segments_per_block: int
    bank_bytes: int
    plan_ms: float
    kernel: str


class Plan:
    """Owns an fdas plan (template bank, twiddles) on one device."""

    def __init__(self, zmax, dz, m=0, seg_len=0, precision="fp32", flags=0, device=None):
        import torch
        self._lib = load()
        self.params = params(zmax, dz, m, seg_len, precision, flags)
        dev = torch.cuda.current_device() if device is None else int(device)
        self.device = dev
        h = C.c_void_p()
        _check(self._lib.fdas_plan(C.byref(h), C.byref(self.params), dev, _stream(dev)), "fdas_plan")
        self._h = h
        self.info = self.get_info()

    def get_info(self) -> Info:
        i = PlanInfo()
        _check(self._lib.fdas_plan_get_info(self._h, C.byref(i)), "fdas_plan_get_info")
        return Info(i.nz, i.m, i.seg_len, i.valid, i.precision, i.flags, i.threads,
                    i.templates_per_block, i.segments_per_block, i.bank_bytes, i.plan_ms,
                    i.kernel.decode())

    @property
    def nz(self) -> int:
        return self.info.nz

    def bank(self):
        """The Fourier-domain bank, natural order, complex64 [nz, L] (testing)."""
        import torch
        out = torch.empty((self.info.nz, self.info.seg_len), dtype=torch.complex64,
                          device=f"cuda:{self.device}")
        _check(self._lib.fdas_plan_bank(self._h, C.c_void_p(out.data_ptr()),
                                        out.numel() * 8, _stream(self.device)), "fdas_plan_bank")
        return out

    def convolve(self, spectrum, out=None, ld=None):
        """power[nz, nbins] (float32) for a complex64 device spectrum."""
        import torch
        if spectrum.dtype != torch.complex64 or not spectrum.is_cuda or spectrum.dim() != 1:
            raise TypeError("spectrum must be a 1-D complex64 CUDA tensor")
        spectrum = spectrum.contiguous()
        nbins = spectrum.numel()
        if out is None:
            ld = nbins if ld is None else int(ld)
            out = torch.empty((self.info.nz, ld), dtype=torch.float32, device=spectrum.device)
        else:
            ld = out.stride(0) if ld is None else int(ld)
            _plane_ok(out, self.info.nz, nbins, ld, spectrum.device)
        _check(self._lib.fdas_convolve(self._h, C.c_void_p(spectrum.data_ptr()), nbins,
                                       C.c_void_p(out.data_ptr()), ld, _stream(spectrum.device)),
               "fdas_convolve")
        return out[:, :nbins] if out.shape[1] != nbins else out

    def candidates(self, spectrum, threshold, capacity=1 << 16, buf=None):
        """Detection epilogue: plane points with power >= threshold.

        Returns (records, count): ``records`` is a device int64 tensor
        [capacity, 2] holding fdas_candidate entries (decode with
        ``decode_candidates``), ``count`` a one-element device int64 tensor
        with the number of points found (records beyond capacity are
        dropped). ``buf`` may pass both tensors back in to reuse them."""
        import torch
        if spectrum.dtype != torch.complex64 or not spectrum.is_cuda or spectrum.dim() != 1:
            raise TypeError("spectrum must be a 1-D complex64 CUDA tensor")
        spectrum = spectrum.contiguous()
        if buf is None:
            rec = torch.empty((capacity, 2), dtype=torch.int64, device=spectrum.device)
            cnt = torch.empty(1, dtype=torch.int64, device=spectrum.device)
        else:
            rec, cnt = buf
            if (rec.dtype != torch.int64 or rec.dim() != 2 or rec.shape[1] != 2
                    or not rec.is_contiguous() or rec.device != spectrum.device
                    or cnt.dtype != torch.int64 or cnt.numel() < 1 or cnt.device != spectrum.device):
                raise TypeError("buf must be (int64 [capacity, 2], int64 [1]) on the spectrum's device")
            capacity = rec.shape[0]
        _check(self._lib.fdas_convolve_candidates(
            self._h, C.c_void_p(spectrum.data_ptr()), spectrum.numel(), float(threshold),
            C.c_void_p(rec.data_ptr()), capacity, C.c_void_p(cnt.data_ptr()),
            _stream(spectrum.device)), "fdas_convolve_candidates")
        return rec, cnt

    def peaks(self, spectrum, threshold, cand_capacity=1 << 16, peak_capacity=1 << 16, buf=None):
        """Detection epilogue with peak picking (see fdas_convolve_peaks).

        Returns (records, counts, workspace, cand_capacity): ``records`` a
        device int64 tensor [peak_capacity, 2] of fdas_candidate entries
        (decode with ``decode_peaks``), ``counts`` a device int64 tensor [2]
        (candidates, peaks found), ``workspace`` the device buffer the search
        used for ``cand_capacity`` candidates. ``buf`` may pass the tuple
        back in to reuse it."""
        import torch
        if spectrum.dtype != torch.complex64 or not spectrum.is_cuda or spectrum.dim() != 1:
            raise TypeError("spectrum must be a 1-D complex64 CUDA tensor")
        spectrum = spectrum.contiguous()
        dev = spectrum.device
        if buf is None:
            nbytes = self._lib.fdas_peaks_workspace_bytes(int(cand_capacity))
            if nbytes == 0:
                raise ValueError(f"candidate capacity {cand_capacity} out of range")
            rec = torch.empty((peak_capacity, 2), dtype=torch.int64, device=dev)
            cnt = torch.empty(2, dtype=torch.int64, device=dev)
            work = torch.empty((nbytes + 15) // 16 * 2, dtype=torch.int64, device=dev)
        else:
            rec, cnt, work, cand_capacity = buf
            if (rec.dtype != torch.int64 or rec.dim() != 2 or rec.shape[1] != 2
                    or not rec.is_contiguous() or rec.device != dev or cnt.dtype != torch.int64
                    or cnt.numel() < 2 or cnt.device != dev or work.device != dev
                    or not work.is_contiguous()):
                raise TypeError("buf must be (int64 [cap, 2], int64 [2], workspace, capacity) "
                                "on the spectrum's device")
            peak_capacity = rec.shape[0]
        _check(self._lib.fdas_convolve_peaks(
            self._h, C.c_void_p(spectrum.data_ptr()), spectrum.numel(), float(threshold),
            C.c_void_p(work.data_ptr()), work.numel() * work.element_size(), int(cand_capacity),
            C.c_void_p(rec.data_ptr()), int(peak_capacity), C.c_void_p(cnt.data_ptr()),
            _stream(dev)), "fdas_convolve_peaks")
        return rec, cnt, work, int(cand_capacity)

    def _series(self, spectra, zmaxs, outs):
        import torch
        n = len(spectra)
        if not (n == len(zmaxs) == len(outs)) or n < 1:
            raise ValueError("need equally many (>= 1) spectra, zmaxs and outputs")
        per = 2 if self.params.flags & FLAG_INTERBIN else 1
        arr = (Series * n)()
        for i, (s, z, o) in enumerate(zip(spectra, zmaxs, outs)):
            if s.dtype != torch.complex64 or not s.is_cuda or s.dim() != 1 or not s.is_contiguous():
                raise TypeError(f"spectrum {i} must be a contiguous 1-D complex64 CUDA tensor")
            span = 2 * float(z) / self.params.dz
            if 0 <= float(z) <= self.params.zmax and abs(span - round(span)) < 1e-6:
                # (other zmax values are the library's to reject)
                _plane_ok(o, per * (int(round(span)) + 1), s.numel(), o.stride(0), s.device)
            arr[i] = Series(C.c_void_p(s.data_ptr()), s.numel(), float(z),
                            C.c_void_p(o.data_ptr()), o.stride(0))
        return arr, n

    def convolve_batch(self, spectra, zmaxs, outs):
        """Batched form: one launch over every series (see fdas_convolve_batch)."""
        arr, n = self._series(spectra, zmaxs, outs)
        _check(self._lib.fdas_convolve_batch(self._h, arr, n, _stream(spectra[0].device)),
               "fdas_convolve_batch")
        return outs

    def convolve_batch_noalloc(self, spectra, zmaxs, outs):
        """The batched form without any device allocation (see
        fdas_convolve_batch_noalloc): same results as convolve_batch."""
        arr, n = self._series(spectra, zmaxs, outs)
        _check(self._lib.fdas_convolve_batch_noalloc(self._h, arr, n,
                                                     _stream(spectra[0].device)),
               "fdas_convolve_batch_noalloc")
        return outs

    def close(self):
        if getattr(self, "_h", None):
            _check(self._lib.fdas_destroy(self._h), "fdas_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def decode_candidates(rec, count):
    """(row, r, power) numpy arrays from the tensors of Plan.candidates
    (`count` the count tensor, or the count itself)."""
    import numpy as np
    n = min(count if isinstance(count, int) else int(count.cpu()[0]), rec.shape[0])
    raw = rec[:n].cpu().numpy()
    lo = raw[:, 0].astype(np.uint64)
    row = (lo & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.int32)
    power = (lo >> np.uint64(32)).astype(np.uint32).view(np.float32)
    return row.astype(np.int64), raw[:, 1].copy(), power.astype(np.float32)


def decode_peaks(rec, counts):
    """(row, r, power) numpy arrays and the two counts (candidates, peaks)
    from the tensors of Plan.peaks."""
    n_cand, n_peak = (int(x) for x in counts.cpu()[:2])
    row, r, power = decode_candidates(rec, n_peak)
    return row, r, power, n_cand, n_peak


def fft_variants(n=0):
    """Names of the compiled standalone FFT forms of length n (0 = all)."""
    k = load().fdas_fft_variants(int(n), None, 0)
    if k < 0:
        _check(k, "fdas_fft_variants")
    buf = C.create_string_buffer(64 * (k + 1))
    load().fdas_fft_variants(int(n), buf, len(buf))
    return [x for x in buf.value.decode().split("\n") if x]


class FFT:
    """Standalone batched complex FFT of length n (the correlation kernel's
    shared-memory FFT on its own)."""

    def __init__(self, n, elems_per_thread=0, device=None):
        import torch
        self._lib = load()
        dev = torch.cuda.current_device() if device is None else int(device)
        self.device = dev
        h = C.c_void_p()
        _check(self._lib.fdas_fft_plan(C.byref(h), int(n), int(elems_per_thread), dev,
                                       _stream(dev)), "fdas_fft_plan")
        self._h = h
        i = FftInfoC()
        _check(self._lib.fdas_fft_get_info(self._h, C.byref(i)), "fdas_fft_get_info")
        self.n, self.elems_per_thread = i.n, i.elems_per_thread
        self.threads, self.transforms_per_block = i.threads, i.transforms_per_block
        self.kernel = i.kernel.decode()

    def __call__(self, x, out=None, direction=-1):
        """Transforms of the rows of a complex64 CUDA tensor [batch, n]
        (unnormalised; direction -1 forward, +1 inverse)."""
        import torch
        if x.dtype != torch.complex64 or not x.is_cuda or x.dim() != 2 or x.shape[1] != self.n:
            raise TypeError(f"need a complex64 CUDA tensor [batch, {self.n}]")
        x = x.contiguous()
        if out is None:
            out = torch.empty_like(x)
        elif (out.dtype != torch.complex64 or out.shape != x.shape or not out.is_contiguous()
              or out.device != x.device):
            raise TypeError(f"out must be a contiguous complex64 tensor {tuple(x.shape)} on {x.device}")
        _check(self._lib.fdas_fft_exec(self._h, C.c_void_p(x.data_ptr()),
                                       C.c_void_p(out.data_ptr()), x.shape[0], int(direction),
                                       _stream(x.device)), "fdas_fft_exec")
        return out

    def close(self):
        if getattr(self, "_h", None):
            _check(self._lib.fdas_fft_destroy(self._h), "fdas_fft_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class FrontEnd:
    """Device front end: real series of n samples (a power of two) -> the
    normalised complex spectrum of n/2 bins the correlation runs on."""

    def __init__(self, n, device=None):
        import torch
        self._lib = load()
        dev = torch.cuda.current_device() if device is None else int(device)
        self.device, self.n = dev, int(n)
        h = C.c_void_p()
        _check(self._lib.fdas_frontend_plan(C.byref(h), self.n, dev, _stream(dev)),
               "fdas_frontend_plan")
        self._h = h

    def __call__(self, series, out=None, stats=None):
        """complex64 spectrum [n/2] of a float32 CUDA series [n]; `stats`, a
        float32 CUDA tensor [2], receives (scale, median |A|^2)."""
        import torch
        if series.dtype != torch.float32 or not series.is_cuda or series.shape != (self.n,):
            raise TypeError(f"need a float32 CUDA tensor [{self.n}]")
        series = series.contiguous()
        if out is None:
            out = torch.empty(self.n // 2, dtype=torch.complex64, device=series.device)
        elif (out.dtype != torch.complex64 or out.numel() != self.n // 2
              or not out.is_contiguous() or out.device != series.device):
            raise TypeError(f"out must be a contiguous complex64 tensor of {self.n // 2} values")
        if stats is not None and (stats.dtype != torch.float32 or stats.numel() < 2
                                  or not stats.is_contiguous() or stats.device != series.device):
            raise TypeError("stats must be a contiguous float32 tensor of 2 values")
        st = C.c_void_p(stats.data_ptr()) if stats is not None else None
        _check(self._lib.fdas_frontend_exec(self._h, C.c_void_p(series.data_ptr()),
                                            C.c_void_p(out.data_ptr()), st,
                                            _stream(series.device)), "fdas_frontend_exec")
        return out

    def close(self):
        if getattr(self, "_h", None):
            _check(self._lib.fdas_frontend_destroy(self._h), "fdas_frontend_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def convolve(spectrum, zmax, dz, m=0, seg_len=0, precision="fp32", flags=0):
    """One-shot: plan, correlate, destroy. Returns power [nz, nbins] float32."""
    with Plan(zmax, dz, m, seg_len, precision, flags, device=spectrum.device.index) as p:
        return p.convolve(spectrum)
