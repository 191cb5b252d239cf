"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments on the host before any device work (CPU only; no compute calls)."""

import ctypes as C
import os
import re

import pytest

from paper_1711_10855_amd import fdas

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fdas.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fdas_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return fdas.load()


def test_every_declared_symbol_is_exported(lib):
    syms = declared_symbols()
    assert len(syms) >= 11
    for s in syms:
        assert hasattr(lib, s), s
    assert set(fdas.EXPORTS) <= set(syms)


def test_status_strings(lib):
    assert lib.fdas_status_string(0) == b"ok"
    assert lib.fdas_status_string(-1) == b"invalid argument"
    assert lib.fdas_status_string(-2) == b"unsupported configuration"
    assert lib.fdas_status_string(12345) == b"unknown status"


@pytest.mark.parametrize("zmax,dz,nz", [(16, 2, 17), (100, 2, 101), (200, 2, 201), (0, 2, 1),
                                        (3, 2, 4), (1.5, 0.5, 7)])
def test_plane_rows(zmax, dz, nz):
    assert fdas.plane_rows(zmax, dz) == nz


@pytest.mark.parametrize("zmax,dz", [(-1, 2), (3, 4), (10, 0), (10, -2), (float("nan"), 2),
                                     (float("inf"), 2), (1e9, 1e-3)])
def test_plane_rows_invalid(zmax, dz):
    with pytest.raises(fdas.FdasError) as e:
        fdas.plane_rows(zmax, dz)
    assert e.value.status == fdas.ERR_INVALID


def test_resolve_defaults():
    r = fdas.resolve(16, 2)
    assert r.m == 64 and r.seg_len >= 256 and r.seg_len > r.m
    r = fdas.resolve(100, 2)
    assert r.m == 256
    r = fdas.resolve(200, 2)
    assert r.m == 512
    r = fdas.resolve(100, 2, 256, 2048)
    assert (r.m, r.seg_len) == (256, 2048)


@pytest.mark.parametrize("kw,status", [
    (dict(m=7), fdas.ERR_INVALID),                  # odd m
    (dict(m=-4), fdas.ERR_INVALID),
    (dict(m=256, seg_len=256), fdas.ERR_INVALID),   # L <= m
    (dict(m=64, seg_len=300), fdas.ERR_UNSUPPORTED),  # not a power of two
    (dict(m=64, seg_len=128), fdas.ERR_UNSUPPORTED),  # below the compiled set
    (dict(m=64, seg_len=32768), fdas.ERR_UNSUPPORTED),
    (dict(precision=7), fdas.ERR_INVALID),
    (dict(flags=0x80), fdas.ERR_INVALID),
    (dict(flags=fdas.FLAG_SPLIT), fdas.ERR_INVALID),  # split is for the mixed precisions
])
def test_resolve_rejects(kw, status):
    with pytest.raises(fdas.FdasError) as e:
        fdas.resolve(16, 2, **kw)
    assert e.value.status == status
    assert fdas.last_error() != ""


def test_interbin_doubles_the_rows(lib):
    assert fdas.plane_rows(16, 2) == 17
    assert fdas.plane_rows(16, 2, fdas.FLAG_INTERBIN) == 34
    r = fdas.resolve(16, 2, 64, 256, "fp32", fdas.FLAG_INTERBIN)
    assert r.flags == fdas.FLAG_INTERBIN
    p = fdas.params(16, 2, 64, 0, "fp32", fdas.FLAG_INTERBIN)
    n = C.c_size_t(0)
    assert lib.fdas_make_templates(C.byref(p), None, C.byref(n), None) == 0
    assert n.value == 34 * 65 * 16


def test_template_size_query_needs_no_device(lib):
    p = fdas.params(16, 2, 64)
    n = C.c_size_t(0)
    assert lib.fdas_make_templates(C.byref(p), None, C.byref(n), None) == 0
    assert n.value == 17 * 65 * 16
    assert lib.fdas_make_templates(C.byref(p), None, None, None) == fdas.ERR_INVALID
    small = C.c_size_t(10)
    # a too-small buffer is rejected before any launch (the pointer is never used)
    assert lib.fdas_make_templates(C.byref(p), C.c_void_p(0x1000), C.byref(small), None) == fdas.ERR_INVALID
    assert small.value == 17 * 65 * 16


def test_null_and_bad_arguments(lib):
    assert lib.fdas_destroy(None) == 0
    assert lib.fdas_plan(None, None, 0, None) == fdas.ERR_INVALID
    h = C.c_void_p()
    bad = fdas.params(3, 4)
    assert lib.fdas_plan(C.byref(h), C.byref(bad), 0, None) == fdas.ERR_INVALID
    assert h.value is None
    assert lib.fdas_plan(C.byref(h), C.byref(fdas.params(16, 2)), -1, None) == fdas.ERR_INVALID
    assert lib.fdas_convolve(None, C.c_void_p(8), 10, C.c_void_p(8), 10, None) == fdas.ERR_INVALID
    assert lib.fdas_convolve_batch(None, None, 0, None) == fdas.ERR_INVALID
    assert lib.fdas_plan_get_info(None, None) == fdas.ERR_INVALID
    assert lib.fdas_plan_bank(None, None, 0, None) == fdas.ERR_INVALID


def test_kernel_variant_listing():
    names = fdas.kernel_variants()
    assert len(names) >= 10
    for L in (256, 512, 1024, 2048, 4096, 8192, 16384):
        sub = fdas.kernel_variants(L, "fp32")
        assert sub and all(f"_L{L}_" in n for n in sub)
    assert fdas.load().fdas_kernel_variants(-1, 0, None, 0) == fdas.ERR_INVALID
    for prec in ("fp16", "bf16"):
        sub = fdas.kernel_variants(4096, prec)
        assert any("_split" in n for n in sub) and any("_split" not in n for n in sub)
    r = fdas.resolve(100, 2, 256, 0, "bf16", fdas.FLAG_SPLIT)
    assert (r.seg_len, r.flags) == (4096, fdas.FLAG_SPLIT)


def test_matrix_core_lengths():
    """The matrix-core kernels exist at 4096 (all forms) and 2048 (FP16 and
    BF16 without the split form); other lengths are refused on the host."""
    for prec in ("fp16", "bf16"):
        assert fdas.kernel_variants(2048, prec) == [f"{prec}_L2048_mfma_w16"]
        assert fdas.resolve(100, 2, 256, 2048, prec).seg_len == 2048
        with pytest.raises(fdas.FdasError) as e:
            fdas.resolve(100, 2, 256, 2048, prec, fdas.FLAG_SPLIT)
        assert e.value.status == fdas.ERR_UNSUPPORTED and "split" in fdas.last_error()
        for L in (1024, 8192):
            with pytest.raises(fdas.FdasError) as e:
                fdas.resolve(100, 2, 256, L, prec)
            assert e.value.status == fdas.ERR_UNSUPPORTED


def test_fft_variant_listing():
    names = fdas.fft_variants()
    assert len(names) >= 10
    assert [n for n in names if n.startswith("fft_L1024_")] == fdas.fft_variants(1024)
    assert {int(v.split("_e")[1].split("_")[0]) for v in fdas.fft_variants(1024)} == {2, 4, 8, 16}
    assert fdas.fft_variants(3) == []


@pytest.mark.parametrize("n,elems,status", [(1000, 0, fdas.ERR_INVALID), (1, 0, fdas.ERR_INVALID),
                                            (1024, 3, fdas.ERR_INVALID),
                                            (1024, -2, fdas.ERR_INVALID),
                                            (1 << 20, 0, fdas.ERR_UNSUPPORTED),
                                            (1024, 32, fdas.ERR_UNSUPPORTED)])
def test_fft_plan_rejects_on_host(lib, n, elems, status):
    h = C.c_void_p(1234)
    assert lib.fdas_fft_plan(C.byref(h), n, elems, 0, None) == status
    assert not h.value  # cleared on failure
    assert lib.fdas_fft_plan(None, 1024, 0, 0, None) == fdas.ERR_INVALID
    assert lib.fdas_fft_plan(C.byref(h), 1024, 0, -1, None) == fdas.ERR_INVALID


def test_fft_exec_and_destroy_reject_null_plan(lib):
    assert lib.fdas_fft_exec(None, None, None, 1, -1, None) == fdas.ERR_INVALID
    assert lib.fdas_fft_destroy(None) == fdas.OK
    assert lib.fdas_fft_get_info(None, None) == fdas.ERR_INVALID


@pytest.mark.parametrize("n", [0, 64, 100, 1000, 1 << 26, -128])
def test_frontend_plan_rejects_on_host(lib, n):
    h = C.c_void_p(1234)
    assert lib.fdas_frontend_plan(C.byref(h), n, 0, None) == fdas.ERR_INVALID
    assert not h.value


def test_frontend_exec_and_destroy_reject_null_plan(lib):
    assert lib.fdas_frontend_plan(None, 1024, 0, None) == fdas.ERR_INVALID
    assert lib.fdas_frontend_plan(C.byref(C.c_void_p()), 1024, -1, None) == fdas.ERR_INVALID
    assert lib.fdas_frontend_exec(None, None, None, None, None) == fdas.ERR_INVALID
    assert lib.fdas_frontend_destroy(None) == fdas.OK


def test_binding_rejects_output_buffers_that_do_not_fit():
    """The binding checks output tensors before their pointers reach a kernel
    (shape, dtype, row stride); exercised on host tensors."""
    import torch
    dev = torch.device("cpu")
    ok = torch.empty((5, 120), dtype=torch.float32)
    fdas._plane_ok(ok, 5, 100, 120, dev)
    fdas._plane_ok(ok[:, :100], 5, 100, 120, dev)          # a column slice keeps stride 120
    for bad, ld in ((torch.empty((4, 120)), 120),              # too few rows
                    (torch.empty((5, 90)), 90),                # rows too short
                    (torch.empty((5, 120), dtype=torch.float64), 120),
                    (torch.empty((120, 5)).t(), 120),          # column stride != 1
                    (ok, 100)):                                 # stride differs from ld
        with pytest.raises((TypeError, ValueError)):
            fdas._plane_ok(bad, 5, 100, ld, dev)


def test_noalloc_batch_rejects_on_host(lib):
    """The allocation-free batch checks its arguments, and its series limit,
    before anything touches the plan or the device (the plan pointer below is
    never dereferenced)."""
    assert lib.fdas_convolve_batch_noalloc(None, None, 0, None) == fdas.ERR_INVALID
    n = 4097
    arr = (fdas.Series * n)()
    for i in range(n):
        arr[i] = fdas.Series(C.c_void_p(0x1000), 10, 0.0, C.c_void_p(0x2000), 10)
    fake = C.c_void_p(0x3000)
    assert lib.fdas_convolve_batch_noalloc(fake, arr, n, None) == fdas.ERR_INVALID
    assert "4096" in fdas.last_error()
    arr[5] = fdas.Series(C.c_void_p(0x1004), 10, 0.0, C.c_void_p(0x2000), 10)  # misaligned
    assert lib.fdas_convolve_batch_noalloc(fake, arr, 10, None) == fdas.ERR_INVALID
    assert "series 5" in fdas.last_error()


def test_peaks_workspace_and_host_checks(lib):
    assert lib.fdas_peaks_workspace_bytes(-1) == 0
    assert lib.fdas_peaks_workspace_bytes((1 << 30) + 1) == 0
    assert lib.fdas_peaks_workspace_bytes(0) == 64 * 12            # the smallest table
    assert lib.fdas_peaks_workspace_bytes(1000) == 1000 * 16 + 2048 * 12
    assert lib.fdas_peaks_workspace_bytes(1024) == 1024 * 16 + 2048 * 12
    assert lib.fdas_convolve_peaks(None, C.c_void_p(8), 10, 1.0, C.c_void_p(16), 1 << 20, 100,
                                   C.c_void_p(16), 10, C.c_void_p(8), None) == fdas.ERR_INVALID


def test_bank_size_query_needs_no_device(lib):
    """fdas_make_templates with FDAS_FLAG_BANK: complex64 [nz][L]; the segment
    length must be known (not left to the autotuner)."""
    n = C.c_size_t(0)
    p = fdas.params(16, 2, 64, 256, "fp32", fdas.FLAG_BANK)
    assert lib.fdas_make_templates(C.byref(p), None, C.byref(n), None) == 0
    assert n.value == 17 * 256 * 8
    p = fdas.params(16, 2, 64, 0, "fp32", fdas.FLAG_BANK | fdas.FLAG_INTERBIN)
    assert lib.fdas_make_templates(C.byref(p), None, C.byref(n), None) == 0
    assert n.value == 34 * fdas.resolve(16, 2, 64).seg_len * 8
    p = fdas.params(16, 2, 64, 0, "fp32", fdas.FLAG_BANK | fdas.FLAG_AUTOTUNE)
    assert lib.fdas_make_templates(C.byref(p), None, C.byref(n), None) == fdas.ERR_INVALID
