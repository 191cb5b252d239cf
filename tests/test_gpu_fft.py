"""GPU parity of the standalone batched FFT (fdas_fft_*) against the FP64
DFT of the oracle, through the C ABI.

Bar: max |X - X_ref| <= 1e-5 * max |X_ref| per batch, for every compiled
form (lengths 256 .. 4096; 2, 4, 8 and 16 elements per thread at n = 1024),
both directions, batches that leave the last block of transforms partly
empty, in place, and the empty batch.
"""

import re

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _forms():
    from paper_1711_10855_amd import fdas
    out = []
    for name in fdas.fft_variants():
        m = re.match(r"fft_L(\d+)_e(\d+)_", name)
        out.append((int(m.group(1)), int(m.group(2)), name))
    return out


def _rand(batch, n, seed):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((batch, n)) + 1j * rng.standard_normal((batch, n))).astype(
        np.complex64)


def _err(got, ref):
    return float(np.max(np.abs(got.astype(np.complex128) - ref)) / np.max(np.abs(ref)))


@pytest.fixture
def fft_form(monkeypatch):
    """Force a compiled FFT form (by name) for plans made inside the test."""
    return lambda name: monkeypatch.setenv("FDAS_FFT_VARIANT", name)


@pytest.mark.parametrize("n,e,name", _forms())
@pytest.mark.parametrize("direction", [-1, 1])
def test_every_form_matches_the_dft(gpu, fft_form, n, e, name, direction):
    import torch
    x = _rand(37, n, seed=n + e + direction)
    print(f"fft {name} direction {direction} batch 37", flush=True)
    fft_form(name)
    with gpu.FFT(n, e) as f:
        assert f.kernel == name and f.elems_per_thread == e
        got = f(torch.from_numpy(x).cuda(), direction=direction).cpu().numpy()
    ref = oracle.dft64(x, direction)
    assert _err(got, ref) <= TOL


def test_default_form_in_place_and_small_batches(gpu):
    import torch
    n = 1024
    with gpu.FFT(n) as f:
        for batch in (1, 3, 4, 5):
            x = _rand(batch, n, seed=batch)
            d = torch.from_numpy(x).cuda()
            f(d, out=d)  # in place
            assert _err(d.cpu().numpy(), oracle.dft64(x, -1)) <= TOL
        empty = torch.empty((0, n), dtype=torch.complex64, device="cuda")
        assert f(empty).shape == (0, n)


def test_round_trip_and_impulse(gpu):
    import torch
    n = 2048
    x = np.zeros((2, n), np.complex64)
    x[0, 0] = 1.0
    x[1, 7] = 1.0
    with gpu.FFT(n) as f:
        X = f(torch.from_numpy(x).cuda())
        k = np.arange(n)
        assert np.max(np.abs(X[0].cpu().numpy() - 1.0)) < 1e-6
        ramp = np.exp(-2j * np.pi * 7 * k / n)
        assert np.max(np.abs(X[1].cpu().numpy() - ramp)) < 2e-6
        y = _rand(9, n, seed=11)
        back = f(f(torch.from_numpy(y).cuda(), direction=-1), direction=1).cpu().numpy() / n
        assert np.max(np.abs(back - y)) < 1e-5 * np.max(np.abs(y))


def test_large_batch_sampled(gpu):
    """The Table 1 shape (100,000 transforms of 1024 points), checked on a
    sample of rows with the oracle."""
    import torch
    n, batch = 1024, 100_000
    rng = np.random.default_rng(5)
    xr = rng.standard_normal((batch, 2 * n), dtype=np.float32)
    x = torch.from_numpy(xr).view(torch.complex64).cuda()
    for e in (2, 4, 8, 16):
        with gpu.FFT(n, e) as f:
            X = f(x)
            torch.cuda.synchronize()
            rows = [0, 1, 4095, 50_000, batch - 2, batch - 1]
            got = X[rows].cpu().numpy()
            ref = oracle.dft64(x[rows].cpu().numpy(), -1)
            assert _err(got, ref) <= TOL, e


def test_partly_overlapping_buffers_are_rejected(gpu):
    import torch
    n = 256
    buf = torch.zeros((5, n), dtype=torch.complex64, device="cuda")
    with gpu.FFT(n) as f:
        lib = gpu.load()
        import ctypes as C
        st = lib.fdas_fft_exec(f._h, C.c_void_p(buf.data_ptr()),
                               C.c_void_p(buf[1:].data_ptr()), 4, -1, None)
        assert st == gpu.ERR_INVALID
        f(buf, out=buf)  # in place is fine
