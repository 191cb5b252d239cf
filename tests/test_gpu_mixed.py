"""Mixed-precision path (16-bit storage, MFMA DFT stages, FP32 accumulation;
optionally hi + lo split products) against the FP64 oracle through the C ABI.
Bar: max |P - P_ref| <= 1e-3 * max(P_ref); the measured error is printed for
every case."""

import numpy as np
import pytest

import oracle
from paper_1711_10855_amd import synth

pytestmark = pytest.mark.gpu

TOL_MIXED = 1e-3


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).cuda()


def rel_err(p, ref):
    return float(np.max(np.abs(p.astype(np.float64) - ref)) / np.max(ref))


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_mixed_bank_matches_oracle(gpu, prec):
    with gpu.Plan(100.0, 2.0, 256, 4096, prec) as p:
        dev = p.bank().cpu().numpy().astype(np.complex128)
    _, h = oracle.templates64(100.0, 2.0, 256)
    ref = oracle.bank_natural(h, 256, 4096)
    err = float(np.max(np.abs(dev - ref)) / np.max(np.abs(ref)))
    print(f"{prec} bank max rel err {err:.2e}")
    assert err <= (1e-3 if prec == "fp16" else 8e-3)


@pytest.mark.parametrize("prec,nbins,zmax,m", [
    ("fp16", 3 * 3840 + 517, 10.0, 256),
    ("fp16", 1000, 6.0, 256),
    ("fp16", 20000, 30.0, 512),
    ("fp16", 9000, 12.0, 100),     # m/2 = 50: every segment takes the per-value stores
])
def test_mixed_full_plane(gpu, prec, nbins, zmax, m):
    a = synth.small_random_spectrum(nbins, seed=nbins)
    ref = oracle.plane_direct(a, zmax, 2.0, m)
    print(f"{prec} nbins={nbins} zmax={zmax} m={m}", flush=True)
    out = gpu.convolve(to_dev(a), zmax, 2.0, m, 4096, prec).cpu().numpy()
    err = rel_err(out, ref)
    print(f"{prec} nbins={nbins}: max|dP|/maxP = {err:.3e}")
    assert err <= TOL_MIXED


def test_mixed_bf16_error_is_reported(gpu):
    """BF16 storage without split products: 8 mantissa bits. The measured
    error is recorded; the 1e-3 bar applies to the split form."""
    a = synth.small_random_spectrum(12000, seed=77)
    ref = oracle.plane_direct(a, 10.0, 2.0, 256)
    out = gpu.convolve(to_dev(a), 10.0, 2.0, 256, 4096, "bf16").cpu().numpy()
    err = rel_err(out, ref)
    print(f"bf16 (no split) max|dP|/maxP = {err:.3e}")
    assert err <= 2e-2


def test_mixed_zero_and_scaled_inputs(gpu):
    import torch
    z = torch.zeros(9000, dtype=torch.complex64, device="cuda")
    out = gpu.convolve(z, 10.0, 2.0, 256, 4096, "fp16")
    assert float(out.abs().max()) == 0.0
    # per-segment power-of-two scaling: results scale exactly with the input
    a = synth.small_random_spectrum(9000, seed=5)
    p1 = gpu.convolve(to_dev(a), 10.0, 2.0, 256, 4096, "fp16").cpu().numpy()
    p2 = gpu.convolve(to_dev(a * 1024.0), 10.0, 2.0, 256, 4096, "fp16").cpu().numpy()
    assert np.array_equal(p1 * (1024.0 ** 2), p2)
    p3 = gpu.convolve(to_dev(a * 1e-12), 10.0, 2.0, 256, 4096, "fp16").cpu().numpy()
    ref = oracle.plane_direct(a.astype(np.complex128) * 1e-12, 10.0, 2.0, 256)
    assert rel_err(p3, ref) <= TOL_MIXED


def test_mixed_workload_sampled_points(gpu):
    """Paper-scale inputs (2^21 bins, nz 101, m 256) through the FP16 MFMA path."""
    a, chirps = synth.single_series("fp32-paper")
    p = gpu.convolve(to_dev(a), 100.0, 2.0, 256, 4096, "fp16").cpu().numpy()
    nz, nbins = p.shape
    rng = np.random.default_rng(12)
    iz = rng.integers(0, nz, 5000)
    r = rng.integers(0, nbins, 5000)
    extra = np.array([0, 1, nbins - 1] + [int(round(c.r0)) for c in chirps])
    iz = np.concatenate([iz, np.repeat(np.arange(nz), extra.size)])
    r = np.concatenate([r, np.tile(extra, nz)])
    ref = oracle.plane_points(a, 100.0, 2.0, 256, iz, r)
    err = float(np.max(np.abs(p[iz, r] - ref)) / ref.max())
    print(f"mixed-paper fp16 sampled max|dP|/maxP = {err:.3e}")
    assert err <= TOL_MIXED


@pytest.mark.parametrize("persistent", ["0", "1"])
def test_mixed_batch_matches_oracle(gpu, monkeypatch, persistent):
    """Flat item grid, and persistent blocks taking items from a counter."""
    import torch
    monkeypatch.setenv("FDAS_BATCH_PERSISTENT", persistent)
    specs = [(9000, 16.0), (1, 4.0), (4100, 0.0), (20000, 10.0), (3841, 16.0)]
    spectra = [synth.small_random_spectrum(n, seed=300 + k) for k, (n, _) in enumerate(specs)]
    outs = [torch.full((int(round(z)) + 1, n + 2), -5.0, dtype=torch.float32, device="cuda")
            for n, z in specs]
    with gpu.Plan(16.0, 2.0, 256, 4096, "fp16") as p:
        p.convolve_batch([to_dev(a) for a in spectra], [z for _, z in specs], outs)
        res = [o.cpu().numpy() for o in outs]
    for (n, z), a, o in zip(specs, spectra, res):
        ref = oracle.plane_direct(a, z, 2.0, 256)
        err = rel_err(o[:, :n], ref)
        print(f"fp16 batch nbins={n} zmax={z} persistent={persistent}: {err:.3e}")
        assert err <= TOL_MIXED
        assert np.all(o[:, n:] == -5.0)


def _mixed_variants():
    from paper_1711_10855_amd import fdas
    return [n for n in fdas.kernel_variants(4096, "fp16")] + \
        [n for n in fdas.kernel_variants(4096, "bf16")]


@pytest.mark.parametrize("name", _mixed_variants())
def test_every_mixed_variant(gpu, name, monkeypatch):
    prec = "bf16" if name.startswith("bf16") else "fp16"
    split = "_split" in name
    monkeypatch.setenv("FDAS_VARIANT", name)
    a = synth.small_random_spectrum(2 * 3840 + 999, seed=31)
    ref = oracle.plane_direct(a, 8.0, 2.0, 256)
    with gpu.Plan(8.0, 2.0, 256, 4096, prec, gpu.FLAG_SPLIT if split else 0) as p:
        assert p.info.kernel == name
        out = p.convolve(to_dev(a)).cpu().numpy()
    err = rel_err(out, ref)
    print(f"{name}: {err:.3e}")
    assert err <= (TOL_MIXED if (prec == "fp16" or split) else 2e-2)


@pytest.mark.parametrize("name", _mixed_variants())
def test_every_mixed_variant_batch(gpu, name, monkeypatch):
    """Each variant in the persistent batched form, with rows padded to a
    multiple of 4 (16-byte stores on whole segments, per-value stores on the
    ragged last one) and untouched padding."""
    import torch
    prec = "bf16" if name.startswith("bf16") else "fp16"
    split = "_split" in name
    monkeypatch.setenv("FDAS_VARIANT", name)
    monkeypatch.setenv("FDAS_BATCH_PERSISTENT", "1")
    specs = [(9000, 16.0), (4100, 0.0), (20000, 10.0)]
    spectra = [synth.small_random_spectrum(n, seed=700 + k) for k, (n, _) in enumerate(specs)]
    outs = [torch.full((int(round(z)) + 1, (n + 3) // 4 * 4 + 4), -5.0, dtype=torch.float32,
                       device="cuda") for n, z in specs]
    with gpu.Plan(16.0, 2.0, 256, 4096, prec, gpu.FLAG_SPLIT if split else 0) as p:
        assert p.info.kernel == name
        p.convolve_batch([to_dev(a) for a in spectra], [z for _, z in specs], outs)
        res = [o.cpu().numpy() for o in outs]
    for (n, z), a, o in zip(specs, spectra, res):
        err = rel_err(o[:, :n], oracle.plane_direct(a, z, 2.0, 256))
        print(f"{name} batch nbins={n} zmax={z}: {err:.3e}")
        assert err <= (TOL_MIXED if (prec == "fp16" or split) else 2e-2)
        assert np.all(o[:, n:] == -5.0)


@pytest.mark.parametrize("name", _mixed_variants())
def test_every_mixed_variant_odd_half(gpu, name, monkeypatch):
    """m = 100: m / 2 is not a multiple of 4, so every segment stores value by
    value."""
    prec = "bf16" if name.startswith("bf16") else "fp16"
    split = "_split" in name
    monkeypatch.setenv("FDAS_VARIANT", name)
    a = synth.small_random_spectrum(9001, seed=37)
    with gpu.Plan(6.0, 2.0, 100, 4096, prec, gpu.FLAG_SPLIT if split else 0) as p:
        assert p.info.kernel == name
        out = p.convolve(to_dev(a)).cpu().numpy()
    err = rel_err(out, oracle.plane_direct(a, 6.0, 2.0, 100))
    print(f"{name} m=100: {err:.3e}")
    assert err <= (TOL_MIXED if (prec == "fp16" or split) else 2e-2)


# ---- hi + lo split products (FDAS_FLAG_SPLIT) -------------------------------

@pytest.mark.parametrize("prec,tol", [("fp16", 1e-7), ("bf16", 1e-7)])
def test_split_bank_matches_oracle(gpu, prec, tol):
    """The split forms keep the bank in FP32: within FP32 rounding of the
    oracle's FP64 bank (relative to its largest value)."""
    with gpu.Plan(100.0, 2.0, 256, 4096, prec, gpu.FLAG_SPLIT) as p:
        assert "_split" in p.info.kernel
        dev = p.bank().cpu().numpy().astype(np.complex128)
    _, h = oracle.templates64(100.0, 2.0, 256)
    ref = oracle.bank_natural(h, 256, 4096)
    err = float(np.max(np.abs(dev - ref)) / np.max(np.abs(ref)))
    print(f"{prec} split bank max rel err {err:.2e}")
    assert err <= tol


@pytest.mark.parametrize("prec,nbins,zmax,m", [
    ("fp16", 3 * 3840 + 517, 10.0, 256),
    ("bf16", 3 * 3840 + 517, 10.0, 256),
    ("bf16", 20000, 30.0, 512),
    ("bf16", 1000, 6.0, 256),
])
def test_split_full_plane(gpu, prec, nbins, zmax, m):
    a = synth.small_random_spectrum(nbins, seed=nbins + 1)
    ref = oracle.plane_direct(a, zmax, 2.0, m)
    print(f"{prec} split nbins={nbins} zmax={zmax} m={m}", flush=True)
    out = gpu.convolve(to_dev(a), zmax, 2.0, m, 4096, prec, gpu.FLAG_SPLIT).cpu().numpy()
    err = rel_err(out, ref)
    print(f"{prec} split nbins={nbins}: max|dP|/maxP = {err:.3e}")
    assert err <= TOL_MIXED


def test_split_workload_sampled_points(gpu):
    """Paper-scale inputs through the BF16 split path."""
    a, chirps = synth.single_series("fp32-paper")
    p = gpu.convolve(to_dev(a), 100.0, 2.0, 256, 4096, "bf16", gpu.FLAG_SPLIT).cpu().numpy()
    nz, nbins = p.shape
    rng = np.random.default_rng(13)
    iz = rng.integers(0, nz, 4000)
    r = rng.integers(0, nbins, 4000)
    extra = np.array([0, 1, nbins - 1] + [int(round(c.r0)) for c in chirps])
    iz = np.concatenate([iz, np.repeat(np.arange(nz), extra.size)])
    r = np.concatenate([r, np.tile(extra, nz)])
    ref = oracle.plane_points(a, 100.0, 2.0, 256, iz, r)
    err = float(np.max(np.abs(p[iz, r] - ref)) / ref.max())
    print(f"mixed-paper bf16 split sampled max|dP|/maxP = {err:.3e}")
    assert err <= TOL_MIXED


def test_split_batch_matches_oracle(gpu):
    import torch
    specs = [(9000, 16.0), (1, 4.0), (4101, 0.0), (20000, 10.0)]
    spectra = [synth.small_random_spectrum(n, seed=400 + k) for k, (n, _) in enumerate(specs)]
    outs = [torch.full((int(round(z)) + 1, n + 3), -5.0, dtype=torch.float32, device="cuda")
            for n, z in specs]
    with gpu.Plan(16.0, 2.0, 256, 4096, "bf16", gpu.FLAG_SPLIT) as p:
        p.convolve_batch([to_dev(a) for a in spectra], [z for _, z in specs], outs)
        res = [o.cpu().numpy() for o in outs]
    for (n, z), a, o in zip(specs, spectra, res):
        ref = oracle.plane_direct(a, z, 2.0, 256)
        err = rel_err(o[:, :n], ref)
        print(f"bf16 split batch nbins={n} zmax={z}: {err:.3e}")
        assert err <= TOL_MIXED
        assert np.all(o[:, n:] == -5.0)


@pytest.mark.parametrize("prec,split", [("bf16", True), ("bf16", False), ("fp16", True)])
def test_zero_and_scaled_inputs_other_forms(gpu, prec, split):
    """Zero input gives a zero plane; a power-of-two input scale scales the
    powers exactly (FP16 through its per-segment scale, BF16 at 4096 points
    through its fixed one, exact while no value leaves FP32's normal range);
    inputs of magnitude 1e-12 and 1e+12 stay within the bar."""
    flags = gpu.FLAG_SPLIT if split else 0
    tol = TOL_MIXED if (prec == "fp16" or split) else 2e-2
    import torch
    z = torch.zeros(9000, dtype=torch.complex64, device="cuda")
    out = gpu.convolve(z, 10.0, 2.0, 256, 4096, prec, flags)
    assert float(out.abs().max()) == 0.0
    a = synth.small_random_spectrum(9000, seed=6)
    p1 = gpu.convolve(to_dev(a), 10.0, 2.0, 256, 4096, prec, flags).cpu().numpy()
    p2 = gpu.convolve(to_dev(a * 1024.0), 10.0, 2.0, 256, 4096, prec, flags).cpu().numpy()
    assert np.array_equal(p1 * (1024.0 ** 2), p2)
    for s in (1e-12, 1e12):
        p3 = gpu.convolve(to_dev(a * s), 10.0, 2.0, 256, 4096, prec, flags).cpu().numpy()
        ref = oracle.plane_direct(a.astype(np.complex128) * s, 10.0, 2.0, 256)
        err = rel_err(p3, ref)
        print(f"{prec} split={split} scale {s:g}: {err:.3e}")
        assert err <= tol
