"""Interbinned plane (FDAS_FLAG_INTERBIN: rows 2i at integer r, 2i + 1 at
r + 1/2) on the GPU against the FP64 oracle, through the C ABI."""

import numpy as np
import pytest

import oracle
from paper_1711_10855_amd import synth

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-4
TOL_MIXED = 1e-3


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).cuda()


def rel_err(p, ref):
    return float(np.max(np.abs(p.astype(np.float64) - ref)) / np.max(ref))


def test_device_half_bin_templates_match_oracle(gpu):
    for zmax, m in ((16.0, 64), (100.0, 256)):
        dev = gpu.make_templates(zmax, 2.0, m, gpu.FLAG_INTERBIN).cpu().numpy()
        _, ref = oracle.templates64(zmax, 2.0, m, interbin=True)
        assert dev.shape == ref.shape
        assert np.max(np.abs(dev - ref)) < 1e-13, (zmax, m)


@pytest.mark.parametrize("L,m,nbins,zmax", [(256, 64, 3 * 192 + 77, 16.0),
                                            (2048, 256, 5000, 30.0)])
def test_fp32_interbinned_plane(gpu, L, m, nbins, zmax):
    a = synth.small_random_spectrum(nbins, seed=nbins)
    ref = oracle.plane_direct(a, zmax, 2.0, m, interbin=True)
    with gpu.Plan(zmax, 2.0, m, L, "fp32", gpu.FLAG_INTERBIN) as p:
        assert p.info.nz == ref.shape[0]
        out = p.convolve(to_dev(a)).cpu().numpy()
    with gpu.Plan(zmax, 2.0, m, L, "fp32") as p:
        plain = p.convolve(to_dev(a)).cpu().numpy()
    err = rel_err(out, ref)
    print(f"fp32 interbin L={L} nbins={nbins}: {err:.3e}")
    assert err <= TOL_FP32
    assert np.array_equal(out[0::2], plain)   # integer rows are the plain plane


@pytest.mark.parametrize("prec,flags", [("fp16", 0), ("bf16", 1)])
def test_mixed_interbinned_plane(gpu, prec, flags):
    a = synth.small_random_spectrum(9000, seed=21)
    ref = oracle.plane_direct(a, 10.0, 2.0, 256, interbin=True)
    f = gpu.FLAG_INTERBIN | (gpu.FLAG_SPLIT if flags else 0)
    out = gpu.convolve(to_dev(a), 10.0, 2.0, 256, 4096, prec, f).cpu().numpy()
    err = rel_err(out, ref)
    print(f"{prec} split={flags} interbin: {err:.3e}")
    assert err <= TOL_MIXED


def test_interbinned_batch(gpu):
    import torch
    specs = [(5000, 16.0), (777, 4.0), (3000, 0.0)]
    spectra = [synth.small_random_spectrum(n, seed=600 + k) for k, (n, _) in enumerate(specs)]
    outs = [torch.full((2 * (int(round(z)) + 1), n + 1), -7.0, dtype=torch.float32, device="cuda")
            for n, z in specs]
    with gpu.Plan(16.0, 2.0, 64, 512, "fp32", gpu.FLAG_INTERBIN) as p:
        p.convolve_batch([to_dev(a) for a in spectra], [z for _, z in specs], outs)
        res = [o.cpu().numpy() for o in outs]
    for (n, z), a, o in zip(specs, spectra, res):
        ref = oracle.plane_direct(a, z, 2.0, 64, interbin=True)
        err = rel_err(o[:, :n], ref)
        print(f"interbin batch nbins={n} zmax={z}: {err:.3e}")
        assert err <= TOL_FP32
        assert np.all(o[:, n:] == -7.0)


def test_interbinned_workload_sampled_points(gpu):
    """Paper-scale inputs, interbinned, FP32 and FP16 forms, sampled points."""
    a, chirps = synth.single_series("fp32-paper")
    rng = np.random.default_rng(14)
    for prec, L, tol in (("fp32", 2048, TOL_FP32), ("fp16", 4096, TOL_MIXED)):
        p = gpu.convolve(to_dev(a), 100.0, 2.0, 256, L, prec, gpu.FLAG_INTERBIN).cpu().numpy()
        rows, nbins = p.shape
        assert rows == 202
        iz = rng.integers(0, rows, 3000)
        r = rng.integers(0, nbins, 3000)
        extra = np.array([0, nbins - 1] + [int(c.r0) for c in chirps])
        iz = np.concatenate([iz, np.repeat(np.arange(rows), extra.size)])
        r = np.concatenate([r, np.tile(extra, rows)])
        ref = oracle.plane_points(a, 100.0, 2.0, 256, iz, r, interbin=True)
        err = float(np.max(np.abs(p[iz, r] - ref)) / ref.max())
        print(f"fp32-paper interbin {prec}: {err:.3e}")
        assert err <= tol
        del p
