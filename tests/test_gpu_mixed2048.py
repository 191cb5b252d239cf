"""The 2048-point matrix-core kernel (FP16 / BF16 storage, radix-8 and two
radix-16 MFMA stages, FP32 accumulation) against the FP64 oracle through the
C ABI. Bar: max |P - P_ref| <= 1e-3 * max(P_ref) for FP16; BF16 (8 mantissa
bits, no split form at this length) is held to 2e-2 and its error printed."""

import numpy as np
import pytest

import oracle
from paper_1711_10855_amd import synth

pytestmark = pytest.mark.gpu

L = 2048
TOL = {"fp16": 1e-3, "bf16": 2e-2}


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).cuda()


def rel_err(p, ref):
    return float(np.max(np.abs(p.astype(np.float64) - ref)) / np.max(ref))


@pytest.mark.parametrize("prec,tol", [("fp16", 1e-3), ("bf16", 8e-3)])
def test_bank_matches_oracle(gpu, prec, tol):
    with gpu.Plan(100.0, 2.0, 256, L, prec) as p:
        assert p.info.kernel == f"{prec}_L2048_mfma_w16"
        dev = p.bank().cpu().numpy().astype(np.complex128)
    _, h = oracle.templates64(100.0, 2.0, 256)
    ref = oracle.bank_natural(h, 256, L)
    err = float(np.max(np.abs(dev - ref)) / np.max(np.abs(ref)))
    print(f"{prec} L2048 bank max rel err {err:.2e}")
    assert err <= tol


@pytest.mark.parametrize("prec,nbins,zmax,m", [
    ("fp16", 3 * 1792 + 517, 10.0, 256),     # three full segments and a ragged tail
    ("fp16", 700, 6.0, 256),                 # less than one segment
    ("fp16", 20000, 30.0, 1024),             # widest filter: half of each segment kept
    ("fp16", 9001, 16.0, 64),
    ("fp16", 7000, 12.0, 100),               # m/2 = 50: every segment takes the per-value stores
    ("bf16", 3 * 1792 + 517, 10.0, 256),
])
def test_full_plane(gpu, prec, nbins, zmax, m):
    a = synth.small_random_spectrum(nbins, seed=nbins + 7)
    ref = oracle.plane_direct(a, zmax, 2.0, m)
    print(f"{prec} L2048 nbins={nbins} zmax={zmax} m={m}", flush=True)
    out = gpu.convolve(to_dev(a), zmax, 2.0, m, L, prec).cpu().numpy()
    err = rel_err(out, ref)
    print(f"  max|dP|/maxP = {err:.3e}")
    assert err <= TOL[prec]


def test_interbin_plane(gpu):
    a = synth.small_random_spectrum(6000, seed=11)
    ref = oracle.plane_direct(a, 8.0, 2.0, 128, True)
    out = gpu.convolve(to_dev(a), 8.0, 2.0, 128, L, "fp16", gpu.FLAG_INTERBIN).cpu().numpy()
    err = rel_err(out, ref)
    print(f"fp16 L2048 interbin: {err:.3e}")
    assert err <= TOL["fp16"]


def test_zero_and_scaled_inputs(gpu):
    import torch
    z = torch.zeros(5000, dtype=torch.complex64, device="cuda")
    assert float(gpu.convolve(z, 10.0, 2.0, 256, L, "fp16").abs().max()) == 0.0
    # the per-segment power-of-two scale makes results scale exactly
    a = synth.small_random_spectrum(5000, seed=6)
    p1 = gpu.convolve(to_dev(a), 10.0, 2.0, 256, L, "fp16").cpu().numpy()
    p2 = gpu.convolve(to_dev(a * 1024.0), 10.0, 2.0, 256, L, "fp16").cpu().numpy()
    assert np.array_equal(p1 * (1024.0 ** 2), p2)


def test_workload_sampled_points(gpu):
    """Paper-scale inputs (2^21 bins, 101 templates, m 256) at L = 2048."""
    a, chirps = synth.single_series("fp32-paper")
    p = gpu.convolve(to_dev(a), 100.0, 2.0, 256, L, "fp16").cpu().numpy()
    nz, nbins = p.shape
    rng = np.random.default_rng(14)
    iz = rng.integers(0, nz, 4000)
    r = rng.integers(0, nbins, 4000)
    extra = np.array([0, 1, nbins - 1] + [int(round(c.r0)) for c in chirps])
    iz = np.concatenate([iz, np.repeat(np.arange(nz), extra.size)])
    r = np.concatenate([r, np.tile(extra, nz)])
    ref = oracle.plane_points(a, 100.0, 2.0, 256, iz, r)
    err = float(np.max(np.abs(p[iz, r] - ref)) / ref.max())
    print(f"fp32-paper inputs, fp16 L2048 sampled max|dP|/maxP = {err:.3e}")
    assert err <= TOL["fp16"]


@pytest.mark.parametrize("persistent", ["0", "1"])
@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_batch_matches_oracle(gpu, monkeypatch, persistent, prec):
    import torch
    monkeypatch.setenv("FDAS_BATCH_PERSISTENT", persistent)
    specs = [(9000, 16.0), (1, 4.0), (1793, 0.0), (20000, 10.0), (1791, 16.0)]
    spectra = [synth.small_random_spectrum(n, seed=500 + k) for k, (n, _) in enumerate(specs)]
    outs = [torch.full((int(round(z)) + 1, n + 2), -5.0, dtype=torch.float32, device="cuda")
            for n, z in specs]
    with gpu.Plan(16.0, 2.0, 256, L, prec) as p:
        p.convolve_batch([to_dev(a) for a in spectra], [z for _, z in specs], outs)
        res = [o.cpu().numpy() for o in outs]
    for (n, z), a, o in zip(specs, spectra, res):
        ref = oracle.plane_direct(a, z, 2.0, 256)
        err = rel_err(o[:, :n], ref)
        print(f"{prec} L2048 batch nbins={n} zmax={z} persistent={persistent}: {err:.3e}")
        assert err <= TOL[prec]
        assert np.all(o[:, n:] == -5.0)


def test_candidates_equal_the_plane(gpu):
    """The detection epilogue of this kernel reports exactly the points of
    its own stored plane at or above the threshold."""
    a = synth.small_random_spectrum(12000, seed=41)
    a[5000:5004] *= 6.0
    with gpu.Plan(16.0, 2.0, 256, L, "fp16") as p:
        plane = p.convolve(to_dev(a)).cpu().numpy()
        rec, cnt = p.candidates(to_dev(a), 4.0, 1 << 18)
        row, r, pw = gpu.decode_candidates(rec, cnt)
    want = set(zip(*np.nonzero(plane >= 4.0)))
    got = set(zip(row.tolist(), r.tolist()))
    assert int(cnt.cpu()[0]) == len(want) == len(got) and got == want
    assert np.array_equal(pw, plane[row, r])


def test_autotuner_may_choose_this_length(gpu, tmp_path, monkeypatch):
    """With no segment length fixed, the FP16 autotuner times both compiled
    matrix-core lengths that keep at least half of each segment."""
    monkeypatch.setenv("FDAS_TUNE_CACHE", str(tmp_path / "tune.txt"))
    a = synth.small_random_spectrum(50000, seed=3)
    with gpu.Plan(16.0, 2.0, 256, 0, "fp16", gpu.FLAG_AUTOTUNE) as p:
        assert p.info.seg_len in (2048, 4096)
        out = p.convolve(to_dev(a)).cpu().numpy()
        print(f"autotuned fp16: {p.info.kernel}")
    assert rel_err(out, oracle.plane_direct(a, 16.0, 2.0, 256)) <= TOL["fp16"]
    lines = (tmp_path / "tune.txt").read_text().splitlines()
    assert lines
