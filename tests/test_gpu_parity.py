"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Bar (plain FP32): max |P - P_ref| <= 1e-4 * max(P_ref), element by element
over the whole plane at sizes the oracle finishes in seconds; at the full
paper-scale workload on oracle-sampled points. FP64 device templates must
match the oracle to 1e-13 absolute; the FP32 bank to FP32 rounding.
"""

import math
import os

import numpy as np
import pytest

import oracle
from paper_1711_10855_amd import synth

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-4


def rel_err(p, ref):
    return float(np.max(np.abs(p.astype(np.float64) - ref)) / np.max(ref))


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).cuda()


@pytest.fixture
def variant_env():
    """Select a compiled kernel variant for plans made inside the test."""
    old = os.environ.get("FDAS_VARIANT")
    yield lambda name: os.environ.__setitem__("FDAS_VARIANT", name)
    if old is None:
        os.environ.pop("FDAS_VARIANT", None)
    else:
        os.environ["FDAS_VARIANT"] = old


def test_device_templates_match_oracle(gpu):
    for zmax, dz, m in [(16, 2, 64), (100, 2, 256), (200, 2, 512), (3, 0.5, 32)]:
        print(f"templates zmax={zmax} dz={dz} m={m}", flush=True)
        dev = gpu.make_templates(zmax, dz, m).cpu().numpy()
        _, ref = oracle.templates64(zmax, dz, m)
        assert np.max(np.abs(dev - ref)) < 1e-13, (zmax, m)


@pytest.mark.parametrize("L,m,zmax", [(256, 64, 16), (2048, 256, 100), (512, 32, 6)])
def test_bank_matches_oracle(gpu, L, m, zmax):
    with gpu.Plan(zmax, 2.0, m, L) as p:
        dev = p.bank().cpu().numpy().astype(np.complex128)
    _, h = oracle.templates64(zmax, 2.0, m)
    ref = oracle.bank_natural(h, m, L)
    assert np.max(np.abs(dev - ref)) <= 1.2e-7 * np.max(np.abs(ref))


@pytest.mark.parametrize("L,m,zmax,flags", [(256, 64, 16, 0), (4096, 512, 200, 0),
                                            (1024, 64, 8, 4)])
def test_make_templates_bank_form(gpu, L, m, zmax, flags):
    """fdas_make_templates with FDAS_FLAG_BANK gives the Fourier-domain bank in
    natural order: the oracle's FP64 bank to FP32 rounding, and exactly the
    values an FP32 plan of the same length stores."""
    bank = gpu.make_bank(zmax, 2.0, m, L, flags).cpu().numpy()
    _, h = oracle.templates64(zmax, 2.0, m, bool(flags & gpu.FLAG_INTERBIN))
    ref = oracle.bank_natural(h, m, L)
    assert bank.shape == ref.shape
    assert np.max(np.abs(bank.astype(np.complex128) - ref)) <= 1.2e-7 * np.max(np.abs(ref))
    with gpu.Plan(zmax, 2.0, m, L, "fp32", flags) as p:
        assert np.array_equal(p.bank().cpu().numpy(), bank)


def test_workload1_full_plane(gpu):
    a, _ = synth.single_series("fp32-small")
    ref = oracle.plane_direct(a, 16.0, 2.0, 64)
    print("fp32-small full plane", flush=True)
    p = gpu.convolve(to_dev(a), 16.0, 2.0, 64, 256).cpu().numpy()
    err = rel_err(p, ref)
    print(f"fp32-small max|dP|/maxP = {err:.3e}")
    assert err <= TOL_FP32


def _variants():
    from paper_1711_10855_amd import fdas
    out = []
    for name in fdas.kernel_variants(0, "fp32"):
        L = int(name.split("_L")[1].split("_")[0])
        out.append((L, name))
    return out


@pytest.mark.parametrize("L,name", _variants())
def test_every_variant_full_plane(gpu, variant_env, L, name):
    # several segments plus a ragged tail, m a quarter of L
    m = max(32, L // 8)
    nbins = 3 * (L - m) + 517
    zmax = 6.0
    a = synth.small_random_spectrum(nbins, seed=L)
    ref = oracle.plane_direct(a, zmax, 2.0, m)
    variant_env(name)
    print(f"variant {name} nbins={nbins} m={m}", flush=True)
    with gpu.Plan(zmax, 2.0, m, L) as p:
        assert p.info.kernel == name
        out = p.convolve(to_dev(a)).cpu().numpy()
    err = rel_err(out, ref)
    print(f"{name}: {err:.3e}")
    assert err <= TOL_FP32


@pytest.mark.parametrize("L,name", _variants())
def test_every_variant_padded_rows_odd_half(gpu, variant_env, L, name):
    """Rows padded by 5 values (row starts not 16-byte aligned), m / 2 odd, a
    ragged last segment: every output lands where the oracle puts it and the
    padding stays untouched."""
    import torch
    m = max(34, L // 8) | 2          # m / 2 odd
    nbins = 2 * (L - m) + 333
    a = synth.small_random_spectrum(nbins, seed=L + 1)
    ref = oracle.plane_direct(a, 4.0, 2.0, m)
    variant_env(name)
    with gpu.Plan(4.0, 2.0, m, L) as p:
        assert p.info.kernel == name
        buf = torch.full((p.nz, nbins + 5), -7.0, dtype=torch.float32, device="cuda")
        p.convolve(to_dev(a), out=buf)
        b = buf.cpu().numpy()
    assert np.all(b[:, nbins:] == -7.0)
    err = rel_err(b[:, :nbins], ref)
    print(f"{name} m={m} padded: {err:.3e}")
    assert err <= TOL_FP32


@pytest.mark.parametrize("nbins", [1, 2, 31, 191, 192, 193, 384, 1000])
def test_edge_lengths(gpu, nbins):
    # U = 192 for L = 256, m = 64: below, at and just past segment boundaries
    a = synth.small_random_spectrum(nbins, seed=nbins)
    ref = oracle.plane_direct(a, 16.0, 2.0, 64)
    out = gpu.convolve(to_dev(a), 16.0, 2.0, 64, 256).cpu().numpy()
    assert rel_err(out, ref) <= TOL_FP32


def test_single_row_zmax0_and_identity(gpu):
    a = synth.small_random_spectrum(5000, seed=3)
    out = gpu.convolve(to_dev(a), 0.0, 2.0, 64, 512).cpu().numpy()
    assert out.shape == (1, 5000)
    ref = np.abs(a.astype(np.complex128)) ** 2
    assert rel_err(out[0], ref) <= TOL_FP32


def test_zero_input_gives_zero_plane(gpu):
    import torch
    z = torch.zeros(4000, dtype=torch.complex64, device="cuda")
    out = gpu.convolve(z, 10.0, 2.0, 32, 256)
    assert float(out.abs().max()) == 0.0


def test_leading_dimension_padding_untouched(gpu):
    import torch
    a = synth.small_random_spectrum(3000, seed=5)
    with gpu.Plan(8.0, 2.0, 64, 256) as p:
        buf = torch.full((p.nz, 3100), -7.0, dtype=torch.float32, device="cuda")
        p.convolve(to_dev(a), out=buf)
        b = buf.cpu().numpy()
    assert np.all(b[:, 3000:] == -7.0)
    ref = oracle.plane_direct(a, 8.0, 2.0, 64)
    assert rel_err(b[:, :3000], ref) <= TOL_FP32


def test_templates_per_block_and_length_invariance(gpu):
    a = synth.small_random_spectrum(20000, seed=8)
    outs = []
    for L in (512, 1024, 4096):
        outs.append(gpu.convolve(to_dev(a), 20.0, 2.0, 128, L).cpu().numpy().astype(np.float64))
    scale = outs[0].max()
    for o in outs[1:]:
        assert np.max(np.abs(o - outs[0])) <= 2e-5 * scale


def test_deterministic(gpu):
    a = to_dev(synth.small_random_spectrum(50000, seed=9))
    with gpu.Plan(30.0, 2.0, 128, 1024) as p:
        o1 = p.convolve(a).cpu().numpy()
        o2 = p.convolve(a).cpu().numpy()
    assert np.array_equal(o1, o2)


def test_conjugate_minus_z_symmetry_on_gpu(gpu):
    a = synth.small_random_spectrum(8000, seed=10)
    with gpu.Plan(24.0, 2.0, 64, 512) as p:
        o = p.convolve(to_dev(a)).cpu().numpy().astype(np.float64)
        oc = p.convolve(to_dev(np.conj(a))).cpu().numpy().astype(np.float64)
    assert np.max(np.abs(o - oc[::-1])) <= 1e-5 * o.max()


def test_workload2_sampled_points(gpu):
    """Paper-scale workload (2^21 bins, nz 101, m 256, L 2048) in the launch
    configuration the benchmark times; checked on sampled points."""
    a, chirps = synth.single_series("fp32-paper")
    print("fp32-paper full-size plane", flush=True)
    p = gpu.convolve(to_dev(a), 100.0, 2.0, 256, 2048).cpu().numpy()
    nz, nbins = p.shape
    assert (nz, nbins) == (101, 1 << 21)
    rng = np.random.default_rng(2)
    iz = rng.integers(0, nz, 6000)
    r = rng.integers(0, nbins, 6000)
    # every row at segment seams, both edges and the injected signals
    U = 2048 - 256
    seams = np.array([s * U + d for s in (0, 1, 2, 500, 1170) for d in (-1, 0, 1) if 0 <= s * U + d < nbins])
    extra_r = np.concatenate([[0, 1, nbins - 1, nbins - 2], seams,
                              [int(round(c.r0)) for c in chirps]])
    iz = np.concatenate([iz, np.repeat(np.arange(nz), extra_r.size)])
    r = np.concatenate([r, np.tile(extra_r, nz)])
    ref = oracle.plane_points(a, 100.0, 2.0, 256, iz, r)
    err = float(np.max(np.abs(p[iz, r].astype(np.float64) - ref))) / float(ref.max())
    print(f"fp32-paper sampled max|dP|/maxP = {err:.3e} over {iz.size} points")
    assert err <= TOL_FP32
    # the injected signals are found where they were put
    for c in chirps:
        row = int(round((c.z0 + 100.0) / 2.0))
        rr = int(round(c.r0))
        win = p[max(0, row - 2):row + 3, rr - 3:rr + 4]
        assert win.max() > 0.3 * c.snr ** 2
