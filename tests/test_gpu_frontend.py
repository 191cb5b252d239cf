"""GPU parity of the device front end (fdas_frontend_*) against the FP64
oracle ``spectrum64``, through the C ABI; and the whole device pipeline
(series -> spectrum -> plane) against the oracle's plane.

Bar: spectrum max |A - A_ref| <= 1e-5 max |A_ref| and <= 1e-4 absolute
(unit noise power), median within 1e-5 relative, for one-transform lengths
and four-step lengths up to the largest supported series (2^25 samples, a
4096 x 4096 split).
"""

import numpy as np
import pytest

import oracle
from paper_1711_10855_amd import synth

pytestmark = pytest.mark.gpu


def _series(n, seed, chirp=True):
    rng = np.random.default_rng(seed)
    ch = [synth.Chirp(0.3 * n / 2 + 0.25, 3.0, 25.0, 0.7)] if chirp else []
    return synth.make_series(n, ch, rng).astype(np.float32)


def _check(gpu, x):
    import torch
    n = x.size
    a_ref, med_ref = oracle.spectrum64(x.astype(np.float64))
    stats = torch.zeros(2, dtype=torch.float32, device="cuda")
    with gpu.FrontEnd(n) as fe:
        a = fe(torch.from_numpy(x).cuda(), stats=stats).cpu().numpy()
    st = stats.cpu().numpy()
    err = np.max(np.abs(a.astype(np.complex128) - a_ref))
    assert err <= 1e-5 * np.max(np.abs(a_ref)) and err <= 1e-4, (n, err)
    assert abs(st[1] - med_ref) <= 1e-5 * med_ref
    assert a[0] == 0
    return a


@pytest.mark.parametrize("n", [128, 1024, 8192, 1 << 14, 1 << 16, 1 << 19, 1 << 22, 1 << 25])
def test_spectrum_matches_oracle(gpu, n):
    print(f"front end n={n}", flush=True)
    _check(gpu, _series(n, seed=n))


def test_paper_workload_series(gpu):
    x, _ = synth.single_series_samples("fp32-paper")
    print("front end fp32-paper series", flush=True)
    _check(gpu, x.astype(np.float32))


def test_in_place_and_repeat(gpu):
    import torch
    n = 1 << 16
    x = _series(n, seed=3)
    a_ref, _ = oracle.spectrum64(x.astype(np.float64))
    with gpu.FrontEnd(n) as fe:
        for _ in range(2):
            buf = torch.from_numpy(x).cuda()
            out = buf.view(torch.complex64)          # the series' own buffer
            fe(buf, out=out)
            a = out.cpu().numpy()
            assert np.max(np.abs(a - a_ref)) <= 1e-5 * np.max(np.abs(a_ref))


def test_zero_series_is_left_unscaled(gpu):
    import torch
    n = 4096
    stats = torch.full((2,), -1.0, dtype=torch.float32, device="cuda")
    with gpu.FrontEnd(n) as fe:
        a = fe(torch.zeros(n, dtype=torch.float32, device="cuda"), stats=stats)
    assert not torch.any(a != 0)
    assert stats.cpu().tolist() == [1.0, 0.0]


def test_device_pipeline_plane(gpu):
    """series -> fdas_frontend -> fdas_convolve (FP32) against the oracle's
    plane of the oracle's spectrum (the small workload: 2^16 samples, z in
    [-16, 16], m 64)."""
    import torch
    x, chirps = synth.single_series_samples("fp32-small")
    x = x.astype(np.float32)
    a_ref, _ = oracle.spectrum64(x.astype(np.float64))
    p_ref = oracle.plane_direct(a_ref, 16.0, 2.0, 64)
    with gpu.FrontEnd(x.size) as fe:
        a = fe(torch.from_numpy(x).cuda())
    with gpu.Plan(16.0, 2.0, 64, 256, "fp32") as p:
        pw = p.convolve(a).cpu().numpy()
    assert np.max(np.abs(pw - p_ref)) <= 1e-4 * np.max(p_ref)
    iz, ir = np.unravel_index(np.argmax(pw), pw.shape)
    assert abs(ir - chirps[0].r0) < 1.5 and abs((-16 + 2 * iz) - chirps[0].z0) <= 1.01


def test_alternating_series_and_outputs(gpu):
    """One plan serves any buffers: alternating two series and two outputs
    gives each its own spectrum and median, repeatedly (the plan's scratch
    carries nothing from one call to the next)."""
    import torch
    n = 1 << 15
    xs = [_series(n, seed=s) for s in (11, 12)]
    refs = [oracle.spectrum64(x.astype(np.float64)) for x in xs]
    devs = [torch.from_numpy(x).cuda() for x in xs]
    outs = [torch.empty(n // 2, dtype=torch.complex64, device="cuda") for _ in range(2)]
    stats = torch.zeros(2, dtype=torch.float32, device="cuda")
    with gpu.FrontEnd(n) as fe:
        for rep in range(3):
            for k in (0, 1):
                fe(devs[k], out=outs[k], stats=stats)
                torch.cuda.synchronize()
                a_ref, med_ref = refs[k]
                a = outs[k].cpu().numpy()
                assert np.max(np.abs(a - a_ref)) <= 1e-5 * np.max(np.abs(a_ref)), (rep, k)
                assert abs(stats.cpu().numpy()[1] - med_ref) <= 1e-5 * med_ref
