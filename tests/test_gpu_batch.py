"""Batched path (one graph-captured launch over many series of uneven length
and per-series zmax; persistent work-queue loop by default, flat work-item
grid with FDAS_BATCH_PERSISTENT=0) against the FP64 oracle, through the C ABI."""

import os

import numpy as np
import pytest

import oracle
from paper_1711_10855_amd import synth

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-4


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).cuda()


def make_batch(plan_zmax, dz, specs):
    import torch
    spectra, zmaxs, outs = [], [], []
    for k, (nbins, zmax, ldpad) in enumerate(specs):
        a = synth.small_random_spectrum(nbins, seed=100 + k)
        nz = int(round(2 * zmax / dz)) + 1
        spectra.append(a)
        zmaxs.append(zmax)
        outs.append(torch.full((nz, nbins + ldpad), -3.0, dtype=torch.float32, device="cuda"))
    return spectra, zmaxs, outs


SPECS = [(5000, 16.0, 0), (1, 8.0, 0), (191, 0.0, 3), (20000, 16.0, 7), (777, 4.0, 0),
         (12345, 10.0, 0), (193, 16.0, 1)]


@pytest.fixture
def env():
    saved = {k: os.environ.get(k) for k in ("FDAS_NO_GRAPH", "FDAS_BATCH_PERSISTENT")}
    yield os.environ
    for k, v in saved.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v


@pytest.mark.parametrize("L,m,persistent", [(256, 64, "0"), (1024, 128, "0"), (256, 64, "1"),
                                             (1024, 128, "1")])
def test_batch_matches_oracle(gpu, env, L, m, persistent):
    env["FDAS_BATCH_PERSISTENT"] = persistent
    spectra, zmaxs, outs = make_batch(16.0, 2.0, SPECS)
    print(f"batch L={L} m={m} nseries={len(SPECS)} persistent={persistent}", flush=True)
    with gpu.Plan(16.0, 2.0, m, L) as p:
        p.convolve_batch([to_dev(a) for a in spectra], zmaxs, outs)
        res = [o.cpu().numpy() for o in outs]
    for a, z, o, (nbins, _, ldpad) in zip(spectra, zmaxs, res, SPECS):
        ref = oracle.plane_direct(a, z, 2.0, m)
        err = float(np.max(np.abs(o[:, :nbins] - ref)) / np.max(ref))
        assert err <= TOL_FP32, (nbins, z, err)
        if ldpad:
            assert np.all(o[:, nbins:] == -3.0)


def test_batch_graph_replays_match_eager(gpu, env):
    import torch
    spectra, zmaxs, outs = make_batch(16.0, 2.0, SPECS)
    dev = [to_dev(a) for a in spectra]
    with gpu.Plan(16.0, 2.0, 64, 512) as p:
        env["FDAS_NO_GRAPH"] = "1"
        p.convolve_batch(dev, zmaxs, outs)
        eager = [o.clone() for o in outs]
        env.pop("FDAS_NO_GRAPH")
        for rep in range(4):
            for o in outs:
                o.fill_(-3.0)  # same as the initial fill: ld padding is never written
            # the program's own eager work between replays
            single = p.convolve(dev[3])
            torch.cuda.synchronize()
            p.convolve_batch(dev, zmaxs, outs)
            torch.cuda.synchronize()
            for o, e in zip(outs, eager):
                assert torch.equal(o, e), f"replay {rep} differs from eager"
            full = p.convolve(dev[3]).cpu().numpy()
            assert np.array_equal(full, single.cpu().numpy())


def test_batch_equals_single_series_calls(gpu):
    spectra, zmaxs, outs = make_batch(16.0, 2.0, SPECS[:4])
    dev = [to_dev(a) for a in spectra]
    with gpu.Plan(16.0, 2.0, 64, 256) as p:
        p.convolve_batch(dev, zmaxs, outs)
        for a, z, o in zip(dev, zmaxs, outs):
            row0 = int(round((16.0 - z) / 2.0))
            full = p.convolve(a).cpu().numpy()[row0:row0 + o.shape[0]]
            got = o[:, :a.numel()].cpu().numpy()
            assert np.max(np.abs(got - full)) <= 1e-6 * max(1.0, float(full.max()))


def test_batch_rejects_bad_series(gpu):
    import torch
    from paper_1711_10855_amd import fdas
    a = to_dev(synth.small_random_spectrum(1000, seed=1))
    with gpu.Plan(16.0, 2.0, 64, 256) as p:
        for bad_z in (18.0, 3.0, -2.0):
            nz = max(1, int(round(2 * abs(bad_z) / 2.0)) + 1)
            o = torch.empty((nz, 1000), dtype=torch.float32, device="cuda")
            with pytest.raises(fdas.FdasError) as e:
                p.convolve_batch([a], [bad_z], [o])
            assert e.value.status == fdas.ERR_INVALID


def test_batch_workload_sample(gpu):
    """Batched workload recipe (uneven lengths, zmax in {32, 64, 100}) on a
    sample of its series, sampled points checked against the oracle."""
    import torch
    specs = synth.batch_specs("batch-fp32", nseries=6)
    spectra = [synth.batch_spectrum("batch-fp32", sp) for sp in specs]
    outs = [torch.empty((int(round(sp.zmax)) + 1, sp.nbins), dtype=torch.float32, device="cuda")
            for sp in specs]
    print("batch-fp32 sample of 6 series", [(sp.nbins, sp.zmax) for sp in specs], flush=True)
    with gpu.Plan(100.0, 2.0, 256, 2048) as p:
        p.convolve_batch([to_dev(a) for a in spectra], [sp.zmax for sp in specs], outs)
        res = [o.cpu().numpy() for o in outs]
    rng = np.random.default_rng(4)
    for sp, a, o in zip(specs, spectra, res):
        nz = o.shape[0]
        iz = rng.integers(0, nz, 1500)
        r = rng.integers(0, sp.nbins, 1500)
        extra = np.array([0, sp.nbins - 1] + [int(round(c.r0)) for c in sp.chirps])
        iz = np.concatenate([iz, np.repeat(np.arange(nz), extra.size)])
        r = np.concatenate([r, np.tile(extra, nz)])
        ref = oracle.plane_points(a, sp.zmax, 2.0, 256, iz, r)
        err = float(np.max(np.abs(o[iz, r] - ref)) / ref.max())
        print(f"series nbins={sp.nbins} zmax={sp.zmax}: {err:.3e}")
        assert err <= TOL_FP32


@pytest.mark.parametrize("prec,split,tol", [("fp16", False, 1e-3), ("bf16", True, 1e-3),
                                           ("fp32", False, TOL_FP32)])
def test_wide_batch_workload_sample(gpu, prec, split, tol):
    """Wide-filter batched recipe (2^21 bins per series, z in [-200, 200],
    m 512) on three of its series in the bench's launch configuration
    (segment length 4096 for the 16-bit forms, the FP32 default otherwise),
    sampled points checked against the oracle."""
    import torch
    specs = synth.batch_specs("batch-mixed-wide", nseries=3)
    spectra = [synth.batch_spectrum("batch-mixed-wide", sp) for sp in specs]
    ld = [(sp.nbins + 63) // 64 * 64 for sp in specs]
    outs = [torch.empty((201, l), dtype=torch.float32, device="cuda")[:, :sp.nbins]
            for sp, l in zip(specs, ld)]
    print(f"batch-mixed-wide sample of 3 series, {prec} split={split}", flush=True)
    flags = gpu.FLAG_SPLIT if split else 0
    with gpu.Plan(200.0, 2.0, 512, 4096 if prec != "fp32" else 0, prec, flags) as p:
        p.convolve_batch([to_dev(a) for a in spectra], [sp.zmax for sp in specs], outs)
        res = [o.cpu().numpy() for o in outs]
    rng = np.random.default_rng(5)
    for sp, a, o in zip(specs, spectra, res):
        iz = rng.integers(0, 201, 1200)
        r = rng.integers(0, sp.nbins, 1200)
        extra = np.array([0, sp.nbins - 1] + [int(round(c.r0)) for c in sp.chirps])
        iz = np.concatenate([iz, np.repeat(np.arange(201), extra.size)])
        r = np.concatenate([r, np.tile(extra, 201)])
        ref = oracle.plane_points(a, 200.0, 2.0, 512, iz, r)
        err = float(np.max(np.abs(o[iz, r] - ref)) / ref.max())
        print(f"{prec} series nbins={sp.nbins}: {err:.3e}")
        assert err <= tol


def test_many_batch_layouts_replay_in_turn(gpu):
    """Twelve distinct batch layouts, each called three times in turn, give
    the same planes every time (each layout keeps its own captured graph and
    descriptor table)."""
    import torch
    layouts = []
    for k in range(12):
        specs = [(300 + 97 * k, 16.0, 0), (1 + k, 8.0, 1), (2000 - 50 * k, 4.0, 0)]
        spectra, zmaxs, outs = make_batch(16.0, 2.0, specs)
        layouts.append(([to_dev(a) for a in spectra], zmaxs, outs))
    with gpu.Plan(16.0, 2.0, 64, 256) as p:
        first = []
        for rep in range(3):
            for k, (dev, zmaxs, outs) in enumerate(layouts):
                for o in outs:
                    o.fill_(-3.0)
                p.convolve_batch(dev, zmaxs, outs)
                torch.cuda.synchronize()
                got = [o.cpu().numpy() for o in outs]
                if rep == 0:
                    first.append(got)
                    for a, z, g in zip(dev, zmaxs, got):
                        row0 = int(round((16.0 - z) / 2.0))
                        full = p.convolve(a).cpu().numpy()[row0:row0 + g.shape[0]]
                        assert np.max(np.abs(g[:, :a.numel()] - full)) <= \
                            1e-6 * max(1.0, float(full.max())), k
                else:
                    for g, f in zip(got, first[k]):
                        assert np.array_equal(g, f), (rep, k)
