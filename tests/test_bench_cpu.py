"""Host-side checks of bench.py that need no GPU: the one-GPU contract, the
oracle pool it times (against a direct oracle call), the sampled points it
checks and the error figure it reports."""

import json
import os
import subprocess
import sys

import numpy as np

import oracle
from paper_1711_10855_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"] and msg["n_gpus"] == 2


def test_unknown_form_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--forms", "fp8"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "unknown forms" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_rel_error():
    import bench
    ref = np.array([1.0, 4.0, 2.0])
    assert bench.rel_error(ref, ref) == 0.0
    assert abs(bench.rel_error(ref + [0, 0, 4e-4], ref) - 1e-4) < 1e-15


def test_pool_dense_equals_the_oracle_plane():
    """Bin ranges with their m/2 halos, put back together, give exactly the
    oracle's own plane (edges included)."""
    import bench
    a = synth.small_random_spectrum(3000, seed=1)
    pool = bench.OraclePool(2)
    try:
        got, dt = pool.dense([("x", a, 16.0, 2.0, 64, 2500)], chunk=700)
        ref = oracle.plane_direct(a, 16.0, 2.0, 64)
        assert got["x"].shape == (17, 2500) and dt > 0
        assert np.array_equal(got["x"], ref[:, :2500])
        # the dense check compares only columns that do not reach past the sample
        full, _ = pool.dense([("y", a, 16.0, 2.0, 64, 3000)], chunk=1024)
        assert np.array_equal(full["y"], ref)
    finally:
        pool.close()


def test_pool_points_redraw_the_batch_series():
    """The workers draw a batched series again from its seed; the oracle's
    points on that series equal those on the parent's copy."""
    import bench
    specs = synth.batch_specs("batch-fp32", 2)
    sp = min(specs, key=lambda s: s.nbins)
    a = synth.batch_spectrum("batch-fp32", sp)
    iz, r = bench.sample_points(sp.nbins, 2 * int(sp.zmax / 2) + 1, sp.zmax, 2.0, sp.chirps,
                                sp.index, 64)
    pool = bench.OraclePool(2)
    try:
        got = pool.points([(7, "batch-fp32", sp, sp.zmax, 2.0, 16, iz, r)])
    finally:
        pool.close()
    assert np.array_equal(got[7], oracle.plane_points(a, sp.zmax, 2.0, 16, iz, r))


def test_sample_points_cover_signals_and_edges():
    import bench
    chirps = [synth.Chirp(1000.4, 7.0, 20.0, 0.0), synth.Chirp(3.2, -31.0, 10.0, 1.0)]
    iz, r = bench.sample_points(5000, 33, 32.0, 2.0, chirps, 3, 100)
    pts = set(zip(iz.tolist(), r.tolist()))
    assert {(19, 1000), (20, 1000), (19, 998), (20, 1002)} <= pts   # z0 = 7 -> rows 19.5
    assert (0, 1) in pts and (0, 5) in pts                          # z0 = -31 -> row 0.5
    assert {(0, 0), (32, 4999), (16, 4998)} <= pts
    assert iz.min() >= 0 and iz.max() < 33 and r.min() >= 0 and r.max() < 5000
    again = bench.sample_points(5000, 33, 32.0, 2.0, chirps, 3, 100)
    assert np.array_equal(again[0], iz) and np.array_equal(again[1], r)
    # with the spectrum: its strongest bins on the rows next to z = 0 (row 16)
    a = np.ones(5000, dtype=np.complex64)
    a[[10, 4999]] = 5.0
    iz, r = bench.sample_points(5000, 33, 32.0, 2.0, [], 3, 0, a)
    pts = set(zip(iz.tolist(), r.tolist()))
    assert {(15, 8), (16, 10), (17, 12), (16, 4997), (17, 4999)} <= pts
    assert iz.min() >= 0 and iz.max() < 33 and r.max() < 5000


def test_pick_series():
    import bench
    specs = synth.batch_specs("batch-fp32", 40)
    pick = bench.pick_series(specs, 8)
    assert len(pick) == len(set(pick)) == 8
    nb = [s.nbins for s in specs]
    assert nb.index(min(nb)) in pick and nb.index(max(nb)) in pick
    assert {specs[i].zmax for i in pick} == {32.0, 64.0, 100.0}


def test_profile_rows_hash_their_own_kernel_sources():
    from paper_1711_10855_amd import profile_summary as ps
    assert "csrc/ols_fp32.hip" in ps.kernel_sources("fp32_L2048_t128_r8.16.16_o2")
    assert "csrc/ols_mixed.hip" in ps.kernel_sources("fp16_L4096_mfma_w16_pfw")
    assert "csrc/ols_mixed2048.hip" in ps.kernel_sources("fp16_L2048_mfma_w16")
    assert ps.source_hash("fp16_L2048_mfma_w16") != ps.source_hash("fp16_L4096_mfma_w16_pfw")


def test_matrix_core_forms_run_at_the_workloads_length():
    import bench
    args = bench.parse([])
    paper, wide = synth.WORKLOADS["fp32-paper"], synth.WORKLOADS["batch-mixed-wide"]
    assert bench.form_seg_len("fp16", paper, args) == 2048
    assert bench.form_seg_len("bf16-split", paper, args) == 4096   # split: 4096 only
    assert bench.form_seg_len("fp16", wide, args) == 4096
