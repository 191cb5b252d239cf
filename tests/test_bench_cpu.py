"""Host-side checks of bench.py that need no GPU: the one-GPU contract and
the error figure it reports against the oracle sample."""

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


def test_error_against_the_oracle_sample():
    """A plane perturbed by a known relative amount reports that amount; rows
    of a shorter series are matched to the bank's central rows."""
    import bench
    a = synth.small_random_spectrum(3000, seed=1)
    p = oracle.plane_direct(a, 16.0, 2.0, 64)
    bumped = p.copy()
    ref_max = p[:, :2048 - 32].max()   # the columns the check compares
    bumped[5, 100] += 3e-5 * ref_max
    base, err = bench.cpu_baseline(a, 16.0, 2.0, 64, 17, 2048,
                                   [("all", bumped[:, :2048].astype(np.float64), 0, 1, 1e-4),
                                    ("central", p[3:14, :2048], 3, 1, 1e-4)])
    assert base["kind"] == "oracle" and base["cores"] == 1
    assert abs(err["all"]["max_abs_err_over_max_ref"] - 3e-5) < 1e-12 and err["all"]["pass"]
    assert err["central"]["max_abs_err_over_max_ref"] == 0.0
    assert err["all"]["points"] == 17 * (2048 - 32)
