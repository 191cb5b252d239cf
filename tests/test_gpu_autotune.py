"""The autotuner (FDAS_FLAG_AUTOTUNE) picks a compiled variant, caches the
choice, and the tuned plan still matches the FP64 oracle."""

import numpy as np
import pytest

import oracle
from paper_1711_10855_amd import synth

pytestmark = pytest.mark.gpu


def test_autotune_choice_is_cached_and_correct(gpu, tmp_path, monkeypatch):
    import torch
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("FDAS_TUNE_CACHE", str(cache))
    monkeypatch.delenv("FDAS_VARIANT", raising=False)
    a = synth.small_random_spectrum(30000, seed=21)
    print("autotune zmax=8 m=64", flush=True)
    with gpu.Plan(8.0, 2.0, 64, 0, "fp32", flags=gpu.FLAG_AUTOTUNE) as p:
        info = p.info
        out = p.convolve(torch.from_numpy(a).cuda()).cpu().numpy()
    print("chose", info.kernel, info.seg_len, info.templates_per_block)
    assert info.seg_len - 64 >= info.seg_len // 2
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and info.kernel in lines[0]
    ref = oracle.plane_direct(a, 8.0, 2.0, 64)
    assert np.max(np.abs(out - ref)) <= 1e-4 * ref.max()
    with gpu.Plan(8.0, 2.0, 64, 0, "fp32", flags=gpu.FLAG_AUTOTUNE) as p2:
        assert p2.info.kernel == info.kernel
        assert p2.info.templates_per_block == info.templates_per_block
    assert len(cache.read_text().splitlines()) == 1   # served from the cache


def test_tune_cache_separates_split_forms(gpu, tmp_path, monkeypatch):
    """A cached choice for the plain 16-bit form is not reused for the hi+lo
    split form (and vice versa): each gets its own line and its own kind of
    kernel."""
    import torch
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("FDAS_TUNE_CACHE", str(cache))
    monkeypatch.delenv("FDAS_VARIANT", raising=False)
    a = synth.small_random_spectrum(20000, seed=22)
    ref = oracle.plane_direct(a, 8.0, 2.0, 64)
    kernels = []
    for flags, tol in ((gpu.FLAG_AUTOTUNE, 1e-3), (gpu.FLAG_AUTOTUNE | gpu.FLAG_SPLIT, 1e-5)):
        print(f"autotune fp16 flags={flags}", flush=True)
        with gpu.Plan(8.0, 2.0, 64, 0, "fp16", flags=flags) as p:
            kernels.append(p.info.kernel)
            out = p.convolve(torch.from_numpy(a).cuda()).cpu().numpy()
        assert np.max(np.abs(out - ref)) <= tol * ref.max()
    assert "_split" not in kernels[0] and "_split" in kernels[1]
    assert len(cache.read_text().splitlines()) == 2


def _median_ms(plan, spec, out, reps=9):
    """Median of individually timed calls after 100 ms of load."""
    import time

    import torch
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 0.1:
        for _ in range(8):
            plan.convolve(spec, out=out)
        torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.convolve(spec, out=out)
        e1.record()
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    return sorted(ms)[reps // 2]


def test_tuned_choice_is_near_the_best_retimed(gpu, tmp_path, monkeypatch):
    """On the 101-template, m = 256 bank, the tuned plan is within 10% of the
    fastest of an independent re-timing of the untuned default plan at every
    admissible segment length, on the 2^20-bin input the tuner itself uses."""
    import torch
    monkeypatch.setenv("FDAS_TUNE_CACHE", str(tmp_path / "tune.txt"))
    monkeypatch.delenv("FDAS_VARIANT", raising=False)
    monkeypatch.delenv("FDAS_ZPB", raising=False)
    spec = torch.from_numpy(synth.small_random_spectrum(1 << 20, seed=23)).cuda()
    out = torch.empty((101, 1 << 20), dtype=torch.float32, device="cuda")
    print("autotune zmax=100 m=256", flush=True)
    with gpu.Plan(100.0, 2.0, 256, 0, "fp32", flags=gpu.FLAG_AUTOTUNE) as p:
        tuned = _median_ms(p, spec, out)
        choice = (p.info.kernel, p.info.seg_len)
    times = {}
    for L in (512, 1024, 2048, 4096):
        print(f"re-time default plan L={L}", flush=True)
        with gpu.Plan(100.0, 2.0, 256, L, "fp32") as p:
            times[(p.info.kernel, L)] = _median_ms(p, spec, out)
    print("tuned", choice, f"{tuned:.4f} ms; re-timed", times)
    assert tuned <= 1.10 * min(times.values())
