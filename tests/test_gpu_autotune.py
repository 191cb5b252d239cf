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
