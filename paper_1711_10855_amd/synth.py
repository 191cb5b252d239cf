"""Seeded synthetic inputs for the FDAS correlation step.

This module holds the workload recipes and the seeded input generators that
both the checker and the HIP path consume. It contains none of the method's
arithmetic (no templates, no correlation): it produces time series of white
noise with injected accelerated sinusoids and turns them into the normalised
complex spectrum the correlation step reads.

Signal model (the meaning of z follows eq. 1, Section 1: the number of bins
the frequency drifts over the observation):

    x_n = N(0, 1) + sum_c a_c cos(2 pi (r0_c s_n + z0_c s_n^2 / 2) + phi_c),
    s_n = n / N - 1/2,   a_c = 2 SNR_c / sqrt(N),

so r0 is the mid-observation frequency in bins and the matched power of each
injection is about SNR^2 after normalisation.

Spectrum: A = rfft(x)[0:N/2] (Nyquist dropped), A_0 = 0, then
A /= sqrt(median(|A_k|^2, k >= 1) / ln 2), which gives the noise unit mean
power (the median of an exponential distribution is ln 2 times its mean).

Seeds: the root is SeedSequence(171110855); workload c (1-based) uses
root.spawn(5)[c-1]; series j of a batched workload uses child j of that.
"""

from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np

SEED_ROOT = 171110855


@dataclass(frozen=True)
class Chirp:
    r0: float
    z0: float
    snr: float
    phi: float


@dataclass
class Workload:
    """One named workload: sizes, filter parameters and how to draw inputs."""
    name: str
    index: int                 # 1-based workload number (seed stream)
    n_samples: int             # time samples of a single series
    zmax: float
    dz: float
    m: int
    seg_len: int
    precision: str = "fp32"   # the workload's main form (bench.py times several)
    nseries: int = 1
    description: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def nbins(self) -> int:
        return self.n_samples // 2

    @property
    def nz(self) -> int:
        return int(round(2 * self.zmax / self.dz)) + 1


WORKLOADS = {
    "fp32-small": Workload(
        "fp32-small", 1, 1 << 16, 16.0, 2.0, 64, 256,
        description="2^16-sample series, one chirp (r0=5000.3, z0=+7, S/N 20); "
                    "32768 bins; z in [-16,16] step 2 (17 templates, width 64); "
                    "segment FFT 256"),
    "fp32-paper": Workload(
        "fp32-paper", 2, 1 << 22, 100.0, 2.0, 256, 2048,
        description="2^22-sample series, 8 chirps (z0 in [-90,90], S/N 8-30); "
                    "2^21 bins; z in [-100,100] step 2 (101 templates, width 256); "
                    "segment FFT 2048"),
    "batch-fp32": Workload(
        "batch-fp32", 3, 1 << 22, 100.0, 2.0, 256, 2048, nseries=512,
        description="512 series of 2^20..2^22 samples, 0-3 chirps each, "
                    "per-series zmax in {32,64,100}, dz 2, one bank (zmax 100, m 256)"),
    "mixed-paper": Workload(
        "mixed-paper", 4, 1 << 22, 100.0, 2.0, 256, 2048, precision="fp16",
        description="fp32-paper inputs, FP16 storage and MFMA DFT stages"),
    "batch-mixed-wide": Workload(
        "batch-mixed-wide", 5, 1 << 22, 200.0, 2.0, 512, 4096, nseries=256,
        precision="fp16",
        description="256 series of 2^22 samples, 0-3 chirps, z in [-200,200] "
                    "step 2 (201 templates, width 512), segment FFT 4096 "
                    "(8192 and 16384 ran slower in plain FP32); the 16-bit "
                    "form that holds 1e-3 unsplit is FP16 (BF16 needs the "
                    "hi+lo split)"),
}


def workload_rng(index: int) -> np.random.SeedSequence:
    return np.random.SeedSequence(SEED_ROOT).spawn(5)[index - 1]


def make_series(n: int, chirps, rng: np.random.Generator,
                noise: bool = True) -> np.ndarray:
    """White N(0,1) noise (float64) plus the given chirps (see module doc)."""
    x = rng.standard_normal(n) if noise else np.zeros(n)
    if chirps:
        s = np.arange(n, dtype=np.float64) / n - 0.5
        for c in chirps:
            a = 2.0 * c.snr / math.sqrt(n)
            x += a * np.cos(2.0 * np.pi * (c.r0 * s + 0.5 * c.z0 * s * s) + c.phi)
    return x


def make_spectrum(x: np.ndarray, normalise: str = "median") -> np.ndarray:
    """rfft, drop Nyquist, zero DC, normalise; returns complex128, N//2 bins.

    ``normalise``: "median" (unit mean noise power from the median), or
    "sqrtn" (divide by sqrt(N), the noise-free reading of the same scale).
    """
    import scipy.fft

    n = x.size
    a = scipy.fft.rfft(np.asarray(x, dtype=np.float64),
                       workers=min(16, os.cpu_count() or 1))[: n // 2]
    a[0] = 0.0
    if normalise == "median":
        p = a[1:].real ** 2 + a[1:].imag ** 2
        a /= math.sqrt(float(np.median(p)) / math.log(2.0))
    elif normalise == "sqrtn":
        a /= math.sqrt(n)
    else:
        raise ValueError(normalise)
    return a


def _draw_chirps(rng, count, nbins, m, zlim, snr_lo, snr_hi):
    out = []
    for _ in range(count):
        r0 = float(rng.uniform(m, nbins - m))
        z0 = float(rng.uniform(-zlim, zlim))
        snr = float(rng.uniform(snr_lo, snr_hi))
        phi = float(rng.uniform(0.0, 2.0 * math.pi))
        out.append(Chirp(r0, z0, snr, phi))
    return out


def single_series_samples(name: str):
    """Time series (float64) and injected chirps of a single-series workload."""
    w = WORKLOADS[name]
    if w.nseries != 1:
        raise ValueError(f"{name} is a batched workload")
    rng = np.random.default_rng(workload_rng(w.index))
    if w.index == 1:
        chirps = [Chirp(5000.3, 7.0, 20.0, float(rng.uniform(0.0, 2.0 * math.pi)))]
    else:
        chirps = _draw_chirps(rng, 8, w.nbins, w.m, 90.0, 8.0, 30.0)
    return make_series(w.n_samples, chirps, rng), chirps


def single_series(name: str):
    """Spectrum (complex64) and injected chirps for a single-series workload."""
    x, chirps = single_series_samples(name)
    a = make_spectrum(x).astype(np.complex64)
    return a, chirps


@dataclass
class SeriesSpec:
    index: int
    n_samples: int
    zmax: float
    chirps: list

    @property
    def nbins(self) -> int:
        return self.n_samples // 2


def batch_specs(name: str, nseries: int | None = None):
    """Per-series sizes, zmax and chirps for a batched workload (no samples)."""
    w = WORKLOADS[name]
    ss = workload_rng(w.index)
    count = w.nseries if nseries is None else int(nseries)
    children = ss.spawn(count)
    specs = []
    for j, child in enumerate(children):
        rng = np.random.default_rng(child.spawn(1)[0])
        if w.index == 3:
            n = int(rng.integers(1 << 20, (1 << 22) + 1))
            n -= n % 2
            zmax = float(rng.choice([32.0, 64.0, 100.0]))
            zlim = 0.9 * zmax
        else:
            n = w.n_samples
            zmax = w.zmax
            zlim = 180.0
        k = int(rng.integers(0, 4))
        chirps = _draw_chirps(rng, k, n // 2, w.m, zlim, 8.0, 30.0)
        specs.append(SeriesSpec(j, n, zmax, chirps))
    return specs


def batch_spectrum(name: str, spec: SeriesSpec) -> np.ndarray:
    """complex64 spectrum of one series of a batched workload (seeded by j).

    The white-noise part is drawn directly in the Fourier domain, where the
    real FFT of N(0,1) samples is exactly i.i.d. complex Gaussian with
    E|A_k|^2 = N for 0 < k < N/2; the chirps are synthesised in time and
    transformed (one FFT per series that has any). DC is zeroed and the
    spectrum is normalised by its median power as for single series.
    """
    import scipy.fft

    w = WORKLOADS[name]
    child = workload_rng(w.index).spawn(w.nseries)[spec.index]
    rng = np.random.default_rng(child)
    n = spec.n_samples
    nb = n // 2
    scale = math.sqrt(n / 2.0)
    a = np.empty(nb, dtype=np.complex128)
    a.real = rng.standard_normal(nb)
    a.imag = rng.standard_normal(nb)
    a *= scale
    if spec.chirps:
        x = make_series(n, spec.chirps, rng, noise=False)
        a += scipy.fft.rfft(x, workers=1)[:nb]
    a[0] = 0.0
    p = a[1:].real ** 2 + a[1:].imag ** 2
    a /= math.sqrt(float(np.median(p)) / math.log(2.0))
    return a.astype(np.complex64)


def batch_inputs(name: str, nseries: int | None = None, workers: int = 16):
    """Specs and complex64 spectra of a batched workload, built in threads."""
    import concurrent.futures as cf

    specs = batch_specs(name, nseries)
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        spectra = list(ex.map(lambda sp: batch_spectrum(name, sp), specs))
    return specs, spectra


def noise_free_chirp_spectrum(n: int, chirp: Chirp) -> np.ndarray:
    """Spectrum of a single noise-free chirp, scaled by 1/sqrt(N) (complex128)."""
    rng = np.random.default_rng(0)
    x = make_series(n, [chirp], rng, noise=False)
    return make_spectrum(x, normalise="sqrtn")


def small_random_spectrum(nbins: int, seed: int) -> np.ndarray:
    """complex64 unit-power complex Gaussian bins (parity cases of any size)."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_ROOT, seed]))
    re = rng.standard_normal(nbins)
    im = rng.standard_normal(nbins)
    return ((re + 1j * im) / math.sqrt(2.0)).astype(np.complex64)
