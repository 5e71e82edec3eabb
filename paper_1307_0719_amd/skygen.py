"""Seeded synthetic skies: unlensed T/E/B and lensing-potential a_lm.

This module is shared by the HIP path's tests/benchmarks and by the CPU
oracle's tests.  It holds no arithmetic of the lensing method itself: only
the input spectra and a seeded complex-Gaussian draw.  It imports nothing
else from this package.

Conventions (stated once, used everywhere):

* a_lm layout: complex128, triangular, m-major.  For 0 <= m <= l <= lmax the
  coefficient a_lm sits at index ``m*(2*lmax+1-m)//2 + l``; only m >= 0 is
  stored, the real-field symmetry a_{l,-m} = (-1)^m conj(a_lm) gives the rest.
  The imaginary part of every m = 0 coefficient is zero.
* Spectra follow the paper's input preparation (Gaussian skies from an
  unlensed power spectrum and a lensing potential, Sec. II.A): here analytic
  stand-ins for the CAMB spectra the paper used, which are not available.
  C_l = 0 for l < 2 for every field.
  T:   C_l = 1e3 / (l(l+1)) * exp(-(l/1500)^2)
  E:   0.05 * C_l^T      (drawn independently of T)
  B:   0
  phi: C_l = A / (l(l+1))^2 with A fixed so that the RMS deflection
       |grad phi| is 2.5 arcmin in expectation over realizations.
* Each realization draws T, E, B, phi in that order from
  ``numpy.random.Generator(PCG64(seed))``; one standard-normal array of shape
  (nalm, 2) per field: a_l0 = sqrt(C_l) g_0 and a_lm = sqrt(C_l/2)(g_0 + i g_1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ARCMIN = math.pi / (180.0 * 60.0)
DEFLECTION_RMS_ARCMIN = 2.5


def nalm(lmax: int) -> int:
    """Number of stored coefficients for band limit lmax."""
    return (lmax + 1) * (lmax + 2) // 2


def alm_index(lmax: int, l, m):
    """Index of a_lm in the triangular m-major layout."""
    return m * (2 * lmax + 1 - m) // 2 + l


def lm_arrays(lmax: int):
    """(l, m) integer arrays in storage order."""
    ls = np.empty(nalm(lmax), dtype=np.int64)
    ms = np.empty(nalm(lmax), dtype=np.int64)
    i = 0
    for m in range(lmax + 1):
        n = lmax + 1 - m
        ls[i:i + n] = np.arange(m, lmax + 1)
        ms[i:i + n] = m
        i += n
    return ls, ms


def cl_tt(lmax: int) -> np.ndarray:
    l = np.arange(lmax + 1, dtype=np.float64)
    c = np.zeros(lmax + 1)
    ll = l[2:]
    c[2:] = 1e3 / (ll * (ll + 1.0)) * np.exp(-(ll / 1500.0) ** 2)
    return c


def cl_ee(lmax: int) -> np.ndarray:
    return 0.05 * cl_tt(lmax)


def cl_bb(lmax: int) -> np.ndarray:
    return np.zeros(lmax + 1)


def cl_phiphi(lmax: int, rms_arcmin: float = DEFLECTION_RMS_ARCMIN) -> np.ndarray:
    """Lensing-potential spectrum scaled to the requested RMS deflection.

    The expected mean-square deflection is sum_l (2l+1)/(4 pi) l(l+1) C_l.
    """
    l = np.arange(lmax + 1, dtype=np.float64)
    c = np.zeros(lmax + 1)
    if lmax < 2:
        return c
    ll = l[2:]
    shape = 1.0 / (ll * (ll + 1.0)) ** 2
    msq = np.sum((2 * ll + 1) / (4 * math.pi) * ll * (ll + 1) * shape)
    amp = (rms_arcmin * ARCMIN) ** 2 / msq
    c[2:] = amp * shape
    return c


def draw_alm(rng: np.random.Generator, cl: np.ndarray, lmax: int) -> np.ndarray:
    """One complex-Gaussian a_lm set with power spectrum cl (layout above)."""
    ls, ms = lm_arrays(lmax)
    g = rng.standard_normal((nalm(lmax), 2))
    c = cl[ls]
    out = np.empty(nalm(lmax), dtype=np.complex128)
    m0 = ms == 0
    out[m0] = np.sqrt(c[m0]) * g[m0, 0]
    mp = ~m0
    out[mp] = np.sqrt(c[mp] / 2.0) * (g[mp, 0] + 1j * g[mp, 1])
    return out


@dataclass
class Sky:
    lmax: int
    seed: int
    alm_T: np.ndarray
    alm_E: np.ndarray | None
    alm_B: np.ndarray | None
    alm_phi: np.ndarray


def make_sky(lmax: int, seed: int, pol: bool = True,
             rms_arcmin: float = DEFLECTION_RMS_ARCMIN) -> Sky:
    """Seeded unlensed sky.  Draw order T, E, B, phi (E/B drawn even when
    pol=False so that T and phi do not depend on the pol flag)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = draw_alm(rng, cl_tt(lmax), lmax)
    e = draw_alm(rng, cl_ee(lmax), lmax)
    b = draw_alm(rng, cl_bb(lmax), lmax)
    p = draw_alm(rng, cl_phiphi(lmax, rms_arcmin), lmax)
    if not pol:
        e = b = None
    return Sky(lmax, seed, t, e, b, p)


def random_alm(lmax: int, seed: int, lmin: int = 0) -> np.ndarray:
    """White unit-variance a_lm (used by unit checks of the harmonic stage);
    m = 0 entries real, entries with l < lmin zero."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ls, ms = lm_arrays(lmax)
    g = rng.standard_normal((nalm(lmax), 2))
    out = g[:, 0] + 1j * g[:, 1]
    out[ms == 0] = g[ms == 0, 0]
    out[ls < lmin] = 0.0
    return out


@dataclass
class Workload:
    """A named workload: band limit, ring grid, Taylor order, fields."""
    name: str
    lmax: int
    ntheta: int
    nphi: int
    order: int
    pol: bool
    seed: int
    precision: str = "fp32"
    extra: dict = field(default_factory=dict)


# The five workloads the method is exercised on (sizes as stated for each).
WORKLOADS = {
    "T256": Workload("T-only lmax=256, 513x1024 rings, order 3, FP64",
                     256, 513, 1024, 3, False, 0, "fp64"),
    "TP2048": Workload("T+Q/U lmax=2048, 2049x4096 rings, orders 1-5, FP32",
                       2048, 2049, 4096, 4, True, 1, "fp32"),
    "TP4096": Workload("T+Q/U lmax=4096, 4097x8192 rings, order 4",
                       4096, 4097, 8192, 4, True, 2, "fp32"),
}


def batch_lmaxes(n: int = 64, seed: int = 3, choices=(512, 1024, 2048, 3000)):
    """lmax per realization for the uneven-lmax batch (uniform draw)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [int(choices[i]) for i in rng.integers(0, len(choices), size=n)]


# ---- learned correction: seeded draws shared by training and its checks ----

CNN_SIZES = [(32, 20 * 9), (32,), (32, 32 * 9), (32,), (3, 32), (3,)]  # (rows, fan_in) of W1 b1 W2 b2 W3 b3


def cnn_init(seed: int) -> np.ndarray:
    """Initial parameter vector of the correction network, float32:
    W1[32][20][3][3], b1[32], W2[32][32][3][3], b2[32], W3[3][32], b3[3]
    uniform in +-1/sqrt(fan_in) of their layer, then three output scales 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    fans = [180, 180, 288, 288, 32, 32]
    parts = []
    for shp, fan in zip(CNN_SIZES, fans):
        n = int(np.prod(shp))
        parts.append(rng.uniform(-1.0, 1.0, n) / math.sqrt(fan))
    parts.append(np.ones(3))
    return np.concatenate(parts).astype(np.float32)


def sample_pixels(npix: int, n: int, seed: int) -> np.ndarray:
    """n distinct output-pixel indices in [0, npix), sorted, int64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(npix, size=min(n, npix), replace=False)).astype(np.int64)
