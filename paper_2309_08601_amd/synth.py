"""Seeded synthetic shear catalogs shaped like the paper's survey workloads.

This module holds only the input model (positions, shape noise, a Gaussian
random shear field, weights).  It contains none of the estimator's
arithmetic, so both the HIP path and the CPU oracle may draw their inputs
from it.

Input recipe (paper Sect. 3: a catalog is positions, complex ellipticities
and weights; ellipticity = shear + noise as an unbiased shear estimate):

* positions uniform in a square field of side L arcmin, snapped to a
  lattice of 2**-16 arcmin and stored as int32 lattice coordinates, so
  that pair separations are exact integers on every implementation;
* ellipticity e = n + s, with n Gaussian per component (sigma_e) and s a
  periodic Gaussian random shear field derived from a convergence field
  with power spectrum P(k) ~ k**-1.5 (P(0) = 0) on a 0.25 arcmin grid,
  rescaled to 0.02 rms, converted to shear with the flat-sky
  Kaiser-Squires kernel and bilinearly interpolated at the galaxy
  positions with periodic wrap;
* weights 1 (small case) or uniform in [0.5, 1.5];
* radial bins log-spaced between theta_min and theta_max.

A Gaussian field has no connected three-point function, so these inputs
exercise load and precision, not science.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

LATTICE_BITS = 16
LATTICE_UNIT = 2.0 ** -LATTICE_BITS  # arcmin per lattice step
SEED_BASE = 230908601
GRF_PIXEL = 0.25  # arcmin


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n_gal: Sequence[int]           # one entry per tomographic bin
    side: float                    # field side, arcmin
    n_bins: int
    theta_min: float
    theta_max: float
    n_max: int
    sigma_e: Sequence[float]       # per tomographic bin
    grf_scale: Sequence[float]     # per tomographic bin
    unit_weights: bool
    seed_index: int
    n_phi: int = 32

    @property
    def n_z(self) -> int:
        return len(self.n_gal)

    def edges(self) -> np.ndarray:
        return np.geomspace(self.theta_min, self.theta_max, self.n_bins + 1)


# The survey-shaped workloads.  The names say what they are; the last one
# has the size, density, binning and n_max of the paper's timing of the
# combined estimator (Sect. 4.1: 3.1e6 ellipticities on 100 deg^2, 33 log
# bins 0.25'-80', n_max = 20).
WORKLOADS = {
    "small_2k": Workload("small_2k", [2000], 60.0, 10, 1.0, 30.0, 10,
                         [0.28], [1.0], True, 0),
    "field_1m": Workload("field_1m", [1_000_000], 600.0, 20, 0.5, 100.0, 30,
                         [0.28], [1.0], False, 1),
    "field_4m": Workload("field_4m", [4_000_000], 1200.0, 30, 0.5, 200.0, 40,
                         [0.28], [1.0], False, 2),
    "tomo_5bin": Workload("tomo_5bin",
                          [300_000, 600_000, 800_000, 700_000, 400_000],
                          600.0, 20, 0.5, 100.0, 30,
                          [0.27, 0.2775, 0.285, 0.2925, 0.30],
                          [0.5, 0.75, 1.0, 1.25, 1.5], False, 3),
    "grad_500k": Workload("grad_500k", [500_000], 420.0, 15, 1.0, 60.0, 20,
                          [0.28], [1.0], False, 4),
    "field_3m_33bins": Workload("field_3m_33bins", [3_100_000], 600.0, 33, 0.25, 80.0, 20,
                                [0.28], [1.0], False, 5),
}


@dataclasses.dataclass
class Catalog:
    """Structure-of-arrays catalog; x, y are int32 lattice coordinates."""
    x: np.ndarray   # int32
    y: np.ndarray   # int32
    g1: np.ndarray  # float32
    g2: np.ndarray  # float32
    w: np.ndarray   # float32

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def subset(self, idx: np.ndarray) -> "Catalog":
        return Catalog(self.x[idx], self.y[idx], self.g1[idx], self.g2[idx], self.w[idx])

    def xy_arcmin(self):
        return self.x.astype(np.float64) * LATTICE_UNIT, self.y.astype(np.float64) * LATTICE_UNIT


def _streams(seed_index: int, n: int = 6) -> List[np.random.Generator]:
    ss = np.random.SeedSequence(SEED_BASE + seed_index)
    return [np.random.default_rng(s) for s in ss.spawn(n)]


def shear_field(side: float, rng: np.random.Generator, rms: float = 0.02,
                pixel: float = GRF_PIXEL) -> np.ndarray:
    """Periodic complex shear field gamma1 + i gamma2 on an (n, n) grid."""
    n = int(round(side / pixel))
    white = rng.standard_normal((n, n))
    kx = np.fft.fftfreq(n, d=pixel) * 2.0 * np.pi
    KX, KY = np.meshgrid(kx, kx, indexing="xy")
    k2 = KX * KX + KY * KY
    amp = np.zeros_like(k2)
    nz = k2 > 0
    amp[nz] = k2[nz] ** (-1.5 / 4.0)  # sqrt(P(k)) with P ~ k^-1.5
    kappa_hat = np.fft.fft2(white) * amp
    kappa = np.fft.ifft2(kappa_hat).real
    kappa *= rms / np.sqrt(np.mean(kappa * kappa))
    kappa_hat = np.fft.fft2(kappa)
    ks = np.zeros_like(kappa_hat)
    ks[nz] = ((KX[nz] ** 2 - KY[nz] ** 2) + 2j * KX[nz] * KY[nz]) / k2[nz]
    return np.fft.ifft2(ks * kappa_hat)


def sample_bilinear(field: np.ndarray, x: np.ndarray, y: np.ndarray, pixel: float) -> np.ndarray:
    """Periodic bilinear interpolation; field[iy, ix] sits at pixel centres."""
    n = field.shape[0]
    fx = x / pixel - 0.5
    fy = y / pixel - 0.5
    ix0 = np.floor(fx).astype(np.int64)
    iy0 = np.floor(fy).astype(np.int64)
    tx = fx - ix0
    ty = fy - iy0
    ix0 %= n
    iy0 %= n
    ix1 = (ix0 + 1) % n
    iy1 = (iy0 + 1) % n
    return ((1 - tx) * (1 - ty) * field[iy0, ix0] + tx * (1 - ty) * field[iy0, ix1]
            + (1 - tx) * ty * field[iy1, ix0] + tx * ty * field[iy1, ix1])


def uniform_positions(n: int, side: float, rng: np.random.Generator):
    top = int(round(side / LATTICE_UNIT))
    x = rng.integers(0, top, size=n, dtype=np.int64).astype(np.int32)
    y = rng.integers(0, top, size=n, dtype=np.int64).astype(np.int32)
    return x, y


def make_catalogs(wl: Workload, with_signal: bool = True, seed_offset: int = 0,
                  n_override: Optional[Sequence[int]] = None) -> List[Catalog]:
    """One catalog per tomographic bin, fully determined by the seed."""
    r_pos, r_noise, r_grf, r_w, _, _ = _streams(wl.seed_index + seed_offset)
    field = shear_field(wl.side, r_grf) if with_signal else None
    counts = list(n_override) if n_override is not None else list(wl.n_gal)
    cats = []
    for z, n in enumerate(counts):
        x, y = uniform_positions(n, wl.side, r_pos)
        noise = r_noise.standard_normal((2, n)) * wl.sigma_e[z]
        g = noise[0] + 1j * noise[1]
        if field is not None:
            xa = x.astype(np.float64) * LATTICE_UNIT
            ya = y.astype(np.float64) * LATTICE_UNIT
            g = g + wl.grf_scale[z] * sample_bilinear(field, xa, ya, GRF_PIXEL)
        if wl.unit_weights:
            w = np.ones(n, dtype=np.float32)
        else:
            w = r_w.uniform(0.5, 1.5, size=n).astype(np.float32)
        cats.append(Catalog(x, y, g.real.astype(np.float32), g.imag.astype(np.float32), w))
    return cats


def random_catalog(n: int, side: float, seed: int, sigma: float = 0.28,
                   unit_weights: bool = False) -> Catalog:
    """Small pure-noise catalog for unit tests."""
    rng = np.random.default_rng(seed)
    x, y = uniform_positions(n, side, rng)
    g = rng.standard_normal((2, n)) * sigma
    w = np.ones(n, np.float32) if unit_weights else rng.uniform(0.5, 1.5, n).astype(np.float32)
    return Catalog(x, y, g[0].astype(np.float32), g[1].astype(np.float32), w)


def centre_sample(n_total: int, n_sample: int, seed: int) -> np.ndarray:
    """Sorted random centre indices (without replacement)."""
    rng = np.random.default_rng(seed)
    n_sample = min(n_sample, n_total)
    return np.sort(rng.choice(n_total, size=n_sample, replace=False)).astype(np.int32)
