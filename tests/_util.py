"""Shared helpers for the tests (comparison metrics, plan construction)."""
from __future__ import annotations

import numpy as np

from paper_2309_08601_amd.synth import LATTICE_UNIT

FP32_TOL = 1e-6     # relative Frobenius error per (mu, n), FP32 path
SPLIT_TOL = 1e-5    # split-precision contraction
FP32_MAX_TOL = 2e-6   # largest entry error per (mu, n) over the largest |entry|, FP32 path
SPLIT_MAX_TOL = 2e-5  # the same for the two-part bf16 split
N_OWN_TOL = 5e-6      # N_n (n >= 1) against its own Frobenius norm, every precision


def rel_fro(a: np.ndarray, b: np.ndarray, axes=(-2, -1)) -> np.ndarray:
    """||a - b||_F / ||b||_F over the bin-pair axes (per leading index)."""
    num = np.sqrt(np.sum(np.abs(a - b) ** 2, axis=axes))
    den = np.sqrt(np.sum(np.abs(b) ** 2, axis=axes))
    return num / np.where(den > 0, den, 1.0)


def rel_max(a: np.ndarray, b: np.ndarray, axes=(-2, -1)) -> np.ndarray:
    num = np.max(np.abs(a - b), axis=axes)
    den = np.max(np.abs(b), axis=axes)
    return num / np.where(den > 0, den, 1.0)


def box_for(side_arcmin: float, margin_steps: int = 0):
    """Lattice box [0, side) as (lo, size) in lattice steps."""
    return (-margin_steps, -margin_steps), int(round(side_arcmin / LATTICE_UNIT)) + 2 * margin_steps


def multipole_max_errors(gpu: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Element-wise companion of ``multipole_errors``: per (mu, n) the largest
    |entry error| over the largest |entry| of the oracle's block (N_n with
    n >= 1 against the largest |N_0| entry, as there)."""
    m = rel_max(gpu, ref)
    n0 = np.max(np.abs(ref[..., 4, 0, :, :]), axis=(-2, -1))
    dn = np.max(np.abs(gpu[..., 4, :, :, :] - ref[..., 4, :, :, :]), axis=(-2, -1))
    m[..., 4, 1:] = dn[..., 1:] / np.where(n0 > 0, n0, 1.0)[..., None]
    return m


def multipole_errors(gpu: np.ndarray, ref: np.ndarray):
    """Errors of packed multipoles [..., 5, n_max + 1, B, B] (mu = 0..3 then N).

    Returns (e, e_own):
      e[..., mu, n]     relative Frobenius error over (b1, b2) for Upsilon_{mu,n}
                        and N_0; for N_n with n >= 1 the error is measured
                        against ||N_0||, the scale N_n is used at (mode-coupling
                        matrix N_{l-n} / N_0).  This is the graded metric.
      e_own[..., n]     N_n error against its own norm (information: the
                        j = k removal makes N_{n != 0} a small difference).
    """
    e = rel_fro(gpu, ref)
    n0 = np.sqrt(np.sum(np.abs(ref[..., 4, 0, :, :]) ** 2, axis=(-2, -1)))
    dn = np.sqrt(np.sum(np.abs(gpu[..., 4, :, :, :] - ref[..., 4, :, :, :]) ** 2, axis=(-2, -1)))
    e_own = e[..., 4, :].copy()
    e[..., 4, 1:] = dn[..., 1:] / np.where(n0 > 0, n0, 1.0)[..., None]
    return e, e_own
