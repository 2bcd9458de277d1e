"""x -> centroid projection of the natural components (TEST INFRASTRUCTURE ONLY).

Porth et al. (2023), Sect. 2.3: eqs. X2Centroid0-X2Centroid3 with the
rotation factors written in the side lengths theta_1, theta_2 and the
opening angle phi (the expressions that follow eq. X2Centroid3):

    A1 = (t1 + t2 e^{-i phi}) / (t1 + t2 e^{i phi})      = (q1*/q1) e^{2 i phi_1}
    A2 = (t2 e^{-i phi} - 2 t1) / (t2 e^{i phi} - 2 t1)  = (q2*/q2) e^{2 i phi_1}
    A3 = (t1 - 2 t2 e^{-i phi}) / (t1 - 2 t2 e^{i phi})  = (q3*/q3) e^{2 i phi_1}

    Gamma_0^cent = Gamma_0^x  A1 A2 A3 e^{3 i phi}
    Gamma_1^cent = Gamma_1^x  A2 A3 / A1 e^{i phi}
    Gamma_2^cent = Gamma_2^x  A1 A3 / A2 e^{3 i phi}
    Gamma_3^cent = Gamma_3^x  A1 A2 / A3 e^{-i phi}

Reading for binned data: the factors are evaluated at one representative
(theta_1, theta_2, phi) per bin -- the caller's radii (default: the centre
of each radial bin) and the centre of each angular bin.  Where a factor's
denominator is exactly zero (a collinear configuration with some q_k = 0,
e.g. t1 = t2 at phi = pi or t2 = 2 t1 at phi = 0; the projection is
undefined there) the output is 0.
"""
from __future__ import annotations

import numpy as np


def centroid_factors(t1, t2, phi):
    """The four conversion factors [4, ...] (broadcast over the inputs)."""
    t1 = np.asarray(t1, dtype=np.float64)
    t2 = np.asarray(t2, dtype=np.float64)
    e = np.exp(1j * np.asarray(phi, dtype=np.float64))
    ec = np.conj(e)
    num = [t1 + t2 * ec, t2 * ec - 2.0 * t1, t1 - 2.0 * t2 * ec]
    den = [t1 + t2 * e, t2 * e - 2.0 * t1, t1 - 2.0 * t2 * e]
    bad = (den[0] == 0) | (den[1] == 0) | (den[2] == 0)
    A = [np.where(bad, 0.0, n / np.where(d == 0, 1.0, d)) for n, d in zip(num, den)]
    A1, A2, A3 = A
    with np.errstate(divide="ignore", invalid="ignore"):
        f = [A1 * A2 * A3 * e ** 3,
             np.where(bad, 0.0, A2 * A3 / np.where(bad, 1.0, A1)) * e,
             np.where(bad, 0.0, A1 * A3 / np.where(bad, 1.0, A2)) * e ** 3,
             np.where(bad, 0.0, A1 * A2 / np.where(bad, 1.0, A3)) * ec]
    return np.stack([np.where(bad, 0.0, v) for v in f])


def x_to_centroid(gamma_phi: np.ndarray, theta: np.ndarray, phi_centres: np.ndarray) -> np.ndarray:
    """gamma_phi[..., 4, B, B, K] in the x-projection -> centroid projection,
    factors at (theta[b1], theta[b2], phi_centres[k])."""
    t1 = np.asarray(theta, dtype=np.float64)[:, None, None]
    t2 = np.asarray(theta, dtype=np.float64)[None, :, None]
    ph = np.asarray(phi_centres, dtype=np.float64)[None, None, :]
    f = centroid_factors(t1, t2, ph)  # [4, B, B, K]
    return gamma_phi * f


def bin_centres(edges) -> np.ndarray:
    """Default representative radius per bin: the arithmetic centre."""
    e = np.asarray(edges, dtype=np.float64)
    return 0.5 * (e[:-1] + e[1:])


def phi_centres(n_phi: int) -> np.ndarray:
    return 2.0 * np.pi * (np.arange(n_phi) + 0.5) / n_phi
