"""Third-order aperture statistics from the centroid-projected 3PCF
(TEST INFRASTRUCTURE ONLY).

Porth et al. (2023), Sect. 4 and Appendix C: the exponential filter Q_theta
(eq. CrittendenQ), the filter functions F_0..F_3 of the natural components
(eq. 3pcftomap3_helpers and the F_0, F_1 expressions that follow, F_2 and F_3
by cyclic permutation of the indices), the four complex correlators
(eqs. MFrom3pcfTheory, MFrom3pcfTheoryb) and the eight real aperture
statistics (eqs. MapTrafo8_1-MapTrafo8_8).

Triangle convention: vertex 1 at the origin, theta_1 = t1 (along x),
theta_2 = t2 e^{i phi}; q_k the centroid-to-vertex vectors (eq. QvecDef).

Reading (the filter assignment): the printed F_1 has its distinguished
index (the unconjugated f and the conjugated q) at vertex 2, so that, with
the paper's own definitions of the aperture measure (eq. MapGamma), the
filter Q (eq. CrittendenQ), the centroid projection and
Gamma_1 = <gamma*(X_1) gamma(X_2) gamma(X_3)> (eq. Gamma1_def), it is the
filter of the component conjugated at vertex 2.  The filter paired with
Gamma_mu (conjugate at vertex mu) and with the correlator whose conjugated
aperture has radius theta_mu is the printed F_1 with its indices rotated so
that the distinguished index is mu.  This is what a direct two-dimensional
integration of one triangle's shear triple against three apertures gives
(the pin in tests/test_oracle_pins.py), for F_0 as printed and for all three
rotations of F_1.
"""
from __future__ import annotations

import numpy as np


def q_vectors(t1, t2, phi):
    v1 = np.asarray(t1, dtype=np.float64) + 0j
    v2 = np.asarray(t2, dtype=np.float64) * np.exp(1j * np.asarray(phi, dtype=np.float64))
    return [-(v1 + v2) / 3.0, (2.0 * v1 - v2) / 3.0, (2.0 * v2 - v1) / 3.0]


def filters(t1, t2, phi, th1, th2, th3):
    """[F_0, F_1, F_2, F_3] at triangle (t1, t2, phi) for aperture radii
    (th1, th2, th3) (broadcast over all inputs)."""
    q = q_vectors(t1, t2, phi)
    th = [np.asarray(th1, dtype=np.float64), np.asarray(th2, dtype=np.float64),
          np.asarray(th3, dtype=np.float64)]
    T2 = np.sqrt((th[0] ** 2 * th[1] ** 2 + th[0] ** 2 * th[2] ** 2 + th[1] ** 2 * th[2] ** 2) / 3.0)  # Theta^2
    T4, T6 = T2 * T2, T2 ** 3
    S = th[0] ** 2 * th[1] ** 2 * th[2] ** 2 / T6
    M = S * np.asarray(t1) * np.asarray(t2) / (2.0 * np.pi * T4)
    aq2 = [np.abs(v) ** 2 for v in q]
    Z = sum((-th[i] ** 2 + 2 * th[(i + 1) % 3] ** 2 + 2 * th[(i + 2) % 3] ** 2) * aq2[i] for i in range(3)) / (6.0 * T4)
    f, g = [], []
    for i in range(3):
        a, b = (i + 1) % 3, (i + 2) % 3
        r = np.conj(q[i]) * (q[a] - q[b]) / aq2[i]
        f.append((th[a] ** 2 + th[b] ** 2) / (2.0 * T2) + r * (th[a] ** 2 - th[b] ** 2) / (6.0 * T2))
        g.append(th[a] ** 2 * th[b] ** 2 / T4 + r * th[i] ** 2 * (th[b] ** 2 - th[a] ** 2) / (3.0 * T4))
    P = aq2[0] * aq2[1] * aq2[2]
    ez = np.exp(-Z)
    F0 = M / 24.0 * P / T6 * np.conj(f[0]) ** 2 * np.conj(f[1]) ** 2 * np.conj(f[2]) ** 2 * ez

    def F1_perm(i1, i2, i3):
        """F_1 with (1, 2, 3) -> (i1, i2, i3)."""
        q1, q2, q3 = q[i1], q[i2], q[i3]
        f1, f2, f3 = f[i1], f[i2], f[i3]
        g2 = g[i2]
        t1s, t3s = th[i1] ** 2, th[i3] ** 2
        term = (P / (24.0 * T6) * np.conj(f3) ** 2 * np.conj(f1) ** 2 * f2 ** 2
                - (1.0 / 9.0) * q3 * q1 * np.conj(q2) ** 2 / T4 * np.conj(f3) * np.conj(f1) * f2 * np.conj(g2)
                + (1.0 / 27.0) * (q3 ** 2 * q1 ** 2 * np.conj(q2) ** 4 / (P * T2) * np.conj(g2) ** 2
                                  + 2.0 * t3s * t1s / T4 * q3 * q1 * np.conj(q2) ** 2 / (aq2[i2] * T2)
                                  * np.conj(f3) * np.conj(f1)))
        return M * ez * term

    # distinguished index (the printed index 2) at vertex mu
    F1 = F1_perm(2, 0, 1)
    F2 = F1_perm(0, 1, 2)
    F3 = F1_perm(1, 2, 0)
    return np.stack([F0, F1, F2, F3])


def q_filter(r, theta):
    """Q_theta(r) = r^2 / (4 pi theta^4) exp(-r^2 / (2 theta^2)) (eq. CrittendenQ)."""
    return r * r / (4.0 * np.pi * theta ** 4) * np.exp(-r * r / (2.0 * theta * theta))


def correlators(gamma_cent, radii_edges, phi_edges, apertures):
    """The four complex correlators <M^3>, <M* M^2>, <M M* M>, <M^2 M*>
    (eqs. MFrom3pcfTheory, MFrom3pcfTheoryb) from a binned Gamma^cent
    [4, B, B, K] by the midpoint rule on the (theta_1, theta_2, phi) bins
    (reading: the representative point of a bin is its arithmetic centre).
    apertures: [T, 3] radii.  Returns [T, 4] complex."""
    e = np.asarray(radii_edges, dtype=np.float64)
    pe = np.asarray(phi_edges, dtype=np.float64)
    tc = 0.5 * (e[:-1] + e[1:])
    dt = np.diff(e)
    pc = 0.5 * (pe[:-1] + pe[1:])
    dp = np.diff(pe)
    T1, T2, P = np.meshgrid(tc, tc, pc, indexing="ij")
    W = dt[:, None, None] * dt[None, :, None] * dp[None, None, :]
    out = np.zeros((len(apertures), 4), dtype=np.complex128)
    for a, (h1, h2, h3) in enumerate(apertures):
        F = filters(T1, T2, P, h1, h2, h3)
        out[a] = np.sum(gamma_cent * F * W[None], axis=(1, 2, 3))
    return out


def aperture_stats(corr):
    """Eqs. MapTrafo8_1-8 from [.., 4] correlators ordered (<M^3>, <M* M^2>,
    <M M* M>, <M^2 M*>): [.., 8] real = <Map^3>, <Mx Map^2>, <Map Mx Map>,
    <Map^2 Mx>, <Map Mx^2>, <Mx Map Mx>, <Mx^2 Map>, <Mx^3>."""
    c0, c1, c2, c3 = (corr[..., k] for k in range(4))
    return np.stack([np.real(c3 + c2 + c1 + c0) / 4, np.imag(c3 + c2 - c1 + c0) / 4,
                     np.imag(c3 - c2 + c1 + c0) / 4, np.imag(-c3 + c2 + c1 + c0) / 4,
                     np.real(c3 + c2 - c1 - c0) / 4, np.real(c3 - c2 + c1 - c0) / 4,
                     np.real(-c3 + c2 + c1 - c0) / 4, np.imag(c3 + c2 + c1 - c0) / 4], axis=-1)
