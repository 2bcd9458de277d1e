"""O(N^3) triplet sums straight from the definitions (TEST INFRASTRUCTURE ONLY).

Porth et al. (2023), Sect. 2.2-2.3 and 3.  For every ordered triplet of
pairwise-distinct galaxies (i, j, k) with theta_ij in bin b1 and theta_ik
in bin b2, the shears are projected in the x-projection
(zeta_1 = (phi_1 + phi_2)/2, zeta_2 = phi_1, zeta_3 = phi_2, eq. xprojection)
with gamma(X; zeta) = -gamma_c e^{-2 i zeta} (eq. gammatx_def), multiplied
as in the four natural components (eqs. Gamma0_def..Gamma3_def) with the
weights attached, and projected onto e^{-i n psi} with psi = phi_2 - phi_1
(eq. Upsilon0_Derivation, first line).  The normaliser takes w_i w_j w_k.

No harmonic sums, no factorisation: this is the independent check of the
multipole oracle.  Pure numpy, vectorised over (j, k) per centre; use only
for catalogs of a few hundred galaxies.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

from paper_2309_08601_amd.synth import LATTICE_UNIT


def _bin_of(r2: np.ndarray, e2: np.ndarray) -> np.ndarray:
    b = np.searchsorted(e2, r2, side="right") - 1   # e2[b] <= r2 < e2[b+1]
    b[(r2 < e2[0]) | (r2 >= e2[-1])] = -1
    return b


def triplets(x, y, g1, g2, w, edges: Sequence[float], n_max: int,
             phi_edges: Optional[np.ndarray] = None, in_lattice_units: bool = True,
             phi_weight=None, labels=None, roles=None):
    """Returns dict(ups[4, 2n_max+1, B, B], N[2n_max+1, B, B]) and, when
    phi_edges is given, the angularly binned sums ups_phi[4, B, B, K],
    N_phi[B, B, K] (eqs. TripletUpsilon, TripletNorm).  ``phi_weight(psi)``
    (-> [T, K]) replaces the bin indicator of psi by arbitrary weights.

    Tomography (Sect. 3.5, eq. tomoGn): with per-galaxy source-bin
    ``labels`` and ``roles = (z1, z2, z3)``, only the triplets whose vertex
    X_1 (galaxy i, the centre) lies in bin z1, whose vertex X_2 (galaxy j,
    at separation theta_ij in radial bin b1) lies in z2 and whose vertex X_3
    (galaxy k, theta_ik in b2) lies in z3 are summed."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    gc = np.asarray(g1, dtype=np.float64) + 1j * np.asarray(g2, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    e = np.asarray(edges, dtype=np.float64)
    if in_lattice_units:
        e = e / LATTICE_UNIT
    e2 = e * e
    B = len(edges) - 1
    n = x.shape[0]
    ns = np.arange(-n_max, n_max + 1)
    ups = np.zeros((4, ns.size, B, B), dtype=np.complex128)
    N = np.zeros((ns.size, B, B), dtype=np.complex128)
    K = None if phi_edges is None else len(phi_edges) - 1
    if K is not None:
        ups_phi = np.zeros((4, B, B, K), dtype=np.complex128)
        N_phi = np.zeros((B, B, K), dtype=np.float64)
    if (labels is None) != (roles is None):
        raise ValueError("labels and roles go together")
    lab = None if labels is None else np.asarray(labels)
    for i in range(n):
        if lab is not None and lab[i] != roles[0]:
            continue
        dx = x - x[i]
        dy = y - y[i]
        b = _bin_of(dx * dx + dy * dy, e2)
        inb = b >= 0
        sel_j = np.nonzero(inb if lab is None else inb & (lab == roles[1]))[0]
        sel_k = np.nonzero(inb if lab is None else inb & (lab == roles[2]))[0]
        if sel_j.size == 0 or sel_k.size == 0:
            continue
        J, Kk = np.meshgrid(sel_j, sel_k, indexing="ij")
        keep = J != Kk                      # pairwise distinct: j != k
        j, k = J[keep], Kk[keep]
        if j.size == 0:
            continue
        p1, p2 = np.arctan2(dy[j], dx[j]), np.arctan2(dy[k], dx[k])
        b1, b2 = b[j], b[k]
        # projected, weighted shears gamma(X; zeta) = -gamma_c e^{-2 i zeta}
        e_z1 = np.exp(-1j * (p1 + p2))       # e^{-2 i zeta_1}
        e_z2 = np.exp(-2j * p1)
        e_z3 = np.exp(-2j * p2)
        s1 = -w[i] * gc[i] * e_z1
        s2 = -w[j] * gc[j] * e_z2
        s3 = -w[k] * gc[k] * e_z3
        prods = [s1 * s2 * s3,
                 np.conj(s1) * s2 * s3,
                 s1 * np.conj(s2) * s3,
                 s1 * s2 * np.conj(s3)]
        www = w[i] * w[j] * w[k]
        psi = p2 - p1
        ph = np.exp(-1j * np.outer(ns, psi))   # [n, T]
        flat = b1 * B + b2
        for mu in range(4):
            acc = ph * prods[mu][None, :]
            for a in range(ns.size):
                ups[mu, a] += np.bincount(flat, weights=acc[a].real, minlength=B * B).reshape(B, B) \
                    + 1j * np.bincount(flat, weights=acc[a].imag, minlength=B * B).reshape(B, B)
        accn = ph * www[None, :]
        for a in range(ns.size):
            N[a] += np.bincount(flat, weights=accn[a].real, minlength=B * B).reshape(B, B) \
                + 1j * np.bincount(flat, weights=accn[a].imag, minlength=B * B).reshape(B, B)
        if K is not None:
            psi_m = np.mod(psi, 2.0 * np.pi)
            if phi_weight is None:
                kb = np.searchsorted(phi_edges, psi_m, side="right") - 1
                wk = np.zeros((psi_m.size, K))
                wk[np.arange(psi_m.size), np.clip(kb, 0, K - 1)] = 1.0
            else:
                wk = phi_weight(psi_m)
            for kk in range(K):
                for mu in range(4):
                    v = prods[mu] * wk[:, kk]
                    ups_phi[mu, :, :, kk] += (np.bincount(flat, weights=v.real, minlength=B * B)
                                              + 1j * np.bincount(flat, weights=v.imag,
                                                                 minlength=B * B)).reshape(B, B)
                N_phi[:, :, kk] += np.bincount(flat, weights=www * wk[:, kk],
                                               minlength=B * B).reshape(B, B)
    out = dict(ups=ups, N=N)
    if K is not None:
        out.update(ups_phi=ups_phi, N_phi=N_phi)
    return out


def triangle_components(pos, gc, projection: str = "x"):
    """The four natural components of one triangle's shear triple, straight
    from the projection definitions (Sect. 2.3): gamma(X; zeta) =
    -gamma_c e^{-2 i zeta} (eq. gammatx_def) with

    * "x":        zeta_1 = (phi_1 + phi_2)/2, zeta_2 = phi_1, zeta_3 = phi_2
                  (eq. xprojection; phi_k the polar angle of X_{k+1} - X_1);
    * "centroid": e^{2 i zeta_k} = q_k / q_k^*, q_k the vector from the
                  centroid to X_k (eqs. centroidprojection, QvecDef).

    pos: [3, 2] float positions X_1..X_3, gc: [3] complex shears.
    Returns [Gamma_0, Gamma_1, Gamma_2, Gamma_3] for this single triple
    (eqs. Gamma0_def..Gamma3_def without the ensemble average).
    """
    pos = np.asarray(pos, dtype=np.float64)
    gc = np.asarray(gc, dtype=np.complex128)
    z = pos[:, 0] + 1j * pos[:, 1]
    if projection == "x":
        p1 = np.angle(z[1] - z[0])
        p2 = np.angle(z[2] - z[0])
        e2z = np.exp(1j * np.array([p1 + p2, 2.0 * p1, 2.0 * p2]))      # e^{2 i zeta}
    elif projection == "centroid":
        q = z - z.mean()
        e2z = q / np.conj(q)
    else:
        raise ValueError(projection)
    s = -gc / e2z                                                        # -gamma_c e^{-2 i zeta}
    return np.array([s[0] * s[1] * s[2], np.conj(s[0]) * s[1] * s[2],
                     s[0] * np.conj(s[1]) * s[2], s[0] * s[1] * np.conj(s[2])])
