"""Differentiable FP64 multipole estimator in plain torch (TEST INFRASTRUCTURE ONLY).

The same definitions as ``multipole.py`` (Porth et al. 2023, eqs. Gn_disc,
Upsilon0_Derivation, Upsilon1-3, 3PCF_Normalization, j = k terms removed),
written with torch CPU ops so that autograd gives the reference gradient of
a scalar loss with respect to every galaxy's g1, g2 and w.  Pair search is a
dense distance matrix: small catalogs only (a few thousand galaxies).

The loss used for the adjoint checks (a reading; the paper defines none):
    L = sum_{mu<4, n>=0, b1, b2} omega |Gamma_{mu,n}(b1,b2) - T_{mu,n}(b1,b2)|^2,
    Gamma = Upsilon / N_0.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np
import torch

from paper_2309_08601_amd.synth import LATTICE_UNIT


def pairs(x: np.ndarray, y: np.ndarray, edges: Sequence[float], chunk: int = 2048):
    """All ordered (centre i, neighbour j, bin b) with e_b <= r < e_{b+1}."""
    e = np.asarray(edges, dtype=np.float64) / LATTICE_UNIT
    e2 = e * e
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    I, J, Bn, DX, DY = [], [], [], [], []
    for s in range(0, x.size, chunk):
        dx = x[None, :] - x[s:s + chunk, None]
        dy = y[None, :] - y[s:s + chunk, None]
        r2 = dx * dx + dy * dy
        b = np.searchsorted(e2, r2, side="right") - 1
        ok = (r2 >= e2[0]) & (r2 < e2[-1])
        ii, jj = np.nonzero(ok)
        I.append(ii + s)
        J.append(jj)
        Bn.append(b[ii, jj])
        DX.append(dx[ii, jj])
        DY.append(dy[ii, jj])
    cat = lambda v: np.concatenate(v) if v else np.zeros(0)  # noqa: E731
    return cat(I).astype(np.int64), cat(J).astype(np.int64), cat(Bn).astype(np.int64), cat(DX), cat(DY)


def multipoles(x, y, g1: torch.Tensor, g2: torch.Tensor, w: torch.Tensor, edges, n_max: int,
               pair_list=None, diag: bool = True, centres=None):
    """Upsilon [4, n_max+1, B, B] and N [n_max+1, B, B] (orders n >= 0),
    complex128, differentiable in g1, g2, w (float64 tensors).

    ``centres`` (indices, optional): the sum over centres i of
    eq. Upsilon0_Derivation taken over that set only (an index listed twice
    counts twice); every galaxy remains a neighbour."""
    B = len(edges) - 1
    n = int(g1.shape[0])
    I, J, Bn, DX, DY = pair_list if pair_list is not None else pairs(x, y, edges)
    I = torch.from_numpy(I)
    J = torch.from_numpy(J)
    Bn = torch.from_numpy(Bn)
    r = np.sqrt(DX * DX + DY * DY)
    z = torch.from_numpy(DX / r + 1j * (DY / r))
    m_lo, m_hi = -n_max - 3, n_max - 1
    orders = list(range(m_lo, m_hi + 1))
    pw = {0: torch.ones_like(z)}
    for m in range(1, max(-m_lo, m_hi, n_max, 6) + 1):
        pw[m] = pw[m - 1] * z
        pw[-m] = torch.conj(pw[m])
    c = w * torch.complex(g1, g2)
    cj = c[J]
    wj = w[J].to(torch.complex128)
    key = I * B + Bn
    Zg = torch.stack([pw[m] for m in orders], dim=1)
    G = torch.zeros((n * B, len(orders)), dtype=torch.complex128).index_add(0, key, cj[:, None] * Zg)
    Zw = torch.stack([pw[m] for m in range(0, n_max + 1)], dim=1)
    W = torch.zeros((n * B, n_max + 1), dtype=torch.complex128).index_add(0, key, wj[:, None] * Zw)
    G = G.reshape(n, B, -1)
    W = W.reshape(n, B, -1)
    gi = lambda m: m - m_lo  # noqa: E731
    if centres is None:
        sel = torch.ones(n, dtype=torch.float64)
    else:
        sel = torch.zeros(n, dtype=torch.float64).index_add(
            0, torch.as_tensor(np.asarray(centres, dtype=np.int64)), torch.ones(len(centres), dtype=torch.float64))
    a = c * sel
    ac = torch.conj(c) * sel
    ups = []
    for nn in range(n_max + 1):
        u0 = -torch.einsum("i,ia,ib->ab", a, G[:, :, gi(nn - 3)], G[:, :, gi(-nn - 3)])
        u1 = -torch.einsum("i,ia,ib->ab", ac, G[:, :, gi(nn - 1)], G[:, :, gi(-nn - 1)])
        u2 = -torch.einsum("i,ia,ib->ab", a, torch.conj(G[:, :, gi(-nn - 1)]), G[:, :, gi(-nn - 3)])
        u3 = -torch.einsum("i,ia,ib->ab", a, G[:, :, gi(nn - 3)], torch.conj(G[:, :, gi(nn - 1)]))
        ups.append(torch.stack([u0, u1, u2, u3]))
    ups = torch.stack(ups, dim=1)  # [4, n_max+1, B, B]
    wc = (w * sel).to(torch.complex128)
    N = torch.stack([torch.einsum("i,ia,ib->ab", wc, W[:, :, k], torch.conj(W[:, :, k]))
                     for k in range(n_max + 1)])
    if diag:
        D6 = torch.zeros(n * B, dtype=torch.complex128).index_add(0, key, cj * cj * pw[-6]).reshape(n, B)
        D2 = torch.zeros(n * B, dtype=torch.complex128).index_add(0, key, cj * cj * pw[-2]).reshape(n, B)
        DA = torch.zeros(n * B, dtype=torch.complex128).index_add(
            0, key, (cj * torch.conj(cj)) * pw[-2]).reshape(n, B)
        DW = torch.zeros(n * B, dtype=torch.complex128).index_add(0, key, wj * wj).reshape(n, B)
        eye = torch.eye(B, dtype=torch.complex128)
        corr = torch.stack([torch.einsum("i,ia->a", a, D6), torch.einsum("i,ia->a", ac, D2),
                            torch.einsum("i,ia->a", a, DA), torch.einsum("i,ia->a", a, DA)])
        ups = ups + corr[:, None, :, None] * eye[None, None]
        N = N - torch.einsum("i,ia->a", wc, DW)[None, :, None] * eye[None]
    return ups, N


def gamma(ups: torch.Tensor, N: torch.Tensor) -> torch.Tensor:
    n0 = N[0].real
    return ups / n0[None, None]


def loss(gam: torch.Tensor, target: torch.Tensor, omega: torch.Tensor) -> torch.Tensor:
    d = gam - target
    return torch.sum(omega * (d.real ** 2 + d.imag ** 2))


def loss_weights(target: torch.Tensor) -> torch.Tensor:
    """omega = 1 / mean_n |T_{mu,n}(b1, b2)|^2 (fixed per (mu, b1, b2))."""
    m = torch.mean(target.real ** 2 + target.imag ** 2, dim=1, keepdim=True)
    return (1.0 / torch.clamp(m, min=1e-300)).expand_as(target.real).contiguous()
