"""Grid-based and combined multipole estimators (TEST INFRASTRUCTURE ONLY).

Porth et al. (2023), Sect. 3.2 (grid-based approximation), Sect. 3.3
(combined estimator, eq. CombinedEstimatorRegridding) and Appendix A
(multi-resolution grids Delta_l = 2^(l-1) Delta_1, blocks of the
(Theta_1, Theta_2) plane).

Definitions used here:
* pixelisation: square pixels of side Delta (lattice steps) anchored at the
  plan box corner; pixel (px, py) of a galaxy at lattice (x, y) is
  floor((x - x0) / Delta), floor((y - y0) / Delta); pixel values are the
  sums (w gamma)^(Delta) = sum_i w_i gamma_i and w^(Delta) = sum_i w_i over
  the galaxies inside (FP64); only non-empty pixels are kept;
* pixel positions: the lower-left corner (x0 + px Delta, y0 + py Delta);
  only differences enter the estimator, so corners and centres give the
  same separations and angles;
* G_n^Delta and W_n^Delta (the convolution of the pixel values with the
  bin kernel e^{i n phi} 1(theta in Theta)) are the discrete harmonic sums
  of eq. (Gn_disc) over the pixel catalog, evaluated at the pixels;
* grid estimator (eq. UpsilonmuGrid): the discrete estimator applied to
  the pixel catalog, including the removal of the degenerate pairs of one
  neighbour pixel on the diagonal b1 = b2 (the reading taken for the
  discrete estimator, applied to pixels);
* combined estimator: every radial bin has a level l (0 = discrete,
  l >= 1 = grid of side Delta_1 2^(l-1)), non-decreasing with the bin.
  A block (b1, b2) is evaluated at the coarser level L = max(l1, l2): the
  finer side's products (w gamma) G (or w W) are mapped onto the level-L
  pixels (regridding) and contracted with the coarse harmonics at the
  pixel -- eq. (CombinedEstimatorRegridding), second and third lines, with
  its leading minus restored, and the same rule for two grids of different
  resolution (the higher resolution is mapped to the coarser grid).
  Blocks with l1 = l2 are the discrete (l = 0) or grid (l >= 1) estimator
  at that level.
"""
from __future__ import annotations

import dataclasses
from typing import Sequence

import numpy as np

from oracle import multipole as mp


@dataclasses.dataclass
class PixelCatalog:
    """Non-empty pixels of one resolution: corners (lattice), FP64 sums."""
    x: np.ndarray      # int64 lattice corner
    y: np.ndarray
    c: np.ndarray      # complex128 sum of w gamma
    w: np.ndarray      # float64 sum of w
    side: int
    # fields read by oracle.multipole.harmonics
    g1: np.ndarray = None
    g2: np.ndarray = None

    def __post_init__(self):
        with np.errstate(divide="ignore", invalid="ignore"):
            g = np.where(self.w != 0, self.c / self.w, 0.0)
        self.g1 = g.real.copy()
        self.g2 = g.imag.copy()

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def pixel_index(x, y, side: int, box_lo):
    """2-D pixel indices of lattice positions (floor division)."""
    px = np.floor_divide(np.asarray(x, np.int64) - int(box_lo[0]), int(side))
    py = np.floor_divide(np.asarray(y, np.int64) - int(box_lo[1]), int(side))
    return px, py


def pixelise(cat, side: int, box_lo):
    """Pixel catalog of side ``side`` and, per galaxy, its pixel's row."""
    px, py = pixel_index(cat.x, cat.y, side, box_lo)
    keys = np.stack([py, px], axis=1)
    uniq, inv = np.unique(keys, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    c = np.zeros(uniq.shape[0], np.complex128)
    w = np.zeros(uniq.shape[0], np.float64)
    ci = cat.w.astype(np.float64) * (cat.g1.astype(np.float64) + 1j * cat.g2.astype(np.float64))
    np.add.at(c, inv, ci)
    np.add.at(w, inv, cat.w.astype(np.float64))
    pc = PixelCatalog(int(box_lo[0]) + uniq[:, 1] * side, int(box_lo[1]) + uniq[:, 0] * side, c, w, side)
    return pc, inv


def _rows_at(units_x, units_y, coarse: PixelCatalog, box_lo):
    """Row of the coarse pixel that holds each unit (galaxy or finer-pixel corner)."""
    px, py = pixel_index(units_x, units_y, coarse.side, box_lo)
    cx, cy = pixel_index(coarse.x, coarse.y, coarse.side, box_lo)
    order = np.lexsort((cx, cy))
    ck = cy[order] * (1 << 32) + cx[order]
    uk = py * (1 << 32) + px
    pos = np.searchsorted(ck, uk)
    assert np.all(ck[np.minimum(pos, ck.size - 1)] == uk), "unit outside every coarse pixel"
    return order[pos]


def _regrid(rows, values, n_rows):
    """Sum of per-unit values [n_units, ...] into their coarse pixels: the
    product with the 0/1 membership matrix M[P, u] = [unit u lies in P]."""
    from scipy.sparse import csr_matrix
    n_units = rows.shape[0]
    M = csr_matrix((np.ones(n_units), (rows, np.arange(n_units))), shape=(n_rows, n_units))
    flat = values.reshape(n_units, -1)
    return np.asarray(M @ flat).reshape((n_rows,) + values.shape[1:])


def _cross_blocks(cf, wf, hf, rows, hL, n_rows, n_max, w_max, fine_is_b1):
    """Blocks between a finer bin set (units: c, w, harmonics hf) and the
    level-L bin set (harmonics hL at the L pixels), regridded to level L.
    Returns ups[4, 2 n_max + 1, Bf, BL] (fine_is_b1) or [.., BL, Bf], and N."""
    gf = lambda m: m - hf["m_lo"]  # noqa: E731
    gl = lambda m: m - hL["m_lo"]  # noqa: E731
    c = cf.astype(np.complex128)[:, None, None]
    # the finer side's products with the centre factor, summed into the
    # level-L pixels (every order at once)
    Ac = _regrid(rows, c * hf["G"], n_rows)                  # sum c G
    Acc = _regrid(rows, np.conj(c) * hf["G"], n_rows)        # sum c* G
    Acj = _regrid(rows, c * np.conj(hf["G"]), n_rows)        # sum c conj G
    Aw = _regrid(rows, wf[:, None, None] * hf["W"], n_rows)  # sum w W
    Bf, BL = hf["G"].shape[1], hL["G"].shape[1]
    # order axis first: every [pixel, bin] slice below is contiguous
    first = lambda a: np.ascontiguousarray(np.moveaxis(a, 2, 0))  # noqa: E731
    Ac, Acc, Acj, Aw = first(Ac), first(Acc), first(Acj), first(Aw)
    GL, WL = first(hL["G"]), first(hL["W"])
    shp = (Bf, BL) if fine_is_b1 else (BL, Bf)
    ups = np.zeros((4, 2 * n_max + 1) + shp, np.complex128)
    N = np.zeros((2 * w_max + 1,) + shp, np.complex128)
    for n in range(-n_max, n_max + 1):
        k = n + n_max
        if fine_is_b1:
            # sum_P [sum_{u in P} X(u, b1)] Y(P, b2), X carrying the centre factor
            ups[0, k] = -Ac[gf(n - 3)].T @ GL[gl(-n - 3)]
            ups[1, k] = -Acc[gf(n - 1)].T @ GL[gl(-n - 1)]
            ups[2, k] = -Acj[gf(-n - 1)].T @ GL[gl(-n - 3)]
            ups[3, k] = -Ac[gf(n - 3)].T @ np.conj(GL[gl(n - 1)])
        else:
            # sum_P X'(P, b1) [sum_{u in P} c_u Y(u, b2)], X' without the centre factor
            ups[0, k] = -GL[gl(n - 3)].T @ Ac[gf(-n - 3)]
            ups[1, k] = -GL[gl(n - 1)].T @ Acc[gf(-n - 1)]
            ups[2, k] = -np.conj(GL[gl(-n - 1)]).T @ Ac[gf(-n - 3)]
            ups[3, k] = -GL[gl(n - 3)].T @ Acj[gf(n - 1)]
    for n in range(-w_max, w_max + 1):
        if fine_is_b1:
            N[n + w_max] = Aw[n + hf["w_max"]].T @ np.conj(WL[n + hL["w_max"]])
        else:
            N[n + w_max] = WL[n + hL["w_max"]].T @ np.conj(Aw[n + hf["w_max"]])
    return ups, N


def check_levels(levels: Sequence[int], n_bins: int):
    lv = [int(v) for v in levels]
    if len(lv) != n_bins or min(lv) < 0 or any(b < a for a, b in zip(lv, lv[1:])):
        raise ValueError("levels: one per bin, >= 0, non-decreasing")
    return lv


def multipoles_combined(cat, edges: Sequence[float], n_max: int, delta: int, levels: Sequence[int],
                        box_lo=(0, 0), w_max=None, diag: bool = True):
    """Combined discrete / multi-resolution grid multipoles of every block.

    delta: Delta_1 in lattice steps; levels[b]: 0 discrete, l >= 1 grid of
    side delta 2^(l-1).  Returns ups[4, 2 n_max + 1, B, B], N[2 w_max + 1,
    B, B] (index n + n_max, n + w_max), npairs (galaxy pairs of the
    discrete bins plus pixel pairs of the grid bins) and the pixel catalogs.
    diag=False keeps the degenerate pairs (the literal sums).
    """
    edges = np.asarray(edges, np.float64)
    B = edges.size - 1
    lv = check_levels(levels, B)
    wm = n_max if w_max is None else int(w_max)
    ups = np.zeros((4, 2 * n_max + 1, B, B), np.complex128)
    N = np.zeros((2 * wm + 1, B, B), np.complex128)
    npairs = 0
    # per level: units (galaxies or pixels), their factors, harmonics of its bins
    units = {}
    for L in sorted(set(lv)):
        bins = [b for b in range(B) if lv[b] == L]
        sub = edges[bins[0]:bins[-1] + 2]
        if L == 0:
            u = cat
            c = cat.w.astype(np.float64) * (cat.g1.astype(np.float64) + 1j * cat.g2.astype(np.float64))
            w = cat.w.astype(np.float64)
        else:
            u, _ = pixelise(cat, delta << (L - 1), box_lo)
            c, w = u.c, u.w
        h = mp.harmonics(u, u, sub, n_max, w_max=wm)
        npairs += int(h["npairs"].sum())
        units[L] = (u, c, w, h, bins)
        # blocks inside the level: the discrete (L = 0) or grid estimator
        uu, nn = mp.upsilon_from_harmonics(c, w, h, h, n_max, diag=diag)
        sl = slice(bins[0], bins[-1] + 1)
        ups[:, :, sl, sl] = uu
        N[:, sl, sl] = nn
    # blocks across levels, regridded to the coarser one
    for L, (uL, cL, wL, hL, binsL) in units.items():
        slL = slice(binsL[0], binsL[-1] + 1)
        for l, (uf, cf, wf, hf, binsf) in units.items():
            if l >= L:
                continue
            slf = slice(binsf[0], binsf[-1] + 1)
            rows = _rows_at(uf.x, uf.y, uL, box_lo)
            u1, n1 = _cross_blocks(cf, wf, hf, rows, hL, uL.n, n_max, wm, True)
            ups[:, :, slf, slL] = u1
            N[:, slf, slL] = n1
            u2, n2 = _cross_blocks(cf, wf, hf, rows, hL, uL.n, n_max, wm, False)
            ups[:, :, slL, slf] = u2
            N[:, slL, slf] = n2
    return dict(ups=ups, N=N, npairs=npairs, units=units)


def multipoles_broadcast(cat, edges, n_max, delta, levels, box_lo=(0, 0), w_max=None):
    """The same blocks from the first line of eq. (CombinedEstimatorRegridding):
    a sum over galaxies with every grid bin's harmonics taken at the galaxy's
    pixel (not divided by the pixel's galaxy count) -- an independent
    arrangement of the sum used to pin the regridding."""
    edges = np.asarray(edges, np.float64)
    B = edges.size - 1
    lv = check_levels(levels, B)
    wm = n_max if w_max is None else int(w_max)
    m_lo, m_hi = mp.g_order_range(n_max)
    G = np.zeros((cat.n, B, m_hi - m_lo + 1), np.complex128)
    W = np.zeros((cat.n, B, 2 * wm + 1), np.complex128)
    D = np.zeros((cat.n, B, 4), np.complex128)
    for L in sorted(set(lv)):
        bins = [b for b in range(B) if lv[b] == L]
        sub = edges[bins[0]:bins[-1] + 2]
        sl = slice(bins[0], bins[-1] + 1)
        if L == 0:
            h = mp.harmonics(cat, cat, sub, n_max, w_max=wm)
            G[:, sl], W[:, sl], D[:, sl] = h["G"], h["W"], h["D"]
        else:
            pc, inv = pixelise(cat, delta << (L - 1), box_lo)
            h = mp.harmonics(pc, pc, sub, n_max, w_max=wm)
            G[:, sl], W[:, sl], D[:, sl] = h["G"][inv], h["W"][inv], h["D"][inv]
    h = dict(G=G, W=W, D=D, m_lo=m_lo, w_max=wm)
    c = cat.w.astype(np.float64) * (cat.g1.astype(np.float64) + 1j * cat.g2.astype(np.float64))
    ups, N = mp.upsilon_from_harmonics(c, cat.w.astype(np.float64), h, h, n_max, diag=True)
    return dict(ups=ups, N=N)


def default_levels(edges, delta_arcmin: float, ratio: float = 20.0, theta_disc: float = 0.0,
                   max_level: int = 8):
    """Level per bin: discrete below theta_disc (lower edge), otherwise the
    coarsest grid with lower edge >= ratio * Delta_l (the accuracy criterion
    Theta >= 20 Delta of Sect. 3.3), discrete if none qualifies."""
    lv = []
    for lo in np.asarray(edges, np.float64)[:-1]:
        best = 0
        if lo >= theta_disc:
            for l in range(1, max_level + 1):
                if lo >= ratio * delta_arcmin * 2 ** (l - 1):
                    best = l
        lv.append(best)
    for i in range(1, len(lv)):
        lv[i] = max(lv[i], lv[i - 1])
    return lv
