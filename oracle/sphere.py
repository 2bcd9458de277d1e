"""Curved-sky catalogs in flat patches (TEST INFRASTRUCTURE ONLY).

Porth et al. (2023), Appendix B: the footprint is cut into rectangular
patches (RA/Dec rectangles here), each patch is rotated so that its centre
lies on the equator at RA = 0, mapped to the plane by the sinusoidal
projection, and extended by theta_max; the multipoles are summed over
patches with centres from each patch's core only (eq. PatchGamma).

Readings:
* the rotation R takes the patch centre (ra0, dec0) to (0, 0): first a
  rotation about the polar axis by -ra0, then about the new y axis by dec0;
* shears (spin 2, in the local (east, north) frame, angles from east
  towards north -- the frame of the projected plane, x east and y north)
  are rotated by the reference-direction change of the rotation (what
  healpy's angle_ref supplies in the paper): with psi the angle from the
  local north at the image point to the image of the original north,
  measured from north towards east, position angles grow by psi, polar
  angles fall by psi, and gamma' = gamma e^{-2 i psi}.  The sinusoidal projection's own skew of the local axes
  (a second-order effect within a patch) is not applied, as in the paper;
* positions in the plane: x = lambda cos(beta), y = beta (rotated longitude
  and latitude, radians -> arcmin), rounded to the lattice;
* core: ra in [ra_lo, ra_hi), dec in [dec_lo, dec_hi) (degrees; the cores
  of a tiling partition the catalog); extended: the core rectangle widened
  by theta_max in dec and by theta_max / cos(dec) in ra at the galaxy's dec
  (contains every galaxy within theta_max of the core on the sphere for
  patches away from the poles).
"""
from __future__ import annotations

import numpy as np

ARCMIN = np.pi / (180.0 * 60.0)


def unit_vectors(ra, dec):
    """Cartesian unit vectors of (ra, dec) in radians."""
    ra = np.asarray(ra, dtype=np.float64)
    dec = np.asarray(dec, dtype=np.float64)
    return np.stack([np.cos(dec) * np.cos(ra), np.cos(dec) * np.sin(ra), np.sin(dec)], axis=-1)


def rotation(ra0, dec0):
    """3x3 matrix taking (ra0, dec0) (radians) to (0, 0)."""
    cz, sz = np.cos(-ra0), np.sin(-ra0)
    Rz = np.array([[cz, -sz, 0.0], [sz, cz, 0.0], [0.0, 0.0, 1.0]])
    cy, sy = np.cos(dec0), np.sin(dec0)
    Ry = np.array([[cy, 0.0, sy], [0.0, 1.0, 0.0], [-sy, 0.0, cy]])   # tilts +z towards +x by dec0
    return Ry @ Rz


def local_basis(v):
    """(east, north) unit tangent vectors at unit vectors v[..., 3]."""
    z = np.array([0.0, 0.0, 1.0])
    e = np.cross(z, v)
    e /= np.linalg.norm(e, axis=-1, keepdims=True)
    n = np.cross(v, e)
    return e, n


def shear_angle(v, R):
    """psi: angle (from north towards east) of R(north at v) in the basis at R v."""
    e, n = local_basis(v)
    w = v @ R.T
    e2, n2 = local_basis(w)
    rn = n @ R.T
    return np.arctan2(np.sum(rn * e2, axis=-1), np.sum(rn * n2, axis=-1))


def project(ra_deg, dec_deg, g1, g2, patch, unit_arcmin, centre=None):
    """One patch: lattice (x, y) relative to the patch centre, rotated
    shears, core mask, extended mask (theta_max taken from patch[4]).
    centre (ra, dec in degrees) overrides the projection centre."""
    ra_lo, ra_hi, dec_lo, dec_hi, theta_max = patch
    if centre is None:
        centre = (0.5 * (ra_lo + ra_hi), 0.5 * (dec_lo + dec_hi))
    ra0 = np.radians(centre[0])
    dec0 = np.radians(centre[1])
    v = unit_vectors(np.radians(ra_deg), np.radians(dec_deg))
    R = rotation(ra0, dec0)
    w = v @ R.T
    lam = np.arctan2(w[:, 1], w[:, 0])
    beta = np.arcsin(np.clip(w[:, 2], -1.0, 1.0))
    x = lam * np.cos(beta) / ARCMIN
    y = beta / ARCMIN
    xl = np.rint(x / unit_arcmin).astype(np.int64)
    yl = np.rint(y / unit_arcmin).astype(np.int64)
    psi = shear_angle(v, R)
    g = (np.asarray(g1, np.float64) + 1j * np.asarray(g2, np.float64)) * np.exp(-2j * psi)
    ra = np.asarray(ra_deg, np.float64)
    dec = np.asarray(dec_deg, np.float64)
    core = (ra >= ra_lo) & (ra < ra_hi) & (dec >= dec_lo) & (dec < dec_hi)
    tm = theta_max / 60.0
    dra = tm / np.cos(np.radians(np.clip(dec, -89.9, 89.9)))
    ext = (ra >= ra_lo - dra) & (ra < ra_hi + dra) & (dec >= dec_lo - tm) & (dec < dec_hi + tm)
    return xl, yl, g.real, g.imag, core, ext


def multipoles_patches(ra_deg, dec_deg, g1, g2, w, patches, theta_max, edges, n_max, unit_arcmin,
                       w_max=None, centre=None):
    """eq. PatchGamma: sum over patches of the multipoles with centres from
    the patch core and neighbours from the extended patch, each patch in its
    own projection (or all in the projection about ``centre``)."""
    from paper_2309_08601_amd.synth import Catalog
    from oracle import multipole as mp
    ups = N = None
    npairs = 0
    for (ra_lo, ra_hi, dec_lo, dec_hi) in patches:
        x, y, h1, h2, core, ext = project(ra_deg, dec_deg, g1, g2,
                                          (ra_lo, ra_hi, dec_lo, dec_hi, theta_max), unit_arcmin, centre)
        idx = np.nonzero(ext)[0]
        if idx.size == 0:
            continue
        sub = Catalog(x[idx].astype(np.int32), y[idx].astype(np.int32), h1[idx].astype(np.float32),
                      h2[idx].astype(np.float32), np.asarray(w, np.float32)[idx])
        cen = np.nonzero(core[idx])[0]
        if cen.size == 0:
            continue
        o = mp.multipoles(sub, edges, n_max, centres=cen, w_max=w_max)
        ups = o["ups"] if ups is None else ups + o["ups"]
        N = o["N"] if N is None else N + o["N"]
        npairs += o["npairs"]
    return dict(ups=ups, N=N, npairs=npairs)
