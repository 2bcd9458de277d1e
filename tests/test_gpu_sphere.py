"""Curved-sky catalogs through flat patches (Appendix B) on the GPU, against
the oracle's patch sum (eq. PatchGamma) with its own rotation, shear
reference-direction change and sinusoidal projection, on a footprint at
Dec 40-44 deg split into four 2 deg x 2 deg patches with theta_max overlap."""
import numpy as np
import pytest

from _util import FP32_TOL, rel_fro

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def t3():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08601_amd import t3 as mod
    return mod


def _sphere_catalog(n, seed):
    rng = np.random.default_rng(seed)
    ra = rng.uniform(150.0, 154.0, n)
    sdec = rng.uniform(np.sin(np.radians(40.0)), np.sin(np.radians(44.0)), n)  # uniform on the sphere
    dec = np.degrees(np.arcsin(sdec))
    g1 = rng.normal(0.0, 0.28, n).astype(np.float32)
    g2 = rng.normal(0.0, 0.28, n).astype(np.float32)
    w = rng.uniform(0.5, 1.5, n).astype(np.float32)
    return ra, dec, g1, g2, w


PATCHES = [(150.0, 152.0, 40.0, 42.0), (152.0, 154.0, 40.0, 42.0), (150.0, 152.0, 42.0, 44.0),
           (152.0, 154.0, 42.0, 44.0)]


@pytest.mark.parametrize("ec", [False, True])
def test_sphere_patches_match_oracle(t3, ec):
    from oracle.sphere import multipoles_patches
    ra, dec, g1, g2, w = _sphere_catalog(6000, seed=404)
    edges = np.geomspace(0.5, 10.0, 6)
    nm, tmax = 6, 10.0
    plan = t3.Plan(edges, nm, box_lo=(-(1 << 23), -(1 << 23)), box_size=1 << 24, edge_correct=ec)
    dev = "cuda"
    ups, npairs = plan.forward_sphere(*(torch.from_numpy(np.ascontiguousarray(a)).to(dev)
                                        for a in (ra, dec, g1, g2, w)), PATCHES, tmax)
    o = multipoles_patches(ra, dec, g1, g2, w, PATCHES, tmax, edges, nm, 2.0 ** -16,
                           w_max=2 * nm if ec else None)
    assert npairs == o["npairs"]
    u4, N = plan.split_ups(ups)
    wm = 2 * nm if ec else nm
    e_u = rel_fro(u4.cpu().numpy(), o["ups"][:, nm:]).max()
    n_ref = o["N"][wm:]
    e_n = (np.linalg.norm((N.cpu().numpy() - n_ref).reshape(n_ref.shape[0], -1), axis=1)
           / np.linalg.norm(n_ref[0])).max()
    print(f"sphere patches (edge-correct={ec}): {npairs} pairs, Upsilon {e_u:.2e}, N_n/N_0 {e_n:.2e}", flush=True)
    assert e_u <= FP32_TOL and e_n <= FP32_TOL
