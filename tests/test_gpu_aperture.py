"""Third-order aperture statistics on the GPU (Sect. 4, Appendix C).

* FP64 integration of a random centroid-projected Gamma against the oracle's
  midpoint rule with the same filters: 1e-12 relative;
* the whole chain on a masked catalog -- edge-corrected multipoles, FP64
  solve, resummation, x -> centroid, aperture statistics -- against the same
  chain in the oracle.  The statistics of a shape-noise catalog are sums
  with heavy cancellation, so the error is measured over the whole output
  vector: ||gpu - oracle|| / ||oracle|| <= 1e-5 (FP32 multipoles at 1e-6
  amplified by the cancellation).
"""
import numpy as np
import pytest

from paper_2309_08601_amd.synth import random_catalog
from _util import box_for

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def t3():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08601_amd import t3 as mod
    return mod


APERTURES = [(1.0, 1.0, 1.0), (1.5, 2.0, 3.0), (3.0, 2.0, 1.5), (2.5, 2.5, 4.0), (4.0, 4.0, 4.0)]


def test_aperture_integration_matches_oracle(t3):
    from oracle.aperture import aperture_stats, correlators
    rng = np.random.default_rng(12)
    edges = np.geomspace(0.3, 20.0, 11)
    B, K, sets = 10, 20, 3
    plan = t3.Plan(edges, 4, box_size=1 << 22)
    g = rng.standard_normal((sets, 4, B, B, K)) + 1j * rng.standard_normal((sets, 4, B, B, K))
    corr, stats = plan.aperture_stats(torch.from_numpy(g).cuda(), APERTURES)
    pe = 2 * np.pi * np.arange(K + 1) / K
    for s in range(sets):
        ref = correlators(g[s], edges, pe, APERTURES)
        got = corr[s].cpu().numpy()
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
        assert np.allclose(stats[s].cpu().numpy(), aperture_stats(ref), rtol=0, atol=1e-12 * np.max(np.abs(ref)))


def test_aperture_chain_end_to_end(t3):
    from oracle import multipole as mp
    from oracle.aperture import aperture_stats, correlators
    from oracle.projection import bin_centres, phi_centres, x_to_centroid
    cat = random_catalog(3000, 40.0, seed=88)
    keep = np.nonzero(cat.x.astype(np.int64) + cat.y.astype(np.int64) > np.percentile(
        cat.x.astype(np.int64) + cat.y.astype(np.int64), 20))[0]
    cat = cat.subset(keep)
    edges = np.geomspace(0.8, 12.0, 7)
    nm, K = 6, 24
    lo, size = box_for(40.0)
    plan = t3.Plan(edges, nm, box_lo=lo, box_size=size, edge_correct=True)
    ups, _ = plan.forward(t3.DeviceCatalog.from_catalog(cat))
    _, gp = plan.normalise_resum(ups, n_phi=K)
    gc = plan.x_to_centroid(gp)
    corr, stats = plan.aperture_stats(gc, APERTURES)
    o = mp.multipoles(cat, edges, nm, w_max=2 * nm)
    g_all = mp.mode_coupling_correct(o["ups"], o["N"], nm)
    g_phi = mp.resum(g_all, nm, mp.phi_bin_edges(K))
    g_cent = x_to_centroid(g_phi, bin_centres(edges), phi_centres(K))
    ref = correlators(g_cent, edges, mp.phi_bin_edges(K), APERTURES)
    e_c = np.linalg.norm(corr.cpu().numpy() - ref) / np.linalg.norm(ref)
    e_s = np.linalg.norm(stats.cpu().numpy() - aperture_stats(ref)) / np.linalg.norm(aperture_stats(ref))
    print(f"aperture chain: correlators {e_c:.2e}, statistics {e_s:.2e}", flush=True)
    assert e_c <= 1e-5 and e_s <= 1e-5
