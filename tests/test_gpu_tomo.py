"""Batched tomography: one stage-1 launch for all neighbour catalogs (one
wavefront per task, or a persistent work queue), one stage-2 launch for all
ordered (Z2, Z3) pairs, the chunk schedule captured as one HIP graph.

* graph replays (with eager work in between) equal the eager schedule bit
  for bit, for both stage-1 launch modes;
* the autotuner's choice reproduces the same multipoles;
* the 5-bin workload (0.3/0.6/0.8/0.7/0.4 M galaxies in 10 deg x 10 deg,
  20 bins 0.5'-100', n_max 30) matches the oracle on 4,000 centres per
  source bin for all 125 ordered triples (relative Frobenius 1e-6, largest
  entry 2e-6, N_n against its own norm 5e-6, per block).
"""
import numpy as np
import pytest

from paper_2309_08601_amd.synth import WORKLOADS, centre_sample, make_catalogs, random_catalog
from _util import FP32_MAX_TOL, FP32_TOL, N_OWN_TOL, box_for, multipole_errors, multipole_max_errors

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def t3():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08601_amd import t3 as mod
    return mod


def _small(t3):
    cats = [random_catalog(n, 40.0, seed=700 + z) for z, n in enumerate([900, 1500, 600, 1200])]
    return cats, [t3.DeviceCatalog.from_catalog(c) for c in cats]


@pytest.mark.parametrize("mode", [0, 1])
def test_graph_replays_equal_eager(t3, mode):
    cats, dcs = _small(t3)
    edges = np.geomspace(1.0, 12.0, 5)
    lo, size = box_for(40.0)
    eager = t3.Plan(edges, 6, box_lo=lo, box_size=size, graph=False, scan_mode=mode)
    ref, np_ref = eager.forward_tomo(dcs)
    ref = ref.clone()
    plan = t3.Plan(edges, 6, box_lo=lo, box_size=size, graph=True, scan_mode=mode)
    for rep in range(3):
        junk = torch.randn(1 << 20, device="cuda").sum()  # unrelated eager work between replays
        torch.cuda.synchronize()
        got, npairs = plan.forward_tomo(dcs)
        assert npairs == np_ref
        assert torch.equal(got, ref), rep
        del junk
    # and the non-tomographic entry point
    u_e, _ = eager.forward(dcs[1])
    u_e = u_e.clone()
    for rep in range(2):
        u_g, _ = plan.forward(dcs[1])
        assert torch.equal(u_g, u_e)


def test_graph_captured_once_and_replayed(t3):
    """The chunk schedule is captured once per plan and geometry and then
    replayed: later calls with the same catalogs, and with new shears on the
    same positions, launch the captured graph without capturing again
    (t3_graph_stats), each replay equal bit for bit to the eager schedule
    with unrelated eager work and synchronisations between replays; a
    different geometry captures anew."""
    from paper_2309_08601_amd.synth import Catalog
    cats, dcs = _small(t3)
    edges = np.geomspace(1.0, 12.0, 5)
    lo, size = box_for(40.0)
    eager = t3.Plan(edges, 6, box_lo=lo, box_size=size, graph=False)
    plan = t3.Plan(edges, 6, box_lo=lo, box_size=size)
    ref, np_ref = eager.forward_tomo(dcs)
    ref = ref.clone()
    for rep in range(3):
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        got, npairs = plan.forward_tomo(dcs)
        assert npairs == np_ref and torch.equal(got, ref), rep
        del junk
    assert plan.graph_stats() == (1, 3)
    cats2 = [Catalog(c.x, c.y, (-0.5 * c.g2).astype(np.float32), (1.3 * c.g1).astype(np.float32), c.w) for c in cats]
    dcs2 = [t3.DeviceCatalog.from_catalog(c) for c in cats2]
    ref2, _ = eager.forward_tomo(dcs2)
    ref2 = ref2.clone()
    for rep in range(2):
        got, _ = plan.forward_tomo(dcs2)
        assert torch.equal(got, ref2), rep
    assert plan.graph_stats() == (1, 5)
    got, _ = plan.forward_tomo(dcs[:3])  # three catalogs: another geometry
    assert plan.graph_stats() == (2, 6)
    ref3, _ = eager.forward_tomo(dcs[:3])
    assert torch.equal(got, ref3)


def test_autotune_keeps_results(t3):
    """The tuner picks among its candidates, caches the choice per shape,
    and every setting it may pick (stage-2 tile shape, lane threshold,
    chunk capacity, launch mode) gives the oracle's multipoles."""
    from oracle import multipole as mp
    cats, dcs = _small(t3)
    edges = np.geomspace(1.0, 12.0, 5)
    lo, size = box_for(40.0)
    o = mp.multipoles_tomo(cats, edges, 6)
    ref = mp.pack_nonneg(o["ups"], o["N"], 6)
    plan = t3.Plan(edges, 6, box_lo=lo, box_size=size)
    best = plan.autotune(dcs, sample_per_bin=300)
    assert best > 0.0
    st = plan.settings()
    print("tuned:", st, f"{best:.3f} ms", flush=True)
    assert st["scan_mode"] in (0, 1) and st["tile_mode"] in (0, 1)
    assert st["lane_neighbours"] in (0.0, 64.0, 128.0) and st["cell_arcmin"] > 0.0
    # every chunk capacity the tuner could try (1/2 and 1/4 of the automatic
    # one) holds the whole 300-centre sample, like the automatic capacity, so
    # none is tried and the capacity stays automatic
    assert st["chunk_centres"] == 0
    ups, npairs = plan.forward_tomo(dcs)
    assert npairs == o["npairs"]
    e, _ = multipole_errors(ups.cpu().numpy(), ref)
    assert e.max() <= FP32_TOL
    # cached: a second plan of the same shape takes the choice without timing
    again = t3.Plan(edges, 6, box_lo=lo, box_size=size)
    assert again.autotune(dcs, sample_per_bin=300) == 0.0
    assert again.settings() == st
    for kw in [dict(tile_mode=1), dict(tile_mode=0, lane_neighbours=64.0), dict(lane=False, chunk_centres=256),
               dict(scan_mode=1, tile_mode=1, chunk_centres=512)]:
        p = t3.Plan(edges, 6, box_lo=lo, box_size=size, **kw)
        ups, npairs = p.forward_tomo(dcs)
        assert npairs == o["npairs"], kw
        e, _ = multipole_errors(ups.cpu().numpy(), ref)
        assert e.max() <= FP32_TOL, (kw, e.max())


def test_tomo_5bin_workload_4k_centres_per_bin(t3):
    """The 5-bin workload (0.3/0.6/0.8/0.7/0.4 M galaxies in 10 deg x 10 deg,
    20 bins 0.5'-100', n_max 30): 4,000 random centres of every source bin
    against every neighbour catalog, all 125 ordered triples, one persistent
    stage-1 launch per chunk, against the oracle (which takes a minute or
    two: it prints a line per source bin)."""
    import time
    from oracle import multipole as mp
    wl = WORKLOADS["tomo_5bin"]
    cats = make_catalogs(wl)
    idx = [centre_sample(c.n, 4000, seed=40 + z) for z, c in enumerate(cats)]
    lo, size = box_for(wl.side)
    plan = t3.Plan(wl.edges(), wl.n_max, box_lo=lo, box_size=size, scan_mode=1)
    ups, npairs = plan.forward_tomo([t3.DeviceCatalog.from_catalog(c) for c in cats],
                                    [torch.from_numpy(i).cuda() for i in idx])
    ups = ups.cpu().numpy()
    nz, nm = len(cats), wl.n_max
    worst = worst_own = 0.0
    pairs = 0
    for z1 in range(nz):
        t0 = time.time()
        cen = cats[z1].subset(idx[z1])
        hs = [mp.harmonics(cen, cats[z], wl.edges(), nm) for z in range(nz)]
        pairs += sum(int(h["npairs"].sum()) for h in hs)
        for z2 in range(nz):
            for z3 in range(nz):
                u, n_ = mp.upsilon_from_harmonics(mp._c_of(cen), cen.w, hs[z2], hs[z3], nm, diag=(z2 == z3))
                ref = mp.pack_nonneg(u, n_, nm)
                e, e_own = multipole_errors(ups[z1, z2, z3], ref)
                m = multipole_max_errors(ups[z1, z2, z3], ref)
                assert e.max() <= FP32_TOL and m.max() <= FP32_MAX_TOL and e_own.max() <= N_OWN_TOL, \
                    (z1, z2, z3, e.max(), m.max(), e_own.max())
                worst = max(worst, e.max())
                worst_own = max(worst_own, e_own.max())
        print(f"tomo_5bin Z1 = {z1}: 4000 centres, oracle {time.time() - t0:.0f} s, worst rel-F so far "
              f"{worst:.3e}, N_n own {worst_own:.3e}", flush=True)
    assert npairs == pairs
