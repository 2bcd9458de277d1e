"""Batched tomography: one stage-1 launch for all neighbour catalogs (one
wavefront per task, or a persistent work queue), one stage-2 launch for all
ordered (Z2, Z3) pairs, the chunk schedule captured as one HIP graph.

* graph replays (with eager work in between) equal the eager schedule bit
  for bit, for both stage-1 launch modes;
* the autotuner's choice reproduces the same multipoles;
* the 5-bin workload (0.3/0.6/0.8/0.7/0.4 M galaxies in 10 deg x 10 deg,
  20 bins 0.5'-100', n_max 30) matches the oracle on a sample of centres
  per source bin for all 125 ordered triples.
"""
import numpy as np
import pytest

from paper_2309_08601_amd.synth import WORKLOADS, centre_sample, make_catalogs, random_catalog
from _util import FP32_TOL, box_for, multipole_errors

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


def test_autotune_keeps_results(t3):
    from oracle import multipole as mp
    cats, dcs = _small(t3)
    edges = np.geomspace(1.0, 12.0, 5)
    lo, size = box_for(40.0)
    plan = t3.Plan(edges, 6, box_lo=lo, box_size=size)
    best = plan.autotune(dcs, sample_per_bin=300)
    assert best >= 0.0
    ups, npairs = plan.forward_tomo(dcs)
    o = mp.multipoles_tomo(cats, edges, 6)
    assert npairs == o["npairs"]
    e, _ = multipole_errors(ups.cpu().numpy(), mp.pack_nonneg(o["ups"], o["N"], 6))
    assert e.max() <= FP32_TOL


def test_tomo_5bin_workload_sampled(t3):
    from oracle import multipole as mp
    wl = WORKLOADS["tomo_5bin"]
    cats = make_catalogs(wl)
    idx = [centre_sample(c.n, 60, seed=40 + z) for z, c in enumerate(cats)]
    lo, size = box_for(wl.side)
    plan = t3.Plan(wl.edges(), wl.n_max, box_lo=lo, box_size=size, scan_mode=1)
    ups, npairs = plan.forward_tomo([t3.DeviceCatalog.from_catalog(c) for c in cats],
                                    [torch.from_numpy(i).cuda() for i in idx])
    o = mp.multipoles_tomo(cats, wl.edges(), wl.n_max, centres=idx)
    assert npairs == o["npairs"]
    e, e_own = multipole_errors(ups.cpu().numpy(), mp.pack_nonneg(o["ups"], o["N"], wl.n_max))
    print(f"tomo_5bin sample: max rel-F {e.max():.3e}, Upsilon {e[..., :4, :].max():.3e}, "
          f"N_n own {e_own.max():.3e}", flush=True)
    assert e.max() <= FP32_TOL
