"""The no-allocation forward pass (t3_forward_noalloc) against t3_forward.

Two calls in a row on one plan, the second with a smaller catalog and a
centre list, each compared with t3_forward on the same input to the parity
bars (relative Frobenius error 1e-6 and largest entry error 2e-6 per
(mu, n)); the pair counts are exact.  The plan holds no device memory of its
own afterwards (every buffer came from the library's static scratch), and
a catalog too large for the scratch is refused before any launch with
T3_ENOMEM, its output untouched.
"""
import numpy as np
import pytest

from paper_2309_08601_amd.synth import WORKLOADS, centre_sample, make_catalogs
from _util import FP32_MAX_TOL, FP32_TOL, box_for, multipole_errors, multipole_max_errors

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def t3():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08601_amd import t3 as mod
    return mod


def _catalog(n, seed_index):
    import dataclasses
    wl = dataclasses.replace(WORKLOADS["field_1m"], name="noalloc", n_gal=[n], side=float(np.sqrt(n / 2.78)),
                             n_bins=12, theta_max=20.0, n_max=20, seed_index=seed_index)
    return wl, make_catalogs(wl)[0]


def _compare(got, ref, label):
    g, r = got.cpu().numpy(), ref.cpu().numpy()
    e, _ = multipole_errors(g, r)
    m = multipole_max_errors(g, r)
    print(f"{label}: rel-F {e.max():.3e}, rel-max {m.max():.3e}, bitwise {bool(np.array_equal(g, r))}", flush=True)
    assert e.max() <= FP32_TOL and m.max() <= FP32_MAX_TOL


def test_noalloc_forward_matches_forward_on_two_calls(t3):
    wl, big = _catalog(300_000, 11)
    lo, size = box_for(wl.side)
    plan = t3.Plan(wl.edges(), wl.n_max, box_lo=lo, box_size=size)
    ref_plan = t3.Plan(wl.edges(), wl.n_max, box_lo=lo, box_size=size)
    d_big = t3.DeviceCatalog.from_catalog(big)
    got, n1 = plan.forward_noalloc(d_big)
    ref, r1 = ref_plan.forward(d_big)
    assert n1 == r1
    _compare(got, ref, "no-alloc call 1 (300k galaxies, all centres)")
    assert plan.workspace_bytes() == (0, 0)
    # second call, smaller: a 40k-galaxy catalog and a centre list
    wl2, small = _catalog(40_000, 12)
    lo2, size2 = box_for(wl2.side)
    assert size2 <= size
    d_small = t3.DeviceCatalog.from_catalog(small)
    idx = torch.from_numpy(centre_sample(small.n, 15_000, seed=5)).cuda()
    got2, n2 = plan.forward_noalloc(d_small, idx)
    ref2, r2 = ref_plan.forward(d_small, idx)
    assert n2 == r2
    _compare(got2, ref2, "no-alloc call 2 (40k galaxies, 15k centres)")
    assert plan.workspace_bytes() == (0, 0)
    # the plan's own path is unaffected by the scratch calls
    again, _ = plan.forward(d_small, idx)
    assert torch.equal(again, ref2)


def test_noalloc_refuses_a_catalog_beyond_the_scratch(t3):
    n = 6_000_000
    side = 1500.0
    lo, size = box_for(side)
    plan = t3.Plan(np.geomspace(1.0, 10.0, 6), 8, box_lo=lo, box_size=size)
    zi = torch.zeros(n, dtype=torch.int32, device="cuda")
    zf = torch.zeros(n, dtype=torch.float32, device="cuda")
    cat = t3.DeviceCatalog.__new__(t3.DeviceCatalog)
    cat.x, cat.y, cat.g1, cat.g2, cat.w, cat.n = zi, zi, zf, zf, zf, n
    out = torch.full((5, 9, 5, 5, 2), 3.0, dtype=torch.float64, device="cuda")
    with pytest.raises(t3.T3Error) as ei:
        plan.forward_noalloc(cat, out=out)
    assert ei.value.code == t3.T3_ENOMEM and "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool(torch.all(out == 3.0))
