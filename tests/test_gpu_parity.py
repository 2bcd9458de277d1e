"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bars per (mu, n) block over (b1, b2), every one asserted:
  * relative Frobenius error 1e-6 for the FP32 path, the three-part bf16
    and the scaled fp16 splits on the survey-sized workloads, 1e-5 for the
    two-part bf16 split (and for the fp16 split on the small cases);
  * largest entry error over the largest |entry| 2e-6 (FP32, three-part
    bf16, fp16), 2e-5 (two-part bf16);
  * N_n (n >= 1) also against its own norm: 5e-6;
  * the normalised Gamma_n at the FP32 bar, 2e-5 for the two-part bf16 split
    (which reaches 1.0e-5 on single Gamma_n blocks: 1e-5 is met by the
    three-part split).
Bin membership and pair counts are exact and compared bit for bit.  The
survey-sized workloads are checked on 20,000-centre samples against stored
oracle references (tests/golden/make_fixtures.py, which calls only the
oracle), and the production configuration (all centres, automatic
65,536-centre chunks, the captured graph) against the oracle on a catalog
of two full chunks and a ragged one.
"""
import numpy as np
import pytest

from paper_2309_08601_amd.synth import (LATTICE_UNIT, WORKLOADS, Catalog, centre_sample,
                                        make_catalogs, random_catalog)
from _util import (FP32_MAX_TOL, FP32_TOL, N_OWN_TOL, SPLIT_MAX_TOL, SPLIT_TOL, box_for, multipole_errors,
                   multipole_max_errors, rel_fro)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def t3():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08601_amd import t3 as mod
    return mod


def _oracle():
    import oracle
    from oracle import multipole as mp
    return oracle, mp


def _pack(o, n_max):
    from oracle import multipole as mp
    return mp.pack_nonneg(o["ups"], o["N"], n_max)


def _check(gpu, ref, tol, label="", max_tol=None):
    """gpu, ref: packed multipoles [..., 5, n_max + 1, B, B]; tol bounds the
    relative Frobenius error per (mu, n), max_tol (default: 2 tol) the
    largest entry error over the largest |entry|."""
    if max_tol is None:
        max_tol = 2 * tol
    e, e_own = multipole_errors(gpu, ref)
    m = multipole_max_errors(gpu, ref)
    worst = np.unravel_index(np.argmax(e), e.shape)
    print(f"{label}: max rel-F {e.max():.3e} at {worst}, Upsilon {e[..., :4, :].max():.3e}, "
          f"N_0 {e[..., 4, 0].max():.3e}, N_n/N_0 {e[..., 4, 1:].max() if e.shape[-1] > 1 else 0:.3e}, "
          f"N_n own {e_own.max():.3e}, max rel-max {m.max():.3e}", flush=True)
    assert e.max() <= tol, (label, e.max(), worst)
    assert m.max() <= max_tol, (label, m.max(), np.unravel_index(np.argmax(m), m.shape))
    assert e_own.max() <= N_OWN_TOL, (label, e_own.max())


def test_harmonics_match_oracle(t3):
    _, mp = _oracle()
    cat = random_catalog(3000, 60.0, seed=7)
    edges = np.geomspace(0.8, 14.0, 7)
    nm = 10
    lo, size = box_for(60.0)
    plan = t3.Plan(edges, nm, box_lo=lo, box_size=size)
    dc = t3.DeviceCatalog.from_catalog(cat)
    idx = centre_sample(cat.n, 300, seed=1)
    G, W, D = plan.harmonics(dc, torch.from_numpy(idx).cuda())
    h = mp.harmonics(cat.subset(idx), cat, edges, nm)
    G = G.cpu().numpy().astype(np.complex128)
    W = W.cpu().numpy().astype(np.complex128)
    D = D.cpu().numpy().astype(np.complex128)
    scale = np.abs(h["G"]).max()
    assert np.abs(G - h["G"]).max() < 2e-6 * scale
    Wo = h["W"][:, :, nm:]
    assert np.abs(W - Wo).max() < 2e-6 * np.abs(Wo).max()
    assert np.abs(D - h["D"]).max() < 2e-6 * np.abs(h["D"]).max()
    # W_0 holds the weight sums exactly up to FP32 rounding; the count of
    # in-bin neighbours is exact
    plan_u = t3.Plan(edges, nm, box_lo=lo, box_size=size)
    ones = Catalog(cat.x, cat.y, cat.g1, cat.g2, np.ones(cat.n, np.float32))
    _, W1, _ = plan_u.harmonics(t3.DeviceCatalog.from_catalog(ones), torch.from_numpy(idx).cuda())
    cnt = mp.harmonics(ones.subset(idx), ones, edges, nm)["W"][:, :, nm].real
    assert np.array_equal(W1[:, :, 0].real.cpu().numpy().astype(np.float64), cnt)


@pytest.mark.parametrize("nm,n_cent", [(10, 301), (10, 302), (30, 303), (30, 304)])
def test_harmonics_wavefront_bins_ragged_quads(t3, nm, n_cent):
    """Every bin on the one-wavefront-per-centre kernel (the lane threshold
    set below any bin's expected count), whose workgroups of four centres
    store their totals as four-centre rows: centre counts 1, 2, 3 and 0
    mod 4, each plane and bin of every centre against the oracle."""
    _, mp = _oracle()
    cat = random_catalog(2500, 50.0, seed=900 + n_cent)
    edges = np.geomspace(0.8, 14.0, 8)
    lo, size = box_for(50.0)
    plan = t3.Plan(edges, nm, box_lo=lo, box_size=size, lane_neighbours=1e-6)
    idx = centre_sample(cat.n, n_cent, seed=n_cent)
    G, W, D = plan.harmonics(t3.DeviceCatalog.from_catalog(cat), torch.from_numpy(idx).cuda())
    h = mp.harmonics(cat.subset(idx), cat, edges, nm)
    G = G.cpu().numpy().astype(np.complex128)
    W = W.cpu().numpy().astype(np.complex128)
    D = D.cpu().numpy().astype(np.complex128)
    eg = np.abs(G - h["G"]).max() / np.abs(h["G"]).max()
    ew = np.abs(W - h["W"][:, :, nm:]).max() / np.abs(h["W"][:, :, nm:]).max()
    ed = np.abs(D - h["D"]).max() / np.abs(h["D"]).max()
    print(f"n_max {nm}, {n_cent} centres: G {eg:.2e}, W {ew:.2e}, D {ed:.2e}", flush=True)
    assert eg < 2e-6 and ew < 2e-6 and ed < 2e-6


# every compiled capacity (8, 12 and 40 are covered elsewhere), and n_max = 28,
# 38, 61 below the capacities 30, 40, 64: there only some of the orders C .. C+3
# that the top pass takes as G_{-m} alone reach a plane
@pytest.mark.parametrize("nm", [0, 3, 10, 14, 20, 24, 28, 30, 32, 38, 48, 61, 64])
def test_forward_small_orders(t3, nm):
    _, mp = _oracle()
    cat = random_catalog(1500, 40.0, seed=100 + nm)
    edges = np.geomspace(1.0, 15.0, 6)
    lo, size = box_for(40.0)
    plan = t3.Plan(edges, nm, box_lo=lo, box_size=size)
    ups, npairs = plan.forward(t3.DeviceCatalog.from_catalog(cat))
    o = mp.multipoles(cat, edges, nm)
    assert npairs == o["npairs"]
    _check(ups.cpu().numpy(), _pack(o, nm), FP32_TOL, f"n_max={nm}")


def test_forward_small_2k_workload(t3):
    """The 2,000-galaxy, 1 deg^2 workload in full (10 bins 1'-30', n_max 10)."""
    _, mp = _oracle()
    wl = WORKLOADS["small_2k"]
    cat = make_catalogs(wl)[0]
    lo, size = box_for(wl.side)
    plan = t3.Plan(wl.edges(), wl.n_max, box_lo=lo, box_size=size)
    ups, npairs = plan.forward(t3.DeviceCatalog.from_catalog(cat))
    o = mp.multipoles(cat, wl.edges(), wl.n_max)
    assert npairs == o["npairs"]
    _check(ups.cpu().numpy(), _pack(o, wl.n_max), FP32_TOL, "small_2k")


def _fixture(name):
    """Stored oracle reference of a 20,000-centre sample (written by
    tests/golden/make_fixtures.py from the oracle alone) and the regenerated
    catalog, which must be the one the reference was computed for."""
    import os
    from golden.make_fixtures import catalog_sha, fixture_path
    path = fixture_path(name)
    if not os.path.exists(path):
        pytest.skip(f"oracle reference {path} not written")
    f = np.load(path, allow_pickle=False)
    wl = WORKLOADS[name]
    cat = make_catalogs(wl)[0]
    assert str(f["catalog_sha256"]) == catalog_sha(cat), "regenerated catalog differs from the reference's"
    return wl, cat, f


# Gamma_n = Upsilon_n / N_0 weights every bin pair equally, so its relative
# error is larger than Upsilon's where a block's few large entries dominate:
# the two-part bf16 split (about 16 bits per operand, 2^-18 representation
# error each) reaches 1.0e-5 on single Gamma_n blocks of the 1M field and is
# held to 2e-5 there; the three-part split meets the FP32 bar.
_PARITY_CASES = [("fp32", FP32_TOL, FP32_MAX_TOL, FP32_TOL), ("bf16x6", FP32_TOL, FP32_MAX_TOL, FP32_TOL),
                 ("bf16x3", SPLIT_TOL, SPLIT_MAX_TOL, 2 * SPLIT_TOL)]


@pytest.mark.parametrize("prec,tol,max_tol,gamma_tol", _PARITY_CASES)
def test_forward_field_1m_20k_centres(t3, prec, tol, max_tol, gamma_tol):
    """1M galaxies in 10 deg x 10 deg, 20 bins 0.5'-100', n_max 30: the GPU
    on 20,000 random centres against the full neighbour catalog."""
    wl, cat, f = _fixture("field_1m")
    lo, size = box_for(wl.side)
    plan = t3.Plan(wl.edges(), wl.n_max, box_lo=lo, box_size=size, precision=prec)
    ups, npairs = plan.forward(t3.DeviceCatalog.from_catalog(cat), torch.from_numpy(f["idx"]).cuda())
    assert npairs == int(f["npairs"])
    _check(ups.cpu().numpy(), f["ref"], tol, f"field_1m 20k centres {prec}", max_tol)
    gn, _ = plan.normalise_resum(ups, with_phi=False)
    eg = rel_fro(gn.cpu().numpy(), f["gamma_n"])
    print(f"field_1m 20k centres {prec}: Gamma_n max rel-F {eg.max():.3e}", flush=True)
    assert eg.max() <= gamma_tol


def test_production_configuration_matches_oracle(t3):
    """The configuration the benchmark times: every galaxy a centre, the
    automatic chunk capacity (65,536 centres at n_max 30), the chunk schedule
    captured as one HIP graph, the stage-2 slicing and XCD balancing at full
    chunk size: 140,000 galaxies at the 1M field's density (two full chunks
    and a ragged one of 8,928), 8 bins 0.5'-12' (inner bins one lane per
    centre, outer bins one wavefront per centre), n_max 30, against the
    oracle over every centre."""
    import dataclasses
    _, mp = _oracle()
    n = 140_000
    # the 1M field's shear and weight model on a field that holds 140k
    # galaxies at the same density
    wl = dataclasses.replace(WORKLOADS["field_1m"], name="field_140k", n_gal=[n],
                             side=float(np.sqrt(n / 2.78)), n_bins=8, theta_max=12.0, seed_index=6)
    cat = make_catalogs(wl)[0]
    edges = wl.edges()
    nm = 30
    side = wl.side
    lo, size = box_for(side)
    plan = t3.Plan(edges, nm, box_lo=lo, box_size=size)
    ups, npairs = plan.forward(t3.DeviceCatalog.from_catalog(cat))
    o = mp.multipoles(cat, edges, nm)
    assert npairs == o["npairs"]
    _check(ups.cpu().numpy(), _pack(o, nm), FP32_TOL, "production configuration, 140k centres")


@pytest.mark.parametrize("prec,tol", [("fp32", FP32_TOL), ("bf16x3", SPLIT_TOL)])
def test_forward_field_3m_33bins_sampled_centres(t3, prec, tol):
    """The combined-estimator timing setup of Sect. 4.1 run through the
    discrete estimator: 3.1M galaxies on 100 deg^2, 33 bins 0.25'-80',
    n_max 20 (bin 32 summed by the edge-bin path), on a sample of centres
    against the full neighbour catalog."""
    _, mp = _oracle()
    wl = WORKLOADS["field_3m_33bins"]
    cat = make_catalogs(wl)[0]
    idx = centre_sample(cat.n, 120, seed=17)
    lo, size = box_for(wl.side)
    plan = t3.Plan(wl.edges(), wl.n_max, box_lo=lo, box_size=size, precision=prec)
    ups, npairs = plan.forward(t3.DeviceCatalog.from_catalog(cat), torch.from_numpy(idx).cuda())
    o = mp.multipoles(cat, wl.edges(), wl.n_max, centres=idx)
    assert npairs == o["npairs"]
    assert tuple(ups.shape[-2:]) == (33, 33)
    _check(ups.cpu().numpy(), _pack(o, wl.n_max), tol, f"field_3m_33bins sample {prec}")


@pytest.mark.parametrize("prec,tol,max_tol,gamma_tol",
                         _PARITY_CASES + [("fp16x3", FP32_TOL, FP32_MAX_TOL, FP32_TOL)])
def test_forward_field_4m_20k_centres(t3, prec, tol, max_tol, gamma_tol):
    """The precision workload: 4M galaxies in 20 deg x 20 deg, 30 bins
    0.5'-200', n_max 40 (the two-pass stage-1 variant; B = 30 nearly fills
    the 32-row MFMA tiles), on 20,000 random centres.  The two-part bf16
    split keeps about 16 bits of each operand: its Frobenius error stays
    below 1e-5 per (mu, n) of Upsilon, its largest entry error and its
    Gamma_n error below 2e-5; the three-part bf16 split (all 24 bits) and
    the scaled fp16 split meet the FP32 bars."""
    wl, cat, f = _fixture("field_4m")
    lo, size = box_for(wl.side)
    plan = t3.Plan(wl.edges(), wl.n_max, box_lo=lo, box_size=size, precision=prec)
    ups, npairs = plan.forward(t3.DeviceCatalog.from_catalog(cat), torch.from_numpy(f["idx"]).cuda())
    assert npairs == int(f["npairs"])
    _check(ups.cpu().numpy(), f["ref"], tol, f"field_4m 20k centres {prec}", max_tol)
    gn, _ = plan.normalise_resum(ups, with_phi=False)
    eg = rel_fro(gn.cpu().numpy(), f["gamma_n"])
    print(f"field_4m 20k centres {prec}: Gamma_n max rel-F {eg.max():.3e}, per mu "
          f"{[float(f'{v:.3e}') for v in eg.max(axis=1)]}", flush=True)
    assert eg.max() <= gamma_tol


@pytest.mark.parametrize("prec,tol", [("bf16x3", SPLIT_TOL), ("fp16x3", SPLIT_TOL), ("bf16x6", FP32_TOL)])
def test_split_precision(t3, prec, tol):
    _, mp = _oracle()
    cat = random_catalog(3999, 60.0, seed=55)  # ragged: the last centre quad holds 3
    edges = np.geomspace(0.7, 20.0, 9)
    nm = 12
    lo, size = box_for(60.0)
    plan = t3.Plan(edges, nm, box_lo=lo, box_size=size, precision=prec)
    ups, _ = plan.forward(t3.DeviceCatalog.from_catalog(cat))
    o = mp.multipoles(cat, edges, nm)
    _check(ups.cpu().numpy(), _pack(o, nm), tol, prec)


def test_normalise_and_resum(t3):
    _, mp = _oracle()
    cat = random_catalog(2500, 50.0, seed=8)
    edges = np.geomspace(1.0, 16.0, 6)
    nm = 8
    lo, size = box_for(50.0)
    plan = t3.Plan(edges, nm, box_lo=lo, box_size=size)
    ups, _ = plan.forward(t3.DeviceCatalog.from_catalog(cat))
    gn, gp = plan.normalise_resum(ups, n_phi=24)
    o = mp.multipoles(cat, edges, nm)
    g_all, _ = mp.normalise(o["ups"], o["N"])
    e = rel_fro(gn.cpu().numpy(), g_all[:, nm:])
    assert e.max() <= FP32_TOL, e.max()
    ref_phi = mp.resum(g_all, nm, mp.phi_bin_edges(24))
    gp = gp.cpu().numpy()
    e = np.sqrt(np.sum(np.abs(gp - ref_phi) ** 2, axis=(1, 2, 3))) / np.sqrt(
        np.sum(np.abs(ref_phi) ** 2, axis=(1, 2, 3)))
    assert e.max() < FP32_TOL


def test_tomography_small(t3):
    _, mp = _oracle()
    cats = [random_catalog(n, 40.0, seed=300 + z) for z, n in enumerate([700, 1200, 900])]
    edges = np.geomspace(1.0, 12.0, 5)
    nm = 6
    lo, size = box_for(40.0)
    plan = t3.Plan(edges, nm, box_lo=lo, box_size=size)
    ups, npairs = plan.forward_tomo([t3.DeviceCatalog.from_catalog(c) for c in cats])
    o = mp.multipoles_tomo(cats, edges, nm)
    assert npairs == o["npairs"]
    _check(ups.cpu().numpy(), mp.pack_nonneg(o["ups"], o["N"], nm), FP32_TOL, "tomo")


def test_edge_cases(t3):
    _, mp = _oracle()
    u = int(round(1.0 / LATTICE_UNIT))
    edges = [1.0, 3.0, 5.0]
    lo, size = box_for(20.0)
    # empty catalog
    plan = t3.Plan(edges, 4, box_lo=lo, box_size=size)
    empty = t3.DeviceCatalog(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32),
                             np.zeros(0, np.float32), np.zeros(0, np.float32))
    ups, npairs = plan.forward(empty)
    assert npairs == 0 and float(ups.abs().max()) == 0.0
    # neighbours exactly on bin edges, a coincident pair, the box corner
    xs = np.array([2 * u, 4 * u, 2 * u, 2 * u + 3 * u, 2 * u, 0, 20 * u - 1], np.int32)
    ys = np.array([2 * u, 2 * u, 5 * u, 6 * u, 2 * u, 0, 20 * u - 1], np.int32)
    n = xs.size
    rng = np.random.default_rng(0)
    cat = Catalog(xs, ys, rng.normal(0, .3, n).astype(np.float32), rng.normal(0, .3, n).astype(np.float32),
                  rng.uniform(.5, 1.5, n).astype(np.float32))
    ups, npairs = plan.forward(t3.DeviceCatalog.from_catalog(cat))
    o = mp.multipoles(cat, edges, 4)
    assert npairs == o["npairs"]
    ref = _pack(o, 4)
    assert np.abs(ups.cpu().numpy() - ref).max() <= 1e-6 * max(np.abs(ref).max(), 1e-30)
    # empty centre list (n_centres == 0 is "no centre", not "all")
    ups, npairs = plan.forward(t3.DeviceCatalog.from_catalog(cat), torch.zeros(0, dtype=torch.int32).cuda())
    assert npairs == 0 and float(ups.abs().max()) == 0.0


def test_errors_are_reported(t3):
    lo, size = box_for(10.0)
    plan = t3.Plan([1.0, 2.0], 3, box_lo=lo, box_size=size)
    bad = t3.DeviceCatalog(np.array([0, size + 5], np.int32), np.array([0, 0], np.int32),
                           np.zeros(2, np.float32), np.zeros(2, np.float32), np.ones(2, np.float32))
    with pytest.raises(t3.T3Error) as ei:
        plan.forward(bad)
    assert ei.value.code == t3.T3_ELATTICE
    good = t3.DeviceCatalog(np.array([0, 5], np.int32), np.array([0, 0], np.int32),
                            np.zeros(2, np.float32), np.zeros(2, np.float32), np.ones(2, np.float32))
    with pytest.raises(t3.T3Error) as ei:
        plan.forward(good, torch.tensor([0, 7], dtype=torch.int32).cuda())
    assert ei.value.code == t3.T3_EINVAL


def test_repeatable_bitwise(t3):
    cat = random_catalog(3000, 50.0, seed=9)
    edges = np.geomspace(1.0, 16.0, 6)
    lo, size = box_for(50.0)
    plan = t3.Plan(edges, 10, box_lo=lo, box_size=size)
    dc = t3.DeviceCatalog.from_catalog(cat)
    a, _ = plan.forward(dc)
    b, _ = plan.forward(dc)
    assert torch.equal(a, b)


@pytest.mark.parametrize("prec,ec", [("fp32", False), ("bf16x6", False), ("fp32", True)])
def test_many_chunks_ragged(t3, prec, ec):
    """Chunks of 256 centres over 1999 galaxies (7 full chunks and a ragged
    one of 207): every chunk's stage-2 partials accumulate into one output."""
    _, mp = _oracle()
    cat = random_catalog(1999, 50.0, seed=73)
    edges = np.geomspace(1.0, 15.0, 7)
    nm = 9
    lo, size = box_for(50.0)
    plan = t3.Plan(edges, nm, box_lo=lo, box_size=size, precision=prec, chunk_centres=256,
                   edge_correct=ec)
    ups, npairs = plan.forward(t3.DeviceCatalog.from_catalog(cat))
    o = mp.multipoles(cat, edges, nm, w_max=2 * nm if ec else None)
    assert npairs == o["npairs"]
    if ec:
        u4, N = plan.split_ups(ups)
        wm = 2 * nm
        ref_u = o["ups"][:, nm:]
        e = rel_fro(u4.cpu().numpy(), ref_u).max()
        dn = np.linalg.norm((N.cpu().numpy() - o["N"][wm:]).reshape(wm + 1, -1), axis=1)
        en = (dn / np.linalg.norm(o["N"][wm])).max()
        print(f"many chunks, edge-correct layout: Upsilon {e:.2e}, N_n/N_0 {en:.2e}", flush=True)
        assert e <= FP32_TOL and en <= FP32_TOL
    else:
        _check(ups.cpu().numpy(), _pack(o, nm), FP32_TOL, f"many chunks {prec}")
