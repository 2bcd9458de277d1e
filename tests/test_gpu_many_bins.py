"""More than 32 radial bins (up to 64): the paper's own runs use 38 and 40
logarithmic bins (Sects. 4-5).  Stage 2 then tiles each B x B block into
four 32 x 32 MFMA tiles; the adjoint, the x -> centroid projection and the
aperture integration carry per-bin tables of up to 64 entries.

Every case is checked against the FP64 oracle with the bars of the other
parity tests (1e-6 FP32, 1e-5 split precision)."""
import numpy as np
import pytest

from paper_2309_08601_amd.synth import LATTICE_UNIT, random_catalog
from _util import FP32_TOL, SPLIT_TOL, box_for, multipole_errors, rel_fro

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def t3():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08601_amd import t3 as mod
    return mod


def _check(gpu, ref, tol, label):
    e, e_own = multipole_errors(gpu, ref)
    print(f"{label}: max rel-F {e.max():.3e}, N_n own {e_own.max():.3e}", flush=True)
    assert e.max() <= tol, (label, e.max())
    assert e_own.max() <= 50 * tol, (label, e_own.max())


@pytest.mark.parametrize("prec,tol", [("fp32", FP32_TOL), ("bf16x6", FP32_TOL), ("bf16x3", SPLIT_TOL),
                                      ("fp16x3", SPLIT_TOL)])
def test_forward_40_bins(t3, prec, tol):
    """40 bins, 512-centre chunks over 3001 galaxies (ragged last chunk)."""
    from oracle import multipole as mp
    cat = random_catalog(3001, 50.0, seed=4001)
    edges = np.geomspace(0.7, 20.0, 41)
    nm = 8
    lo, size = box_for(50.0)
    plan = t3.Plan(edges, nm, box_lo=lo, box_size=size, precision=prec, chunk_centres=512)
    ups, npairs = plan.forward(t3.DeviceCatalog.from_catalog(cat))
    o = mp.multipoles(cat, edges, nm)
    assert npairs == o["npairs"]
    assert tuple(ups.shape[-2:]) == (40, 40)
    _check(ups.cpu().numpy(), mp.pack_nonneg(o["ups"], o["N"], nm), tol, f"B=40 {prec}")


@pytest.mark.parametrize("B,keep_jk", [(33, False), (37, True), (41, False), (64, True), (64, False)])
def test_forward_33_and_64_bins(t3, B, keep_jk):
    """One bin past a tile (edge bins on the vector ALUs), 37 bins with the
    j = k terms kept (their diagonal entries 32-36 come from the edge sums),
    41 bins (the first size with four MFMA tiles) and the largest plan (with
    and without the j = k terms, which touch only the diagonal blocks)."""
    from oracle import multipole as mp
    cat = random_catalog(2500, 45.0, seed=4100 + B)
    edges = np.geomspace(0.5, 18.0, B + 1)
    nm = 5
    lo, size = box_for(45.0)
    plan = t3.Plan(edges, nm, box_lo=lo, box_size=size, keep_jk=keep_jk)
    ups, npairs = plan.forward(t3.DeviceCatalog.from_catalog(cat))
    o = mp.multipoles(cat, edges, nm, diag=not keep_jk)
    assert npairs == o["npairs"]
    _check(ups.cpu().numpy(), mp.pack_nonneg(o["ups"], o["N"], nm), FP32_TOL, f"B={B} keep_jk={keep_jk}")


def test_tomography_36_bins(t3):
    from oracle import multipole as mp
    cats = [random_catalog(n, 40.0, seed=4200 + z) for z, n in enumerate([900, 1300])]
    edges = np.geomspace(0.8, 14.0, 37)
    nm = 4
    lo, size = box_for(40.0)
    plan = t3.Plan(edges, nm, box_lo=lo, box_size=size)
    ups, npairs = plan.forward_tomo([t3.DeviceCatalog.from_catalog(c) for c in cats])
    o = mp.multipoles_tomo(cats, edges, nm)
    assert npairs == o["npairs"]
    _check(ups.cpu().numpy(), mp.pack_nonneg(o["ups"], o["N"], nm), FP32_TOL, "tomo B=36")


def test_normalise_resum_centroid_40_bins(t3):
    from oracle import multipole as mp
    from oracle.projection import bin_centres, phi_centres, x_to_centroid
    cat = random_catalog(2500, 50.0, seed=4300)
    edges = np.geomspace(1.0, 16.0, 41)
    nm, K = 6, 16
    lo, size = box_for(50.0)
    plan = t3.Plan(edges, nm, box_lo=lo, box_size=size)
    ups, _ = plan.forward(t3.DeviceCatalog.from_catalog(cat))
    gn, gp = plan.normalise_resum(ups, n_phi=K)
    o = mp.multipoles(cat, edges, nm)
    g_all, _ = mp.normalise(o["ups"], o["N"])
    e = rel_fro(gn.cpu().numpy(), g_all[:, nm:])
    assert e.max() <= FP32_TOL, e.max()
    ref_phi = mp.resum(g_all, nm, mp.phi_bin_edges(K))
    ep = np.sqrt(np.sum(np.abs(gp.cpu().numpy() - ref_phi) ** 2, axis=(1, 2, 3))) / np.sqrt(
        np.sum(np.abs(ref_phi) ** 2, axis=(1, 2, 3)))
    assert ep.max() <= FP32_TOL, ep.max()
    rng = np.random.default_rng(3)
    g = rng.standard_normal((2, 4, 40, 40, K)) + 1j * rng.standard_normal((2, 4, 40, 40, K))
    got = plan.x_to_centroid(torch.from_numpy(g).cuda()).cpu().numpy()
    ref = x_to_centroid(g, bin_centres(edges), phi_centres(K))
    assert rel_fro(got, ref, axes=(-3, -2, -1)).max() < 1e-13


def test_edge_correction_40_bins(t3):
    from oracle import multipole as mp
    cat = random_catalog(5000, 50.0, seed=4400)
    keep = np.nonzero(cat.x.astype(np.int64) > np.percentile(cat.x.astype(np.int64), 15))[0]
    cat = cat.subset(keep)
    edges = np.geomspace(2.0, 20.0, 41)
    nm = 5
    lo, size = box_for(50.0)
    plan = t3.Plan(edges, nm, box_lo=lo, box_size=size, edge_correct=True)
    ups, _ = plan.forward(t3.DeviceCatalog.from_catalog(cat))
    gn, _ = plan.normalise_resum(ups, n_phi=8)
    o = mp.multipoles(cat, edges, nm, w_max=2 * nm)
    ref_all = mp.mode_coupling_correct(o["ups"], o["N"], nm)
    e = rel_fro(gn.cpu().numpy(), ref_all[:, nm:])
    print(f"edge-corrected Gamma_n, B=40: {e.max():.2e}", flush=True)
    assert e.max() <= 2 * FP32_TOL


def test_aperture_40_bins(t3):
    from oracle.aperture import aperture_stats, correlators
    rng = np.random.default_rng(44)
    edges = np.geomspace(0.3, 20.0, 41)
    B, K, sets = 40, 12, 2
    plan = t3.Plan(edges, 4, box_size=1 << 22)
    g = rng.standard_normal((sets, 4, B, B, K)) + 1j * rng.standard_normal((sets, 4, B, B, K))
    aps = [(1.0, 1.0, 1.0), (1.5, 2.0, 3.0), (4.0, 4.0, 4.0)]
    corr, stats = plan.aperture_stats(torch.from_numpy(g).cuda(), aps)
    pe = 2 * np.pi * np.arange(K + 1) / K
    for s in range(sets):
        ref = correlators(g[s], edges, pe, aps)
        got = corr[s].cpu().numpy()
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
        assert np.allclose(stats[s].cpu().numpy(), aperture_stats(ref), rtol=0,
                           atol=1e-12 * np.max(np.abs(ref)))


def test_adjoint_40_bins(t3):
    """Gradient through 40 bins against the FP64 autograd oracle."""
    from oracle import autodiff as ad
    cat = random_catalog(900, 30.0, seed=4501)
    tgt = random_catalog(900, 30.0, seed=4502)
    edges = np.geomspace(1.0, 10.0, 41)
    nm = 4
    pl = ad.pairs(cat.x, cat.y, edges)
    t = lambda a: torch.tensor(np.asarray(a, dtype=np.float64))  # noqa: E731
    uT, NT = ad.multipoles(tgt.x, tgt.y, t(tgt.g1), t(tgt.g2), t(tgt.w), edges, nm)
    T = ad.gamma(uT, NT).detach()
    om = ad.loss_weights(T)
    g1 = t(cat.g1).requires_grad_(True)
    g2 = t(cat.g2).requires_grad_(True)
    w = t(cat.w).requires_grad_(True)
    u, N = ad.multipoles(cat.x, cat.y, g1, g2, w, edges, nm, pair_list=pl)
    Lr = ad.loss(ad.gamma(u, N), T, om)
    Lr.backward()
    lo, size = box_for(30.0)
    plan = t3.Plan(edges, nm, box_lo=lo, box_size=size)
    dev = "cuda"
    x = torch.from_numpy(cat.x).to(dev)
    y = torch.from_numpy(cat.y).to(dev)
    q1 = torch.from_numpy(cat.g1.copy()).to(dev).requires_grad_(True)
    q2 = torch.from_numpy(cat.g2.copy()).to(dev).requires_grad_(True)
    qw = torch.from_numpy(cat.w.copy()).to(dev).requires_grad_(True)
    gam = torch.view_as_complex(t3.GammaMultipoles.apply(q1, q2, qw, x, y, plan))
    d = gam - T.to(dev)
    L = torch.sum(om.to(dev) * (d.real ** 2 + d.imag ** 2))
    L.backward()
    assert abs(float(L) - float(Lr)) < 1e-5 * float(Lr)
    for got, ref, name in ((q1.grad, g1.grad, "g1"), (q2.grad, g2.grad, "g2"), (qw.grad, w.grad, "w")):
        got = got.cpu().numpy()
        ref = ref.numpy()
        e = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print(f"B=40 grad {name}: rel-norm {e:.2e}", flush=True)
        assert e < 2e-5, (name, e)


@pytest.mark.parametrize("method", ["direct", "fft"])
def test_combined_40_bins(t3, method):
    from oracle import grid as og
    cat = random_catalog(4000, 50.0, seed=4600)
    edges = np.geomspace(1.0, 14.0, 41)
    nm = 4
    levels = [0] * 20 + [1] * 10 + [2] * 10
    box_lo = (-777, 31)
    delta = int(0.25 / LATTICE_UNIT)
    plan = t3.Plan(edges, nm, box_lo=box_lo, box_size=1 << 23)
    ups, _ = plan.forward_grid(t3.DeviceCatalog.from_catalog(cat), delta, levels, method=method)
    o = og.multipoles_combined(cat, edges, nm, delta, levels, box_lo=box_lo, w_max=nm)
    B = 40
    ref = np.concatenate([o["ups"][:, nm:].reshape(4 * (nm + 1), B, B), o["N"][nm:]], axis=0)
    got = ups.cpu().numpy().reshape(ref.shape)
    u_err = rel_fro(got[:4 * (nm + 1)], ref[:4 * (nm + 1)]).max()
    n0 = np.linalg.norm(ref[4 * (nm + 1)])
    n_err = max(np.linalg.norm(got[4 * (nm + 1) + k] - ref[4 * (nm + 1) + k]) / n0 for k in range(nm + 1))
    print(f"combined B=40 ({method}): Upsilon {u_err:.2e}, N_n/N_0 {n_err:.2e}", flush=True)
    assert u_err <= FP32_TOL and n_err <= FP32_TOL


@pytest.mark.parametrize("prec,tol", [("bf16x3", SPLIT_TOL), ("fp16x3", SPLIT_TOL), ("bf16x6", FP32_TOL)])
def test_forward_33_bins_split_precision(t3, prec, tol):
    """33 bins: the first 32 x 32 tile on split-precision MFMA, the 65 outputs
    per block that involve bin 32 in FP64 on the vector ALUs, with N_n to
    2 n_max (edge correction) so that the N side covers more orders than
    Upsilon."""
    from oracle import multipole as mp
    cat = random_catalog(2800, 45.0, seed=4700)
    edges = np.geomspace(0.6, 18.0, 34)
    nm = 6
    lo, size = box_for(45.0)
    plan = t3.Plan(edges, nm, box_lo=lo, box_size=size, precision=prec, edge_correct=True, chunk_centres=1024)
    ups, npairs = plan.forward(t3.DeviceCatalog.from_catalog(cat))
    o = mp.multipoles(cat, edges, nm, w_max=2 * nm)
    assert npairs == o["npairs"]
    got = ups.cpu().numpy()
    ref_u = o["ups"][:, nm:]
    e = rel_fro(got[:4 * (nm + 1)].reshape(4, nm + 1, 33, 33), ref_u)
    n_ref = o["N"][2 * nm:]
    n_got = got[4 * (nm + 1):]
    n0 = np.linalg.norm(n_ref[0])
    en = max(np.linalg.norm(n_got[k] - n_ref[k]) / n0 for k in range(2 * nm + 1))
    print(f"B=33 {prec}: Upsilon {e.max():.2e}, N_n/N_0 {en:.2e}", flush=True)
    assert e.max() <= tol and en <= FP32_TOL


def test_adjoint_64_bins_large_order(t3):
    """64 bins at n_max = 40: the coefficient step's LDS (64 KiB and more)
    needs the raised dynamic-LDS limit; gradient against the FP64 autograd
    oracle, with the planes kept by the forward."""
    from oracle import autodiff as ad
    cat = random_catalog(700, 30.0, seed=4801)
    tgt = random_catalog(700, 30.0, seed=4802)
    edges = np.geomspace(0.8, 12.0, 65)
    nm = 40
    pl = ad.pairs(cat.x, cat.y, edges)
    t = lambda a: torch.tensor(np.asarray(a, dtype=np.float64))  # noqa: E731
    uT, NT = ad.multipoles(tgt.x, tgt.y, t(tgt.g1), t(tgt.g2), t(tgt.w), edges, nm)
    T = ad.gamma(uT, NT).detach()
    om = ad.loss_weights(T)
    g1 = t(cat.g1).requires_grad_(True)
    g2 = t(cat.g2).requires_grad_(True)
    w = t(cat.w).requires_grad_(True)
    u, N = ad.multipoles(cat.x, cat.y, g1, g2, w, edges, nm, pair_list=pl)
    Lr = ad.loss(ad.gamma(u, N), T, om)
    Lr.backward()
    lo, size = box_for(30.0)
    plan = t3.Plan(edges, nm, box_lo=lo, box_size=size, keep_planes=True)
    dev = "cuda"
    x = torch.from_numpy(cat.x).to(dev)
    y = torch.from_numpy(cat.y).to(dev)
    q1 = torch.from_numpy(cat.g1.copy()).to(dev).requires_grad_(True)
    q2 = torch.from_numpy(cat.g2.copy()).to(dev).requires_grad_(True)
    qw = torch.from_numpy(cat.w.copy()).to(dev).requires_grad_(True)
    gam = torch.view_as_complex(t3.GammaMultipoles.apply(q1, q2, qw, x, y, plan))
    d = gam - T.to(dev)
    L = torch.sum(om.to(dev) * (d.real ** 2 + d.imag ** 2))
    L.backward()
    assert abs(float(L) - float(Lr)) < 1e-5 * float(Lr)
    for got, ref, name in ((q1.grad, g1.grad, "g1"), (q2.grad, g2.grad, "g2"), (qw.grad, w.grad, "w")):
        got = got.cpu().numpy()
        ref = ref.numpy()
        e = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print(f"B=64 n_max=40 grad {name}: rel-norm {e:.2e}", flush=True)
        assert e < 2e-5, (name, e)
