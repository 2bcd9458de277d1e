"""The hand-written adjoint (t3_normalise_backward + t3_backward) on the GPU.

* elementwise against the FP64 autograd oracle on a small catalog;
* against central finite differences of the GPU forward (exact for the
  shears: the loss is quadratic in each gamma_j);
* on the 500k-galaxy, 7 deg x 7 deg workload (15 bins 1'-60', n_max 20):
  finite differences of the GPU forward on 64 random galaxies of the full
  catalog, the FP64 autograd oracle on a 5,000-galaxy sub-catalog, and
  exact identities that hold at any size:
    - Gamma is homogeneous of degree 3 in the shears:
          sum_j g . dL/dg_j = 6 sum omega Re(conj(Gamma - T) Gamma);
    - Gamma is homogeneous of degree 0 in the weights: sum_j w_j dL/dw_j = 0;
    - a common phase rotation of every shear, gamma -> gamma e^{i eps},
      turns Gamma_0 by e^{3 i eps} and Gamma_{1,2,3} by e^{i eps}:
          sum_j (g1 dL/dg2 - g2 dL/dg1) = sum 2 omega Re(conj(Gamma - T) i k_mu Gamma),
      k = (3, 1, 1, 1).
Tolerances: 2e-5 (norm-relative) against the oracle; 1e-4 for the
full-size identities (FP32 gradients summed over 5e5 galaxies).
"""
import numpy as np
import pytest

from paper_2309_08601_amd.synth import LATTICE_UNIT, WORKLOADS, make_catalogs, random_catalog
from _util import box_for

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def t3():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08601_amd import t3 as mod
    return mod


def _loss_torch(gam, T, om):
    d = gam - T
    return torch.sum(om * (d.real ** 2 + d.imag ** 2))


def _gpu_loss_and_grad(t3, plan, cat, T, om):
    dev = "cuda"
    x = torch.from_numpy(cat.x).to(dev)
    y = torch.from_numpy(cat.y).to(dev)
    g1 = torch.from_numpy(cat.g1.copy()).to(dev).requires_grad_(True)
    g2 = torch.from_numpy(cat.g2.copy()).to(dev).requires_grad_(True)
    w = torch.from_numpy(cat.w.copy()).to(dev).requires_grad_(True)
    gam = torch.view_as_complex(t3.GammaMultipoles.apply(g1, g2, w, x, y, plan))
    L = _loss_torch(gam, T.to(dev), om.to(dev))
    L.backward()
    return L.detach(), gam.detach(), g1.grad.cpu().numpy(), g2.grad.cpu().numpy(), w.grad.cpu().numpy()


def test_normalise_backward_matches_autograd(t3):
    rng = np.random.default_rng(1)
    nm, B = 4, 3
    plan = t3.Plan(np.geomspace(1, 5, B + 1), nm, box_size=1 << 20)
    ups = torch.from_numpy(rng.standard_normal((5, nm + 1, B, B, 2)))
    ups[4, 0, :, :, 0] = torch.from_numpy(rng.uniform(1, 2, (B, B)))
    ups[4, 0, :, :, 1] = 0
    gg = torch.from_numpy(rng.standard_normal((4, nm + 1, B, B, 2)))
    got = plan.normalise_backward(ups.cuda(), gg.cuda()).cpu()
    u = ups.clone().requires_grad_(True)
    uc = torch.view_as_complex(u)
    gam = uc[:4] / uc[4, 0].real[None, None]
    gam_r = torch.view_as_real(gam)
    (gam_r * gg).sum().backward()
    assert torch.allclose(got, u.grad, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("keep", [False, True])
def test_backward_matches_fp64_autograd_oracle(t3, keep):
    """keep: the backward takes the planes the forward kept (three chunks of
    512 centres, the last ragged; forward as a captured graph) instead of
    recomputing stage 1."""
    from oracle import autodiff as ad
    cat = random_catalog(1500, 40.0, seed=501)
    tgt = random_catalog(1500, 40.0, seed=502)
    edges = np.geomspace(1.0, 12.0, 6)
    nm = 8
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
    lo, size = box_for(40.0)
    plan = t3.Plan(edges, nm, box_lo=lo, box_size=size, keep_planes=keep, chunk_centres=512 if keep else 0)
    L, _, d1, d2, dw = _gpu_loss_and_grad(t3, plan, cat, T, om)
    assert abs(float(L) - float(Lr)) < 1e-5 * float(Lr)
    for got, ref, name in ((d1, g1.grad, "g1"), (d2, g2.grad, "g2"), (dw, w.grad, "w")):
        ref = ref.numpy()
        e = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        m = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"grad {name}: rel-norm {e:.2e}, rel-max {m:.2e}", flush=True)
        assert e < 2e-5 and m < 1e-4, (name, e, m)


def test_kept_planes_follow_the_catalog(t3):
    """With kept planes the backward reuses the last forward's planes only
    when it is given that forward's catalog and nothing rebuilt the plan's
    catalog in between; otherwise it recomputes stage 1.  Gradients agree
    with a plan that keeps nothing either way (to rounding: FP32 atomics)."""
    rng = np.random.default_rng(7)
    cats = [random_catalog(1200, 35.0, seed=s) for s in (601, 602)]
    edges = np.geomspace(1.0, 10.0, 6)
    nm = 6
    lo, size = box_for(35.0)
    keep = t3.Plan(edges, nm, box_lo=lo, box_size=size, keep_planes=True, chunk_centres=512, timing=True)
    ref = t3.Plan(edges, nm, box_lo=lo, box_size=size, chunk_centres=512)
    dA, dB = (t3.DeviceCatalog.from_catalog(c) for c in cats)
    gups = torch.from_numpy(rng.standard_normal((5, nm + 1, 5, 5)) + 1j * rng.standard_normal((5, nm + 1, 5, 5)))
    gups = gups.cuda()

    def close(a, b):
        for x, y in zip(a, b):
            x, y = x.cpu().numpy(), y.cpu().numpy()
            assert np.linalg.norm(x - y) <= 1e-5 * np.linalg.norm(y)

    def stage1_launches():
        return keep.stage_times()[1][1]

    keep.forward(dA)
    got = keep.backward(dA, gups)
    assert stage1_launches() == 0
    close(got, ref.backward(dA, gups))
    keep.forward(dB)
    got = keep.backward(dA, gups)  # kept planes are B's: recompute
    assert stage1_launches() > 0
    close(got, ref.backward(dA, gups))
    got = keep.backward(dA, gups)  # the last call rebuilt the catalog: recompute
    assert stage1_launches() > 0
    keep.forward(dB)
    got = keep.backward(dB, gups)
    assert stage1_launches() == 0
    close(got, ref.backward(dB, gups))


def test_backward_largest_order_matches_fp64_autograd_oracle(t3):
    """n_max = 64: the largest compiled transpose-scan variant."""
    from oracle import autodiff as ad
    cat = random_catalog(700, 30.0, seed=511)
    tgt = random_catalog(700, 30.0, seed=512)
    edges = np.geomspace(1.0, 8.0, 5)
    nm = 64
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
    L, _, d1, d2, dw = _gpu_loss_and_grad(t3, plan, cat, T, om)
    assert abs(float(L) - float(Lr)) < 1e-5 * float(Lr)
    for got, ref, name in ((d1, g1.grad, "g1"), (d2, g2.grad, "g2"), (dw, w.grad, "w")):
        ref = ref.numpy()
        e = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print(f"n_max 64 grad {name}: rel-norm {e:.2e}", flush=True)
        assert e < 2e-5, (name, e)


def test_backward_matches_finite_differences_of_gpu_forward(t3):
    cat = random_catalog(2000, 45.0, seed=601)
    tgt = random_catalog(2000, 45.0, seed=602)
    edges = np.geomspace(1.0, 14.0, 6)
    nm = 10
    lo, size = box_for(45.0)
    plan = t3.Plan(edges, nm, box_lo=lo, box_size=size)
    Tu, _ = plan.forward(t3.DeviceCatalog.from_catalog(tgt))
    T, _ = plan.normalise_resum(Tu, with_phi=False)
    T = T.cpu()
    om = 1.0 / torch.clamp(torch.mean(T.real ** 2 + T.imag ** 2, dim=1, keepdim=True), min=1e-300)
    om = om.expand_as(T.real).contiguous()
    L0, _, d1, d2, _ = _gpu_loss_and_grad(t3, plan, cat, T, om)

    def L_of(g1, g2):
        c = t3.DeviceCatalog(cat.x, cat.y, g1, g2, cat.w)
        u, _ = plan.forward(c)
        g, _ = plan.normalise_resum(u, with_phi=False)
        return float(_loss_torch(g.cpu(), T, om))

    rng = np.random.default_rng(9)
    h = 0.05
    for j in rng.choice(cat.n, 12, replace=False):
        for which, grad in ((0, d1), (1, d2)):
            a = [cat.g1.astype(np.float64).copy(), cat.g2.astype(np.float64).copy()]
            ap = [v.copy() for v in a]
            am = [v.copy() for v in a]
            ap[which][j] += h
            am[which][j] -= h
            fd = (L_of(*[v.astype(np.float32) for v in ap]) - L_of(*[v.astype(np.float32) for v in am])) / (2 * h)
            g = float(grad[j])
            scale = np.abs(grad).max()
            assert abs(fd - g) <= 1e-2 * max(abs(g), 0.05 * scale), (j, which, fd, g)


def test_backward_exact_identities_at_500k(t3):
    wl = WORKLOADS["grad_500k"]
    cat = make_catalogs(wl)[0]
    tgt = make_catalogs(wl, seed_offset=100)[0]
    lo, size = box_for(wl.side)
    plan = t3.Plan(wl.edges(), wl.n_max, box_lo=lo, box_size=size)
    Tu, _ = plan.forward(t3.DeviceCatalog.from_catalog(tgt))
    T, _ = plan.normalise_resum(Tu, with_phi=False)
    T = T.cpu()
    om = 1.0 / torch.clamp(torch.mean(T.real ** 2 + T.imag ** 2, dim=1, keepdim=True), min=1e-300)
    om = om.expand_as(T.real).contiguous()
    L, gam, d1, d2, dw = _gpu_loss_and_grad(t3, plan, cat, T, om)
    gam = gam.cpu()
    D = gam - T
    g1 = cat.g1.astype(np.float64)
    g2 = cat.g2.astype(np.float64)
    w = cat.w.astype(np.float64)
    # degree 3 in the shears
    lhs = float(np.dot(g1, d1) + np.dot(g2, d2))
    rhs = float(6.0 * torch.sum(om * (D.real * gam.real + D.imag * gam.imag)))
    print(f"shear homogeneity: {lhs:.6e} vs {rhs:.6e}", flush=True)
    assert abs(lhs - rhs) <= 1e-4 * abs(rhs)
    # degree 0 in the weights
    lw = float(np.dot(w, dw))
    scale = float(np.sum(np.abs(w * dw)))
    print(f"weight homogeneity: {lw:.3e} (scale {scale:.3e})", flush=True)
    assert abs(lw) <= 1e-4 * scale
    # common phase rotation of the shears
    k = torch.tensor([3.0, 1.0, 1.0, 1.0], dtype=torch.float64)[:, None, None, None]
    ig = k * torch.complex(-gam.imag, gam.real)
    rhs2 = float(2.0 * torch.sum(om * (D.real * ig.real + D.imag * ig.imag)))
    lhs2 = float(np.dot(g1, d2) - np.dot(g2, d1))
    print(f"phase rotation: {lhs2:.6e} vs {rhs2:.6e}", flush=True)
    assert abs(lhs2 - rhs2) <= 1e-4 * max(abs(rhs2), 1e-3 * abs(rhs))


def test_backward_fp64_gradient_on_5k_subcatalog_of_500k(t3):
    """The differentiation workload's shear and weight model (7 deg x 7 deg,
    15 bins 1'-60', n_max 20) on a random 5,000-galaxy sub-catalog of the
    500k catalog: every galaxy's gradient against the FP64 autograd oracle,
    the target from the same sub-catalog of the second-seed catalog."""
    from oracle import autodiff as ad
    from paper_2309_08601_amd.synth import centre_sample
    wl = WORKLOADS["grad_500k"]
    sub = centre_sample(wl.n_gal[0], 5000, seed=77)
    cat = make_catalogs(wl)[0].subset(sub)
    tgt = make_catalogs(wl, seed_offset=100)[0].subset(sub)
    edges, nm = wl.edges(), wl.n_max
    t = lambda a: torch.tensor(np.asarray(a, dtype=np.float64))  # noqa: E731
    uT, NT = ad.multipoles(tgt.x, tgt.y, t(tgt.g1), t(tgt.g2), t(tgt.w), edges, nm)
    T = ad.gamma(uT, NT).detach()
    om = ad.loss_weights(T)
    g1, g2, w = (t(v).requires_grad_(True) for v in (cat.g1, cat.g2, cat.w))
    u, N = ad.multipoles(cat.x, cat.y, g1, g2, w, edges, nm)
    Lr = ad.loss(ad.gamma(u, N), T, om)
    Lr.backward()
    lo, size = box_for(wl.side)
    plan = t3.Plan(edges, nm, box_lo=lo, box_size=size)
    L, _, d1, d2, dw = _gpu_loss_and_grad(t3, plan, cat, T, om)
    assert abs(float(L) - float(Lr)) < 1e-5 * float(Lr)
    for got, ref, name in ((d1, g1.grad, "g1"), (d2, g2.grad, "g2"), (dw, w.grad, "w")):
        ref = ref.numpy()
        e = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        m = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"5k sub-catalog grad {name}: rel-norm {e:.2e}, rel-max {m:.2e}", flush=True)
        assert e < 2e-5 and m < 1e-4, (name, e, m)


def test_backward_matches_finite_differences_at_500k(t3):
    """Central finite differences of the GPU forward on 64 random galaxies
    of the full 500k catalog.  After the j = k removal every distinct
    triplet holds a galaxy at most once, so Upsilon and N_0 are linear in
    each galaxy's c_j and w_j, and only centres within the outer bin edge of
    galaxy j (j included) see it: the forward over exactly those centres,
    with one parameter of j moved by +-h, gives the derivative of the full
    Upsilon and N_0 exactly for any h (h = 10 for the shears, where the
    moved galaxy then dominates the sums it enters, 0.4 for the weight), and
    the loss then follows by the chain rule through Gamma = Upsilon / N_0 of
    the full forward."""
    wl = WORKLOADS["grad_500k"]
    cat = make_catalogs(wl)[0]
    tgt = make_catalogs(wl, seed_offset=100)[0]
    edges, nm = wl.edges(), wl.n_max
    lo, size = box_for(wl.side)
    plan = t3.Plan(edges, nm, box_lo=lo, box_size=size)
    Tu, _ = plan.forward(t3.DeviceCatalog.from_catalog(tgt))
    T, _ = plan.normalise_resum(Tu, with_phi=False)
    T = T.cpu()
    om = 1.0 / torch.clamp(torch.mean(T.real ** 2 + T.imag ** 2, dim=1, keepdim=True), min=1e-300)
    om = om.expand_as(T.real).contiguous()
    _, _, d1, d2, dw = _gpu_loss_and_grad(t3, plan, cat, T, om)
    dc = t3.DeviceCatalog.from_catalog(cat)
    U0, _ = plan.forward(dc)
    U0 = U0.cpu().numpy()
    n0 = U0[4, 0].real
    gam = U0[:4] / n0
    dev = gam - T.numpy()
    omn = om.numpy()
    e2hi = (edges[-1] / LATTICE_UNIT) ** 2
    x64, y64 = cat.x.astype(np.int64), cat.y.astype(np.int64)
    rng = np.random.default_rng(19)
    worst = {0: 0.0, 1: 0.0, 2: 0.0}
    scales = {k: np.abs(v).max() for k, v in ((0, d1), (1, d2), (2, dw))}
    for j in rng.choice(cat.n, 64, replace=False):
        near = np.nonzero((x64 - x64[j]) ** 2 + (y64 - y64[j]) ** 2 < e2hi)[0].astype(np.int32)
        cidx = torch.from_numpy(near).cuda()
        for which, arr, h, grad in ((0, dc.g1, 10.0, d1), (1, dc.g2, 10.0, d2), (2, dc.w, 0.4, dw)):
            v0 = float(arr[j])
            U = []
            for sgn in (1, -1):
                arr[j] = v0 + sgn * h
                u, _ = plan.forward(dc, cidx)
                U.append(u.cpu().numpy())
            arr[j] = v0
            D = (U[0] - U[1]) / (2 * h)
            dG = D[:4] / n0 if which < 2 else (D[:4] - gam * D[4, 0].real) / n0
            fd = float(np.sum(2.0 * omn * (dev.real * dG.real + dev.imag * dG.imag)))
            g = float(grad[j])
            err = abs(fd - g) / max(abs(g), 0.05 * scales[which])
            worst[which] = max(worst[which], err)
            assert err <= (2e-4 if which < 2 else 1e-3), (int(j), which, fd, g)
    print(f"500k finite differences, worst relative error g1 {worst[0]:.2e}, g2 {worst[1]:.2e}, "
          f"w {worst[2]:.2e}", flush=True)
