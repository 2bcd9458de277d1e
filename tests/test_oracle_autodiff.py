"""Pins of the differentiable FP64 oracle (reference gradient of the adjoint).

* its forward equals the C-core oracle (independent implementation);
* its gradient equals central finite differences of the loss: exact for
  the shears up to rounding, because after removing j = k every
  pairwise-distinct triplet holds a galaxy at most once, so Upsilon (and
  Gamma = Upsilon / N_0, N_0 free of shears) is linear in each gamma_j and
  the loss quadratic; for the weights (N_0 depends on w) with a small step.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import autodiff as ad  # noqa: E402
from oracle import multipole as mp  # noqa: E402
from paper_2309_08601_amd.synth import random_catalog  # noqa: E402

EDGES = np.geomspace(1.0, 10.0, 5)
NM = 5


@pytest.fixture(scope="module")
def setup(oracle_lib):
    cat = random_catalog(220, 25.0, seed=77)
    tgt = random_catalog(220, 25.0, seed=78)
    pl = ad.pairs(cat.x, cat.y, EDGES)
    t = lambda a: torch.tensor(np.asarray(a, dtype=np.float64))  # noqa: E731
    u_t, N_t = ad.multipoles(cat.x, cat.y, t(tgt.g1), t(tgt.g2), t(tgt.w), EDGES, NM, pair_list=pl)
    T = ad.gamma(u_t, N_t).detach()
    om = ad.loss_weights(T)
    return cat, pl, T, om, t


def _L(cat, pl, T, om, t, g1, g2, w):
    u, N = ad.multipoles(cat.x, cat.y, g1, g2, w, EDGES, NM, pair_list=pl)
    return ad.loss(ad.gamma(u, N), T, om)


def test_forward_matches_c_oracle(setup):
    cat, pl, T, om, t = setup
    u, N = ad.multipoles(cat.x, cat.y, t(cat.g1), t(cat.g2), t(cat.w), EDGES, NM, pair_list=pl)
    o = mp.multipoles(cat, EDGES, NM)
    ref = o["ups"][:, NM:]
    assert np.abs(u.detach().numpy() - ref).max() < 1e-12 * np.abs(ref).max()
    refN = o["N"][NM:2 * NM + 1]
    assert np.abs(N.detach().numpy() - refN).max() < 1e-12 * np.abs(refN).max()


def test_gradient_matches_finite_differences(setup):
    cat, pl, T, om, t = setup
    g1 = t(cat.g1).requires_grad_(True)
    g2 = t(cat.g2).requires_grad_(True)
    w = t(cat.w).requires_grad_(True)
    L = _L(cat, pl, T, om, t, g1, g2, w)
    L.backward()
    rng = np.random.default_rng(3)
    for j in rng.choice(cat.n, 6, replace=False):
        for which, grad, h in ((0, g1.grad, 0.05), (1, g2.grad, 0.05), (2, w.grad, 1e-4)):
            vals = []
            for sgn in (1, -1):
                a = [t(cat.g1), t(cat.g2), t(cat.w)]
                a[which] = a[which].clone()
                a[which][j] += sgn * h
                with torch.no_grad():
                    vals.append(float(_L(cat, pl, T, om, t, *a)))
            fd = (vals[0] - vals[1]) / (2 * h)
            g = float(grad[j])
            tol = (1e-9 if which < 2 else 1e-6) * max(abs(g), 1e-3 * float(L))
            assert abs(fd - g) <= tol, (j, which, fd, g)


def test_centre_subset_forward_and_gradient(setup):
    """A centre subset (the sum over centres i restricted to a set, every
    galaxy still a neighbour) equals the C-core oracle's centre list, an
    index listed twice counts twice, and the gradient (which still reaches
    galaxies outside the set through their neighbours' harmonic sums)
    equals central finite differences."""
    cat, pl, T, om, t = setup
    rng = np.random.default_rng(12)
    sub = np.sort(rng.choice(cat.n, 90, replace=False))
    u, N = ad.multipoles(cat.x, cat.y, t(cat.g1), t(cat.g2), t(cat.w), EDGES, NM, pair_list=pl, centres=sub)
    o = mp.multipoles(cat, EDGES, NM, centres=sub)
    ref = o["ups"][:, NM:]
    assert np.abs(u.detach().numpy() - ref).max() < 1e-12 * np.abs(ref).max()
    assert np.abs(N.detach().numpy() - o["N"][NM:2 * NM + 1]).max() < 1e-12 * np.abs(o["N"]).max()
    dup = np.concatenate([sub, sub[:7]])
    u2, _ = ad.multipoles(cat.x, cat.y, t(cat.g1), t(cat.g2), t(cat.w), EDGES, NM, pair_list=pl, centres=dup)
    o2 = mp.multipoles(cat, EDGES, NM, centres=dup)
    assert np.abs(u2.detach().numpy() - o2["ups"][:, NM:]).max() < 1e-12 * np.abs(o2["ups"]).max()
    g1 = t(cat.g1).requires_grad_(True)
    g2 = t(cat.g2).requires_grad_(True)
    w = t(cat.w).requires_grad_(True)

    def L_of(a1, a2, aw):
        uu, NN = ad.multipoles(cat.x, cat.y, a1, a2, aw, EDGES, NM, pair_list=pl, centres=sub)
        return ad.loss(ad.gamma(uu, NN), T, om)

    L = L_of(g1, g2, w)
    L.backward()
    outside = np.setdiff1d(np.arange(cat.n), sub)
    assert float(np.abs(g1.grad.numpy()[outside]).max()) > 0
    for j in list(rng.choice(sub, 3, replace=False)) + list(rng.choice(outside, 3, replace=False)):
        for which, grad, h in ((0, g1.grad, 0.05), (1, g2.grad, 0.05), (2, w.grad, 1e-4)):
            vals = []
            for sgn in (1, -1):
                a = [t(cat.g1), t(cat.g2), t(cat.w)]
                a[which] = a[which].clone()
                a[which][j] += sgn * h
                with torch.no_grad():
                    vals.append(float(L_of(*a)))
            fd = (vals[0] - vals[1]) / (2 * h)
            g = float(grad[j])
            tol = (1e-9 if which < 2 else 1e-6) * max(abs(g), 1e-3 * float(L))
            assert abs(fd - g) <= tol, (j, which, fd, g)
