"""Stage 2 on blocks of at most 24 bins, where the complex product is one
real product of 2B x 2B on 16 x 16 MFMA tiles (T = ceil(2B / 16) tiles per
side), and the first size past them (B = 25, the 32 x 32 tiles).

The cases cover every tile count (T = 1, 2, 3), full tiles (B = 8, 16, 24)
and ragged ones, the j = k terms removed and kept, slices of several centre
blocks with a ragged last block, chunked calls, and the normaliser orders
past n_max (N_n for n <= 2 n_max, computed four orders per workgroup: full
and ragged last groups).  Bars as the other FP32 parity tests: relative
Frobenius error 1e-6 and largest entry error 2e-6 per (mu, n), N_n against
its own norm 5e-6; a block of one bin has one entry, whose error is held to
the entry bar."""
import numpy as np
import pytest

from paper_2309_08601_amd.synth import random_catalog
from _util import (FP32_MAX_TOL, FP32_TOL, N_OWN_TOL, SPLIT_MAX_TOL, SPLIT_TOL, box_for, multipole_errors,
                   multipole_max_errors, rel_fro, rel_max)

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def t3():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_08601_amd import t3 as mod
    return mod


def _check(gpu, ref, label, tol=FP32_TOL, max_tol=FP32_MAX_TOL):
    e, e_own = multipole_errors(gpu, ref)
    m = multipole_max_errors(gpu, ref)
    print(f"{label}: max rel-F {e.max():.3e}, max rel-max {m.max():.3e}, N_n own {e_own.max():.3e}", flush=True)
    # a 1 x 1 block's Frobenius error is its one entry's error: the entry bar
    if gpu.shape[-1] == 1:
        tol = max_tol
    assert e.max() <= tol, (label, e.max(), np.unravel_index(np.argmax(e), e.shape))
    assert m.max() <= max_tol, (label, m.max(), np.unravel_index(np.argmax(m), m.shape))
    assert e_own.max() <= N_OWN_TOL, (label, e_own.max())


@pytest.mark.parametrize("B,nm,keep_jk,chunk", [(1, 6, False, None), (4, 7, True, None), (8, 5, False, 512),
                                                (9, 9, False, None), (13, 4, True, None), (16, 6, False, None),
                                                (17, 3, False, 768), (20, 10, False, None), (24, 5, True, None),
                                                (25, 5, False, None)])
def test_forward_small_blocks(t3, B, nm, keep_jk, chunk):
    from oracle import multipole as mp
    cat = random_catalog(2300, 45.0, seed=5100 + B)
    edges = np.geomspace(0.5, 18.0, B + 1)
    lo, size = box_for(45.0)
    kw = {} if chunk is None else {"chunk_centres": chunk}
    plan = t3.Plan(edges, nm, box_lo=lo, box_size=size, keep_jk=keep_jk, **kw)
    ups, npairs = plan.forward(t3.DeviceCatalog.from_catalog(cat))
    o = mp.multipoles(cat, edges, nm, diag=not keep_jk)
    assert npairs == o["npairs"]
    _check(ups.cpu().numpy(), mp.pack_nonneg(o["ups"], o["N"], nm), f"B={B} n_max={nm} keep_jk={keep_jk}")


@pytest.mark.parametrize("B,nm", [(3, 4), (12, 5), (20, 6), (23, 7)])
def test_extended_normaliser_small_blocks(t3, B, nm):
    """N_n for n <= 2 n_max: 2 n_max + 1 orders in groups of four, the last
    group holding one (n_max 4, 6) or three (n_max 5, 7) of them."""
    from oracle import multipole as mp
    cat = random_catalog(2000, 40.0, seed=5200 + B)
    edges = np.geomspace(0.6, 15.0, B + 1)
    lo, size = box_for(40.0)
    plan = t3.Plan(edges, nm, box_lo=lo, box_size=size, edge_correct=True)
    ups, npairs = plan.forward(t3.DeviceCatalog.from_catalog(cat))
    o = mp.multipoles(cat, edges, nm, w_max=2 * nm)
    assert npairs == o["npairs"]
    u4, Ng = plan.split_ups(ups)
    u4 = u4.cpu().numpy()
    Ng = Ng.cpu().numpy()
    e_u = rel_fro(u4, o["ups"][:, nm:])
    m_u = rel_max(u4, o["ups"][:, nm:])
    n_ref = o["N"][2 * nm:]
    n0 = np.linalg.norm(n_ref[0])
    e_n = np.linalg.norm((Ng - n_ref).reshape(Ng.shape[0], -1), axis=1) / n0
    m_n = np.abs(Ng - n_ref).reshape(Ng.shape[0], -1).max(axis=1) / np.abs(n_ref[0]).max()
    print(f"B={B} n_max {nm}: Upsilon {e_u.max():.2e} (max {m_u.max():.2e}), N_n/N_0 {e_n.max():.2e} "
          f"(max {m_n.max():.2e}), orders 0..{2 * nm}", flush=True)
    assert e_u.max() <= FP32_TOL and e_n.max() <= FP32_TOL
    assert m_u.max() <= FP32_MAX_TOL and m_n.max() <= FP32_MAX_TOL


_SPLITS = {"bf16x3": (SPLIT_TOL, SPLIT_MAX_TOL), "fp16x3": (SPLIT_TOL, SPLIT_MAX_TOL),
           "bf16x6": (FP32_TOL, FP32_MAX_TOL)}


@pytest.mark.parametrize("prec", sorted(_SPLITS))
@pytest.mark.parametrize("B,nm", [(5, 6), (12, 4), (20, 8)])
def test_split_precision_small_blocks(t3, prec, B, nm):
    """The split products on the 16 x 16 x 32 tiles (two part products per
    MFMA), one case per tile count, j = k terms removed; bars as for the
    32 x 32 split kernel (1e-5 for the two-part splits, FP32 bars for the
    three-part bf16 split)."""
    from oracle import multipole as mp
    tol, max_tol = _SPLITS[prec]
    cat = random_catalog(2300, 45.0, seed=5300 + B)
    edges = np.geomspace(0.5, 18.0, B + 1)
    lo, size = box_for(45.0)
    plan = t3.Plan(edges, nm, box_lo=lo, box_size=size, precision=prec)
    ups, npairs = plan.forward(t3.DeviceCatalog.from_catalog(cat))
    o = mp.multipoles(cat, edges, nm)
    assert npairs == o["npairs"]
    _check(ups.cpu().numpy(), mp.pack_nonneg(o["ups"], o["N"], nm), f"B={B} n_max={nm} {prec}", tol, max_tol)
