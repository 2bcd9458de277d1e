"""Writes the stored oracle references of the sampled-centre parity tests.

Calls only the FP64 CPU oracle (``oracle/``) and the seeded catalog
generator; nothing here touches the HIP library.  For each workload the
file holds the centre sample, the exact in-range pair count, the packed
multipoles [5, n_max + 1, B, B] (Upsilon_{0..3,n} and N_n, n >= 0,
complex128) and the normalised Gamma_{mu,n} = Upsilon_{mu,n} / N_0, plus a
SHA-256 of the catalog arrays so that a test can confirm it regenerated the
same inputs.

    python tests/golden/make_fixtures.py [field_1m] [field_4m]
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import multipole as mp  # noqa: E402
from paper_2309_08601_amd.synth import WORKLOADS, centre_sample, make_catalogs  # noqa: E402

# centre samples of the sampled-centre parity tests (20,000 centres each)
SAMPLES = {"field_1m": (20000, 21), "field_4m": (20000, 23)}


def catalog_sha(cat) -> str:
    h = hashlib.sha256()
    for a in (cat.x, cat.y, cat.g1, cat.g2, cat.w):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def fixture_path(name: str) -> str:
    n, seed = SAMPLES[name]
    return os.path.join(HERE, f"oracle_{name}_{n // 1000}k_centres.npz")


def make(name: str) -> str:
    wl = WORKLOADS[name]
    n, seed = SAMPLES[name]
    t0 = time.time()
    cat = make_catalogs(wl)[0]
    idx = centre_sample(cat.n, n, seed=seed)
    o = mp.multipoles(cat, wl.edges(), wl.n_max, centres=idx)
    ref = mp.pack_nonneg(o["ups"], o["N"], wl.n_max)
    gam, _ = mp.normalise(o["ups"], o["N"])
    path = fixture_path(name)
    np.savez(path, idx=idx, npairs=np.int64(o["npairs"]), ref=ref, gamma_n=gam[:, wl.n_max:],
             catalog_sha256=np.array(catalog_sha(cat)), workload=np.array(name))
    print(f"{name}: {n} centres, {o['npairs']} pairs, {time.time() - t0:.0f} s -> {path}", flush=True)
    return path


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(SAMPLES)):
        make(name)
