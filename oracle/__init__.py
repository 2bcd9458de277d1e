"""CPU oracle for the multipole estimator of the shear three-point function.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the HIP path (``paper_2309_08601_amd``) other than the seeded
input generator, which holds none of the estimator's arithmetic.

Everything here is FP64 and follows Porth et al. (2023):

* ``brute``     -- O(N^3) triplet sums straight from the definitions of the
                   natural components in the x-projection (Sect. 2.2-2.3,
                   eqs. Gamma0_def..Gamma3_def, xprojection, TripletUpsilon,
                   TripletNorm) -- the independent pin for ``multipole``.
* ``multipole`` -- per-centre harmonic sums (C core, eq. Gn_disc / W_n),
                   the multipoles Upsilon_{mu,n} and N_n for every
                   |n| <= n_max (eqs. Upsilon0_Derivation, Upsilon1-3,
                   3PCF_Normalization) with the j = k terms removed,
                   tomographic triples (eq. tomoGn), normalisation,
                   mode-coupling solve (eqs. ModeCoupling,
                   GammaMultipolesWithEC) and resummation onto angular bins
                   (eq. Gamma0_binned).
* ``autodiff``  -- the same forward written in differentiable torch FP64,
                   used as the reference gradient for the adjoint.
"""
from .multipole import (  # noqa: F401
    squared_edges, harmonics, upsilon_from_harmonics, multipoles, multipoles_tomo,
    normalise, mode_coupling_correct, resum, phi_bin_edges, g_order_range,
    pack_nonneg, build_lib, ORACLE_LIB,
)
