"""MI355X implementation of the multipole estimator of the shear
three-point correlation function (Porth et al. 2023).

``paper_2309_08601_amd.t3`` binds the HIP library (C ABI in include/t3pcf.h);
``paper_2309_08601_amd.synth`` generates seeded synthetic catalogs.
The binding is imported lazily so that the input generator can be used on
machines without the built library.
"""
__all__ = ["synth", "t3", "build"]
