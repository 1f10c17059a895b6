"""MAFOD (multi-scale anisotropic fourth-order diffusion) on MI355X.

The filter runs in the HIP library ``libmf4d.so`` (C ABI in include/mf4d.h);
``paper_1611_06906_amd.mf4d`` is its Python binding. ``synth`` holds the
seeded input generators. Importing the package itself loads nothing.
"""
__all__ = ["mf4d", "synth"]
