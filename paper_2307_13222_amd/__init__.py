"""MI355X-native matrix-free H*v, Lanczos and cTPQ engine for spin-1/2 and
Hubbard lattice models (the iterative-method core of HPhi, arXiv:2307.13222).

Importing the package loads nothing native; the HIP library is loaded on the
first call through :mod:`paper_2307_13222_amd.api`.
"""
__all__ = ["workloads"]
