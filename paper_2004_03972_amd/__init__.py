"""HQA-MD on MI355X: the hot path of Hybrid Quantum Annealing via Molecular Dynamics.

The compute runs in the HIP library ``libhqa.so`` (``csrc/``) behind the C-ABI
declared in ``include/hqa.h``; :mod:`paper_2004_03972_amd.hqa` is a thin ctypes
binding with the same names.  :mod:`paper_2004_03972_amd.instances` holds the
seeded synthetic instance recipes.
"""
