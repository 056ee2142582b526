"""Pauli-sum operator-state engine for AMD MI355X (gfx950).

The numerical work lives in the HIP library ``libpbs.so`` (C ABI declared
in include/pbs.h); ``api`` is its Python binding.
"""
