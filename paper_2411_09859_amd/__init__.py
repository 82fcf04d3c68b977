"""Skew-symmetric LTL^T factorization and Pfaffians on AMD MI355X (gfx950).

The compute path is the HIP library ``libskltlt.so`` built from ``csrc/``;
``binding`` marshals arguments to its C ABI (declared in ``include/skltlt.h``).
Importing this package does not load the library; ``binding.lib()`` does, and
raises if it is missing.
"""
__all__ = ["binding", "inputs"]
