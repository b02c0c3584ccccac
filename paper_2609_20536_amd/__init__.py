"""HOTRG coarse-graining of the 2D generalized XY model on MI355X (gfx950).

The compute path lives in the C-ABI library ``libgxyhotrg.so`` built from
``csrc/``; :mod:`paper_2609_20536_amd.hotrg` is its thin ctypes binding.
Importing this package loads nothing: the binding is imported on demand.
"""

__all__ = ["workloads", "hotrg"]
