"""Independent CPU oracle for the symmetry-sector H.v, basis and Lanczos.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the product library (``paper_1804_05028_amd``) and never imports it; the
two meet only in the seeded inputs of ``ed_inputs``.

Contents
--------
* ``bruteforce``: plain C brute force (``orc.c``), wrapped with ctypes --
  representatives by applying every group element, the sector basis, the
  scatter-form H.v, and per-row matrix elements for sampled checks.
* ``definition``: the sector matrix straight from the definition of
  symmetry-adapted states, B^dagger H B, with B built column by column in the
  full fixed-Sz basis (small N only).
* ``dimension``: sector dimensions from the character formula.
* ``lanczos``: the plain three-term Lanczos recurrence in NumPy, FP64.

Every function cites the passage of Wietek & Laeuchli (arXiv:1804.05028) that
it follows.  Parity status of each function is recorded in its module
docstring; none is "parity unpinned".
"""
