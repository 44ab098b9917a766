"""Kahler-Dirac-preconditioned adaptive multigrid for the staggered Dirac
operator on AMD MI355X (gfx950): a HIP library behind a C ABI (include/kdmg.h)
with a thin Python binding.  Importing `paper_1801_07823_amd.kdmg` loads the
built library and fails loudly if it is missing."""

__all__ = ["kdmg"]
