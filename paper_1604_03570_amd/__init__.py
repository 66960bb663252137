"""boxtile: single-level BoxLib MultiFab hot path (FillBoundary, heat step, red-black
Gauss-Seidel, reductions) on MI355X (gfx950), behind the C-ABI library libboxtile.so.

Importing the package loads nothing; ``paper_1604_03570_amd.boxtile`` is the Python
binding over the C-ABI and ``paper_1604_03570_amd.inputs`` the seeded synthetic
input generators.
"""
__all__ = ["boxtile", "inputs"]
