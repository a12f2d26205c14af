"""MI355X-native G-QAOA on random 3-SAT (Zhang et al., arXiv 2402.02585).

The compute path lives in ``libgqaoa.so`` (HIP kernels for gfx950 behind a
C ABI declared in include/gqaoa.h). ``paper_2402_02585_amd.gqaoa`` is the thin
Python binding with the same function names; importing this package does not
load the library, so the seeded generators in ``instances`` stay usable on a
machine without a GPU.
"""
__all__ = ["instances", "gqaoa"]
