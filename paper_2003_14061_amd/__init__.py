"""MI355X-native short-range molecular dynamics (Rapaport, arXiv:2003.14061).

The GPU work lives in ``libmd.so`` (hand-written HIP for gfx950 behind a C
ABI, see ``include/md.h``).  ``paper_2003_14061_amd.md`` is the thin Python
binding; ``paper_2003_14061_amd.inputs`` builds seeded initial states.
Importing the package does not load the GPU library.
"""
__all__ = ["inputs", "md"]
