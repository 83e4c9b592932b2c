"""MI355X (gfx950) library for the coherent hyperspin machine (arXiv 2308.02329).

``paper_2308_02329_amd.api`` binds the C ABI of ``libchym.so`` (see
include/chym.h); ``paper_2308_02329_amd.synth`` draws seeded synthetic
inputs.  Importing the package does not load the library; the first API call
does, and raises if it is missing.
"""
__all__ = ["api", "synth"]
