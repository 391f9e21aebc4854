"""MI355X-native DG-AMR hot path (arXiv 2404.16648): HIP library + thin binding.

``dg`` binds the C ABI of ``libdgamr.so`` (include/dg.h); ``synth`` holds the
seeded synthetic input generators; ``build`` compiles the library for gfx950.
"""
