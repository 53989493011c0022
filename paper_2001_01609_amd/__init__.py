"""MI355X library for Parareal applied to 2D Rayleigh-Benard convection.

The compute path is librbc.so (HIP, gfx950) behind the C ABI in
include/rbc.h; ``paper_2001_01609_amd.rbc`` is its Python binding.
"""
