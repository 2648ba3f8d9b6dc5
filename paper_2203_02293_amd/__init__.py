"""MI355X-native improved two-stream radiative transfer (THOR+HELIOS hot path).

``paper_2203_02293_amd.rt``     ctypes binding of the C-ABI (include/rt.h)
``paper_2203_02293_amd.build``  hipcc build of the gfx950 library
``paper_2203_02293_amd.synth``  seeded synthetic inputs (no method arithmetic)

Importing the package loads nothing; the HIP library is loaded on first use
of ``rt`` and its absence is an error, never a fallback.
"""
