"""MI355X-native real-space AMOEBA pair engine (neighbour lists, permanent
multipoles, Thole-damped induced-dipole PCG, Halgren 14-7 / LJ 12-6 vdW,
Ewald point charges), after arXiv 1906.01211.

The compute lives in ``libtk.so`` (hand-written HIP for gfx950 behind a
C-ABI declared in ``include/tk.h``); ``paper_1906_01211_amd.tk`` is the thin
ctypes binding, ``paper_1906_01211_amd.synth`` the seeded input generator.
Importing this package loads nothing; ``tk.load()`` loads the library and
raises if it is missing.
"""
__all__ = ["synth", "tk"]
