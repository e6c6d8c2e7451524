"""MI355X-native 3D fast super-resolution (Fourier-domain Tikhonov and TV-ADMM).

The solver runs in ``libsr3d.so`` (hand-written HIP for gfx950, C ABI declared
in ``include/sr3d.h``). ``paper_2010_15491_amd.sr3d`` is the thin ctypes
binding. Nothing is imported here, so the input generators in
``paper_2010_15491_amd.phantom`` can be used without loading the library.
"""
