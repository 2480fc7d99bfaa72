"""pfsh: MI355X-native hot path of PFASST-SH (IMEX SDC for the rotating
shallow-water equations in a spherical-harmonic basis).

The compute path is the C-ABI library ``libpfsh.so`` (hand-written HIP for
gfx950, declared in ``include/pfsh.h``); ``paper_1904_05988_amd.pfsh`` is the
thin ctypes binding over it.  ``inputs`` draws the seeded synthetic states.
"""
