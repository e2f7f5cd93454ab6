"""MI355X-native on-the-fly training-data generator for binary-black-hole
likelihood-free inference (AMPLFI, section 3.2 of the paper).

Every step runs in hand-written HIP kernels for gfx950 behind the C-ABI
library ``libgwgen.so`` (declared in ``include/gwgen.h``).  This package holds
the thin ctypes binding (``gwgen``) and the seeded synthetic inputs
(``inputs``).  The binding loads the library on first use and raises if it
has not been built: there is no CPU fallback.
"""
