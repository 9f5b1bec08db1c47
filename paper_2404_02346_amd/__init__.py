"""MI355X-native wave lattice Boltzmann computation of the acoustic radiation force.

Hot path in hand-written HIP for gfx950 behind the C ABI of include/lb_wave.h
(liblbwave.so); this package is its thin ctypes binding.  Method:
Castro-Avila et al., "A lattice Boltzmann approach for acoustic manipulation"
(arXiv 2404.02346).
"""
from .lbwave import (LBError, LBWave, STORAGE, cavity_calibrate, check,  # noqa: F401
                     lib, make_descs, stream_copy, workspace_bytes)
