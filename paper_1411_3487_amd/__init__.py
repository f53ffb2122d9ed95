"""MI355X (gfx950) mode-amplitude Langevin dynamics of semiflexible chains
(Panja, Barkema & van Leeuwen, arXiv:1411.3487).

The simulation runs in the HIP library libdnamodes.so (C ABI in
include/dnamodes.h); this package holds the build script, a ctypes binding
(``_lib``) and the seeded synthetic input generators (``inputs``).
"""
from ._lib import (Context, DMError, coarse_grain, load, DM_FP64, DM_FP32, DM_BF16X3,  # noqa: F401
                   DM_OBS_CHAIN, DM_OBS_MODES, DM_OBS_ACCUM, DM_OBS_RESET)

# dsDNA in the paper's reduced units (Sec. II.A) and its maximal time steps
# per chain length (Table 1; 96/192/384 bp take the next shorter length's).
NU_DSDNA = 0.35
T_STAR_DSDNA = 0.034
DTAU_MAX = {64: 10.0, 96: 10.0, 128: 50.0, 192: 50.0, 256: 100.0, 384: 100.0, 512: 100.0}
