"""MI355X (gfx950) corner-transfer-matrix library for iPEPS environments.

The computation lives in ``libctm.so`` (hand-written HIP kernels behind the C
interface declared in ``include/ctm.h``); this package only marshals arguments.
"""
from .binding import CTM, MLP, SimpleUpdate, CtmError, fidelity, load, LIB_PATH, EXPORTS  # noqa: F401
