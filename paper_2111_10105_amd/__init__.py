"""MI355X (gfx950) spatio-temporal dynamic-mesh compressor.

The compute path is the HIP library libdmc.so behind the C ABI in
include/dmc.h; `dmc` is its ctypes binding.  Importing this package does not
load the library; the first call does, and fails loudly if it is not built.
"""
from . import dmc  # noqa: F401
from .dmc import (Context, DmcError, Mesh, Params, compress_sequence, decode_sequence,  # noqa: F401
                  decode_window, encode_window, make_params, parse_record)
