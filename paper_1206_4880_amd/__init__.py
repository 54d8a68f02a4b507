"""MI355X (gfx950) range-domain matching search of a PIFS fractal encoder
with the dynamic fractal-dimension domain pool (Revathy & Jayamohan).

The compute path is the HIP library ``libfic.so`` (C ABI in include/fic.h);
``fic`` is its thin ctypes binding. Calls raise when the library or a device
is missing: there is no CPU fallback.
"""
from . import fic  # noqa: F401
from .fic import (CODE_DTYPE, Context, FicError, batch_workspace_bytes,  # noqa: F401
                  build_domain_pool, decode_pifs, decode_quadtree, encode, encode_batch,
                  encode_color, encode_pifs, encode_quadtree, fd_classify, unpack_codes)

__all__ = ["fic", "CODE_DTYPE", "Context", "FicError", "batch_workspace_bytes",
           "build_domain_pool", "decode_pifs", "decode_quadtree", "encode_color",
           "encode_quadtree",
           "encode", "encode_batch", "encode_pifs", "fd_classify", "unpack_codes"]
