"""MI355X-native subdomain-levelset deflated PCG (arXiv 1510.02148) behind a C-ABI.

``psl``       -- ctypes binding of libpsl (include/psl.h), same names as the C entry points.
``pipeline``  -- convenience chaining of those calls for one permeability field.
``build``     -- hipcc build of libpsl.so for gfx950.
"""
__all__ = ["psl", "pipeline", "build"]
