"""MI355X-native coupled-channel R-matrix internal-region solver.

``hprmat``   -- ctypes binding of the C ABI (include/hprmat.h, libhprmat.so)
``pipeline`` -- persistent device buffers and the per-energy call sequence
``build``    -- hipcc build of the library for gfx950
"""
