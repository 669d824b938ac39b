"""MI355X (gfx950) offered-ILP streaming-load library.

``ilpsweep``  ctypes binding of the C ABI in ``include/ilpsweep.h`` (the HIP
              kernels live in ``csrc/`` and are built into ``libilpsweep.so``)
``stats``     sweep statistics: medians, K=2->8 decline, peak K, knee and
              regime rule, residency screen, Little's-law accounting
``rocprof``   parser for rocprofv3 counter CSVs (the counter audit)
"""
