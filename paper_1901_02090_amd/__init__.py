"""MI355X-native adaptive BDDC for RT0/P0 flow in heterogeneous porous media.

The numerical work runs in the HIP library ``libbddc.so`` (C ABI declared in
``include/bddc.h``); this package only marshals arguments.
"""
from .bddc import Solver, Server, BddcError, estimate_bytes, set_allocator, load_library, LIB_PATH  # noqa: F401
