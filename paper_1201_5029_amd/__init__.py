"""MI355X-native symplectic FRW lattice library (HIP/gfx950) after
Sainio, arXiv:1201.5029.  The compute lives in libsymlat.so (C ABI in
include/symlat.h); this package is its thin Python binding."""
from .symlat import (  # noqa: F401
    Lattice, Batch, Linear, STENCILS, SymlatError, load, composition_weights, stability_limit,
    footprint_bytes, transient_bytes, device_memory, from_recipe, EXPORTS,
)
