"""MI355X-native REANN message-passing energy / force library (Python side).

The work runs in ``libreann.so`` (hand-written HIP kernels for gfx950 behind the C ABI
in include/reann.h); this package only marshals arguments.  See ``_binding`` for the
host- and device-pointer entry points and ``autograd`` for the torch wrapper.
"""
from ._binding import (BF16, FP8, FP32, FP64, Context, Model, NeighborList, Plan, ReannError,  # noqa: F401
                       Server, build_neighbors, energy_forces, load)

load()   # fail loudly at import when the library has not been built
