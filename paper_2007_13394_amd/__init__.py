"""MI355X-native particle-mesh step of FastPM with massive-neutrino particles.

The compute path is libpm.so (hand-written HIP kernels for gfx950 behind a
C ABI declared in include/pm.h); ``pm`` is its thin Python binding, taking
torch tensors for device memory and the current HIP stream.
"""
