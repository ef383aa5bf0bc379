"""MI355X-native multipath Metropolis engine for the classical Heisenberg model.

The engine is the C ABI of include/mmc.h (libmmc.so, HIP kernels for gfx950); the
`mmc` module binds it. Nothing is loaded at import time.
"""
