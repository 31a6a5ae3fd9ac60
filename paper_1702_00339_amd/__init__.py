"""MI355X-native lattice core-Hamiltonian solver (block-circulant / Toeplitz).

``lhf`` is the ctypes binding of the HIP library liblhf.so (C ABI in
include/lhf.h); ``pipeline`` runs the periodic hot path on torch device
buffers.  Importing the package does not load the library; the first call
does, and fails loudly if it has not been built.
"""
