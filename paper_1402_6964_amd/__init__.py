"""MI355X-native single-pass TSQR and Gaussian projection for near-separable
NMF of tall-and-skinny matrices (Benson, Lee, Rajwa, Gleich).

The compute path is the HIP library ``libtsnmf.so`` (sources in ``csrc/``,
C ABI in ``include/tsnmf.h``); ``tsnmf`` is its thin Python binding and
``synth`` the seeded workload generators.
"""
