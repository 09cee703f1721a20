"""MI355X-native TENO-AA8/10 compressible-Euler right-hand side.

The compute path is the HIP library ``libtenoaa.so`` (sources in ``csrc/``,
C ABI in ``include/tenoaa.h``); ``tenoaa`` is its thin Python binding over
torch device memory and streams, and ``inputs`` draws the seeded synthetic
workloads.
"""
