"""MI355X-native Flux Reconstruction right-hand side (HIP kernels for gfx950 behind a C ABI).

Importing the package loads nothing native; ``paper_2408_16509_amd.frmi`` opens the
built library (``libfrmi.so``) and raises if it is missing.
"""
