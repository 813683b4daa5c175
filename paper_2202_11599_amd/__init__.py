"""NysADMM hot path for AMD MI355X (gfx950).

The compute lives in a HIP shared library (libnysadmm.so) behind a C ABI
declared in include/nysadmm.h; `paper_2202_11599_amd.nysadmm` is the thin
ctypes binding with the same entry-point names.  `synth` draws the seeded
synthetic workloads.  Importing this package loads nothing; the library is
loaded on first use of the binding and a missing build raises.
"""
