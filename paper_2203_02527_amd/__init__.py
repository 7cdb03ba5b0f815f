"""MI355X (gfx950) library for 0th persistent homology barcodes.

The computation lives in libph0.so (HIP kernels behind the C ABI of
include/ph0.h); ``paper_2203_02527_amd.ph0`` is its ctypes binding and
``paper_2203_02527_amd.synth`` draws the seeded workloads.  Importing the
package loads nothing; the binding loads the library on first use and
fails if it has not been built.
"""
