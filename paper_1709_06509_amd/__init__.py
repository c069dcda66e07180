"""Hierarchical, fast-converging min-sum BP stereo on MI355X (gfx950).

The GPU path lives in libbpstereo.so (HIP kernels behind the C ABI of
include/bpstereo.h); ``paper_1709_06509_amd.bpstereo`` is its Python binding and
``paper_1709_06509_amd.synth`` makes seeded synthetic stereo pairs.  Importing this
package loads nothing; the binding loads the library on first use.
"""
