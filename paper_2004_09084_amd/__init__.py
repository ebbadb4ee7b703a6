"""MI355X-native layered belief-propagation decoding of QC-MET-LDPC codes.

The compute path is the HIP library ``libqcmet.so`` (kernels for gfx950 and
a C ABI, see include/qcmet.h); ``paper_2004_09084_amd.qcmet`` is its Python
binding.  Importing this package loads nothing; ``workload`` draws the
seeded synthetic inputs.
"""
