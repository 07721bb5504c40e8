"""Grid Hashing Neighborhood (GHN) KNN on MI355X (gfx950).

`paper_2004_02290_amd.binding` is the Python binding of the HIP library
libghn.so (C ABI in include/ghn.h); `paper_2004_02290_amd.workloads` holds the
seeded input generators.
"""
