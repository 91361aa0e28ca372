"""MI355X-native field-split additive-Schwarz GMG-GMRES solver for the
linearized monolithic FSI system (Q2/Q1, nested structured meshes).

The compute path is the C-ABI library ``libfsgmg.so`` (HIP kernels for gfx950
plus host C++ setup); ``paper_1909_13201_amd.fsgmg`` is its thin ctypes
binding.  ``paper_1909_13201_amd.inputs`` describes the seeded synthetic
workloads.  Importing the package does not load the library.
"""
