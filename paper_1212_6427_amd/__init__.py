"""MI355X (gfx950) implementation of the incompressible Inertial Coupling
Method step: a C-ABI library of hand-written HIP kernels (libicm.so, built
by paper_1212_6427_amd.build) and its ctypes binding (paper_1212_6427_amd.icm).
"""
