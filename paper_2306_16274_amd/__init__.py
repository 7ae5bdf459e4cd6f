"""MI355X (gfx950) HIP implementation of the fused time step of the non-orthogonal
MRT lattice Boltzmann method with the pseudopotential multiphase model
(Fei et al., arXiv 2306.16274), behind the C ABI of include/lbm.h.

Submodules: ``lbm`` (ctypes binding, one function per C entry point), ``build``
(hipcc build of liblbm_hip.so), ``serving`` (continuous-batching request loop).
"""
