"""MI355X-native hot path of the 3D central-moment lattice Boltzmann method
(Premnath & Banerjee, arXiv:1202.6081): a HIP library (libcmlbm.so, C ABI in
include/cmlbm.h) and its Python binding.

Submodules are imported on demand: ``cmlbm`` (ctypes binding), ``autograd``
(differentiable runs with checkpoint-and-recompute), ``build`` (hipcc build).
"""
__all__ = ["cmlbm", "build"]
