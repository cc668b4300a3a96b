"""MI355X-native hot path of the adaptive POD method for magnetic polarizability
tensor spectral signatures (arXiv 2307.05590): HIP kernels behind the C ABI in
include/mpt.h, with a thin ctypes binding in paper_2307_05590_amd.mpt."""

__all__ = ["mpt"]
