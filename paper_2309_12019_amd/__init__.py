"""MI355X-native hot path of the dissipative-WENO-stabilised RKDG scheme
(Vedral, arXiv 2309.12019): HIP kernels for gfx950 behind the C ABI of
include/dgweno.h, with a thin ctypes binding (paper_2309_12019_amd.dgweno).

The binding is imported lazily so that the seeded workload module
(paper_2309_12019_amd.inputs) can be used without a GPU or a built library.
"""
__all__ = ["inputs", "dgweno"]
