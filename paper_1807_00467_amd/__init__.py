"""MI355X (gfx950) library for the dense registration objective of DIS-CO
(Ruehaak et al., arXiv 1807.00467): NGF distance, curvature, volume-change control
and keypoint terms (eq. 1, 5, 7-11), their gradients, matrix-free Gauss-Newton
products and one Gauss-Newton/PCG step, as hand-written HIP kernels behind the C ABI
in include/disco.h.

`paper_1807_00467_amd.disco` is the ctypes binding; importing it fails loudly when
the HIP library has not been built.
"""
__all__ = ["disco"]
