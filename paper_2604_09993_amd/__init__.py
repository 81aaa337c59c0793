"""MI355X-native interval linearize-and-discretize for CI-SCvx (arxiv 2604.09993).

The hot path (RK4 of the time-dilated augmented system with its variational
equations, defects, and the reverse-mode sweep) runs in hand-written HIP
kernels for gfx950 behind the C ABI of include/cis.h (libcis.so).  This
package holds the ctypes binding (``_lib``), the torch-facing calls
(``api``), the in-tree build (``build``) and the seeded synthetic inputs
(``synth``).
"""
__all__ = ["synth", "api", "build"]
