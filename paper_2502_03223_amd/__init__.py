"""MI355X-native GRHD Runge-Kutta substep (Lam & Shibata, arXiv 2502.03223,
Sec. II.C): hand-written gfx950 HIP kernels behind the C ABI of
include/grhd.h, with a thin ctypes binding in ``grhd``."""
__all__ = ["grhd"]
