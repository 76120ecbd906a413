"""MI355X-native hot path of the 3D Edge-Based Interface Tracking method
(Pan et al., arXiv 2509.26361): direction-split interface advection and
Front2VOF as hand-written HIP kernels for gfx950 behind the C ABI of
``include/ebit.h``.

Modules: ``ebit`` (binding of the C ABI), ``inputs`` (seeded workloads),
``build`` (hipcc build step)."""
__all__ = ["ebit", "inputs", "build"]
