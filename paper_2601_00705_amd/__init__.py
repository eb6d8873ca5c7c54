"""MI355X-native differentiable 3D Gaussian-splatting rasterizer (gfx950 HIP).

The renderer of RGS-SLAM (arXiv 2601.00705): projection with EWA covariance
(Eq. proj), tile binning with an LDS radix sort, front-to-back compositing
(Eq. alpha) and its backward, including the SE(3) pose tangent (Eqs. muCjac,
muIjac, sigmaIjac).  Every step runs in the HIP kernels of ``libgsr.so``;
this package only marshals arguments.  Submodules are imported lazily so
that ``scenes`` (input synthesis) loads without the native library.
"""
import importlib

__all__ = ["lib", "render", "scenes", "build"]


def __getattr__(name):
    if name in ("lib", "render", "scenes", "build", "autotune"):
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
