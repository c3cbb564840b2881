"""MI355X (gfx950) asymmetric adaptive fast multipole method for the 2D
logarithmic potential, after Engblom, "On well-separated sets and fast
multipole methods".

The computation lives in the HIP library ``libfmm2d.so`` (C ABI in
``include/fmm2d.h``); ``paper_1006_2269_amd.fmm.FMM2D`` is its Python
binding.  Importing this package does not load the library or torch;
``paper_1006_2269_amd.workloads`` holds the seeded synthetic inputs.
"""

__all__ = ["FMM2D", "FMM2DError"]


def __getattr__(name):
    if name in ("FMM2D", "FMM2DError"):
        from . import fmm

        return getattr(fmm, name)
    raise AttributeError(name)
