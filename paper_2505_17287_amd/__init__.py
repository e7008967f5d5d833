"""MI355X-native ghost-cell immersed-boundary projection (classification, image-point
stencils, multigrid pressure Poisson solve, velocity correction).

The compiled HIP library is loaded lazily by :mod:`paper_2505_17287_amd.ibm` on first use,
so importing the input generators does not touch the GPU path.
"""
__all__ = ["inputs", "ibm"]
