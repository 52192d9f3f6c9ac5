"""MI355X-native triple Gaussian splatting (GS^3, Bi et al. 2024).

The hot path (projection, tile binning, shadow splatting, shading with the
two MLPs, camera splatting and their adjoints) runs in hand-written HIP
kernels for gfx950 behind the C-ABI library ``libgs3.so``. ``gs3`` is the thin
ctypes binding; ``synth`` draws the seeded synthetic inputs.

Importing the package loads nothing; ``paper_2410_11419_amd.gs3`` loads the
library and raises if it has not been built.
"""
__all__ = ["gs3", "synth"]
