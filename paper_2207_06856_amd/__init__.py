"""MI355X-native low-precision Gaussian-process solves.

The compute lives in ``libgpmi.so`` (HIP, gfx950) behind the C ABI declared in
``include/gpmi.h``; ``paper_2207_06856_amd.gpmi`` is its Python binding and
``paper_2207_06856_amd.synth`` draws the seeded synthetic workloads.  The
library is loaded on first use, so importing the package needs no GPU.
"""

__all__ = ["gpmi", "synth", "build"]
