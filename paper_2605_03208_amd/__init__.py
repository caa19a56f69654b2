"""MI355X-native snapshot and validation hot path for VA-faithful kernel capture.

Submodules:
  ``kc``        -- ctypes binding over the HIP C-ABI library ``libkc.so``
  ``build``     -- compiles the HIP sources for gfx950 into ``libkc.so``
  ``workloads`` -- seeded synthetic inputs (layouts, contents, perturbations)
  ``autotune``  -- launch-shape search and its cache
  ``serve``     -- continuous-batching validation request loop

Importing the package loads nothing; ``kc`` loads the library on first use
and raises if it is missing.
"""

__all__ = ["kc", "build", "workloads", "autotune", "serve"]
