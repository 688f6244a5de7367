"""MI355X (gfx950) differentiable triangle-soup rasterizer with stochastic
opacity masking (DiffSoup, arXiv 2603.27151).

Submodules:
  workloads -- seeded synthetic inputs (no rasterizer arithmetic)
  _lib      -- ctypes binding of libdiffsoup.so (the C ABI in include/diffsoup.h)
  raster    -- torch-facing API and the autograd function
  serve     -- continuous-batching render server
  autotune  -- tile-size autotuner
The package import itself loads nothing, so that the input generators can be
used without a GPU.
"""
