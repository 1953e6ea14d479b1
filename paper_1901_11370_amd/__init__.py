"""MI355X-native geometric multigrid for quadtree/octree block grids.

The GPU library (HIP kernels for gfx950 behind a C ABI, ``include/mg.h``) is loaded on
first use by :mod:`paper_1901_11370_amd.mg`; importing this package does not load it.
"""
