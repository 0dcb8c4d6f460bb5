"""pk: an MI355X-native spatially-binned software rasterizer.

The sort-middle tiled renderer of Piko (Sec. 4.4): vertex transform and
triangle setup, AssignBin of triangles to screen tiles, and a per-tile Process
stage (fixed-point edge-function coverage, 64-bit depth test, Gouraud /
textured / deferred shading), as hand-written HIP kernels for gfx950 behind a
C ABI (``include/pk.h``).  The binding loads ``libpk.so`` on first use.
"""
