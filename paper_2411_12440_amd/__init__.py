"""lsplat: tile-based differentiable rasterizer of 3D Linear Splatting
(arXiv 2411.12440) for AMD MI355X.

Modules:
  build       compile liblsplat.so (hipcc, gfx950)
  binding     ctypes binding of the C ABI in include/lsplat.h
  rasterizer  torch-facing wrapper (workspace, stages, autograd.Function)
  scenes      seeded synthetic scenes and cameras (inputs only)
The HIP library is loaded when `binding` (or `rasterizer`) is imported; that
import fails loudly if the library has not been built.
"""
