"""MI355X-native sparse-voxel rasterizer (SVRaster, arXiv 2412.04459).

Submodules:
  scenes  seeded synthetic scenes and cameras (numpy only)
  _abi    ctypes binding of include/svraster.h (libsvraster.so)
  render  device scene, rasterizer and torch.autograd.Function
  build   hipcc build of lib/libsvraster.so for gfx950
"""
__all__ = ["scenes", "render", "build"]
