"""CPU oracle for the voxel-anchored Gaussian rasterizer (arXiv 2403.11247).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product path never imports this
package, and this package never imports the product's kernels or binding.

Contents:
  raster.c / raster.py  FP64 tiled renderer + FP32 key path + FP64 adjoint (C, via ctypes)
  brute.py              per-pixel brute force over every Gaussian (numpy FP64)
                        and the same formula under torch FP64 autograd
  decode.py             anchor decode, mask and codebook gather (numpy FP64) and its adjoint
"""
