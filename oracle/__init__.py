"""CPU oracle for the 3DGStream Stage-1 step: TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct reference implementations in float64, written
from the paper and sharing no code with the HIP library:

  raster.c / raster.py  3D-Gaussian projection, per-pixel alpha blending and
                        their adjoint (Sec. 3, Eq. 2-4; Sec. 4.1 transform)
  ntc.py                multi-resolution hash encoding + MLP of the Neural
                        Transformation Cache and its adjoint (Sec. 4.1, Eq. 5)
  loss.py               Stage-1 loss (1 - lambda) L1 + lambda D-SSIM (Eq. 6)
  optim.py              Adam and the warm-up loss (Eq. 7)

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
anything here.  The product path never does.
"""
