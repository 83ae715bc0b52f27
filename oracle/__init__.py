"""FP64 CPU oracle of NL-RMM-GKS on the angle-parameterised parallel-beam projector.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call or link anything in this
package.  The product path (the HIP library and its Python binding) never
does, and this package imports nothing from the product.

Contents
  strip_oracle.c  FP64 projector, backprojector, angle derivative (C, OpenMP)
  projector.py    ctypes wrapper and build step for strip_oracle.c
  method.py       FP64 NumPy implementation of the method: regulariser, MM-GKS
                  enlarge/compress, discrepancy principle, Gauss-Newton (AltMin),
                  variable projection, streaming and dynamic drivers.
  optical_flow.py FP64 optical-flow regulariser: velocity estimation per frame pair,
                  bilinear warps, the motion rows of the dynamic operator Theta.
  pat.py          FP64 photoacoustic circular-means operator with a global radial shift,
                  its transpose and its derivative in the shift.
"""
