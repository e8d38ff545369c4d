"""MI355X-native double-distribution lattice Boltzmann solver for two-phase
flow in porous media (Chai, Liang, Du, Shi, arXiv:1808.07554).

  paper_1808_07554_amd.lbtp    ctypes binding of liblbtp (include/lbtp.h)
  paper_1808_07554_amd.inputs  seeded synthetic workloads
  paper_1808_07554_amd.build   hipcc build of liblbtp.so for gfx950

Importing the package loads neither torch nor the HIP library.
"""
__all__ = ["lbtp", "inputs", "build"]
