"""MI355X (gfx950) implementation of the incompressible D3Q14 / D3Q18
multiple-relaxation-time lattice Boltzmann step of arXiv 1503.03337.

  lbm       Python binding of liblbm.so (include/lbm.h)
  inputs    seeded synthetic inputs (no method arithmetic)
  params    relaxation vectors and flow set-ups in lattice units
  build     hipcc build of liblbm.so
"""
