"""FP64 CPU oracle for the incompressible D3Q14 / D3Q18 MRT lattice Boltzmann
step (arXiv 1503.03337) -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It shares no code with the GPU library
and never imports it; the GPU library never imports this.

Contents:
  lbm_oracle.c   the lattice step, written plainly from the paper (FP64)
  runner.py      ctypes loader for it, plus numpy conveniences
  analytic.py    the paper's analytic duct solutions and its error norm
  build.py       compiles lbm_oracle.c with gcc
"""
