"""MI355X (gfx950) ghost-cell multigrid Poisson solver on level-set domains with mixed
Dirichlet/Neumann boundary conditions (Coco and Russo, arXiv 1111.0983).

The solver lives in the HIP shared library ``libghostmg.so`` behind the C ABI of
``include/ghostmg.h``; :mod:`paper_1111_0983_amd.ghostmg` is its ctypes binding.
"""
