"""MI355X (gfx950) implementation of the Jacobian-free Newton-GMRES solver with
the FV-subgrid multigrid preconditioner for well-balanced DG (arXiv 2505.24504).

The compute path is the HIP library ``libjfmg.so`` behind the C-ABI declared in
``include/jfmg.h``; ``paper_2505_24504_amd.jfmg`` is its thin ctypes binding.
"""
