"""FP64 CPU oracle for the multigrid-ISDF exchange path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the package smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the GPU
library (it never loads it); the only common inputs come from the seeded
generators in ``workloads``.

It is a plain, slow, step-by-step NumPy/SciPy transcription of the method
of Smyser, White and Sharma, "Use of multigrids to reduce the cost of
performing interpolative separable density fitting" (arXiv 2404.09373):

  plan.py      levels, periodic images, atom-centred windows and the
               local (L) / global (G) / non-local (N) function sets
               (section "Computational details", Eqs. rcut and Ggrid,
               Eq. "mg product density")
  basis.py     periodic Gaussian basis values on each level grid
  isdf.py      pair-density Gram M(R,R') (Eq. M(R,R)), greedy pivoted
               Cholesky point selection, least-squares fitting functions
               (Eq. lsqr)
  coulomb.py   Coulomb metric (xi|xi') by FFT Poisson solves (Eq. (xi|xi'))
  exchange.py  four-term multigrid THC exchange matrix (Eq. ints)
  brute.py     exact exchange from every pair density, no ISDF, computed
               two ways (pair tensor and occupied-orbital Poisson solves)
  universal.py the universal grid with every point as a fitting function:
               diffuse-diffuse exchange from occupied pair densities by FFT
               (occ-RI), (R_U|R_U') never stored
  mlp.py       FP64 forward/backward of the point-scoring network
  pipeline.py  the whole fit + exchange with per-stage timers

Readings taken where the paper is silent or garbled are listed in the
docstrings of the functions that take them.
"""
