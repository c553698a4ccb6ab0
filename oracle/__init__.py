"""Plain FP64 CPU oracle for the steady one-group RTE solved by FGMRES with the
ROMSAD preconditioner (arXiv 2410.08735).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke entry point and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the HIP library and never calls it.

Every function follows the paper step by step with no blocking, fusion or
reordering beyond what the paper states; sparse direct solves and dense least
squares stand in where the paper only fixes the mathematical result.

Modules
  quadrature   S_N rules (section 2.1)
  dg           upwind DG operators by numerical quadrature (sections 2.2-2.3, App. A)
  transport    sweeps, T, b~, A~ and the fully coupled system (sections 2.3, 3.1-3.2)
  dsa          fully / partially consistent DSA (App. A, extended to X-Y)
  fgmres       Alg. 1 (flexible GMRES) with restarts
  rom          ROMSAD preconditioner, xi recurrence, snapshots, MGS with
               truncation, greedy ROM construction (section 4, App. B)
  mlp          the learned flexible preconditioner's network (no paper passage:
               a plain MLP with GELU, forward and backward by hand)
"""
