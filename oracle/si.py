"""Source iteration with synthetic acceleration (section 3): the left-
preconditioned Richardson iteration on the memory-efficient system,

    r^(l) = phi^(l,*) - phi^(l-1) = b~ - A~ phi^(l-1)     (one transport sweep)
    phi^(l) = phi^(l-1) + M_l^{-1} r^(l),

with M_l^{-1} = I + C^{-1} Sigma_s the SA preconditioner of iteration l (the
ROMSAD switch applies M_ROM for l <= window, M_DSA after it).  The iteration
stops when ||r^(l)||_2 <= rtol ||b~||_2 (the SI criterion stated with the
pin-cell comparison of section 5.2); phi^(l-1) is then returned.

Test infrastructure only (see the package docstring).
"""
import numpy as np


class SiResult:
    def __init__(self):
        self.x = None
        self.iterations = 0      # preconditioner applications
        self.residuals = []      # ||r^(l)|| / ||b~||, l = 1, 2, ...
        self.converged = False


def si(A_apply, b, precond, rtol=1e-8, max_iter=100):
    """precond(l, r) returns M_l^{-1} r with l the 1-based iteration index."""
    res = SiResult()
    x = np.zeros_like(b)
    bn = np.linalg.norm(b)
    if bn == 0.0:
        res.x, res.converged = x, True
        return res
    for l in range(1, max_iter + 1):
        r = b - A_apply(x)
        rel = np.linalg.norm(r) / bn
        res.residuals.append(rel)
        if rel <= rtol:
            res.converged = True
            break
        x = x + precond(l, r)
        res.iterations += 1
    res.x = x
    return res
