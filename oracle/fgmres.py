"""Flexible GMRES, Alg. 1 (section 4.2), with restarts.

Stopping test (the paper leaves it open): after each Arnoldi step the least
squares problem min ||beta e_1 - H~ y||_2 is solved with a library routine
and the iteration stops when its residual is <= rtol * ||b~||_2.  At the end
of a cycle the true residual b~ - A~ phi is evaluated; if it is still above
rtol * ||b~|| the method restarts from the current phi (Alg. 1's non-zero
initial-guess branch).  A lucky breakdown (H_{j+1,j} <= 1e-14 ||w||) ends the
cycle with the columns built so far.
"""
import numpy as np


class FgmresResult:
    def __init__(self):
        self.x = None
        self.iterations = 0        # preconditioned Arnoldi steps, all cycles
        self.a_applies = 0         # applications of A~ (one transport sweep each)
        self.cycles = 0
        self.history = []          # LS residual estimate / ||b|| after each step
        self.true_relres = None
        self.converged = False
        self.first_cycle = None    # dict(V, Z, H, beta, x0, j) of cycle 1


def fgmres(A_apply, b, precond, m=30, rtol=1e-8, x0=None, max_cycles=50, keep_first=False):
    """Solve A x = b.  precond(j, v) returns z_j = M_j^{-1} v with j the 1-based
    iteration index inside the current cycle."""
    res = FgmresResult()
    nb = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    if nb == 0.0:
        res.x = x
        res.true_relres = 0.0
        res.converged = True
        return res
    r_next = None
    for cycle in range(max_cycles):
        res.cycles += 1
        if r_next is not None:
            r0 = r_next                    # true residual of the previous cycle
        elif np.linalg.norm(x) == 0.0:
            r0 = b.copy()
        else:
            r0 = b - A_apply(x)
            res.a_applies += 1
        beta = np.linalg.norm(r0)
        if beta <= rtol * nb:
            res.converged = True
            break
        V = [r0 / beta]
        Z = []
        H = np.zeros((m + 1, m))
        j_done = 0
        for j in range(1, m + 1):
            z = precond(j, V[j - 1])
            Z.append(z)
            w = A_apply(z)
            res.a_applies += 1
            wn0 = np.linalg.norm(w)
            for i in range(1, j + 1):  # modified Gram-Schmidt
                H[i - 1, j - 1] = w @ V[i - 1]
                w = w - H[i - 1, j - 1] * V[i - 1]
            H[j, j - 1] = np.linalg.norm(w)
            res.iterations += 1
            j_done = j
            e1 = np.zeros(j + 1)
            e1[0] = beta
            y, *_ = np.linalg.lstsq(H[:j + 1, :j], e1, rcond=None)
            est = np.linalg.norm(e1 - H[:j + 1, :j] @ y)
            res.history.append(est / nb)
            if H[j, j - 1] <= 1e-14 * wn0:
                break
            V.append(w / H[j, j - 1])
            if est <= rtol * nb:
                break
        e1 = np.zeros(j_done + 1)
        e1[0] = beta
        y, *_ = np.linalg.lstsq(H[:j_done + 1, :j_done], e1, rcond=None)
        if cycle == 0 and keep_first:
            res.first_cycle = dict(V=[v.copy() for v in V], Z=[z.copy() for z in Z],
                                   H=H[:j_done + 1, :j_done].copy(), beta=beta,
                                   x0=x.copy(), j=j_done)
        x = x + np.stack(Z, 1) @ y
        r_next = b - A_apply(x)
        res.a_applies += 1
        res.true_relres = np.linalg.norm(r_next) / nb
        if res.true_relres <= rtol:
            res.converged = True
            break
    res.x = x
    return res
