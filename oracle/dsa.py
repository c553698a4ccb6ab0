"""Diffusion synthetic acceleration (section 3.1 equation of the low-order
correction, section 3.2 SA preconditioner M^{-1} = I + C^{-1} Sigma_s, App. A).

App. A derives the fully consistent (FC) DSA in slab geometry: insert the P1
ansatz delta psi_j = delta phi + 3 Omega_j . delta J into the upwind DG
correction equation and take its zeroth and first discrete angular moments.
In X-Y geometry the paper does not print the equations; the reading used
here takes the same two steps literally with the 2D ordinates:

  zeroth moment (weight 1):
    [E + Sigma_t - Sigma_s] dphi + 3 sum_f [E_f + m_f Sigma_t] dJ_f = Sigma_s v
  first moment (weight Omega_d, d = x, y):
    [E_d + m_d (Sigma_t - Sigma_s)] dphi + 3 sum_f [E_df + a_df Sigma_t] dJ_f
        = m_d Sigma_s v
  with E = sum_j w_j D_j, E_f = sum_j w_j Omega_f D_j,
       E_df = sum_j w_j Omega_d Omega_f D_j, m_f = sum_j w_j Omega_f,
       a_df = sum_j w_j Omega_d Omega_f.

In 1D with a symmetric rule these are exactly App. A's two moment equations.
`fc_system_appA` builds the same FC system from App. A's D_C / D_J form
(D_j = sum_e Omega_e (D_C^e - sgn(Omega_e)/2 D_J^e)); the partially consistent
(PC) variant drops the D_J terms from the first-moment rows (App. A, last
paragraph).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import dg


def _axes(P):
    return [0] if P.mesh.dim == 1 else [0, 1]


def _om(P, e):
    return P.ox if e == 0 else P.oy


def fc_system(P):
    """FC-DSA matrix from the angular moments of the assembled upwind D_j."""
    ax = _axes(P)
    n = P.ndof
    Sa = P.St - P.Ss
    E = sum(P.w[j] * P.D(j) for j in range(P.nord))
    Ef = {f: sum(P.w[j] * _om(P, f)[j] * P.D(j) for j in range(P.nord)) for f in ax}
    Edf = {(d, f): sum(P.w[j] * _om(P, d)[j] * _om(P, f)[j] * P.D(j) for j in range(P.nord))
           for d in ax for f in ax}
    m = {f: float(np.sum(P.w * _om(P, f))) for f in ax}
    a = {(d, f): float(np.sum(P.w * _om(P, d) * _om(P, f))) for d in ax for f in ax}
    rows = [[E + Sa] + [3.0 * (Ef[f] + m[f] * P.St) for f in ax]]
    for d in ax:
        rows.append([Ef[d] + m[d] * Sa] + [3.0 * (Edf[(d, f)] + a[(d, f)] * P.St) for f in ax])
    return sp.bmat(rows, format="csc"), m


def _moments(P):
    ax = _axes(P)
    w = P.w
    O = {e: _om(P, e) for e in ax}
    mom = dict(
        m={f: np.sum(w * O[f]) for f in ax},
        a={(d, f): np.sum(w * O[d] * O[f]) for d in ax for f in ax},
        beta={e: 0.5 * np.sum(w * np.abs(O[e])) for e in ax},
        b={(e, f): np.sum(w * np.abs(O[e]) * O[f]) for e in ax for f in ax},
        t={(d, e, f): np.sum(w * O[d] * O[e] * O[f]) for d in ax for e in ax for f in ax},
        c={(d, e, f): np.sum(w * O[d] * np.abs(O[e]) * O[f]) for d in ax for e in ax for f in ax},
        bm={(d, e): np.sum(w * O[d] * np.abs(O[e])) for d in ax for e in ax},
    )
    return mom


def fc_system_appA(P, partially_consistent=False):
    """Same moment system written with App. A's central-flux and jump
    operators (tensor extension per axis).  With partially_consistent=True the
    D_J terms of the first-moment rows are dropped (PC-DSA)."""
    ax = _axes(P)
    mom = _moments(P)
    DC, DJ = {}, {}
    for e in ax:
        DC[e], DJ[e] = dg.central_and_jump(P.mesh, e)
    Sa = P.St - P.Ss
    Z = sp.csc_matrix((P.ndof, P.ndof))
    # zeroth moment
    E = sum(mom["m"][e] * DC[e] - mom["beta"][e] * DJ[e] for e in ax)
    row0 = [E + Sa]
    for f in ax:
        Ef = sum(mom["a"][(e, f)] * DC[e] - 0.5 * mom["b"][(e, f)] * DJ[e] for e in ax)
        row0.append(3.0 * (Ef + mom["m"][f] * P.St))
    rows = [row0]
    kj = 0.0 if partially_consistent else 1.0
    for d in ax:
        Ed = sum(mom["a"][(d, e)] * DC[e] - kj * 0.5 * mom["bm"][(d, e)] * DJ[e] for e in ax)
        row = [Ed + mom["m"][d] * Sa]
        for f in ax:
            Edf = sum(mom["t"][(d, e, f)] * DC[e] - kj * 0.5 * mom["c"][(d, e, f)] * DJ[e]
                      for e in ax)
            row.append(3.0 * (Edf + mom["a"][(d, f)] * P.St))
        rows.append(row)
    return sp.bmat(rows, format="csc"), mom["m"]


class DSA:
    """M_DSA^{-1} v = v + dphi, dphi from the FC (or PC) moment system with
    right-hand side Sigma_s v (zeroth row) and m_d Sigma_s v (first-moment rows)."""

    def __init__(self, P, variant="fc"):
        self.P = P
        if variant == "fc":
            K, m = fc_system(P)
        elif variant == "fc_appA":
            K, m = fc_system_appA(P)
        elif variant == "pc":
            K, m = fc_system_appA(P, partially_consistent=True)
        else:
            raise ValueError(variant)
        self.K = K
        self.m = m
        self.lu = spla.splu(K)

    def correction(self, v):
        P = self.P
        s = P.Ss @ v
        rhs = np.concatenate([s] + [self.m[d] * s for d in _axes(P)])
        return self.lu.solve(rhs)[:P.ndof]

    def apply(self, v):
        return v + self.correction(v)
