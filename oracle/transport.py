"""Discrete ordinates + upwind DG transport (sections 2.3, 3.1, 3.2).

  sweep          psi_j = (D_j + Sigma_t)^{-1} q_j for every ordinate, by a
                 sparse direct solve (the transport sweep's exact result; the
                 paper's sweep is one block Gauss-Seidel pass in upwind order,
                 section 3.1)
  T_apply        T q = sum_j w_j (D_j + Sigma_t)^{-1} q    (memory-efficient SI)
  b_tilde        b~ = sum_j w_j (D_j + Sigma_t)^{-1} G~_j   (G~_j = G + g_j^(bc))
  A_tilde_apply  (I - T Sigma_s) phi                         (memory-efficient system)
  full_system    the fully coupled psi-space matrix A and b (equation of A psi = b)
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import dg
from .quadrature import make_rule


class Problem:
    """One parameter instance: mesh, quadrature, cross sections, source."""

    def __init__(self, spec):
        self.spec = spec
        self.mesh = dg.Mesh.of(spec)
        self.ox, self.oy, self.w = make_rule(spec["quad"])
        self.nord = len(self.w)
        if "sigma_fields" in spec:
            # cross sections that vary inside the cells (section 5.3): sigma_t(x) =
            # sum_f theta_t,f s_f(x), sigma_s(x) = sum_f theta_s,f s_f(x) with the
            # shape functions s_f and coefficients sigma_t / sigma_s of the spec
            self.field_mats = [dg.field_matrix(self.mesh, f) for f in spec["sigma_fields"]]
            tt = np.asarray(spec["sigma_t"], dtype=np.float64)
            ts = np.asarray(spec["sigma_s"], dtype=np.float64)
            self.St = sum(t * M for t, M in zip(tt, self.field_mats))
            self.Ss = sum(t * M for t, M in zip(ts, self.field_mats))
        else:
            region = np.asarray(spec["region"])
            self.sig_t_cell = np.asarray(spec["sigma_t"], dtype=np.float64)[region]
            self.sig_s_cell = np.asarray(spec["sigma_s"], dtype=np.float64)[region]
            self.St = dg.sigma_matrix(self.mesh, self.sig_t_cell)
            self.Ss = dg.sigma_matrix(self.mesh, self.sig_s_cell)
        self.G = np.asarray(spec["source"], dtype=np.float64)
        self.g = spec.get("inflow", 0.0)
        self._D = [None] * self.nord
        self._lu = [None] * self.nord

    @property
    def ndof(self):
        return self.mesh.ndof

    def D(self, j):
        if self._D[j] is None:
            self._D[j] = dg.advection(self.mesh, self.ox[j], self.oy[j]).tocsc()
        return self._D[j]

    def lu(self, j):
        if self._lu[j] is None:
            self._lu[j] = spla.splu((self.D(j) + self.St).tocsc())
        return self._lu[j]

    def gbc(self, j, g=None):
        g = self.g if g is None else g
        if isinstance(g, dict):
            if not any(float(v) for v in g.values()):
                return np.zeros(self.ndof)
        elif not callable(g) and float(g) == 0.0:
            return np.zeros(self.ndof)
        return dg.inflow_vector(self.mesh, self.ox[j], self.oy[j], g)


def sweep(P, q, store_psi=False):
    """psi_j = (D_j + Sigma_t)^{-1} q_j; q is isotropic [ndof] or per ordinate
    [nord, ndof].  Returns (phi = sum_j w_j psi_j, psi or None)."""
    q = np.asarray(q, dtype=np.float64)
    phi = np.zeros(P.ndof)
    psi = np.empty((P.nord, P.ndof)) if store_psi else None
    for j in range(P.nord):
        qj = q[j] if q.ndim == 2 else q
        pj = P.lu(j).solve(qj)
        phi += P.w[j] * pj
        if store_psi:
            psi[j] = pj
    return phi, psi


def T_apply(P, q):
    return sweep(P, q)[0]


def b_tilde(P, g=None):
    """b~ = sum_j w_j (D_j + Sigma_t)^{-1} (G + g_j^(bc))."""
    q = np.stack([P.G + P.gbc(j, g) for j in range(P.nord)])
    return sweep(P, q)[0]


def A_tilde_apply(P, phi):
    """(I - T Sigma_s) phi."""
    return phi - T_apply(P, P.Ss @ phi)


def scalar_flux(P, psi):
    """phi = Q psi = sum_j w_j psi_j (numerical integration in angle)."""
    return np.tensordot(P.w, psi, axes=(0, 0))


def full_system(P, g=None):
    """Fully coupled psi-space system A psi = b: block (j, k) is
    delta_jk (D_j + Sigma_t) - w_k Sigma_s, right-hand side G~_j."""
    n = P.nord
    rows = []
    for j in range(n):
        row = []
        for k in range(n):
            blk = -P.w[k] * P.Ss
            if j == k:
                blk = blk + P.D(j) + P.St
            row.append(blk)
        rows.append(row)
    A = sp.bmat(rows, format="csc")
    b = np.concatenate([P.G + P.gbc(j, g) for j in range(n)])
    return A, b


def dense_A_tilde(P):
    """Columns of (I - T Sigma_s) applied to unit vectors (tiny grids only)."""
    n = P.ndof
    return np.stack([A_tilde_apply(P, e) for e in np.eye(n)], 1)
