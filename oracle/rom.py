"""ROMSAD: the ROM-enhanced synthetic acceleration preconditioner and its
greedy offline construction (section 4, App. B).

A reduced basis U_r (N_Omega N_DOF x r, orthonormal) is held as an array
U[r, nord, ndof]; U_{r,j} = U[:, j, :].T.
  W_1 = sum_j U_{r,j},  W_w = sum_j w_j U_{r,j}                (section 4.3)
  M_ROM^{-1} v = v + W_w (U_r^T A U_r)^{-1} W_1^T Sigma_s v      (eq. of M_ROM)
  M_j = M_ROM for 1 <= j <= window, M_DSA otherwise               (ROMSAD switch)
"""
import numpy as np

from . import transport as tr


def W1(U):
    return U.sum(axis=1)                      # [r, ndof]


def Ww(P, U):
    return np.tensordot(P.w, U, axes=(0, 1))  # [r, ndof]


def A_psi_apply(P, psi):
    """Fully coupled operator of section 2.3 on psi[nord, ndof]:
    (A psi)_j = (D_j + Sigma_t) psi_j - Sigma_s sum_k w_k psi_k."""
    phi = tr.scalar_flux(P, psi)
    s = P.Ss @ phi
    return np.stack([P.D(j) @ psi[j] + P.St @ psi[j] - s for j in range(P.nord)])


def reduced_operator(P, U):
    """U_r^T A U_r formed with explicit products by A (no affine shortcut)."""
    r = U.shape[0]
    AU = np.stack([A_psi_apply(P, U[k]) for k in range(r)])
    return np.einsum("ijn,kjn->ik", U, AU)


def rom_correction(P, U, v, Ar=None):
    """delta phi = W_w (U^T A U)^{-1} W_1^T Sigma_s v  (eq. of C_ROM)."""
    if U.shape[0] == 0:
        return np.zeros_like(v)
    Ar = reduced_operator(P, U) if Ar is None else Ar
    g = W1(U) @ (P.Ss @ v)
    c = np.linalg.solve(Ar, g)
    return Ww(P, U).T @ c


class Romsad:
    """The nonlinear ROMSAD preconditioner for one parameter instance."""

    def __init__(self, P, U, dsa, window):
        self.P, self.U, self.dsa, self.window = P, U, dsa, window
        self.Ar = reduced_operator(P, U) if U.shape[0] else None

    def rom_apply(self, v):
        return v + rom_correction(self.P, self.U, v, self.Ar)

    def __call__(self, j, v):
        if j <= self.window and self.U.shape[0] > 0:
            return self.rom_apply(v)
        return self.dsa.apply(v)


def affine_terms(P, U, n_regions):
    """Affine pieces of U^T A(mu) U (eq. of the affine assumption):
    U^T A U = A_D + sum_R a_{t,R} G_R - sum_R a_{s,R} S_R,
    A_D = sum_j U_j^T D_j U_j, G_R = sum_j U_j^T M_R U_j, S_R = W_1^T M_R W_w.
    Piecewise-constant cross sections: a = sigma_{t,R}, sigma_{s,R} and M_R the
    mass matrix restricted to region R.  Cross sections varying inside the
    cells (section 5.3): a = the coefficients of the shape functions s_R and
    M_R the mass matrix weighted by s_R."""
    from . import dg
    r = U.shape[0]
    AD = np.zeros((r, r))
    for j in range(P.nord):
        AD += U[:, j, :] @ (P.D(j) @ U[:, j, :].T)
    Gs, Ss = [], []
    w1, ww = W1(U), Ww(P, U)
    if "sigma_fields" in P.spec:
        mats = P.field_mats
    else:
        region = np.asarray(P.spec["region"])
        mats = [dg.sigma_matrix(P.mesh, (region == R).astype(np.float64)) for R in range(n_regions)]
    for MR in mats:
        Gs.append(sum(U[:, j, :] @ (MR @ U[:, j, :].T) for j in range(P.nord)))
        Ss.append(w1 @ (MR @ ww.T))
    return AD, np.array(Gs), np.array(Ss)


# ---- offline: snapshots (section 4.4.1) -------------------------------------------

def xi_recurrence(first_cycle, phi, window):
    """xi^(1) = (phi - phi^(0)) / ||r^(0)||;
    xi^(l) = (z^(l-1) - sum_{i<l} H_{i,l-1} xi^(i)) / H_{l,l-1}, l >= 2
    (equations of the FGMRES corrections), for l = 1..window (fewer if the
    first cycle ended earlier)."""
    fc = first_cycle
    H, Z, beta = fc["H"], fc["Z"], fc["beta"]
    xis = [(phi - fc["x0"]) / beta]
    for l in range(2, min(window, fc["j"] + 1) + 1):
        acc = Z[l - 2].copy()
        for i in range(1, l):
            acc -= H[i - 1, l - 2] * xis[i - 1]
        xis.append(acc / H[l - 1, l - 2])
    return xis


def snapshot_corrections(P, xis):
    """delta psi_j^(l) = (D_j + Sigma_t)^{-1} Sigma_s xi^(l) (equation of the
    psi correction under FGMRES): one psi-storing sweep per xi."""
    return [tr.sweep(P, P.Ss @ xi, store_psi=True)[1] for xi in xis]


def mgs_truncate(U, psi, eps_qr=1e-13):
    """App. B: orthogonalise psi against the columns of U (modified
    Gram-Schmidt) and append it, normalised, if the remainder exceeds eps_qr."""
    u = psi.copy()
    for i in range(U.shape[0]):
        R = np.vdot(U[i], u)
        u = u - R * U[i]
    nu = np.linalg.norm(u)
    if nu > eps_qr:
        return np.concatenate([U, (u / nu)[None]], 0), True
    return U, False


# ---- offline: greedy (section 4.4.2) -------------------------------------------

def residual_indicator(P, U, eta0, Ar=None):
    """R_mu = max_j ||(D_j + Sigma_t) dpsi_j - Sigma_s dphi - eta0||_2 with
    U^T A U c = W_1^T eta0, dpsi = U c, dphi = W_w c  (eq. of the greedy ROM
    solve and eq. of the residual indicator)."""
    Ar = reduced_operator(P, U) if Ar is None else Ar
    c = np.linalg.solve(Ar, W1(U) @ eta0)
    dpsi = np.tensordot(c, U, axes=(0, 0))
    dphi = Ww(P, U).T @ c
    s = P.Ss @ dphi
    return max(np.linalg.norm(P.D(j) @ dpsi[j] + P.St @ dpsi[j] - s - eta0)
               for j in range(P.nord))


class GreedyReport:
    def __init__(self):
        self.sampled = []
        self.max_residual = []
        self.r_history = []
        self.truncated = 0


def greedy(train_specs, window=2, mu1_index=0, eps_rom=1e-9, n_giter=16, eps_qr=1e-13,
           rtol_hf=1e-11, m_hf=60):
    """Greedy ROM construction of section 4.4.2 with the FGMRES-DSA
    high-fidelity solver (zero initial guess)."""
    from . import dsa as dsa_mod
    from . import fgmres as fg
    probs = [tr.Problem(s) for s in train_specs]
    # step 1: right-hand sides and eta0 for every training parameter
    bt = [tr.b_tilde(P) for P in probs]
    eta0 = [P.Ss @ b for P, b in zip(probs, bt)]
    nord, ndof = probs[0].nord, probs[0].ndof
    U = np.zeros((0, nord, ndof))
    rep = GreedyReport()
    sampled = [mu1_index]
    k = 1
    while True:
        P = probs[sampled[-1]]
        # step 2(a): high-fidelity solve and xi recurrence
        D = dsa_mod.DSA(P)
        res = fg.fgmres(lambda x: tr.A_tilde_apply(P, x), bt[sampled[-1]],
                        lambda j, v: D.apply(v), m=m_hf, rtol=rtol_hf, keep_first=True)
        xis = xi_recurrence(res.first_cycle, res.x, window)
        # step 2(b): angular flux corrections
        snaps = snapshot_corrections(P, xis)
        # step 2(c): MGS with truncation
        for s in snaps:
            U, added = mgs_truncate(U, s, eps_qr)
            rep.truncated += 0 if added else 1
        rep.r_history.append(U.shape[0])
        if k == n_giter:
            break
        # step 3: greedy sampling over unsampled training parameters
        best, best_i = -1.0, None
        for i, Pi in enumerate(probs):
            if i in sampled:
                continue
            R = residual_indicator(Pi, U, eta0[i])
            if R > best:          # strict: ties keep the lowest index
                best, best_i = R, i
        rep.max_residual.append(best)
        if best_i is None or best < eps_rom:
            break
        sampled.append(best_i)
        k += 1
    rep.sampled = sampled
    return U, rep


# ---- training rows of the learned correction (no paper passage) -----------------

def learned_correction_rows(P, U, first_cycle, phi, window, mu_feat):
    """Rows (x, t) for l < window: x = [mu_feat, g / ||g||], g = W_1^T Sigma_s v^(l);
    t = c / ||g|| with c the least-squares coefficients of xi^(l) - v^(l) (the ideal
    scalar flux correction, from the density relation) in span(W_w)."""
    xis = xi_recurrence(first_cycle, phi, window)
    w1, ww = W1(U), Ww(P, U)
    X, T = [], []
    for l, xi in enumerate(xis):
        v = first_cycle["V"][l]
        g = w1 @ (P.Ss @ v)
        c, *_ = np.linalg.lstsq(ww.T, xi - v, rcond=None)
        nrm = np.linalg.norm(g)
        X.append(np.concatenate([mu_feat, g / nrm]))
        T.append(c / nrm)
    return np.array(X), np.array(T)
