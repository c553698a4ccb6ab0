"""Pins of the oracle's FGMRES, DSA, ROMSAD, greedy and MLP against library
routines, exactness properties and identities fixed by the paper."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import dsa, mlp, rom
from oracle import fgmres as fg
from oracle import transport as tr
from synth import tiny_1d, tiny_2d


def _At(P):
    return lambda x: tr.A_tilde_apply(P, x)


# ---------------------------------------------------------------- FGMRES (Alg. 1)
def test_fgmres_identity_matches_library_gmres():
    """Unpreconditioned: residual history equals scipy's GMRES on the dense A~."""
    P = tr.Problem(tiny_2d(seed=1, nx=3, ny=3, quad=("cl", 4, 2, False)))
    At = tr.dense_A_tilde(P)
    b = tr.b_tilde(P)
    res = fg.fgmres(_At(P), b, lambda j, v: v, m=36, rtol=1e-12)
    hist = []
    spla.gmres(At, b, rtol=1e-12, restart=36, maxiter=1,
               callback=lambda r: hist.append(r), callback_type="pr_norm")
    n = min(len(hist), len(res.history))
    assert n >= 5
    np.testing.assert_allclose(res.history[:n], hist[:n], rtol=1e-5, atol=1e-11)
    np.testing.assert_allclose(At @ res.x, b, rtol=0, atol=1e-11 * np.linalg.norm(b))


def test_fgmres_linear_preconditioner_is_right_gmres():
    """With M_j = M fixed, FGMRES = right-preconditioned GMRES (section 4.2)."""
    P = tr.Problem(tiny_2d(seed=2, nx=3, ny=3, quad=("cl", 4, 2, False)))
    At = tr.dense_A_tilde(P)
    b = tr.b_tilde(P)
    Minv = np.eye(P.ndof) + 0.3 * np.random.default_rng(3).standard_normal((P.ndof, P.ndof)) / P.ndof
    res = fg.fgmres(_At(P), b, lambda j, v: Minv @ v, m=36, rtol=1e-12)
    hist = []
    spla.gmres(At @ Minv, b, rtol=1e-12, restart=36, maxiter=1,
               callback=lambda r: hist.append(r), callback_type="pr_norm")
    n = min(len(hist), len(res.history))
    np.testing.assert_allclose(res.history[:n], hist[:n], rtol=1e-5, atol=1e-11)


def test_flexible_arnoldi_relation_and_sweep_count():
    """A~ Z_j = V_{j+1} H~_j with orthonormal V; zero initial guess costs
    1 + iterations sweeps (b~ plus one per step), plus the true-residual check."""
    P = tr.Problem(tiny_2d(seed=4, nx=4, ny=3, quad=("cl", 4, 2, True)))
    b = tr.b_tilde(P)
    rng = np.random.default_rng(5)
    pc = lambda j, v: v + 0.1 * j * np.tanh(v) + 0.01 * rng.standard_normal(v.shape)  # nonlinear
    res = fg.fgmres(_At(P), b, pc, m=5, rtol=1e-30, max_cycles=1, keep_first=True)
    fc = res.first_cycle
    V = np.stack(fc["V"], 1)
    Z = np.stack(fc["Z"], 1)
    AZ = np.stack([tr.A_tilde_apply(P, z) for z in fc["Z"]], 1)
    assert np.abs(V.T @ V - np.eye(V.shape[1])).max() < 1e-9   # MGS, residual ~1e-6
    np.testing.assert_allclose(AZ, V @ fc["H"], atol=1e-12 * np.abs(AZ).max())
    assert res.a_applies == res.iterations + 1  # steps + final true residual
    assert all(np.diff(res.history) <= 1e-15)


def test_fgmres_restarts_match_library_restarted_gmres():
    """Restart branch: GMRES(4) for 4 cycles from the true residual of each
    cycle's end (Alg. 1 with a non-zero initial guess) gives scipy's restarted
    GMRES iterate and its per-step residual history across the restarts."""
    P = tr.Problem(tiny_2d(seed=7, nx=3, ny=3, quad=("cl", 4, 2, False)))
    At = tr.dense_A_tilde(P)
    b = tr.b_tilde(P)
    res = fg.fgmres(_At(P), b, lambda j, v: v, m=4, rtol=1e-15, max_cycles=4)
    hist = []
    x, _ = spla.gmres(At, b, rtol=1e-15, atol=0.0, restart=4, maxiter=4,
                      callback=lambda r: hist.append(r), callback_type="pr_norm")
    assert res.cycles == 4 and res.iterations == 16 and len(hist) == 16
    np.testing.assert_allclose(res.history, hist, rtol=1e-4, atol=1e-14)
    assert np.linalg.norm(res.x - x) <= 1e-12 * np.linalg.norm(x)
    # every restart continues from the previous cycle's iterate: the history
    # falls through each cycle boundary instead of starting over
    assert res.history[4] < res.history[3] and res.history[8] < res.history[7]


def test_fgmres_lucky_breakdown_pure_absorber():
    """Breakdown branch: without scattering A~ = I, so the first Arnoldi step
    gives H_21 = 0 and the cycle ends with one column and phi = b~."""
    spec = tiny_2d(seed=3, nx=3, ny=3, quad=("cl", 4, 2, True))
    spec = dict(spec, sigma_s=np.zeros_like(spec["sigma_s"]))
    P = tr.Problem(spec)
    b = tr.b_tilde(P)
    res = fg.fgmres(_At(P), b, lambda j, v: v, m=10, rtol=1e-30, max_cycles=1, keep_first=True)
    assert res.iterations == 1 and res.first_cycle["j"] == 1
    assert abs(res.first_cycle["H"][1, 0]) <= 1e-14 * abs(res.first_cycle["H"][0, 0])
    np.testing.assert_allclose(res.x, b, rtol=0, atol=1e-15 * np.abs(b).max())
    assert res.true_relres <= 1e-15


def test_fgmres_breakdown_on_an_invariant_subspace():
    """b in a two-dimensional invariant subspace of A: the Krylov space stops
    growing at step 2, the breakdown test ends the cycle there and the
    two-column least-squares solve is the exact solution."""
    n = 12
    A = np.diag(np.arange(1.0, n + 1.0))
    Q, _ = np.linalg.qr(np.random.default_rng(11).standard_normal((n, n)))
    A = Q @ A @ Q.T
    b = Q[:, 0] + Q[:, 1]
    res = fg.fgmres(lambda x: A @ x, b, lambda j, v: v, m=10, rtol=1e-30, max_cycles=1, keep_first=True)
    assert res.iterations == 2 and res.first_cycle["j"] == 2
    exact = Q[:, 0] + 0.5 * Q[:, 1]
    np.testing.assert_allclose(res.x, exact, rtol=0, atol=1e-13)


# ---------------------------------------------------------------- Adam (Kingma and Ba)
def _adam_run(grads, lr=1e-3, p0=0.25):
    params = [[np.array([[p0]]), np.array([0.0])]]
    state = {}
    out = []
    for g in grads:
        mlp.adam_step(params, [[np.array([[g]]), np.array([0.0])]], state, lr=lr)
        out.append(params[0][0][0, 0])
    return np.array(out)


def test_adam_first_step_is_a_signed_lr_step():
    """Bias correction makes the first update -lr g / (|g| + eps) whatever the
    gradient's size."""
    for g in (3.0, -2e-3, 7e5):
        p = _adam_run([g], lr=1e-2)
        assert abs((0.25 - p[0]) - 1e-2 * g / (abs(g) + 1e-8)) <= 1e-16


def test_adam_constant_gradient_moves_lr_per_step():
    """With a constant gradient the corrected moments are g and g^2 at every
    step, so each of 6 steps moves the parameter by lr g / (|g| + eps)."""
    p = _adam_run([0.5] * 6, lr=1e-3)
    steps = -np.diff(np.concatenate([[0.25], p]))
    np.testing.assert_allclose(steps, 1e-3 * 0.5 / (0.5 + 1e-8), rtol=1e-12)


def test_adam_second_step_by_hand():
    """g = 1 then g = -1 (beta1 = 0.9, beta2 = 0.999): m_2 = 0.09 - 0.1 = -0.01,
    m_2 / (1 - 0.81) = -1/19; v_2 = 0.000999 + 0.001 = 0.001999 = 1 - 0.999^2,
    so the corrected second moment is exactly 1 and the step is +lr/19."""
    p = _adam_run([1.0, -1.0], lr=1e-2)
    assert abs((p[1] - p[0]) - 1e-2 / 19.0 / (1.0 + 1e-8)) <= 1e-15


# ---------------------------------------------------------------- DSA (App. A)
@pytest.mark.parametrize("spec", [tiny_1d(nx=7, n_ord=2), tiny_2d(seed=3, nx=4, ny=3, quad=("cl", 3, 2, False))])
def test_fc_dsa_exact_when_p1_is_exact(spec):
    """S2 in 1D and CL(3,2) in X-Y: the P1 ansatz spans every angular flux,
    so FC-DSA is the ideal correction: M_DSA^{-1} A~ = I, and GMRES-DSA
    converges in one step."""
    P = tr.Problem(spec)
    D = dsa.DSA(P)
    At = tr.dense_A_tilde(P)
    Minv = np.stack([D.apply(e) for e in np.eye(P.ndof)], 1)
    assert np.abs(Minv @ At - np.eye(P.ndof)).max() < 1e-12
    res = fg.fgmres(_At(P), tr.b_tilde(P), lambda j, v: D.apply(v), m=10, rtol=1e-12)
    assert res.iterations == 1


@pytest.mark.parametrize("spec", [tiny_1d(nx=8, n_ord=8), tiny_2d(seed=6, nx=5, ny=5, quad=("cl", 8, 4, True))])
def test_fc_dsa_two_constructions_agree_and_contract(spec):
    """Moments of the assembled upwind D_j == App. A's D_C / D_J form; the
    error propagator I - M^{-1} A~ contracts (spectral radius well below 1)."""
    P = tr.Problem(spec)
    A1, _ = dsa.fc_system(P)
    A2, _ = dsa.fc_system_appA(P)
    assert abs(A1 - A2).max() < 1e-12 * abs(A1).max()
    D = dsa.DSA(P)
    At = tr.dense_A_tilde(P)
    E = np.eye(P.ndof) - np.stack([D.apply(e) for e in np.eye(P.ndof)], 1) @ At
    rho = max(abs(np.linalg.eigvals(E)))
    assert rho < 0.35


@pytest.mark.parametrize("spec", [tiny_1d(nx=8, n_ord=8), tiny_2d(seed=6, nx=5, ny=5, quad=("cl", 8, 4, True)),
                                  tiny_2d(seed=7, nx=4, ny=3, quad=("cl", 6, 3, False))])
def test_pc_dsa_first_moment_rows_keep_only_the_central_flux(spec):
    """PC-DSA (App. A, last paragraph) drops the jump operator from the
    first-moment rows.  Built independently: the central part of the assembled
    upwind operator, C(Omega) = (D(Omega) - D(-Omega)) / 2 from the operators of
    the two mirrored directions, replaces D_j in the first-moment rows of the
    angular-moment construction; this equals the D_C / D_J form with the jump
    terms dropped, and differs from FC-DSA."""
    from oracle import dg
    P = tr.Problem(spec)
    ax = [0] if P.mesh.dim == 1 else [0, 1]
    om = {0: P.ox, 1: P.oy}
    Dn = [dg.advection(P.mesh, -P.ox[j], -P.oy[j]).tocsc() for j in range(P.nord)]
    C = [0.5 * (P.D(j) - Dn[j]) for j in range(P.nord)]
    Sa = P.St - P.Ss
    m = {f: float(np.sum(P.w * om[f])) for f in ax}
    a = {(d, f): float(np.sum(P.w * om[d] * om[f])) for d in ax for f in ax}
    E = sum(P.w[j] * P.D(j) for j in range(P.nord))
    Ef = {f: sum(P.w[j] * om[f][j] * P.D(j) for j in range(P.nord)) for f in ax}
    rows = [[E + Sa] + [3.0 * (Ef[f] + m[f] * P.St) for f in ax]]
    for d in ax:
        Cd = sum(P.w[j] * om[d][j] * C[j] for j in range(P.nord))
        Cdf = {f: sum(P.w[j] * om[d][j] * om[f][j] * C[j] for j in range(P.nord)) for f in ax}
        rows.append([Cd + m[d] * Sa] + [3.0 * (Cdf[f] + a[(d, f)] * P.St) for f in ax])
    K = sp.bmat(rows, format="csc").toarray()
    Kpc = dsa.fc_system_appA(P, partially_consistent=True)[0].toarray()
    Kfc = dsa.fc_system_appA(P)[0].toarray()
    assert np.abs(K - Kpc).max() < 1e-12 * np.abs(Kpc).max()
    assert np.abs(Kfc - Kpc).max() > 1e-3 * np.abs(Kfc).max()


# ---------------------------------------------------------------- ROMSAD (section 4)
def _family(n=5, nx=4, ny=4, quad=("cl", 4, 2, True)):
    specs = []
    for k in range(n):
        s = dict(tiny_2d(seed=0, nx=nx, ny=ny, quad=quad))
        s["sigma_s"] = s["sigma_s"] * (1 + 0.4 * k)
        s["sigma_t"] = s["sigma_s"] + 0.3
        specs.append(s)
    return specs


def test_xi_recurrence_identities():
    """A~ xi^(l) = v^(l) (eq. of xi) and T Sigma_s xi = xi - v (eq. of the
    density relation)."""
    P = tr.Problem(_family()[1])
    D = dsa.DSA(P)
    res = fg.fgmres(_At(P), tr.b_tilde(P), lambda j, v: D.apply(v), m=40, rtol=1e-13, keep_first=True)
    xis = rom.xi_recurrence(res.first_cycle, res.x, 3)
    assert len(xis) == 3
    for l, xi in enumerate(xis):
        v = res.first_cycle["V"][l]
        assert np.linalg.norm(tr.A_tilde_apply(P, xi) - v) < 1e-10
        assert np.linalg.norm(tr.T_apply(P, P.Ss @ xi) - (xi - v)) < 1e-10


def test_rom_exact_when_span_contains_ideal_correction():
    """If U_r spans the ideal correction delta psi(v), M_ROM^{-1} v = A~^{-1} v."""
    P = tr.Problem(_family()[2])
    v = np.random.default_rng(9).standard_normal(P.ndof)
    At = tr.dense_A_tilde(P)
    xi = np.linalg.solve(At, v)
    dpsi = rom.snapshot_corrections(P, [xi])[0]
    U, _ = rom.mgs_truncate(np.zeros((0, P.nord, P.ndof)), dpsi)
    z = v + rom.rom_correction(P, U, v)
    np.testing.assert_allclose(z, xi, rtol=0, atol=1e-11 * np.abs(xi).max())


def test_mgs_truncation():
    rng = np.random.default_rng(1)
    U = np.zeros((0, 3, 10))
    a, b = rng.standard_normal((3, 10)), rng.standard_normal((3, 10))
    U, added1 = rom.mgs_truncate(U, a)
    U, added2 = rom.mgs_truncate(U, b)
    U, added3 = rom.mgs_truncate(U, 2.0 * a - 0.5 * b)   # in the span: truncated
    assert (added1, added2, added3) == (True, True, False)
    G = np.einsum("inm,knm->ik", U, U)
    assert np.abs(G - np.eye(2)).max() < 1e-14


def test_greedy_rank_affine_and_sampled_residual():
    """r = k * window when nothing is truncated; U orthonormal; the affine
    region-wise reduced operator equals the dense projection; the ROM is
    exact on sampled parameters (FGMRES-ROMSAD converges in one step)."""
    specs = _family(5)
    U, rep = rom.greedy(specs, window=2, eps_rom=0.0, n_giter=3)
    assert rep.r_history == [2, 4, 6] and rep.truncated == 0
    assert len(set(rep.sampled)) == 3 and rep.sampled[0] == 0
    assert np.abs(np.einsum("inm,knm->ik", U, U) - np.eye(6)).max() < 1e-8
    assert all(np.diff(rep.max_residual) < 0)
    P = tr.Problem(specs[rep.sampled[1]])
    Ar = rom.reduced_operator(P, U)
    AD, G, S = rom.affine_terms(P, U, 2)
    Aff = AD + sum(P.spec["sigma_t"][R] * G[R] - P.spec["sigma_s"][R] * S[R] for R in range(2))
    assert np.abs(Ar - Aff).max() < 1e-12 * np.abs(Ar).max()
    R = rom.Romsad(P, U, dsa.DSA(P), window=2)
    res = fg.fgmres(_At(P), tr.b_tilde(P), R, m=20, rtol=1e-8)
    assert res.iterations == 1
    b = tr.b_tilde(P)
    assert rom.residual_indicator(P, U, P.Ss @ b) < 1e-7 * np.linalg.norm(P.Ss @ b)


def test_greedy_samples_the_brute_force_argmax():
    """Each greedy step (section 4.4.2, step 3) samples the unsampled training
    parameter with the largest residual indicator, recomputed here from the
    assembled psi-space matrix: a dense Galerkin solve in the span of the
    basis of that step, its residual against the isotropic eta_0, and the
    largest per-ordinate 2-norm; the report holds that maximum."""
    specs = _family(6)
    U, rep = rom.greedy(specs, window=2, eps_rom=0.0, n_giter=4)
    assert rep.truncated == 0 and len(rep.sampled) == 4
    probs = [tr.Problem(s) for s in specs]
    nord, ndof = probs[0].nord, probs[0].ndof
    mats = [tr.full_system(P)[0] for P in probs]
    eta0 = [P.Ss @ tr.b_tilde(P) for P in probs]
    for k in range(1, len(rep.sampled)):
        Uk = U[:2 * k].reshape(2 * k, -1).T  # after k steps the basis is its first 2k vectors
        vals = {}
        for i in range(len(probs)):
            if i in rep.sampled[:k]:
                continue
            e = np.tile(eta0[i], nord)
            AU = mats[i] @ Uk
            c = np.linalg.solve(Uk.T @ AU, Uk.T @ e)
            vals[i] = np.linalg.norm((AU @ c - e).reshape(nord, ndof), axis=1).max()
        best = max(vals, key=lambda i: (vals[i], -i))
        assert rep.sampled[k] == best, (k, rep.sampled, vals)
        assert abs(rep.max_residual[k - 1] - vals[best]) <= 1e-8 * vals[best]


def test_learned_rows_exact_on_a_sampled_parameter():
    """Training rows: on a parameter whose own snapshots span U, xi - v is the
    density-relation correction W_w^T U^T dpsi, so the least-squares target
    reproduces it exactly; features carry the unit vector g / ||g||."""
    specs = _family(4)
    U, rep = rom.greedy(specs, window=2, eps_rom=0.0, n_giter=2)
    P = tr.Problem(specs[rep.sampled[1]])
    D = dsa.DSA(P)
    res = fg.fgmres(_At(P), tr.b_tilde(P), lambda j, v: D.apply(v), m=60, rtol=1e-11, keep_first=True)
    mu = np.array([0.3, 0.7])
    X, T = rom.learned_correction_rows(P, U, res.first_cycle, res.x, 2, mu)
    xis = rom.xi_recurrence(res.first_cycle, res.x, 2)
    ww = rom.Ww(P, U)
    for l in range(2):
        v = res.first_cycle["V"][l]
        g = rom.W1(U) @ (P.Ss @ v)
        np.testing.assert_allclose(X[l, :2], mu)
        assert abs(np.linalg.norm(X[l, 2:]) - 1.0) < 1e-14
        c = T[l] * np.linalg.norm(g)
        err = np.linalg.norm(ww.T @ c - (xis[l] - v)) / np.linalg.norm(xis[l] - v)
        assert err < 1e-8, err


def test_learned_rows_are_least_squares_fits():
    """Off the sampled set the target is the least-squares fit: its residual is
    orthogonal to every column of W_w (a transposed operand breaks this)."""
    specs = _family(4)
    U, _ = rom.greedy(specs, window=2, eps_rom=0.0, n_giter=2)
    spec = dict(specs[1], sigma_s=specs[1]["sigma_s"] * 1.3, sigma_t=specs[1]["sigma_t"] * 1.3)
    P = tr.Problem(spec)
    D = dsa.DSA(P)
    res = fg.fgmres(_At(P), tr.b_tilde(P), lambda j, v: D.apply(v), m=60, rtol=1e-11, keep_first=True)
    X, T = rom.learned_correction_rows(P, U, res.first_cycle, res.x, 2, np.zeros(1))
    xis = rom.xi_recurrence(res.first_cycle, res.x, 2)
    ww = rom.Ww(P, U)
    for l in range(2):
        v = res.first_cycle["V"][l]
        g = rom.W1(U) @ (P.Ss @ v)
        resid = ww.T @ (T[l] * np.linalg.norm(g)) - (xis[l] - v)
        assert np.abs(ww @ resid).max() < 1e-10 * np.linalg.norm(ww) * np.linalg.norm(xis[l] - v)


# ---------------------------------------------------------------- MLP
def test_mlp_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    params = mlp.init([5, 7, 6, 3], rng)
    X = rng.standard_normal((4, 5))
    Y = rng.standard_normal((4, 3))
    out, cache = mlp.forward(params, X)
    grads = mlp.backward(params, cache, out, Y)
    h = 1e-6
    for li in range(len(params)):
        for k in range(2):
            p = params[li][k]
            flat = p.reshape(-1)
            for idx in rng.choice(flat.size, size=min(5, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp = mlp.mse(mlp.forward(params, X)[0], Y)
                flat[idx] = old - h
                lm = mlp.mse(mlp.forward(params, X)[0], Y)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - grads[li][k].reshape(-1)[idx]) < 1e-7 * max(1.0, abs(fd))


def test_gelu_special_values():
    # gelu(0) = 0, gelu'(0) = 1/2, gelu(x) -> x for large x, -> 0 for very negative x
    assert mlp.gelu(np.array(0.0)) == 0.0
    assert abs(mlp.gelu_grad(np.array(0.0)) - 0.5) < 1e-15
    assert abs(mlp.gelu(np.array(10.0)) - 10.0) < 1e-12
    assert abs(mlp.gelu(np.array(-10.0))) < 1e-12
    # gelu(1) = Phi(1) = 0.8413447460685429 (standard normal CDF at 1)
    assert abs(mlp.gelu(np.array(1.0)) - 0.8413447460685429) < 1e-15


# ---------------------------------------------------------------- SI-SA
def test_si_with_the_exact_inverse_converges_in_one_step():
    from oracle import si
    P = tr.Problem(tiny_2d(seed=4, nx=4, ny=3, quad=("cl", 4, 2, False)))
    At = tr.dense_A_tilde(P)
    b = tr.b_tilde(P)
    res = si.si(_At(P), b, lambda l, r: np.linalg.solve(At, r), rtol=1e-12)
    assert res.iterations == 1 and res.converged
    np.testing.assert_allclose(res.x, np.linalg.solve(At, b), rtol=1e-12, atol=1e-14)


def test_unaccelerated_si_contracts_by_the_scattering_ratio():
    """Infinite-medium-like case (uniform c = sigma_s / sigma_t): plain SI
    reduces the residual by at most c per sweep, and its limit is the dense
    solution."""
    from oracle import si
    spec = tiny_2d(seed=5, nx=5, ny=5, quad=("cl", 8, 4, True), n_regions=1)
    spec["sigma_t"] = np.array([2.0])
    spec["sigma_s"] = np.array([1.6])
    P = tr.Problem(spec)
    res = si.si(_At(P), tr.b_tilde(P), lambda l, r: r, rtol=1e-10, max_iter=200)
    assert res.converged
    ratios = np.array(res.residuals[1:]) / np.array(res.residuals[:-1])
    assert ratios.max() <= 0.8 + 1e-12
    np.testing.assert_allclose(res.x, np.linalg.solve(tr.dense_A_tilde(P), tr.b_tilde(P)), rtol=1e-8)


def test_si_dsa_exact_for_slab_s2():
    """1D S2 with fully consistent DSA: M_DSA^{-1} = A~^{-1}, one SI step."""
    from oracle import si
    P = tr.Problem(tiny_1d(seed=2, nx=6, n_ord=2))
    D = dsa.DSA(P)
    res = si.si(_At(P), tr.b_tilde(P), lambda l, r: D.apply(r), rtol=1e-12)
    assert res.iterations == 1


# ---------------------------------------------------------------- cross sections varying inside cells (5.3)
def _vs_spec(seed, nx, ny, quad, mu):
    spec = tiny_2d(seed=seed, nx=nx, ny=ny, quad=quad)
    shape = lambda x, y: 0.5 + x * x + 0.3 * x * y
    return dict(spec, sigma_fields=[shape, lambda x, y: np.ones_like(x)],
                sigma_t=np.array([mu, 0.1]), sigma_s=np.array([0.9 * mu, 0.05]))


def test_fc_dsa_exact_with_varying_sigma():
    """CL(3,2): the P1 ansatz spans every angular flux whatever the cross
    sections, so FC-DSA with the varying mass matrices is still the ideal
    correction (M_DSA^{-1} A~ = I)."""
    P = tr.Problem(_vs_spec(3, 4, 3, ("cl", 3, 2, False), 5.0))
    D = dsa.DSA(P)
    At = tr.dense_A_tilde(P)
    Minv = np.stack([D.apply(e) for e in np.eye(P.ndof)], 1)
    assert np.abs(Minv @ At - np.eye(P.ndof)).max() < 1e-12


def test_affine_terms_with_shape_fields_equal_dense_projection():
    """sigma_t = mu s + 0.1, sigma_s = 0.9 mu s + 0.05 with s varying inside
    the cells: A_D + sum_f theta_t,f G_f - theta_s,f S_f equals U^T A(mu) U,
    and the greedy ROM is exact on its sampled parameters."""
    fam = [_vs_spec(4, 5, 4, ("cl", 8, 4, True), mu) for mu in (2.0, 4.0, 6.0, 8.0)]
    U, rep = rom.greedy(fam, window=2, eps_rom=0.0, n_giter=2)
    for mu in (3.0, 7.5):
        P = tr.Problem(_vs_spec(4, 5, 4, ("cl", 8, 4, True), mu))
        Ar = rom.reduced_operator(P, U)
        AD, G, S = rom.affine_terms(P, U, 2)
        Aff = AD + sum(P.spec["sigma_t"][f] * G[f] - P.spec["sigma_s"][f] * S[f] for f in range(2))
        assert np.abs(Ar - Aff).max() < 1e-12 * np.abs(Ar).max()
    P = tr.Problem(fam[rep.sampled[1]])
    res = fg.fgmres(_At(P), tr.b_tilde(P), rom.Romsad(P, U, dsa.DSA(P), window=2), m=20, rtol=1e-8)
    assert res.iterations == 1
