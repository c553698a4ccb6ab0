"""Pins of the oracle's quadrature, DG operators and transport sweep against
facts fixed by the paper and by mathematics (closed forms, invariants,
conservation, brute force)."""
import numpy as np
import pytest

from oracle import dg
from oracle import transport as tr
from oracle.quadrature import chebyshev_legendre, slab_gl
from synth import tiny_1d, tiny_2d


# ---------------------------------------------------------------- quadrature (section 2.1)
@pytest.mark.parametrize("nt,nz,folded", [(4, 2, False), (16, 16, True), (16, 8, True), (30, 6, False)])
def test_cl_moments(nt, nz, folded):
    ox, oy, w = chebyshev_legendre(nt, nz, folded)
    assert len(w) == nt * (nz // 2 if folded else nz)
    assert abs(w.sum() - 1.0) < 1e-14                      # normalised rule
    assert abs((w * ox).sum()) < 1e-14 and abs((w * oy).sum()) < 1e-14
    # (1/4pi) int Omega_x^2 = (1/4pi) int Omega_y^2 = 1/3 (exact for nz >= 2)
    assert abs((w * ox ** 2).sum() - 1 / 3) < 1e-14
    assert abs((w * oy ** 2).sum() - 1 / 3) < 1e-14
    assert np.all(ox ** 2 + oy ** 2 <= 1 + 1e-14)


def test_cl_ordering_and_angles():
    ox, oy, w = chebyshev_legendre(4, 2)
    th = np.arctan2(oy, ox) % (2 * np.pi)
    # j = (j2 - 1) N_theta + j1 with theta_j1 = (2 j1 - 1) pi / N_theta
    np.testing.assert_allclose(th[:4], (2 * np.arange(1, 5) - 1) * np.pi / 4, atol=1e-14)
    np.testing.assert_allclose(th[4:], th[:4], atol=1e-14)


def test_gl_exactness():
    x, _, w = slab_gl(8)
    for k in range(16):  # exact up to degree 2n-1 = 15; (1/2) int_{-1}^{1} x^k
        exact = 0.0 if k % 2 else 1.0 / (k + 1)
        assert abs((w * x ** k).sum() - exact) < 1e-14


def test_folded_rule_same_transport():
    base = tiny_2d(seed=3, nx=3, ny=3, quad=("cl", 4, 4, False))
    fold = dict(base, quad=("cl", 4, 4, True))
    Pa, Pb = tr.Problem(base), tr.Problem(fold)
    q = np.random.default_rng(0).standard_normal(Pa.ndof)
    np.testing.assert_allclose(tr.T_apply(Pa, q), tr.T_apply(Pb, q), rtol=1e-13, atol=1e-14)


# ---------------------------------------------------------------- DG operators (2.2-2.3, App. A)
@pytest.mark.parametrize("spec", [tiny_1d(nx=5, n_ord=4), tiny_2d(nx=4, ny=3)])
def test_mass_is_identity_in_orthonormal_basis(spec):
    m = dg.Mesh.of(spec)
    np.testing.assert_allclose(dg.mass_local(m), np.eye(m.nloc), atol=1e-14)


@pytest.mark.parametrize("spec", [tiny_1d(nx=5, n_ord=4), tiny_2d(nx=4, ny=3, quad=("cl", 6, 2, False))])
def test_appA_identity(spec):
    """App. A: D_j = sum_e Omega_e (D_C^e - sgn(Omega_e)/2 D_J^e), which holds
    when D_C, D_J include both boundary faces; D_C is then skew-symmetric."""
    P = tr.Problem(spec)
    m = P.mesh
    ops = [dg.central_and_jump(m, e) for e in range(m.dim)]
    for j in range(P.nord):
        om = [P.ox[j], P.oy[j]]
        R = sum(om[e] * (ops[e][0] - np.sign(om[e]) / 2 * ops[e][1]) for e in range(m.dim))
        assert abs(P.D(j) - R).max() < 1e-13
    for DC, DJ in ops:
        assert abs(DC + DC.T).max() < 1e-13
        assert abs(DJ - DJ.T).max() < 1e-13


def test_appA_printed_face_range_breaks_identity():
    """With the face sum printed in App. A (omitting x_{1/2}) the identity
    fails on the first cell, which motivates including both boundary faces."""
    P = tr.Problem(tiny_1d(nx=5, n_ord=4))
    DC, DJ = dg.central_and_jump(P.mesh, 0, include_boundary_faces=False)
    j = int(np.argmin(P.ox))          # x_{1/2} is the outflow face for Omega_x < 0
    R = P.ox[j] * (DC + 0.5 * DJ)
    assert abs(P.D(j) - R).max() > 1e-3


def test_advection_block_closed_form():
    """Quadrature-assembled 1D upwind block for Omega = +1 equals the hand-derived
    (1/h)[[1, sqrt3], [-sqrt3, 3]] in the orthonormal Legendre basis; the
    coupling to the upwind neighbour is -(1/h)[[1, sqrt3], [-sqrt3, -3]]."""
    m = dg.Mesh(1, 4, 1, (0.0, 2.0, 0.0, 1.0))
    D = dg.advection(m, 1.0, 0.0).toarray()
    h = 0.5
    r3 = np.sqrt(3.0)
    np.testing.assert_allclose(D[2:4, 2:4], np.array([[1, r3], [-r3, 3]]) / h, atol=1e-13)
    np.testing.assert_allclose(D[2:4, 0:2], -np.array([[1, r3], [-r3, -3]]) / h, atol=1e-13)
    assert np.all(D[0:2, 2:] == 0)  # first cell depends on nothing downstream


# ---------------------------------------------------------------- sweep (section 3.1)
def test_sweep_mms_bilinear_reproduced():
    """Upwind DG reproduces any continuous bilinear psi* exactly when the
    source is Omega.grad psi* + sigma_t psi* and the inflow is psi*."""
    spec = tiny_2d(seed=1, nx=5, ny=4, quad=("cl", 6, 2, False), n_regions=3)
    P = tr.Problem(spec)
    m = P.mesh
    sig = P.sig_t_cell
    coef = np.random.default_rng(2).standard_normal((P.nord, 4))
    q = np.empty((P.nord, P.ndof))
    exact = np.empty((P.nord, P.ndof))
    for j in range(P.nord):
        a, b, c, d = coef[j]
        f = lambda x, y: a + b * x + c * y + d * x * y
        src = lambda x, y: (P.ox[j] * (b + d * y) + P.oy[j] * (c + d * x)
                            + sig[:, None] * f(x, y))
        q[j] = dg.project(m, src) + P.gbc(j, f)
        exact[j] = dg.project(m, f)
    _, psi = tr.sweep(P, q, store_psi=True)
    np.testing.assert_allclose(psi, exact, rtol=0, atol=1e-12 * np.abs(exact).max())


def test_sweep_constant_state():
    spec = tiny_2d(seed=4, nx=4, ny=4, quad=("cl", 8, 2, True), inflow=0.0)
    spec = dict(spec, sigma_s=np.zeros(2), sigma_t=np.array([2.0, 2.0]))
    spec["source"] = dg.project(dg.Mesh.of(spec), lambda x, y: 3.0 + 0 * x)
    spec["inflow"] = 1.5
    P = tr.Problem(spec)
    phi = tr.b_tilde(P)
    np.testing.assert_allclose(phi, dg.project(P.mesh, lambda x, y: 1.5 + 0 * x), atol=1e-13)


def test_sweep_pure_absorber_second_order():
    """Pure absorber slab, G = 1, zero inflow: psi(x, mu) = (1 - exp(-s x/mu))/s
    for mu > 0 (mirror for mu < 0).  The DG error decays at least like h^2."""
    errs = []
    s = 3.0
    for nx in (16, 32, 64, 128):
        spec = dict(dim=1, nx=nx, ny=1, box=(0.0, 1.0, 0.0, 1.0), quad=("gl", 4),
                    region=np.zeros(nx, np.int32), sigma_t=np.array([s]), sigma_s=np.array([0.0]),
                    source=None, inflow=0.0)
        m = dg.Mesh.of(spec)
        spec["source"] = dg.project(m, lambda x, y: np.ones_like(x))
        P = tr.Problem(spec)
        _, psi = tr.sweep(P, P.G, store_psi=True)
        e = 0.0
        for j in range(P.nord):
            mu = P.ox[j]
            ex = (lambda x, y, mu=mu: (1 - np.exp(-s * x / mu)) / s) if mu > 0 else \
                 (lambda x, y, mu=mu: (1 - np.exp(-s * (1 - x) / -mu)) / s)
            e = max(e, np.linalg.norm(psi[j] - dg.project(m, ex)))
        errs.append(e)
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8) and 1.9 < rates[-1] < 3.1, rates


def _boundary_outflow(P, psi_j, j):
    """sum over boundary faces of int (Omega.n)^+ psi_j, by evaluating the DG
    function on the faces (independent of the assembled matrices)."""
    m = P.mesh
    gx, gw = np.polynomial.legendre.leggauss(3)
    r3 = np.sqrt(3.0)
    out = 0.0
    ox, oy = P.ox[j], P.oy[j]
    c = psi_j.reshape(m.ny, m.nx, m.nloc)
    if m.dim == 1:
        if ox > 0:
            out += ox * (c[0, -1, 0] + r3 * c[0, -1, 1]) / np.sqrt(m.hx)
        else:
            out += -ox * (c[0, 0, 0] - r3 * c[0, 0, 1]) / np.sqrt(m.hx)
        return out

    def trace(cc, sx, sy):
        return (cc[..., 0] + r3 * sx * cc[..., 1] + r3 * sy * cc[..., 2]
                + 3 * sx * sy * cc[..., 3]) / np.sqrt(m.hx * m.hy)
    for g, w in zip(gx, gw):
        if ox > 0:
            out += ox * w * m.hy / 2 * trace(c[:, -1], 1.0, g).sum()
        elif ox < 0:
            out += -ox * w * m.hy / 2 * trace(c[:, 0], -1.0, g).sum()
        if oy > 0:
            out += oy * w * m.hx / 2 * trace(c[-1, :], g, 1.0).sum()
        elif oy < 0:
            out += -oy * w * m.hx / 2 * trace(c[0, :], g, -1.0).sum()
    return out


@pytest.mark.parametrize("spec", [tiny_1d(nx=6, n_ord=8, inflow=0.7),
                                  tiny_2d(seed=5, nx=5, ny=4, quad=("cl", 8, 4, True), inflow=0.4)])
def test_sweep_particle_balance(spec):
    """sum_j w_j outflow_j + int sigma_t phi = int q + inflow (one sweep with
    q = Sigma_s phi_in + G), from integrating the DG equation with eta = 1."""
    P = tr.Problem(spec)
    m = P.mesh
    vol = np.sqrt(m.hx * m.hy)        # int over a cell of eta_0 is sqrt(|T|)
    phi_in = np.random.default_rng(7).uniform(0, 1, P.ndof)
    q0 = P.Ss @ phi_in + P.G
    qs = np.stack([q0 + P.gbc(j) for j in range(P.nord)])
    phi, psi = tr.sweep(P, qs, store_psi=True)
    outflow = sum(P.w[j] * _boundary_outflow(P, psi[j], j) for j in range(P.nord))
    absorb = (P.sig_t_cell * phi.reshape(-1, m.nloc)[:, 0]).sum() * vol
    src = q0.reshape(-1, m.nloc)[:, 0].sum() * vol
    inflow = sum(P.w[j] * P.gbc(j).reshape(-1, m.nloc)[:, 0].sum() * vol for j in range(P.nord))
    assert abs(outflow + absorb - src - inflow) < 1e-12 * (abs(src) + abs(inflow))


def test_sweep_residual():
    P = tr.Problem(tiny_2d(seed=6, nx=6, ny=5, quad=("cl", 8, 2, True)))
    q = np.random.default_rng(1).standard_normal(P.ndof)
    _, psi = tr.sweep(P, q, store_psi=True)
    for j in range(P.nord):
        r = (P.D(j) + P.St) @ psi[j] - q
        assert np.linalg.norm(r) < 1e-13 * np.linalg.norm(q)


# ---------------------------------------------------------------- systems (2.3, 3.2)
@pytest.mark.parametrize("spec", [tiny_1d(nx=4, n_ord=4, inflow=0.3),
                                  tiny_2d(seed=2, nx=3, ny=3, quad=("cl", 4, 2, False), inflow=0.2)])
def test_memory_efficient_system_equals_coupled(spec):
    """phi = Q A^{-1} b (fully coupled system) equals A~^{-1} b~ (brute force)."""
    P = tr.Problem(spec)
    A, b = tr.full_system(P)
    psi = np.linalg.solve(A.toarray(), b).reshape(P.nord, -1)
    phi = tr.scalar_flux(P, psi)
    At = tr.dense_A_tilde(P)
    np.testing.assert_allclose(np.linalg.solve(At, tr.b_tilde(P)), phi, rtol=1e-12, atol=1e-14)


def test_infinite_medium_equilibrium():
    """Uniform medium with inflow g = G / sigma_a: phi == G / sigma_a exactly."""
    spec = tiny_2d(seed=8, nx=4, ny=4, quad=("cl", 8, 2, True))
    spec = dict(spec, sigma_s=np.array([2.0, 2.0]), sigma_t=np.array([2.5, 2.5]))
    m = dg.Mesh.of(spec)
    spec["source"] = dg.project(m, lambda x, y: 0.8 + 0 * x)
    spec["inflow"] = 0.8 / 0.5
    P = tr.Problem(spec)
    At = tr.dense_A_tilde(P)
    phi = np.linalg.solve(At, tr.b_tilde(P))
    np.testing.assert_allclose(phi, dg.project(m, lambda x, y: 1.6 + 0 * x), atol=1e-12)


def test_separable_source_generator_matches_quadrature_projection():
    """The factorised config-3 source moments equal the 4x4 Gauss projection."""
    from synth import cfg3_problem, cfg3_sources, cfg3_train_test
    _, te = cfg3_train_test(n_test=3)
    for mu in te:
        a = cfg3_problem(mu, n=12)["source"]
        b = cfg3_sources(mu[None], 12)[0]
        assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max()


def test_side_inflow_is_linear_and_matches_constant_inflow():
    """Per-side inflow: the four sides together give the constant-inflow term,
    and each side's term is nonzero only for directions entering through it."""
    from oracle import dg
    spec = tiny_2d(seed=3, nx=4, ny=3, quad=("cl", 8, 2, False))
    P = tr.Problem(spec)
    for j in range(P.nord):
        parts = [dg.inflow_vector(P.mesh, P.ox[j], P.oy[j], {side: 0.7}) for side in "LRBT"]
        whole = dg.inflow_vector(P.mesh, P.ox[j], P.oy[j], 0.7)
        np.testing.assert_allclose(sum(parts), whole, rtol=1e-14, atol=1e-15)
        assert (np.abs(parts[0]).max() > 0) == (P.ox[j] > 0)
        assert (np.abs(parts[1]).max() > 0) == (P.ox[j] < 0)
        assert (np.abs(parts[2]).max() > 0) == (P.oy[j] > 0)
        assert (np.abs(parts[3]).max() > 0) == (P.oy[j] < 0)


# ---------------------------------------------------------------- cross sections varying inside cells (5.3)
def _poly_sigma(x, y):
    return 1.0 + 0.5 * x * x + 0.3 * x * y * y + 0.2 * y


def _field_spec(seed=3, nx=5, ny=4, quad=("cl", 6, 2, False), fields=None, coef_t=(1.3, 0.4), coef_s=(0.6, 0.2),
                box=(0.0, 1.0, 0.0, 1.0)):
    spec = tiny_2d(seed=seed, nx=nx, ny=ny, quad=quad)
    spec = dict(spec, box=box, sigma_fields=fields or [_poly_sigma, lambda x, y: np.ones_like(x)],
                sigma_t=np.array(coef_t), sigma_s=np.array(coef_s))
    return spec


def test_field_matrix_constant_and_piecewise_constant():
    """A shape function constant on every cell gives the piecewise-constant
    mass matrix sigma_matrix of the cell values (the quadrature integrates
    the degree-2 basis products exactly)."""
    m = dg.Mesh(2, 5, 4, (0.0, 1.0, 0.0, 2.0))
    vals = 1.0 + 0.1 * np.arange(m.ncell)
    f = lambda x, y: 1.0 + 0.1 * (np.floor(y / m.hy) * m.nx + np.floor(x / m.hx))
    A = dg.field_matrix(m, f).toarray()
    B = dg.sigma_matrix(m, vals).toarray()
    assert np.abs(A - B).max() < 1e-13


def test_field_matrix_linear_shape_closed_form():
    """f = x: the cell block is x_c I plus h_x / (2 sqrt 3) coupling the x-even
    and x-odd Legendre modes with the same y-mode (int s (sqrt3 s) ds / 2 =
    1/sqrt3 on [-1, 1] scaled by h_x / 2)."""
    m = dg.Mesh(2, 3, 2, (0.0, 1.5, -1.0, 1.0))
    A = dg.field_matrix(m, lambda x, y: x).toarray()
    for c in range(m.ncell):
        i = c % m.nx
        xc = (i + 0.5) * m.hx
        blk = A[4 * c:4 * c + 4, 4 * c:4 * c + 4]
        want = xc * np.eye(4)
        for p0, p1 in ((0, 1), (2, 3)):  # dof p + 2q: (0,1) and (2,3) differ in the x-mode
            want[p0, p1] = want[p1, p0] = m.hx / (2.0 * np.sqrt(3.0))
        np.testing.assert_allclose(blk, want, atol=1e-14)


def test_sweep_mms_bilinear_with_varying_sigma():
    """Upwind DG with a cross section varying inside the cells (a polynomial
    sigma_t, integrated exactly) still reproduces a continuous bilinear psi*
    whose source is Omega.grad psi* + sigma_t psi* (projected from its strong
    form, independently of the assembled Sigma_t)."""
    spec = _field_spec()
    P = tr.Problem(spec)
    m = P.mesh
    ct = spec["sigma_t"]
    sig = lambda x, y: ct[0] * _poly_sigma(x, y) + ct[1]
    coef = np.random.default_rng(2).standard_normal((P.nord, 4))
    q = np.empty((P.nord, P.ndof))
    exact = np.empty((P.nord, P.ndof))
    for j in range(P.nord):
        a, b, c, d = coef[j]
        f = lambda x, y: a + b * x + c * y + d * x * y
        src = lambda x, y: P.ox[j] * (b + d * y) + P.oy[j] * (c + d * x) + sig(x, y) * f(x, y)
        q[j] = dg.project(m, src) + P.gbc(j, f)
        exact[j] = dg.project(m, f)
    _, psi = tr.sweep(P, q, store_psi=True)
    np.testing.assert_allclose(psi, exact, rtol=0, atol=1e-12 * np.abs(exact).max())


def test_sweep_particle_balance_with_varying_sigma():
    """sum_j w_j outflow_j + int sigma_t phi_h = int q + inflow, with the
    absorption integrated from the DG function and sigma_t(x) pointwise (an
    8 x 8 Gauss rule, exact for this polynomial sigma_t)."""
    spec = dict(_field_spec(seed=5, quad=("cl", 8, 4, True)), inflow=0.4)
    P = tr.Problem(spec)
    m = P.mesh
    vol = np.sqrt(m.hx * m.hy)
    phi_in = np.random.default_rng(7).uniform(0, 1, P.ndof)
    q0 = P.Ss @ phi_in + P.G
    qs = np.stack([q0 + P.gbc(j) for j in range(P.nord)])
    phi, psi = tr.sweep(P, qs, store_psi=True)
    outflow = sum(P.w[j] * _boundary_outflow(P, psi[j], j) for j in range(P.nord))
    g8, w8 = np.polynomial.legendre.leggauss(8)
    r3 = np.sqrt(3.0)
    ct = spec["sigma_t"]
    absorb = 0.0
    for c in range(m.ncell):
        i, k = c % m.nx, c // m.nx
        co = phi[4 * c:4 * c + 4]
        for a_, wa in zip(g8, w8):
            for b_, wb in zip(g8, w8):
                x = (i + 0.5 + 0.5 * a_) * m.hx
                y = (k + 0.5 + 0.5 * b_) * m.hy
                val = (co[0] + r3 * a_ * co[1] + r3 * b_ * co[2] + 3 * a_ * b_ * co[3]) / vol
                absorb += wa * wb * m.hx * m.hy / 4 * (ct[0] * _poly_sigma(x, y) + ct[1]) * val
    src = q0.reshape(-1, m.nloc)[:, 0].sum() * vol
    inflow = sum(P.w[j] * P.gbc(j).reshape(-1, m.nloc)[:, 0].sum() * vol for j in range(P.nord))
    assert abs(outflow + absorb - src - inflow) < 1e-12 * (abs(src) + abs(inflow))
