"""GPU parity of DSA, FGMRES, ROMSAD and the greedy builder against the oracle."""
import os

import numpy as np
import pytest

from oracle import dsa as odsa
from oracle import fgmres as ofg
from oracle import rom as orom
from oracle import transport as tr
from synth import cfg1, tiny_1d, tiny_2d


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


def _family(n=5, nx=5, ny=4, quad=("cl", 8, 4, True), seed=0):
    specs = []
    for k in range(n):
        s = dict(tiny_2d(seed=seed, nx=nx, ny=ny, quad=quad))
        s["sigma_s"] = s["sigma_s"] * (1 + 0.4 * k)
        s["sigma_t"] = s["sigma_s"] + 0.3 + 0.05 * k
        specs.append(s)
    return specs


# ------------------------------------------------------------------ DSA
@pytest.mark.gpu
def test_dsa_apply_parity():
    import paper_2410_08735_amd as rt
    specs = [tiny_2d(seed=1, nx=6, ny=5, quad=("cl", 8, 4, True), n_regions=3),
             tiny_2d(seed=2, nx=4, ny=7, quad=("cl", 3, 2, False), n_regions=2),
             tiny_2d(seed=3, nx=9, ny=9, quad=("cl", 16, 4, True), n_regions=2)]
    B = rt.Batch(specs)
    st, ss = B.sigma()
    rng = np.random.default_rng(4)
    v = [rng.standard_normal(n) for n in B.ndofs]
    z, iters = rt.dsa_apply(B, st, ss, B.pack(v), inner_tol=1e-14, inner_max=3000, restart=60)
    for k, spec in enumerate(specs):
        ref = odsa.DSA(tr.Problem(spec)).apply(v[k])
        assert rel(B.unpack(z)[k], ref) <= 1e-11, (k, rel(B.unpack(z)[k], ref), iters)


@pytest.mark.gpu
def test_dsa_apply_parity_symmetric_rules():
    """Reflection-symmetric rules only (the structured multigrid path), on grids
    that coarsen several times."""
    import paper_2410_08735_amd as rt
    specs = [tiny_2d(seed=5, nx=16, ny=8, quad=("cl", 8, 4, True), n_regions=3),
             tiny_2d(seed=6, nx=12, ny=12, quad=("cl", 16, 4, True), n_regions=2)]
    B = rt.Batch(specs)
    st, ss = B.sigma()
    rng = np.random.default_rng(7)
    v = [rng.standard_normal(n) for n in B.ndofs]
    z, iters = rt.dsa_apply(B, st, ss, B.pack(v), inner_tol=1e-14, inner_max=3000, restart=60)
    for k, spec in enumerate(specs):
        ref = odsa.DSA(tr.Problem(spec)).apply(v[k])
        assert rel(B.unpack(z)[k], ref) <= 1e-11, (k, rel(B.unpack(z)[k], ref), iters)
    # one V-cycle (no post-smoothing on the finest level) already approximates
    # the DSA correction
    z1, _ = rt.dsa_apply(B, st, ss, B.pack(v), inner_tol=0.0, inner_max=1, restart=0)
    for k, spec in enumerate(specs):
        ref = odsa.DSA(tr.Problem(spec)).apply(v[k])
        err = rel(B.unpack(z1)[k] - v[k], ref - v[k])
        print(f"one FP32 V-cycle, instance {k}: rel err {err:.3e}")
        assert err <= 0.6
    # stationary V-cycles in FP32 converge to the exact correction up to FP32 rounding
    z40, _ = rt.dsa_apply(B, st, ss, B.pack(v), inner_tol=0.0, inner_max=40, restart=0)
    for k, spec in enumerate(specs):
        ref = odsa.DSA(tr.Problem(spec)).apply(v[k])
        err = rel(B.unpack(z40)[k] - v[k], ref - v[k])
        print(f"stationary FP32 V-cycles, instance {k}: rel err {err:.2e}")
        assert err <= 2e-5, (k, err)


@pytest.mark.gpu
def test_dsa_fp32_vcycles_with_an_hbm_backed_tail_level():
    """96 x 48 cells: the 48 x 24 level is too large for LDS next to the coarser
    ones, so the V-cycle's LDS launch keeps its x in LDS only while it smooths
    and its b in global memory; stationary FP32 V-cycles still converge to the
    oracle's exact DSA correction (slowly on these optically thin cells: a
    contraction of about 0.95 per cycle, as a CPU model of the same cycle
    shows, so 400 cycles)."""
    import paper_2410_08735_amd as rt
    spec = tiny_2d(seed=5, nx=96, ny=48, quad=("cl", 8, 4, True), n_regions=3)
    B = rt.Batch([spec, spec])
    st, ss = B.sigma()
    rng = np.random.default_rng(11)
    v = [rng.standard_normal(n) for n in B.ndofs]
    ref = odsa.DSA(tr.Problem(spec))
    for n_cyc, bound in ((400, 2e-5), (40, 0.05), (1, 0.9)):
        z, _ = rt.dsa_apply(B, st, ss, B.pack(v), inner_tol=0.0, inner_max=n_cyc, restart=0)
        for k in range(2):
            err = rel(B.unpack(z)[k] - v[k], ref.apply(v[k]) - v[k])
            print(f"{n_cyc} FP32 V-cycles, 96 x 48, instance {k}: rel err {err:.2e}", flush=True)
            assert err <= bound, (n_cyc, k, err)


@pytest.mark.gpu
def test_dsa_apply_parity_1d():
    import paper_2410_08735_amd as rt
    specs = [tiny_1d(seed=1, nx=12, n_ord=8), tiny_1d(seed=2, nx=7, n_ord=2)]
    B = rt.Batch(specs)
    st, ss = B.sigma()
    rng = np.random.default_rng(5)
    v = [rng.standard_normal(n) for n in B.ndofs]
    z, _ = rt.dsa_apply(B, st, ss, B.pack(v), inner_tol=1e-14, inner_max=2000, restart=60)
    for k, spec in enumerate(specs):
        ref = odsa.DSA(tr.Problem(spec)).apply(v[k])
        assert rel(B.unpack(z)[k], ref) <= 1e-11


@pytest.mark.gpu
def test_pc_dsa_apply_parity():
    """Partially consistent DSA (App. A: no D_J terms in the first-moment rows)
    against the oracle's PC system, on general and reflection-symmetric rules
    and in slab geometry; the PC correction differs from the FC one."""
    import paper_2410_08735_amd as rt
    for specs in ([tiny_2d(seed=1, nx=6, ny=5, quad=("cl", 8, 4, True), n_regions=3),
                   tiny_2d(seed=2, nx=4, ny=7, quad=("cl", 3, 2, False), n_regions=2),
                   tiny_2d(seed=6, nx=12, ny=12, quad=("cl", 16, 4, True), n_regions=2)],
                  # reflection-symmetric rules only: the structured multigrid kernels
                  [tiny_2d(seed=5, nx=16, ny=8, quad=("cl", 8, 4, True), n_regions=3),
                   tiny_2d(seed=6, nx=12, ny=12, quad=("cl", 16, 4, True), n_regions=2)],
                  [tiny_1d(seed=1, nx=12, n_ord=8), tiny_1d(seed=2, nx=7, n_ord=4)]):
        B = rt.Batch(specs)
        st, ss = B.sigma()
        rng = np.random.default_rng(8)
        v = [rng.standard_normal(n) for n in B.ndofs]
        z, iters = rt.dsa_apply(B, st, ss, B.pack(v), inner_tol=1e-14, inner_max=3000, restart=60,
                                variant="pc")
        zf, _ = rt.dsa_apply(B, st, ss, B.pack(v), inner_tol=1e-14, inner_max=3000, restart=60)
        for k, spec in enumerate(specs):
            P = tr.Problem(spec)
            ref = odsa.DSA(P, "pc").apply(v[k])
            err = rel(B.unpack(z)[k], ref)
            print(f"PC-DSA {spec['dim']}D instance {k}: rel err {err:.2e}, iterations {iters[k]}")
            assert err <= 1e-11, (k, err, iters)
            assert rel(B.unpack(zf)[k], odsa.DSA(P).apply(v[k])) <= 1e-11
            assert rel(B.unpack(z)[k], B.unpack(zf)[k]) > 1e-6


@pytest.mark.gpu
def test_fc_dsa_needs_fewer_iterations_than_pc_dsa():
    """FC-DSA preconditioning takes fewer GMRES iterations than PC-DSA (the
    paper's remark opening section 5 and its variable-scattering table); on
    the section 5.2 pin-cell problem the ordering holds with exact DSA solves."""
    import paper_2410_08735_amd as rt
    from synth import pincell_problem, pincell_sets
    _, te_mu = pincell_sets()
    B = rt.Batch([pincell_problem(m) for m in te_mu])
    st, ss = B.sigma()
    common = dict(m=60, max_cycles=10, sweep_dtype="f64", rtol=1e-11, dsa_inner_max=1000, dsa_restart=60,
                  dsa_inner_tol=1e-12)
    it = {}
    for var in ("fc", "pc"):
        print(f"pin-cell GMRES-{var.upper()}-DSA", flush=True)
        _, stats, ret = rt.fgmres_solve(B, st, ss, B.source(), None,
                                        rt.SolveOptions(precond="dsa", dsa_variant=var, **common))
        assert ret == 0 and all(s["true_relres"] <= common["rtol"] for s in stats)
        it[var] = float(np.mean([s["iterations"] for s in stats]))
    print(f"pin-cell, exact DSA: mean iterations FC {it['fc']:.1f}, PC {it['pc']:.1f}")
    assert it["fc"] < it["pc"], it


@pytest.mark.gpu
def test_pc_dsa_rejects_unknown_variant_and_stationary_cycles():
    import paper_2410_08735_amd as rt
    B = rt.Batch([tiny_2d(seed=1, nx=4, ny=4, quad=("cl", 8, 4, True))])
    st, ss = B.sigma()
    with pytest.raises(rt.RteError):
        rt.check(rt.L.lib().rte_dsa_apply(B.h, rt._ptr(st), rt._ptr(ss), rt._ptr(B.zeros()),
                                          rt._ptr(B.zeros()), 1e-10, 10, 10, 2, None,
                                          rt._stream()), "rte_dsa_apply")
    # PC solves need the Krylov method: no stationary V-cycles
    with pytest.raises(rt.RteError):
        rt.dsa_apply(B, st, ss, B.zeros(), inner_tol=0.0, inner_max=1, restart=0, variant="pc")
    with pytest.raises(rt.RteError):
        rt.fgmres_solve(B, st, ss, B.source(), None,
                        rt.SolveOptions(precond="dsa", dsa_restart=0, dsa_inner_max=1, dsa_variant="pc"))


# ------------------------------------------------------------------ FGMRES
def _oracle_solve(spec, precond="dsa", rtol=1e-13, m=60, U=None, window=2, dsa_variant="fc"):
    P = tr.Problem(spec)
    b = tr.b_tilde(P)
    if precond == "none":
        pc = lambda j, v: v
    elif precond in ("dsa", "pc-dsa"):
        D = odsa.DSA(P, "pc" if precond == "pc-dsa" else "fc")
        pc = lambda j, v: D.apply(v)
    else:
        pc = orom.Romsad(P, U, odsa.DSA(P, dsa_variant), window)
    return ofg.fgmres(lambda x: tr.A_tilde_apply(P, x), b, pc, m=m, rtol=rtol)


@pytest.mark.gpu
@pytest.mark.parametrize("precond", ["none", "dsa", "pc-dsa"])
def test_fgmres_fp64_parity(precond):
    import paper_2410_08735_amd as rt
    specs = [tiny_2d(seed=1, nx=7, ny=6, quad=("cl", 8, 4, True), n_regions=3, inflow=0.2),
             tiny_2d(seed=2, nx=5, ny=5, quad=("cl", 12, 2, True), n_regions=2),
             tiny_2d(seed=3, nx=4, ny=6, quad=("cl", 3, 2, False), n_regions=2)]
    B = rt.Batch(specs)
    st, ss = B.sigma()
    opts = rt.SolveOptions(precond="dsa" if precond == "pc-dsa" else precond, m=60, max_cycles=5,
                           sweep_dtype="f64", rtol=1e-13, dsa_inner_max=2000, dsa_restart=60,
                           dsa_inner_tol=1e-14, dsa_variant="pc" if precond == "pc-dsa" else "fc")
    phi, stats, _ = rt.fgmres_solve(B, st, ss, B.source(), B.inflow(), opts)
    for k, spec in enumerate(specs):
        ref = _oracle_solve(spec, precond)
        assert stats[k]["status"] == 0 and stats[k]["true_relres"] <= 1e-13
        assert rel(B.unpack(phi)[k], ref.x) <= 1e-11
        assert abs(stats[k]["iterations"] - ref.iterations) <= 1, (stats[k], ref.iterations)
    # CL(3,2): FC-DSA is exact, one iteration
    if precond == "dsa":
        assert stats[2]["iterations"] == 1


@pytest.mark.gpu
def test_fgmres_fp32_sweeps_refined_to_1e8():
    """FP32 cycles (b~ from an FP32 sweep), FP64 true residuals T (G + Sigma_s phi) - phi,
    with and without inflow."""
    import paper_2410_08735_amd as rt
    specs = [tiny_2d(seed=s, nx=12, ny=10, quad=("cl", 16, 4, True), n_regions=2, inflow=0.3 * (s % 2))
             for s in range(4)]
    B = rt.Batch(specs)
    st, ss = B.sigma()
    opts = rt.SolveOptions(precond="dsa", m=30, max_cycles=10, sweep_dtype="f32", rtol=1e-8,
                           dsa_inner_max=200, dsa_restart=30, dsa_inner_tol=1e-10)
    phi, stats, ret = rt.fgmres_solve(B, st, ss, B.source(), B.inflow(), opts)
    assert ret == 0
    for k, spec in enumerate(specs):
        assert stats[k]["true_relres"] <= 1e-8
        # one FP32 sweep per iteration and one for b~; one FP64 sweep per
        # cycle's true residual T (G + Sigma_s phi) - phi; at least two cycles
        assert stats[k]["sweeps_f32"] == stats[k]["iterations"] + 1, stats[k]
        assert stats[k]["sweeps_f64"] == stats[k]["cycles"] >= 2, stats[k]
        ref = _oracle_solve(spec, "dsa", rtol=1e-13)
        assert rel(B.unpack(phi)[k], ref.x) <= 1e-6


@pytest.mark.gpu
def test_fgmres_fp32_with_one_vcycle_dsa_on_partial_tiles():
    """The production configuration (FP32 cycles, one FP32 V-cycle per DSA
    application, whose finest level runs in 24 x 24 tiles) on grids that leave
    partial tiles: the solution matches the oracle's FGMRES-DSA to FP32-cycle
    accuracy."""
    import paper_2410_08735_amd as rt
    specs = [tiny_2d(seed=21, nx=40, ny=32, quad=("cl", 8, 4, True), n_regions=3, inflow=0.2),
             tiny_2d(seed=22, nx=30, ny=26, quad=("cl", 8, 4, True), n_regions=2),
             tiny_2d(seed=23, nx=18, ny=18, quad=("cl", 12, 2, True), n_regions=2)]
    B = rt.Batch(specs)
    st, ss = B.sigma()
    opts = rt.SolveOptions(precond="dsa", m=30, max_cycles=10, sweep_dtype="f32", rtol=1e-8,
                           dsa_inner_max=1, dsa_restart=0)
    phi, stats, ret = rt.fgmres_solve(B, st, ss, B.source(), B.inflow(), opts)
    assert ret == 0
    for k, spec in enumerate(specs):
        assert stats[k]["true_relres"] <= 1e-8
        ref = _oracle_solve(spec, "dsa", rtol=1e-12)
        err = rel(B.unpack(phi)[k], ref.x)
        print(f"instance {k}: {stats[k]['iterations']} iterations, rel err {err:.2e}")
        assert err <= 1e-6, (k, err)


@pytest.mark.gpu
@pytest.mark.parametrize("precond", ["none", "dsa"])
@pytest.mark.parametrize("sweep_dtype", ["f64", "f32"])
def test_fgmres_degenerate_instances_in_one_batch(precond, sweep_dtype):
    """Degenerate instances beside an ordinary one: a zero right-hand side
    (no source, no inflow) is solved by phi = 0 with no iteration; a pure
    absorber (Sigma_s = 0) makes A~ the identity, so phi = b~ = T G~; a
    problem driven by inflow alone matches the oracle."""
    import paper_2410_08735_amd as rt
    normal = tiny_2d(seed=31, nx=9, ny=7, quad=("cl", 8, 4, True), n_regions=3)
    zero = dict(tiny_2d(seed=32, nx=6, ny=5, quad=("cl", 8, 4, True), n_regions=2))
    zero["source"] = np.zeros_like(zero["source"])
    absorber = dict(tiny_2d(seed=33, nx=7, ny=8, quad=("cl", 8, 4, True), n_regions=2))
    absorber["sigma_t"] = absorber["sigma_t"] - absorber["sigma_s"]
    absorber["sigma_s"] = np.zeros_like(absorber["sigma_s"])
    inflow_only = dict(tiny_2d(seed=34, nx=8, ny=6, quad=("cl", 8, 4, True), n_regions=2, inflow=0.5))
    inflow_only["source"] = np.zeros_like(inflow_only["source"])
    specs = [normal, zero, absorber, inflow_only]
    B = rt.Batch(specs)
    st, ss = B.sigma()
    f32 = sweep_dtype == "f32"
    opts = rt.SolveOptions(precond=precond, m=60, max_cycles=10, sweep_dtype=sweep_dtype,
                           rtol=1e-8 if f32 else 1e-13, dsa_inner_max=2000, dsa_restart=60,
                           dsa_inner_tol=1e-14)
    phi, stats, ret = rt.fgmres_solve(B, st, ss, B.source(), B.inflow(), opts)
    assert ret == 0
    out = B.unpack(phi)
    print([(s["iterations"], s["cycles"], s["true_relres"]) for s in stats])
    assert np.all(out[1] == 0.0)
    assert stats[1]["iterations"] == 0 and stats[1]["true_relres"] == 0.0
    assert stats[1]["status"] == 0
    # A~ = I: one iteration per cycle; FP32 cycles need a second, FP64-residual cycle
    assert stats[2]["status"] == 0
    assert stats[2]["iterations"] == stats[2]["cycles"] == (2 if f32 else 1), stats[2]
    b_abs = tr.b_tilde(tr.Problem(absorber))
    assert rel(out[2], b_abs) <= (1e-8 if f32 else 1e-13)
    for k in (0, 3):
        assert stats[k]["status"] == 0 and stats[k]["true_relres"] <= (1e-8 if f32 else 1e-13)
        ref = _oracle_solve(specs[k], precond, rtol=1e-13)
        assert rel(out[k], ref.x) <= (1e-6 if f32 else 1e-11), k
        if not f32:
            assert abs(stats[k]["iterations"] - ref.iterations) <= 1, (k, stats[k], ref.iterations)


@pytest.mark.gpu
def test_arnoldi_in_registers_matches_the_chunked_kernels():
    """The Arnoldi step keeps w in registers (one launch per step) for
    instances of up to 48 Ki DoFs and runs one launch per projection above
    that.  The same 110^2 instance (48,400 DoFs, the largest register tile)
    solved alone and beside a 112^2 instance (50,176 DoFs, which sends the
    whole batch to the chunked kernels) takes the same iterations and the two
    fluxes agree to rounding; the exact FP64 DSA makes the preconditioner the
    same in both batches."""
    import paper_2410_08735_amd as rt
    a = tiny_2d(seed=41, nx=110, ny=110, quad=("cl", 8, 2, True), n_regions=3, inflow=0.2)
    b = tiny_2d(seed=42, nx=112, ny=112, quad=("cl", 8, 2, True), n_regions=2)
    opts = rt.SolveOptions(precond="dsa", m=30, max_cycles=10, sweep_dtype="f64", rtol=1e-12,
                           dsa_inner_max=2000, dsa_restart=60, dsa_inner_tol=1e-14)
    out = []
    for specs in ([a], [a, b]):
        B = rt.Batch(specs)
        assert max(B.ndofs) == (48400 if len(specs) == 1 else 50176)
        st, ss = B.sigma()
        phi, stats, ret = rt.fgmres_solve(B, st, ss, B.source(), B.inflow(), opts)
        assert ret == 0 and all(s["true_relres"] <= 1e-12 for s in stats), stats
        out.append((B.unpack(phi)[0], int(stats[0]["iterations"])))
    print(f"iterations {out[0][1]} (registers) and {out[1][1]} (chunked), "
          f"flux difference {rel(out[0][0], out[1][0]):.2e}")
    assert abs(out[0][1] - out[1][1]) <= 1
    assert rel(out[0][0], out[1][0]) <= 1e-10


@pytest.mark.gpu
def test_iteration_limit_reports_not_converged():
    """Out of iterations: FGMRES (one cycle of 3) and SI (2 iterations) return
    the not-converged warning, per instance and as the call's status, with the
    iterate reached and its true residual: GMRES(3) after one cycle equals the
    oracle's, and the reported residual is that of the returned phi."""
    import paper_2410_08735_amd as rt
    from paper_2410_08735_amd import _lib
    specs = [tiny_2d(seed=51, nx=7, ny=6, quad=("cl", 8, 4, True), n_regions=3),
             tiny_2d(seed=52, nx=5, ny=8, quad=("cl", 6, 2, False), n_regions=2, inflow=0.3)]
    B = rt.Batch(specs)
    st, ss = B.sigma()
    common = dict(sweep_dtype="f64", rtol=1e-12, dsa_inner_max=2000, dsa_restart=60, dsa_inner_tol=1e-14)
    for solver, opts in (("fgmres", rt.SolveOptions(precond="none", m=3, max_cycles=1, **common)),
                         ("si", rt.SolveOptions(precond="dsa", max_cycles=2, **common))):
        fn = rt.fgmres_solve if solver == "fgmres" else rt.si_solve
        phi, stats, ret = fn(B, st, ss, B.source(), B.inflow(), opts)
        assert ret == _lib.RTE_WNOTCONV, solver
        out = B.unpack(phi)
        for k, spec in enumerate(specs):
            assert stats[k]["status"] == _lib.RTE_WNOTCONV, (solver, k, stats[k])
            assert stats[k]["iterations"] == (3 if solver == "fgmres" else 2), (solver, k, stats[k])
            P = tr.Problem(spec)
            b = tr.b_tilde(P)
            res = np.linalg.norm(b - tr.A_tilde_apply(P, out[k])) / np.linalg.norm(b)
            assert res > 1e-12
            assert abs(stats[k]["true_relres"] - res) <= 1e-9 * res, (solver, k, stats[k], res)
            if solver == "fgmres":
                ref = ofg.fgmres(lambda x: tr.A_tilde_apply(P, x), b, lambda j, v: v, m=3, rtol=1e-12,
                                 max_cycles=1)
                assert rel(out[k], ref.x) <= 1e-11, k


@pytest.mark.gpu
def test_cfg1_gmres30_dsa():
    """Slab, 128 P1 cells, S16, GMRES(30)-DSA to 1e-8 (FP64)."""
    import paper_2410_08735_amd as rt
    spec = cfg1()
    B = rt.Batch([spec])
    st, ss = B.sigma()
    opts = rt.SolveOptions(precond="dsa", m=30, max_cycles=10, sweep_dtype="f64", rtol=1e-8,
                           dsa_inner_max=500, dsa_restart=60, dsa_inner_tol=1e-13)
    phi, stats, ret = rt.fgmres_solve(B, st, ss, B.source(), None, opts)
    assert ret == 0 and stats[0]["true_relres"] <= 1e-8
    ref = _oracle_solve(spec, "dsa", rtol=1e-8, m=30)
    assert abs(stats[0]["iterations"] - ref.iterations) <= 1
    tight = _oracle_solve(spec, "dsa", rtol=1e-13, m=30)
    assert rel(B.unpack(phi)[0], tight.x) <= 1e-6


# ------------------------------------------------------------------ ROMSAD
@pytest.fixture(scope="module")
def oracle_rom():
    specs = _family(5)
    U, rep = orom.greedy(specs, window=2, eps_rom=0.0, n_giter=3, rtol_hf=1e-11)
    return specs, U, rep


@pytest.mark.gpu
def test_romsad_apply_and_affine_terms_parity(oracle_rom):
    import torch

    import paper_2410_08735_amd as rt
    specs, U, _ = oracle_rom
    B = rt.Batch(specs)
    st, ss = B.sigma()
    rom = rt.Rom.from_basis(B, torch.from_numpy(U.reshape(-1)).cuda())
    assert rom.rank == U.shape[0]
    P0 = tr.Problem(specs[0])
    ex = rom.export(P0.nord, P0.ndof, 2)
    AD, G, S = orom.affine_terms(P0, U, 2)
    assert rel(ex["AD"], AD) <= 1e-12 and rel(ex["G"], G) <= 1e-12 and rel(ex["S"], S) <= 1e-12
    assert rel(ex["W1"], orom.W1(U)) <= 1e-14 and rel(ex["Ww"], orom.Ww(P0, U)) <= 1e-14
    rng = np.random.default_rng(3)
    v = [rng.standard_normal(n) for n in B.ndofs]
    z = B.unpack(rt.romsad_apply(rom, B, st, ss, B.pack(v)))
    for k, spec in enumerate(specs):
        P = tr.Problem(spec)
        ref = v[k] + orom.rom_correction(P, U, v[k])
        assert rel(z[k], ref) <= 1e-12


@pytest.mark.gpu
def test_romsad_apply_parity_many_instances_long_vectors():
    """One ROM of rank > 16 for a batch of 21 instances (two groups of 16 on the
    matrix-core projection, the second partial) on a 20 x 15 grid (1,200 DoFs:
    five 256-DoF chunks, the last ragged), against the oracle's ROM correction."""
    import torch

    import paper_2410_08735_amd as rt
    specs = _family(9, nx=20, ny=15)
    U, _ = orom.greedy(specs, window=2, eps_rom=0.0, n_giter=9, rtol_hf=1e-11)
    assert U.shape[0] > 16  # two rank-column blocks
    test = _family(21, nx=20, ny=15, seed=0)
    B = rt.Batch(test)
    st, ss = B.sigma()
    rom = rt.Rom.from_basis(B, torch.from_numpy(U.reshape(-1)).cuda())
    rng = np.random.default_rng(11)
    v = [rng.standard_normal(n) for n in B.ndofs]
    z = B.unpack(rt.romsad_apply(rom, B, st, ss, B.pack(v)))
    for k in (0, 7, 15, 16, 20):
        P = tr.Problem(test[k])
        ref = v[k] + orom.rom_correction(P, U, v[k])
        assert rel(z[k], ref) <= 1e-12, (k, rel(z[k], ref))


@pytest.mark.gpu
@pytest.mark.parametrize("dsa_variant", ["fc", "pc"])
def test_fgmres_romsad_parity(oracle_rom, dsa_variant):
    """FGMRES-ROMSAD with FC-DSA, and with PC-DSA after the window (the
    FGMRES-PC-ROMSAD of the variable-scattering comparison)."""
    import torch

    import paper_2410_08735_amd as rt
    specs, U, rep = oracle_rom
    test = _family(6, seed=0)[5:] + [dict(_family(5)[1], sigma_s=_family(5)[1]["sigma_s"] * 1.1,
                                          sigma_t=_family(5)[1]["sigma_t"] * 1.1)]
    B = rt.Batch(test + [specs[rep.sampled[1]]])
    st, ss = B.sigma()
    rom = rt.Rom.from_basis(B, torch.from_numpy(U.reshape(-1)).cuda())
    opts = rt.SolveOptions(precond="romsad", m=40, max_cycles=5, sweep_dtype="f64", rtol=1e-12,
                           window=2, dsa_inner_max=2000, dsa_restart=60, dsa_inner_tol=1e-14,
                           dsa_variant=dsa_variant)
    phi, stats, ret = rt.fgmres_solve(B, st, ss, B.source(), None, opts, rom=rom)
    assert ret == 0
    for k, spec in enumerate(B.problems):
        ref = _oracle_solve(spec, "romsad", rtol=1e-12, U=U, dsa_variant=dsa_variant)
        assert rel(B.unpack(phi)[k], ref.x) <= 1e-10
        assert abs(stats[k]["iterations"] - ref.iterations) <= 1
        assert stats[k]["pc_rom"] >= 1
    assert stats[-1]["iterations"] == 1   # sampled parameter: the ROM is exact


@pytest.fixture(scope="module")
def oracle_rom_pair():
    """Two geometries (grid and quadrature), each with its own oracle greedy ROM."""
    fa = _family(4)
    fb = _family(4, nx=6, ny=6, quad=("cl", 4, 4, True), seed=2)
    Ua, _ = orom.greedy(fa, window=2, eps_rom=0.0, n_giter=2, rtol_hf=1e-11)
    Ub, _ = orom.greedy(fb, window=2, eps_rom=0.0, n_giter=3, rtol_hf=1e-11)
    return fa, fb, Ua, Ub


@pytest.mark.gpu
def test_rom_set_on_uneven_batch(oracle_rom_pair):
    """One batch mixing both geometries: romsad_apply and FGMRES-ROMSAD with a
    ROM set equal the oracle with each instance's own ROM."""
    import torch

    import paper_2410_08735_amd as rt
    fa, fb, Ua, Ub = oracle_rom_pair
    roma = rt.Rom.from_basis(rt.Batch(fa[:1]), torch.from_numpy(Ua.reshape(-1)).cuda())
    romb = rt.Rom.from_basis(rt.Batch(fb[:1]), torch.from_numpy(Ub.reshape(-1)).cuda())
    scale = lambda sp, f: dict(sp, sigma_s=sp["sigma_s"] * f, sigma_t=sp["sigma_t"] * f)
    mixed = [scale(fb[1], 1.2), scale(fa[2], 0.9), fa[0], scale(fb[3], 1.05), scale(fa[1], 1.1)]
    which = [1, 0, 0, 1, 0]
    B = rt.Batch(mixed)
    st, ss = B.sigma()
    rs = rt.Rom.set(B, [roma, romb], which)
    assert rs.rank == max(Ua.shape[0], Ub.shape[0])
    with pytest.raises(rt.RteError):
        rt.Rom.set(B, [roma, romb], [0, 0, 0, 1, 0])  # instance 0 is not on grid a
    Us = [Ua, Ub]
    rng = np.random.default_rng(8)
    v = [rng.standard_normal(n) for n in B.ndofs]
    z = B.unpack(rt.romsad_apply(rs, B, st, ss, B.pack(v)))
    for k, spec in enumerate(mixed):
        P = tr.Problem(spec)
        assert rel(z[k], v[k] + orom.rom_correction(P, Us[which[k]], v[k])) <= 1e-12, k
    opts = rt.SolveOptions(precond="romsad", m=40, max_cycles=5, sweep_dtype="f64", rtol=1e-12,
                           window=2, dsa_inner_max=2000, dsa_restart=60, dsa_inner_tol=1e-14)
    phi, stats, ret = rt.fgmres_solve(B, st, ss, B.source(), None, opts, rom=rs)
    assert ret == 0
    for k, spec in enumerate(mixed):
        ref = _oracle_solve(spec, "romsad", rtol=1e-12, U=Us[which[k]])
        assert rel(B.unpack(phi)[k], ref.x) <= 1e-10, k
        assert abs(stats[k]["iterations"] - ref.iterations) <= 1, (k, stats[k], ref.iterations)
    assert stats[2]["iterations"] == 1   # fa[0] was sampled by its greedy: the ROM is exact


@pytest.mark.gpu
def test_greedy_matches_oracle(oracle_rom, tmp_path):
    import paper_2410_08735_amd as rt
    specs, U, rep = oracle_rom
    B = rt.Batch(specs)
    st, ss = B.sigma()
    rom, grep = rt.romsad_build_greedy(B, st, ss, B.source(), None, window=2, mu1_index=0,
                                       eps_rom=0.0, n_giter=3, eps_qr=1e-13, hf_rtol=1e-11,
                                       hf_dsa_tol=1e-13)
    assert grep["sampled"] == rep.sampled, (grep, rep.sampled)
    assert grep["rank"] == U.shape[0]
    # same span: M_ROM^{-1} v agrees (invariant under U -> U Q)
    rng = np.random.default_rng(8)
    v = [rng.standard_normal(n) for n in B.ndofs]
    z = B.unpack(rt.romsad_apply(rom, B, st, ss, B.pack(v)))
    for k, spec in enumerate(specs):
        ref = v[k] + orom.rom_correction(tr.Problem(spec), U, v[k])
        assert rel(z[k], ref) <= 1e-7, rel(z[k], ref)
    # save / load round trip
    path = str(tmp_path / "rom.bin")
    rom.save(path)
    rom2 = rt.Rom.load(path)
    z2 = B.unpack(rt.romsad_apply(rom2, B, st, ss, B.pack(v)))
    for k in range(len(specs)):
        assert np.array_equal(z[k], z2[k])


@pytest.mark.gpu
@pytest.mark.timeout(420)
def test_full_size_checkerboard_romsad_sampled():
    """The benchmark's workload at full size (96^2 cells, 128 ordinates, 256 test
    parameters, greedy ROM from 64 training parameters, FP32 sweeps, one
    V-cycle per DSA, ROM window in the first cycle only): every instance
    reaches true relative residual 1e-8, for a sampled instance the oracle's
    own operator confirms the residual of the returned flux, and two
    instances' fluxes match the oracle's FGMRES-DSA solutions (rtol 1e-11,
    solved in processes of their own beside the GPU work) to 1e-6."""
    import paper_2410_08735_amd as rt
    from oracle_refs import OracleRefs
    from synth import cfg3_problem, cfg3_train_test
    tr_mu, te_mu = cfg3_train_test()
    refs = OracleRefs([cfg3_problem(te_mu[k]) for k in (7, 200)], 1e-11)
    Btr = rt.Batch([cfg3_problem(m) for m in tr_mu])
    st, ss = Btr.sigma()
    rom, rep = rt.romsad_build_greedy(Btr, st, ss, Btr.source(), None, window=2, n_giter=16)
    assert rep["rank"] == 32 and rep["sampled"][0] == 0
    del Btr, st, ss
    specs = [cfg3_problem(m) for m in te_mu]
    B = rt.Batch(specs)
    st, ss = B.sigma()
    opts = rt.SolveOptions(precond="romsad", m=30, max_cycles=10, sweep_dtype="f32", rtol=1e-8, window=2,
                           dsa_inner_max=1, dsa_restart=0, window_cycles=1)
    phi, stats, ret = rt.fgmres_solve(B, st, ss, B.source(), None, opts, rom=rom)
    assert ret == 0
    assert all(s["true_relres"] <= 1e-8 for s in stats)
    k = 131
    P = tr.Problem(specs[k])
    b = tr.b_tilde(P)
    r = b - tr.A_tilde_apply(P, B.unpack(phi)[k])
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1.05e-8
    for k, (x, rr) in zip((7, 200), refs.get()):
        assert rr <= 1e-11
        err = rel(B.unpack(phi)[k], x)
        print(f"instance {k}: rel err vs oracle {err:.2e}")
        assert err <= 1e-6, (k, err)


@pytest.mark.gpu
def test_graph_replayed_operator_matches_eager():
    """FGMRES with the operator application captured in HIP graphs: two solves
    in a row (the second only replays) and eager work in between give results
    bitwise equal to the eager solve."""
    import torch

    import paper_2410_08735_amd as rt
    specs = _family(3, nx=9, ny=7)
    B = rt.Batch(specs)
    st, ss = B.sigma()
    common = dict(precond="dsa", m=20, max_cycles=6, sweep_dtype="f32", rtol=1e-9, dsa_inner_max=1,
                  dsa_restart=0)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        G = B.source()
        eager, st_e, _ = rt.fgmres_solve(B, st, ss, G, None, rt.SolveOptions(**common))
        g1, st_1, _ = rt.fgmres_solve(B, st, ss, G, None, rt.SolveOptions(use_graph=True, **common))
        junk = rt.apply_A(B, st, ss, G)  # eager work between the replays
        g2, st_2, _ = rt.fgmres_solve(B, st, ss, G, None, rt.SolveOptions(use_graph=True, **common))
    side.synchronize()
    assert bool((eager == g1).all()) and bool((eager == g2).all())
    assert [s["iterations"] for s in st_e] == [s["iterations"] for s in st_2]
    assert all(s["true_relres"] <= 1e-9 for s in st_2)
    del junk
    # on the null stream the option falls back to eager launches
    g0, _, _ = rt.fgmres_solve(B, st, ss, B.source(), None, rt.SolveOptions(use_graph=True, **common))
    assert bool((g0 == eager).all())


@pytest.mark.gpu
@pytest.mark.timeout(420)
def test_pincell_problem_reproduces_the_papers_sweep_counts():
    """Section 5.2 as specified (80^2, CL(30,6), 5 x 5 training grid, mu_1 at its
    centre, window 2, eps_ROM 1e-10, rtol 1e-11, exact-solve DSA): the average
    sweep counts of GMRES-DSA and FGMRES-ROMSAD on 10 fresh parameters are
    close to the paper's table (differences in the discretisation details and
    the random test draws allow some slack)."""
    import json

    import paper_2410_08735_amd as rt
    from oracle_refs import OracleRefs
    from synth import pincell_problem, pincell_sets
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "pincell_online.json")))
    tr_mu, te_mu = pincell_sets()
    refs = OracleRefs([pincell_problem(te_mu[0])], gold["rtol"])
    Btr = rt.Batch([pincell_problem(m) for m in tr_mu])
    st, ss = Btr.sigma()
    h = 2.0 / 80  # the paper's eps_ROM refers to a basis sqrt(h_x h_y) times the orthonormal one
    rom, rep = rt.romsad_build_greedy(Btr, st, ss, Btr.source(), None, window=gold["window"], mu1_index=0,
                                      eps_rom=gold["eps_rom"] / h, n_giter=25, hf_rtol=1e-11, hf_dsa_tol=1e-12)
    # the printed tolerance taken literally in this library's orthonormal basis
    _, rep_lit = rt.romsad_build_greedy(Btr, st, ss, Btr.source(), None, window=gold["window"], mu1_index=0,
                                        eps_rom=gold["eps_rom"], n_giter=25, hf_rtol=1e-11, hf_dsa_tol=1e-12)
    del Btr, st, ss
    print(f"pin-cell greedy: eps_ROM / h samples {len(rep['sampled'])} (rank {rep['rank']}), "
          f"eps_ROM literal samples {len(rep_lit['sampled'])} (rank {rep_lit['rank']})")
    assert len(rep_lit["sampled"]) >= len(rep["sampled"])
    assert abs(len(rep["sampled"]) - gold["greedy_sampled"]) <= 1, rep["sampled"]
    assert rep["rank"] == 2 * len(rep["sampled"]) - rep["truncated"]
    B = rt.Batch([pincell_problem(m) for m in te_mu])
    st, ss = B.sigma()
    common = dict(m=60, max_cycles=10, sweep_dtype="f64", rtol=gold["rtol"], window=gold["window"],
                  dsa_inner_max=1000, dsa_restart=60, dsa_inner_tol=1e-12)
    n = {}
    for pc, kw in (("dsa", {}), ("romsad", dict(rom=rom))):
        phi, stats, ret = rt.fgmres_solve(B, st, ss, B.source(), None, rt.SolveOptions(precond=pc, **common), **kw)
        assert ret == 0 and all(s["true_relres"] <= gold["rtol"] for s in stats)
        n[pc] = 1 + np.mean([s["iterations"] for s in stats])
    assert abs(n["dsa"] - gold["gmres_dsa_nsweep"]) <= 1.5, n
    assert abs(n["romsad"] - gold["fgmres_romsad_nsweep"]) <= 1.0, n
    # the first test parameter's FGMRES-ROMSAD flux against the oracle's solution
    (x, rr), = refs.get()
    err = rel(B.unpack(phi)[0], x)
    print(f"pin-cell test parameter 0: rel err vs oracle {err:.2e}")
    assert rr <= gold["rtol"] and err <= 1e-8, err


@pytest.mark.gpu
@pytest.mark.parametrize("precond", ["none", "dsa", "pc-dsa", "romsad"])
def test_si_solve_parity(oracle_rom, precond):
    """Source iteration with synthetic acceleration against the oracle's SI
    (FC-DSA, PC-DSA, ROMSAD)."""
    import torch

    from oracle import si as osi

    import paper_2410_08735_amd as rt
    specs, U, _ = oracle_rom
    test = [dict(s, sigma_s=s["sigma_s"] * f, sigma_t=s["sigma_t"] * f) for s, f in zip(specs[:3], (1.0, 1.1, 0.8))]
    B = rt.Batch(test)
    st, ss = B.sigma()
    rom = rt.Rom.from_basis(B, torch.from_numpy(U.reshape(-1)).cuda()) if precond == "romsad" else None
    opts = rt.SolveOptions(precond="dsa" if precond == "pc-dsa" else precond, max_cycles=400,
                           sweep_dtype="f64", rtol=1e-11, window=1, dsa_inner_max=2000, dsa_restart=60,
                           dsa_inner_tol=1e-14, dsa_variant="pc" if precond == "pc-dsa" else "fc")
    phi, stats, ret = rt.si_solve(B, st, ss, B.source(), None, opts, rom=rom)
    assert ret == 0
    for k, spec in enumerate(test):
        P = tr.Problem(spec)
        D = odsa.DSA(P, "pc" if precond == "pc-dsa" else "fc")
        if precond == "none":
            pc = lambda l, r: r
        elif precond in ("dsa", "pc-dsa"):
            pc = lambda l, r: D.apply(r)
        else:
            R = orom.Romsad(P, U, D, 1)
            pc = lambda l, r: R(l, r)
        ref = osi.si(lambda x: tr.A_tilde_apply(P, x), tr.b_tilde(P), pc, rtol=1e-11, max_iter=400)
        assert ref.converged
        assert abs(stats[k]["iterations"] - ref.iterations) <= 1, (k, stats[k]["iterations"], ref.iterations)
        assert rel(B.unpack(phi)[k], ref.x) <= 1e-9
        assert stats[k]["true_relres"] <= 1e-11
        if precond != "none":
            assert stats[k]["pc_dsa"] + stats[k]["pc_rom"] == stats[k]["iterations"]


@pytest.mark.gpu
def test_zero_right_hand_side_beside_an_ordinary_instance_romsad_and_si(oracle_rom):
    """A zero right-hand side in a batch with an ordinary instance: FGMRES-ROMSAD
    and source iteration (DSA, ROMSAD) return phi = 0 for it with no iteration
    and solve the other as the oracle does."""
    import torch

    from oracle import si as osi

    import paper_2410_08735_amd as rt
    specs, U, _ = oracle_rom
    zero = dict(specs[1], source=np.zeros_like(specs[1]["source"]))
    test = [specs[0], zero]
    B = rt.Batch(test)
    st, ss = B.sigma()
    rom = rt.Rom.from_basis(B, torch.from_numpy(U.reshape(-1)).cuda())
    P = tr.Problem(specs[0])
    D = odsa.DSA(P)
    common = dict(sweep_dtype="f64", rtol=1e-11, dsa_inner_max=2000, dsa_restart=60, dsa_inner_tol=1e-14)
    runs = [("fgmres", "romsad", rt.SolveOptions(precond="romsad", m=60, max_cycles=5, window=2, **common)),
            ("si", "dsa", rt.SolveOptions(precond="dsa", max_cycles=400, **common)),
            ("si", "romsad", rt.SolveOptions(precond="romsad", max_cycles=400, window=1, **common))]
    for solver, precond, opts in runs:
        fn = rt.fgmres_solve if solver == "fgmres" else rt.si_solve
        phi, stats, ret = fn(B, st, ss, B.source(), None, opts, rom=rom if precond == "romsad" else None)
        assert ret == 0, (solver, precond)
        out = B.unpack(phi)
        assert np.all(out[1] == 0.0), (solver, precond)
        assert stats[1]["iterations"] == 0 and stats[1]["status"] == 0, (solver, precond, stats[1])
        assert stats[0]["status"] == 0 and stats[0]["true_relres"] <= 1e-11, (solver, precond, stats[0])
        if solver == "fgmres":
            ref = _oracle_solve(specs[0], "romsad", rtol=1e-11, U=U, window=2)
        else:
            pc = (lambda l, r: D.apply(r)) if precond == "dsa" else orom.Romsad(P, U, D, 1)
            ref = osi.si(lambda x: tr.A_tilde_apply(P, x), tr.b_tilde(P), pc, rtol=1e-11, max_iter=400)
        assert abs(stats[0]["iterations"] - ref.iterations) <= 1, (solver, precond, stats[0], ref.iterations)
        assert rel(out[0], ref.x) <= 1e-9, (solver, precond)


@pytest.mark.gpu
def test_pincell_fgmres_si_comparison_matches_the_paper():
    """Section 5.2's FGMRES / SI comparison (window 1, eps_ROM 1e-7, hardest test
    parameter): the sampled count, the relative residual after the first
    correction of all four solvers, and the sweep counts of GMRES-DSA, SI-DSA
    and FGMRES-ROMSAD agree with the paper's table.  (The paper reports SI-
    ROMSAD stagnating; here it converges, which is not asserted either way.)"""
    import json

    import paper_2410_08735_amd as rt
    from synth import pincell_problem, pincell_sets
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "pincell_compare.json")))
    tr_mu, _ = pincell_sets()
    Btr = rt.Batch([pincell_problem(m) for m in tr_mu])
    st, ss = Btr.sigma()
    h = 2.0 / 80
    rom, rep = rt.romsad_build_greedy(Btr, st, ss, Btr.source(), None, window=1, mu1_index=0,
                                      eps_rom=gold["eps_rom"] / h, n_giter=25, hf_rtol=1e-11, hf_dsa_tol=1e-12)
    del Btr, st, ss
    assert len(rep["sampled"]) == gold["greedy_sampled"] and rep["rank"] == gold["rom_dimension"]
    B = rt.Batch([pincell_problem(gold["mu"])])
    st, ss = B.sigma()
    base = dict(m=60, max_cycles=10, sweep_dtype="f64", rtol=1e-11, window=1, dsa_inner_max=1000, dsa_restart=60,
                dsa_inner_tol=1e-12)
    got = {}
    for name, solver, pc, kw in (("gmres_dsa", rt.fgmres_solve, "dsa", {}), ("si_dsa", rt.si_solve, "dsa", {}),
                                 ("fgmres_romsad", rt.fgmres_solve, "romsad", dict(rom=rom)),
                                 ("si_romsad", rt.si_solve, "romsad", dict(rom=rom))):
        _, s1, _ = solver(B, st, ss, B.source(), None, rt.SolveOptions(precond=pc, **dict(base, m=1, max_cycles=1)),
                          **kw)
        ref = gold["relres_after_first_correction"][name]
        assert abs(s1[0]["true_relres"] / ref - 1.0) <= 0.05, (name, s1[0]["true_relres"], ref)
        if name != "si_romsad":
            full = dict(base, max_cycles=100) if solver is rt.si_solve else base
            _, s, _ = solver(B, st, ss, B.source(), None, rt.SolveOptions(precond=pc, **full), **kw)
            got[name] = 1 + s[0]["iterations"]
            assert s[0]["true_relres"] <= 1e-11
    for name, tol in (("gmres_dsa", 1), ("si_dsa", 3), ("fgmres_romsad", 1)):
        assert abs(got[name] - gold["n_sweep"][name]) <= tol, (name, got[name])


@pytest.mark.gpu
def test_two_material_problem_reproduces_the_papers_table():
    """Section 5.4 (left-side parametric inflow, 64^2, CL(60,6), 9 x 11 training
    grid): greedy sample count and rank, and average sweep counts near the table."""
    import json

    import paper_2410_08735_amd as rt
    from synth import twomat_problem, twomat_sets
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "twomat_online.json")))
    tr_mu, te_mu = twomat_sets()
    Btr = rt.Batch([twomat_problem(m) for m in tr_mu])
    st, ss = Btr.sigma()
    h = 2.0 / 64
    rom, rep = rt.romsad_build_greedy(Btr, st, ss, Btr.source(), Btr.inflow(), window=gold["window"], mu1_index=0,
                                      eps_rom=gold["eps_rom"] / h, n_giter=32, hf_rtol=1e-11, hf_dsa_tol=1e-12)
    # the printed tolerance taken literally in this library's orthonormal basis
    # (an empirical check of the basis-scaling reading: it samples more)
    _, rep_lit = rt.romsad_build_greedy(Btr, st, ss, Btr.source(), Btr.inflow(), window=gold["window"],
                                        mu1_index=0, eps_rom=gold["eps_rom"], n_giter=32, hf_rtol=1e-11,
                                        hf_dsa_tol=1e-12)
    del Btr, st, ss
    print(f"two-material greedy: eps_ROM / h samples {len(rep['sampled'])} (rank {rep['rank']}), "
          f"eps_ROM literal samples {len(rep_lit['sampled'])} (rank {rep_lit['rank']})")
    assert len(rep["sampled"]) == gold["greedy_sampled"] and rep["rank"] == gold["rom_dimension"]
    assert len(rep_lit["sampled"]) >= len(rep["sampled"])
    B = rt.Batch([twomat_problem(m) for m in te_mu])
    st, ss = B.sigma()
    common = dict(m=60, max_cycles=10, sweep_dtype="f64", rtol=gold["rtol"], window=gold["window"],
                  dsa_inner_max=1000, dsa_restart=60, dsa_inner_tol=1e-12)
    n = {}
    for pc, kw in (("dsa", {}), ("romsad", dict(rom=rom))):
        _, stats, ret = rt.fgmres_solve(B, st, ss, B.source(), B.inflow(), rt.SolveOptions(precond=pc, **common),
                                        **kw)
        assert ret == 0 and all(s["true_relres"] <= gold["rtol"] for s in stats)
        n[pc] = 1 + np.mean([s["iterations"] for s in stats])
    assert abs(n["dsa"] - gold["gmres_dsa_nsweep"]) <= 1.0, n
    assert abs(n["romsad"] - gold["fgmres_romsad_nsweep"]) <= 1.0, n
