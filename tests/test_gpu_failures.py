"""Failure conventions of the solvers (per-instance statuses, the DSA fallback of
a singular reduced operator, validation of the cross sections), GMRES(1), the
GPU Adam step against the oracle's, and the recapture of cached operator
graphs after the sweep plan changes.  Every failure is forced from the host
with ordinary inputs; no kernel is made to fault."""
import numpy as np
import pytest

from oracle import dsa as odsa
from oracle import fgmres as ofg
from oracle import mlp as omlp
from oracle import rom as orom
from oracle import transport as tr
from synth import tiny_2d


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


def _exact(spec):
    P = tr.Problem(spec)
    return np.linalg.solve(tr.dense_A_tilde(P), tr.b_tilde(P))


def _dsa_opts(rt, **kw):
    base = dict(precond="dsa", m=40, max_cycles=4, sweep_dtype="f64", rtol=1e-12, dsa_inner_max=2000,
                dsa_restart=60, dsa_inner_tol=1e-14)
    base.update(kw)
    return rt.SolveOptions(**base)


@pytest.mark.gpu
def test_nan_source_stops_only_its_instance():
    """A NaN in one instance's source gives that instance RTE_ENONFINITE and no
    iteration; the other instance of the batch solves as on its own."""
    import torch

    import paper_2410_08735_amd as rt
    specs = [tiny_2d(seed=1, nx=6, ny=5, quad=("cl", 8, 4, True), n_regions=2),
             tiny_2d(seed=2, nx=5, ny=5, quad=("cl", 8, 4, True), n_regions=2)]
    B = rt.Batch(specs)
    st, ss = B.sigma()
    G = B.source()
    G[B.offsets[1] + 7] = float("nan")
    print("case: NaN in the source of instance 1 of 2, FGMRES-DSA FP64", flush=True)
    phi, stats, ret = rt.fgmres_solve(B, st, ss, G, None, _dsa_opts(rt))
    assert ret == 1  # RTE_WNOTCONV: outputs and statistics written
    assert stats[1]["status"] == rt._lib.RTE_ENONFINITE and stats[1]["iterations"] == 0
    assert stats[0]["status"] == 0 and stats[0]["true_relres"] <= 1e-12
    assert rel(B.unpack(phi)[0], _exact(specs[0])) <= 1e-10
    del torch


@pytest.mark.gpu
def test_invalid_cross_sections_rejected():
    """Out-of-range cross sections give RTE_EINVAL: checked on the host by a
    call that tunes the sweep plans (the first, on a fresh batch), and by a
    kernel once the plans are tuned."""
    import paper_2410_08735_amd as rt
    specs = [tiny_2d(seed=1, nx=4, ny=4, quad=("cl", 8, 4, True), n_regions=2)]
    B = rt.Batch(specs)
    st, ss = B.sigma()
    t = st.clone()
    t[0, 1] = -1.0
    with pytest.raises(rt.RteError) as e:  # host check (untuned plans)
        rt.fgmres_solve(B, t, ss, B.source(), None, _dsa_opts(rt))
    assert e.value.status == rt._lib.RTE_EINVAL
    _, stats, ret = rt.fgmres_solve(B, st, ss, B.source(), None, _dsa_opts(rt))  # tunes the plans
    assert ret == 0 and B.sweep_plan("f64")["tuned"]
    for bad_t, bad_s in ((0.0, None), (-1.0, None), (float("nan"), None), (None, -0.5), (None, float("inf"))):
        t, s = st.clone(), ss.clone()
        if bad_t is not None:
            t[0, 1] = bad_t
        if bad_s is not None:
            s[0, 0] = bad_s
        with pytest.raises(rt.RteError) as e:
            rt.fgmres_solve(B, t, s, B.source(), None, _dsa_opts(rt))
        assert e.value.status == rt._lib.RTE_EINVAL
        with pytest.raises(rt.RteError):
            rt.si_solve(B, t, s, B.source(), None, _dsa_opts(rt))


@pytest.mark.gpu
def test_singular_reduced_operator_falls_back_to_dsa():
    """A basis whose two columns are equal makes U^T A(mu) U singular for every
    mu: FGMRES-ROMSAD flags it and runs DSA wherever it would run the ROM
    solve, so it reproduces GMRES-DSA exactly."""
    import torch

    import paper_2410_08735_amd as rt
    specs = [tiny_2d(seed=3, nx=5, ny=4, quad=("cl", 8, 4, True), n_regions=2),
             tiny_2d(seed=4, nx=5, ny=4, quad=("cl", 8, 4, True), n_regions=2)]
    specs[1]["region"] = specs[0]["region"]
    B = rt.Batch(specs)
    st, ss = B.sigma()
    P = tr.Problem(specs[0])
    rng = np.random.default_rng(9)
    u = rng.standard_normal(P.nord * P.ndof)
    u /= np.linalg.norm(u)
    U = np.stack([u, u])
    rom = rt.Rom.from_basis(B, torch.from_numpy(U.reshape(-1)).cuda())
    print("case: duplicated-column basis, FGMRES-ROMSAD FP64 vs GMRES-DSA", flush=True)
    phi_r, s_r, ret_r = rt.fgmres_solve(B, st, ss, B.source(), None, _dsa_opts(rt, precond="romsad", window=2),
                                        rom=rom)
    phi_d, s_d, ret_d = rt.fgmres_solve(B, st, ss, B.source(), None, _dsa_opts(rt))
    assert ret_r == 0 and ret_d == 0
    for k in range(2):
        assert s_r[k]["rom_singular"] == 1 and s_r[k]["pc_rom"] == 0, s_r[k]
        assert s_r[k]["pc_dsa"] == s_r[k]["iterations"] == s_d[k]["iterations"]
        assert rel(B.unpack(phi_r)[k], B.unpack(phi_d)[k]) <= 1e-14
        assert rel(B.unpack(phi_r)[k], _exact(specs[k])) <= 1e-10
    # the standalone operator reports the singular reduced operator
    with pytest.raises(rt.RteError) as e:
        rt.romsad_apply(rom, B, st, ss, B.source())
    assert e.value.status == rt._lib.RTE_ESINGULAR


@pytest.mark.gpu
def test_unhappy_breakdown_stops_the_instance():
    """With the breakdown threshold at 1.5 ||H(:, j)|| every first Arnoldi step
    counts as a breakdown whose rotated diagonal is not above the threshold: the
    singular column is dropped, phi stays at the initial guess (zero) and the
    status is RTE_EBREAKDOWN."""
    import paper_2410_08735_amd as rt
    specs = [tiny_2d(seed=5, nx=4, ny=5, quad=("cl", 8, 4, True), n_regions=2)]
    B = rt.Batch(specs)
    st, ss = B.sigma()
    print("case: breakdown threshold 1.5, FGMRES-DSA FP64", flush=True)
    phi, stats, ret = rt.fgmres_solve(B, st, ss, B.source(), None, _dsa_opts(rt, breakdown_tol=1.5))
    assert ret == 1
    s = stats[0]
    assert s["status"] == rt._lib.RTE_EBREAKDOWN and s["iterations"] == 1 and s["cycles"] == 1, s
    assert float(phi.abs().max()) == 0.0
    assert abs(s["true_relres"] - 1.0) <= 1e-12


@pytest.mark.gpu
def test_gmres1_restarted_matches_oracle():
    """m = 1: every cycle is one preconditioned step from the true residual."""
    import paper_2410_08735_amd as rt
    specs = [tiny_2d(seed=6, nx=5, ny=4, quad=("cl", 8, 4, True), n_regions=2),
             tiny_2d(seed=7, nx=3, ny=6, quad=("cl", 6, 2, False), n_regions=3)]
    B = rt.Batch(specs)
    st, ss = B.sigma()
    print("case: GMRES(1)-DSA FP64, 2 instances", flush=True)
    phi, stats, ret = rt.fgmres_solve(B, st, ss, B.source(), None, _dsa_opts(rt, m=1, max_cycles=60, rtol=1e-11))
    assert ret == 0
    for k, spec in enumerate(specs):
        P = tr.Problem(spec)
        D = odsa.DSA(P)
        ref = ofg.fgmres(lambda x: tr.A_tilde_apply(P, x), tr.b_tilde(P), lambda j, v: D.apply(v), m=1,
                         rtol=1e-11, max_cycles=60)
        assert ref.converged
        assert stats[k]["iterations"] == stats[k]["cycles"]
        assert abs(stats[k]["iterations"] - ref.iterations) <= 1, (stats[k], ref.iterations)
        assert rel(B.unpack(phi)[k], ref.x) <= 1e-9


def _flat(params):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params])


@pytest.mark.gpu
def test_adam_step_matches_oracle():
    """Two GPU Adam steps on oracle gradients (FP64 backward of the oracle's
    network, rounded to FP32) against the oracle's Adam on the same gradients."""
    import torch

    import paper_2410_08735_amd as rt
    rng = np.random.default_rng(21)
    sizes = [36, 64, 64, 32]
    params = omlp.init(sizes, rng)
    for W, b in params:
        b[:] = 0.1 * rng.standard_normal(b.shape)
    p64 = [[W.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)] for W, b in params]
    m = rt.Mlp(36, 64, 2, 32)
    m.set_params(_flat(p64).astype(np.float32))
    ref = [[W.copy(), b.copy()] for W, b in p64]
    state = {}
    start = _flat(p64)
    for step in range(2):
        X = rng.standard_normal((50, 36))
        Y = rng.standard_normal((50, 32))
        out, cache = omlp.forward(ref, X)
        g = omlp.backward(ref, cache, out, Y)
        gf = _flat(g).astype(np.float32)
        g32 = [[gw.astype(np.float32).astype(np.float64), gb.astype(np.float32).astype(np.float64)]
               for gw, gb in g]
        omlp.adam_step(ref, g32, state, lr=1e-2)
        m.adam_step(torch.from_numpy(gf).cuda(), lr=1e-2)
        got = m.get_params()[0].astype(np.float64)
        want = _flat(ref)
        print(f"Adam step {step + 1}: rel err of the update {rel(got - start, want - start):.2e}")
        assert rel(got - start, want - start) <= 1e-5


@pytest.mark.gpu
def test_graphs_recaptured_after_a_new_sweep_plan():
    """Setting a sweep plan reallocates the plan's device tables: a following
    graph-replayed solve captures again (it must not replay the old graphs) and
    still equals the eager solve."""
    import torch

    import paper_2410_08735_amd as rt
    specs = [tiny_2d(seed=s, nx=7, ny=6, quad=("cl", 8, 4, True), n_regions=2) for s in (1, 2)]
    B = rt.Batch(specs)
    st, ss = B.sigma()
    common = dict(precond="dsa", m=12, max_cycles=6, sweep_dtype="f32", rtol=1e-9, dsa_inner_max=1, dsa_restart=0)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        G = B.source()
        eager, _, _ = rt.fgmres_solve(B, st, ss, G, None, rt.SolveOptions(**common))
        g1, _, _ = rt.fgmres_solve(B, st, ss, G, None, rt.SolveOptions(use_graph=True, **common))
        side.synchronize()
        c1 = rt.graph_captures()
        g2, _, _ = rt.fgmres_solve(B, st, ss, G, None, rt.SolveOptions(use_graph=True, **common))
        side.synchronize()
        assert rt.graph_captures() == c1  # replays only
        plan = B.sweep_plan("f32")
        B.set_sweep_plan("f32", plan["variant"], plan["G"], plan["threads"], plan["opl"])
        g3, _, _ = rt.fgmres_solve(B, st, ss, G, None, rt.SolveOptions(use_graph=True, **common))
        side.synchronize()
        assert rt.graph_captures() > c1
    side.synchronize()
    assert bool((eager == g1).all()) and bool((eager == g2).all()) and bool((eager == g3).all())
