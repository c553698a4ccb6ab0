#!/usr/bin/env python3
"""Benchmark of the FGMRES-ROMSAD hot path on one MI355X.

Workload (the parametric checkerboard family at 96x96 Q1 cells, 128
ordinates): a greedy ROM (r <= 32) is built offline from 64 training
parameters, then one step = a batched FGMRES-ROMSAD solve of all 256 test
parameters to FP64 true relative residual 1e-8, with FP32 sweeps and FP64
Krylov.  Inputs are resident in HBM before the timed region.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "FGMRES solves/s to rel-res 1e-8 (MLP vs ROMSAD vs plain); sweep GDoF/s"
# Algorithmic FP32 sweep arithmetic per cell and ordinate: the low end of the
# 70-100 flops of a cell-ordinate of the upwind DG Q1 sweep (about 16 for the
# inflow right-hand side, 40-60 for the local 4x4 solve, 8 for the outgoing
# traces, 8 for the weighted quadrature sum; an FMA counts as two).
SWEEP_FLOPS_PER_CELL_ORD = 70.0
# What the FP32 kernel executes per cell-ordinate: 8 FMA for the right-hand
# side, 10 FMA and 4 multiplies for the local solve with its per-(region,
# ordinate) coefficients formed once per work item, 4 FMA for the traces, 4 FMA
# for the weighted sum (16 + 24 + 8 + 8).
SWEEP_EXECUTED_FLOPS_PER_CELL_ORD = 56.0
PEAK_FP32_VECTOR = 157.3e12   # MI355X published FP32 vector peak (packed two-wide FMA), FLOP/s
# FP32 ALU ceiling of the unpacked instructions this library emits (it is built
# without packed FP32): 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz.
PEAK_FP32_ALU = 256 * 4 * 16 * 2 * 2.4e9
PEAK_FP64_VECTOR = 78.6e12
PEAK_HBM = 8.0e12             # MI355X published HBM3E bandwidth, B/s
# HBM bytes per FULL launch (all 256 instances active) of the FP32 sweep at
# the default workload (96^2, 128 ordinates), from FETCH_SIZE and WRITE_SIZE
# counter passes scaled by what the counters read for a 512 MiB copy, keyed by
# (variant, G, ordinates per lane, threads) and valid for the kernel version
# SWEEP_KERNEL_VERSION the passes measured (profiles/sweep2d_f32_cfg3_96sq_b256_hbm_traffic.md).
SWEEP_KERNEL_VERSION = "rows-v3"
SWEEP_F32_TRAFFIC_BYTES = {
    # FETCH_SIZE 109901.9 KiB x 1.9999 + WRITE_SIZE 199229.4 KiB x 1.0
    ("rows-v3", 1, 8, 4, 768): 419019.4 * 1024,
}
# VALU lane instructions per cell-ordinate of a full launch (SQ_INSTS_VALU x 64
# / cell-ordinates, profiles/sweep2d_f32_cfg3_96sq_b256_sq_counters.md)
SWEEP_F32_VALU_LANE_INSTS = {("rows-v3", 1, 8, 4, 768): 201327616.0 * 64 / 301989888.0}
# Algorithmic HBM bytes per cell and instance of one sweep: read the 4 source
# moments (FP64, 32 B), write the 4 scalar-flux moments (FP64, 32 B), and the
# cell's cross-section data (8 B).  Angular fluxes never leave the chip.
SWEEP_ALG_BYTES_PER_CELL = 72.0


def _json(obj):
    """One JSON line; numpy scalars as plain numbers."""
    return json.dumps(obj, default=lambda o: o.item() if hasattr(o, "item") else str(o))


def plan_key(plan):
    return (plan["variant"], plan["G"], plan["opl"], plan["threads"])


def sweep_kernel_name(plan):
    """The FP32 sweep kernel the autotuned plan launches (as rocprofv3 names it)."""
    if plan["variant"] == 1:
        return f"rte::sweep2d_rows_kernel<float, {plan['G']}, {plan['opl']}, *, true> ({plan['threads']} threads)"
    return f"rte::sweep2d_kernel<float, {plan['G']}, {plan['opl']}> ({plan['threads']} threads)"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _oracle_job(job):
    """CPU worker (one process, one BLAS thread): the oracle's FGMRES-DSA solve
    (FP64, sparse-direct sweeps and DSA) of one instance to rtol 1e-8, timed
    from its problem description to the solution (the CPU baseline), then
    continued from that iterate to rtol 1e-12 (the reference flux against
    which the GPU's results are stated).  kind "sweep": one oracle sweep
    (b~ = T G) of the instance instead, timed."""
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle import dsa, fgmres, transport
    from synth import cfg2, cfg3_problem
    kind, key, mu, n, n_z = job
    t0 = time.perf_counter()
    if kind == "sweep":
        P = transport.Problem(cfg2())
        transport.b_tilde(P)
        return dict(kind=kind, key=key, t=time.perf_counter() - t0, dof=P.ndof * P.nord)
    P = transport.Problem(cfg3_problem(mu, n=n, n_z=n_z))
    b = transport.b_tilde(P)
    D = dsa.DSA(P)
    A = lambda x: transport.A_tilde_apply(P, x)
    pc = lambda j, v: D.apply(v)
    r = fgmres.fgmres(A, b, pc, m=30, rtol=1e-8)
    t1 = time.perf_counter()
    ref = fgmres.fgmres(A, b, pc, m=30, rtol=1e-12, x0=r.x)
    return dict(kind=kind, key=key, t=t1 - t0, iterations=r.iterations, phi=ref.x,
                ref_relres=ref.true_relres, converged=bool(r.converged))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_oracle_jobs(jobs, procs):
    """All oracle jobs in one pool, the largest first; returns their results and the pool's wall time."""
    t = time.perf_counter()
    ctx = mp.get_context("spawn")
    order = sorted(jobs, key=lambda j: -(j[3] or 0) ** 2)
    with ctx.Pool(procs) as pool:
        res = list(pool.imap_unordered(_oracle_job, order))
    return res, time.perf_counter() - t


def rel_err(gpu, ref):
    import numpy as np
    return float(np.linalg.norm(gpu - ref) / np.linalg.norm(ref))


def error_summary(gpu_phis, res, key_prefix):
    """max / mean relative L2 error of GPU fluxes against the oracle's 1e-12 references."""
    import numpy as np
    refs = {r["key"]: r["phi"] for r in res if r["kind"] == "solve" and r["key"][0] == key_prefix}
    out = {}
    for leg, phis in gpu_phis.items():
        e = [rel_err(phis[k], refs[(key_prefix, k)]) for k in sorted(phis) if (key_prefix, k) in refs]
        if e:
            out[leg] = {"max": float(np.max(e)), "mean": float(np.mean(e)), "instances": len(e)}
    return out


def _solve_timed(rt, torch, B, st, ss, G, opts, rom=None, mlp=None, mu=None, reps=1, keep=()):
    """Mean time of `reps` batched solves; keep: instances whose flux of the last
    solve is returned (host copies) for the error against the oracle."""
    import numpy as np
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        phi, stats, _ = rt.fgmres_solve(B, st, ss, G, None, opts, rom=rom, mlp=mlp, mu=mu)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    ok = int(np.count_nonzero(stats["true_relres"] <= 1e-8))
    if keep:
        parts = B.unpack(phi)
        return dt, ok, stats, {k: parts[k].copy() for k in keep}
    return dt, ok, stats


def learned_leg(args, common):
    """The learned preconditioner on the 128^2 x 128 workload: a greedy ROM from
    config-3-law training parameters, correction snapshots from FGMRES-ROMSAD
    solves on fresh parameters, network training on the GPU, then FGMRES with
    the network (ROMSAD fallback), FGMRES-ROMSAD and GMRES-DSA on fresh test
    parameters, all on the same batch and GPU."""
    import numpy as np
    import torch

    import paper_2410_08735_amd as rt
    from synth import cfg3_box_centre, cfg3_features, cfg3_problem, cfg3_sigma, cfg3_sources, cfg5_sets
    n, nb = args.mlp_grid, args.mlp_batch
    tr_mu, sn_mu, te_mu = cfg5_sets(n_train=args.n_train, n_snap=args.mlp_snap, n_test=args.mlp_test)
    out = {"grid": n, "snap_params": len(sn_mu), "test_params": len(te_mu)}

    def inputs(mus):
        st, ss = cfg3_sigma(mus)
        G = cfg3_sources(mus, n)
        f = cfg3_features(mus)
        return (torch.from_numpy(st).cuda(), torch.from_numpy(ss).cuda(),
                torch.from_numpy(G.reshape(-1)).cuda(), torch.from_numpy(f).cuda())

    # offline 1: greedy ROM
    base = cfg3_problem(cfg3_box_centre(), n=n)
    Btr = rt.Batch([base] * len(tr_mu))
    st, ss, G, _ = inputs(tr_mu)
    torch.cuda.synchronize()
    t = time.perf_counter()
    rom, grep = rt.romsad_build_greedy(Btr, st, ss, G, None, window=2, mu1_index=0, eps_rom=1e-9,
                                       n_giter=args.n_giter, eps_qr=1e-13, hf_rtol=1e-11)
    torch.cuda.synchronize()
    out["greedy_s"], out["rank"] = time.perf_counter() - t, grep["rank"]
    del Btr
    log(f"learned: ROM rank {grep['rank']} at {n}^2 in {out['greedy_s']:.1f} s")

    # offline 2: snapshot rows from FGMRES-ROMSAD solves on fresh parameters
    B = rt.Batch([base] * nb)
    snap_opts = rt.SolveOptions(precond="romsad", **common)
    Xs, Ts = [], []
    torch.cuda.synchronize()
    t = time.perf_counter()
    for b0 in range(0, len(sn_mu) - nb + 1, nb):
        st, ss, G, f = inputs(sn_mu[b0:b0 + nb])
        X, T, valid = rt.mlp_snapshots(B, st, ss, G, rom, snap_opts, f)
        keep = valid.bool()
        Xs.append(X[keep])
        Ts.append(T[keep])
    X, T = torch.cat(Xs), torch.cat(Ts)
    torch.cuda.synchronize()
    out["snapshots"], out["snapshot_s"] = int(X.shape[0]), time.perf_counter() - t
    log(f"learned: {X.shape[0]} snapshot rows in {out['snapshot_s']:.1f} s")

    # offline 3: training on the GPU (BF16 matrix cores, FP32 master weights, Adam)
    r = rom.rank
    net = rt.Mlp(4 + r, 256, 4, r)
    net.init(seed=7)
    torch.cuda.synchronize()
    t = time.perf_counter()
    if args.only_mlp:  # counter passes: training between markers 1 and 2
        rt.prof_mark(1)
    hist = net.train(X, T, epochs=args.mlp_epochs, batch=256, lr=args.mlp_lr, seed=11)
    if args.only_mlp:
        rt.prof_mark(2)
    torch.cuda.synchronize()
    out["train_s"], out["epochs"] = time.perf_counter() - t, args.mlp_epochs
    out["loss_first_last"] = [float(hist[0]), float(hist[-1])]
    log(f"learned: trained {args.mlp_epochs} epochs in {out['train_s']:.1f} s, loss {hist[0]:.3e} -> "
        f"{hist[-1]:.3e}")

    # online: the three preconditioners on the same fresh test batch
    Bt = B if len(te_mu) == nb else rt.Batch([base] * len(te_mu))
    st, ss, G, f = inputs(te_mu)
    res = {}
    phis = {}
    for name, pc, kw in (("mlp", "mlp", dict(rom=rom, mlp=net, mu=f)), ("romsad", "romsad", dict(rom=rom)),
                         ("plain_dsa", "dsa", {})):
        opts = rt.SolveOptions(precond=pc, **common)
        rt.fgmres_solve(Bt, st, ss, G, None, opts, **kw)  # warm-up (autotune, DSA hierarchy)
        if args.only_mlp and name == "mlp":  # counter passes: the FGMRES-MLP solves between markers 3 and 4
            rt.prof_mark(3)
        dt, ok, stats, phis[name] = _solve_timed(rt, torch, Bt, st, ss, G, opts, reps=args.steps,
                                                 keep=range(min(4, len(te_mu))), **kw)
        if args.only_mlp and name == "mlp":
            rt.prof_mark(4)
        its = np.array([s["iterations"] for s in stats])
        rr = np.array([s["true_relres"] for s in stats])
        res[name] = {"value": ok / dt, "unit": "solves/s", "ms_per_step": dt * 1e3, "converged": ok,
                     "iterations_mean": float(its.mean()), "iterations_max": int(its.max()),
                     "max_true_relres": float(rr.max())}
        if name == "mlp":
            res[name]["fallbacks"] = int(sum(s["pc_fallback"] for s in stats))
            res[name]["mlp_applies"] = int(sum(s["pc_mlp"] for s in stats))
            jd = np.array([s["mlp_rom_diff"] for s in stats])
            res[name]["mlp_rom_rel_diff_mean"] = float(jd.mean())
            res[name]["mlp_rom_rel_diff_max"] = float(jd.max())
        log(f"learned: {name}: {ok / dt:.1f} solves/s, iterations mean {its.mean():.2f} max {its.max()}, "
            f"converged {ok}/{len(stats)}")
    out.update(res)
    out["_phis"] = phis
    out["_oracle_jobs"] = [("solve", ("cfg5", k), te_mu[k], n, 16) for k in range(min(4, len(te_mu)))]
    return out


def uneven_leg(args, common):
    """The uneven batch: 512 instances on grids of 32^2..128^2 with 64 or 128
    ordinates (checkerboard law), one greedy ROM per (grid, ordinates) group
    joined in a ROM set, all instances solved together: every sweep is one
    launch over the whole batch."""
    import numpy as np
    import torch

    import paper_2410_08735_amd as rt
    from synth import cfg3_box_centre, cfg3_mu, cfg3_problem, cfg4_batch
    items = cfg4_batch(n_inst=args.uneven_n)
    groups = sorted({(g, no) for g, no, _ in items})
    nz = {64: 8, 128: 16}
    rng = np.random.default_rng(40)
    roms = []
    torch.cuda.synchronize()
    t = time.perf_counter()
    for g, no in groups:
        tr = np.concatenate([cfg3_box_centre()[None], cfg3_mu(rng, args.n_train - 1)], 0)
        Btr = rt.Batch([cfg3_problem(m, n=g, n_z=nz[no]) for m in tr])
        st, ss = Btr.sigma()
        rom, _ = rt.romsad_build_greedy(Btr, st, ss, Btr.source(), None, window=2, mu1_index=0, eps_rom=1e-9,
                                        n_giter=args.n_giter, eps_qr=1e-13, hf_rtol=1e-11)
        roms.append(rom)
        del Btr, st, ss
    torch.cuda.synchronize()
    offline = time.perf_counter() - t
    B = rt.Batch([cfg3_problem(m, n=g, n_z=nz[no]) for g, no, m in items])
    which = [groups.index((g, no)) for g, no, _ in items]
    rs = rt.Rom.set(B, roms, which)
    st, ss = B.sigma()
    G = B.source()
    out = {"instances": len(items), "groups": [f"{g}^2 x {no}" for g, no in groups], "hip_graphs": True,
           "dof_total": int(sum(B.ndofs)), "greedy_s_total": offline,
           "ranks": [r.rank for r in roms]}
    side = torch.cuda.Stream()  # graph capture needs a created stream
    first = [which.index(gi) for gi in range(len(groups))]  # one instance per (grid, ordinates) group
    phis = {}
    for name, pc, kw in (("romsad", "romsad", dict(rom=rs)), ("plain_dsa", "dsa", {})):
        opts = rt.SolveOptions(precond=pc, use_graph=True, **common)
        with torch.cuda.stream(side):
            rt.fgmres_solve(B, st, ss, G, None, opts, **kw)  # warm-up: autotune, DSA hierarchy, captures
            dt, ok, stats, phis[name] = _solve_timed(rt, torch, B, st, ss, G, opts, reps=args.steps, keep=first,
                                                     **kw)
        its = np.array([s["iterations"] for s in stats])
        out[name] = {"value": ok / dt, "unit": "solves/s", "ms_per_step": dt * 1e3, "converged": ok,
                     "iterations_mean": float(its.mean()), "iterations_max": int(its.max())}
        log(f"uneven: {name}: {ok / dt:.1f} solves/s, iterations mean {its.mean():.2f}, converged {ok}/{len(stats)}")
    cells_ord = sum(nd // 4 * no for nd, no in zip(B.ndofs, B.n_ords))
    for dt_name in ("f32", "f64"):
        rt.sweep(B, st, G, dtype=dt_name)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(5):
            rt.sweep(B, st, G, dtype=dt_name)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t) / 5
        out[f"sweep_gdof_s_{dt_name}"] = 4 * cells_ord / el / 1e9
        out[f"sweep_plan_{dt_name}"] = B.sweep_plan(dt_name)
    log(f"uneven: sweep GDoF/s f32 {out['sweep_gdof_s_f32']:.0f} plan {out['sweep_plan_f32']}, "
        f"f64 {out['sweep_gdof_s_f64']:.0f} plan {out['sweep_plan_f64']}")
    out["_phis"] = phis
    out["_oracle_jobs"] = [("solve", ("cfg4", k), items[k][2], items[k][0], nz[items[k][1]]) for k in first]
    return out


def pincell_leg(args):
    """The paper's pin-cell problem (section 5.2) as specified there: 80^2 cells,
    CL(30,6), 25 training parameters on a uniform grid, mu_1 = (0.275, 0.275),
    window 2, eps_ROM = 1e-10, rtol 1e-11, 10 test parameters; the DSA is solved
    to 1e-12 (exact-solve DSA, as with the paper's AMG).  Reports the average
    sweep count 1 + iterations, the paper's n_sweep metric, next to its table
    values (GMRES-DSA 15.5, FGMRES-ROMSAD 5.1, 22 sampled, rank 44)."""
    import numpy as np
    import torch

    import paper_2410_08735_amd as rt
    from synth import pincell_problem, pincell_sets
    tr_mu, te_mu = pincell_sets()
    # the paper's eps_ROM applies to the residual indicator of a basis that is
    # sqrt(h_x h_y) = h times the orthonormal one used here
    h = 2.0 / 80
    Btr = rt.Batch([pincell_problem(m) for m in tr_mu])
    st, ss = Btr.sigma()
    torch.cuda.synchronize()
    t = time.perf_counter()
    rom, rep = rt.romsad_build_greedy(Btr, st, ss, Btr.source(), None, window=2, mu1_index=0, eps_rom=1e-10 / h,
                                      n_giter=25, eps_qr=1e-13, hf_rtol=1e-11, hf_dsa_tol=1e-12)
    torch.cuda.synchronize()
    out = {"greedy_s": time.perf_counter() - t, "sampled": len(rep["sampled"]), "rank": rep["rank"],
           "paper": {"gmres_dsa_nsweep": 15.5, "fgmres_romsad_nsweep": 5.1, "sampled": 22, "rank": 44}}
    _, lit = rt.romsad_build_greedy(Btr, st, ss, Btr.source(), None, window=2, mu1_index=0, eps_rom=1e-10,
                                    n_giter=25, eps_qr=1e-13, hf_rtol=1e-11, hf_dsa_tol=1e-12)
    out["literal_eps"] = {"sampled": len(lit["sampled"]), "rank": int(lit["rank"])}
    del Btr, st, ss
    B = rt.Batch([pincell_problem(m) for m in te_mu])
    st, ss = B.sigma()
    G = B.source()
    exact = dict(m=60, max_cycles=10, sweep_dtype="f64", rtol=1e-11, window=2, dsa_inner_max=1000,
                 dsa_restart=60, dsa_inner_tol=1e-12)
    vcycle = dict(exact, dsa_inner_max=1, dsa_restart=0, dsa_inner_tol=1e-6)
    for name, pc, kw, common in (("gmres_dsa", "dsa", {}, exact), ("fgmres_romsad", "romsad", dict(rom=rom), exact),
                                 ("gmres_dsa_vcycle", "dsa", {}, vcycle),
                                 ("fgmres_romsad_vcycle", "romsad", dict(rom=rom), vcycle)):
        opts = rt.SolveOptions(precond=pc, **common)
        dt, ok, stats = _solve_timed(rt, torch, B, st, ss, G, opts, reps=1, **kw)
        its = np.array([s["iterations"] for s in stats])
        rr = np.array([s["true_relres"] for s in stats])
        out[name] = {"nsweep_mean": float(1 + its.mean()), "ms": dt * 1e3, "max_true_relres": float(rr.max()),
                     "converged": int((rr <= 1e-11).sum())}
        log(f"pin-cell: {name}: n_sweep {1 + its.mean():.2f}, {dt * 1e3:.1f} ms, max relres {rr.max():.2e}")
    log(f"pin-cell: greedy sampled {out['sampled']}, rank {out['rank']}, {out['greedy_s']:.1f} s")

    # the FGMRES / SI comparison of section 5.2: window 1, eps_ROM 1e-7, the
    # hardest test parameter (mu_a, mu_s) = (0.065886, 0.11397)
    Btr = rt.Batch([pincell_problem(m) for m in tr_mu])
    st, ss = Btr.sigma()
    rom1, rep1 = rt.romsad_build_greedy(Btr, st, ss, Btr.source(), None, window=1, mu1_index=0, eps_rom=1e-7 / h,
                                        n_giter=25, eps_qr=1e-13, hf_rtol=1e-11, hf_dsa_tol=1e-12)
    _, lit1 = rt.romsad_build_greedy(Btr, st, ss, Btr.source(), None, window=1, mu1_index=0, eps_rom=1e-7,
                                     n_giter=25, eps_qr=1e-13, hf_rtol=1e-11, hf_dsa_tol=1e-12)
    del Btr, st, ss
    B1 = rt.Batch([pincell_problem((0.065886, 0.11397))])
    st, ss = B1.sigma()
    G = B1.source()
    cmp = {"sampled": len(rep1["sampled"]), "rank": rep1["rank"],
           "literal_eps": {"sampled": len(lit1["sampled"]), "rank": int(lit1["rank"])},
           "paper": {"gmres_dsa": 15, "si_dsa": 49, "fgmres_romsad": 10, "si_romsad": "100 (not converged)",
                     "first_correction_relres": {"gmres_dsa": 6.23e-2, "si_dsa": 1.17e-1,
                                                 "fgmres_romsad": 4.87e-6, "si_romsad": 4.90e-6},
                     "sampled": 13, "rank": 13}}
    one = dict(exact, window=1)
    for name, solver, pc, kw in (("gmres_dsa", rt.fgmres_solve, "dsa", {}), ("si_dsa", rt.si_solve, "dsa", {}),
                                 ("fgmres_romsad", rt.fgmres_solve, "romsad", dict(rom=rom1)),
                                 ("si_romsad", rt.si_solve, "romsad", dict(rom=rom1))):
        full = dict(one, max_cycles=100) if solver is rt.si_solve else one
        _, stats, _ = solver(B1, st, ss, G, None, rt.SolveOptions(precond=pc, **full), **kw)
        first = dict(one, m=1, max_cycles=1)
        _, s1, _ = solver(B1, st, ss, G, None, rt.SolveOptions(precond=pc, **first), **kw)
        cmp[name] = {"n_sweep": 1 + int(stats[0]["iterations"]), "converged": bool(stats[0]["true_relres"] <= 1e-11),
                     "true_relres": float(stats[0]["true_relres"]),
                     "first_correction_relres": float(s1[0]["true_relres"])}
        log(f"pin-cell compare: {name}: n_sweep {1 + stats[0]['iterations']}, relres {stats[0]['true_relres']:.2e}, "
            f"after the first correction {s1[0]['true_relres']:.2e}")
    out["si_comparison"] = cmp
    return out


def twomat_leg(args):
    """The paper's two-material problem with parametric inflow (section 5.4):
    64^2 cells, CL(60,6), 9 x 11 training grid, mu_1 = (3, 1), window 2,
    eps_ROM = 1e-9 (in the paper's basis scaling), rtol 1e-11, 10 test
    parameters, exact-solve DSA; the paper's table: GMRES-DSA 10.0 sweeps,
    FGMRES-ROMSAD 4.3, 9 sampled, rank 18."""
    import numpy as np
    import torch

    import paper_2410_08735_amd as rt
    from synth import twomat_problem, twomat_sets
    tr_mu, te_mu = twomat_sets()
    h = 2.0 / 64
    Btr = rt.Batch([twomat_problem(m) for m in tr_mu])
    st, ss = Btr.sigma()
    torch.cuda.synchronize()
    t = time.perf_counter()
    rom, rep = rt.romsad_build_greedy(Btr, st, ss, Btr.source(), Btr.inflow(), window=2, mu1_index=0,
                                      eps_rom=1e-9 / h, n_giter=32, eps_qr=1e-13, hf_rtol=1e-11, hf_dsa_tol=1e-12)
    torch.cuda.synchronize()
    out = {"greedy_s": time.perf_counter() - t, "sampled": len(rep["sampled"]), "rank": rep["rank"],
           "paper": {"gmres_dsa_nsweep": 10.0, "fgmres_romsad_nsweep": 4.3, "sampled": 9, "rank": 18}}
    _, lit = rt.romsad_build_greedy(Btr, st, ss, Btr.source(), Btr.inflow(), window=2, mu1_index=0, eps_rom=1e-9,
                                    n_giter=32, eps_qr=1e-13, hf_rtol=1e-11, hf_dsa_tol=1e-12)
    out["literal_eps"] = {"sampled": len(lit["sampled"]), "rank": int(lit["rank"])}
    del Btr, st, ss
    B = rt.Batch([twomat_problem(m) for m in te_mu])
    st, ss = B.sigma()
    exact = dict(m=60, max_cycles=10, sweep_dtype="f64", rtol=1e-11, window=2, dsa_inner_max=1000,
                 dsa_restart=60, dsa_inner_tol=1e-12)
    for name, pc, kw in (("gmres_dsa", "dsa", {}), ("fgmres_romsad", "romsad", dict(rom=rom))):
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, stats, _ = rt.fgmres_solve(B, st, ss, B.source(), B.inflow(), rt.SolveOptions(precond=pc, **exact), **kw)
        torch.cuda.synchronize()
        its = np.array([s["iterations"] for s in stats])
        rr = np.array([s["true_relres"] for s in stats])
        out[name] = {"nsweep_mean": float(1 + its.mean()), "ms": (time.perf_counter() - t) * 1e3,
                     "max_true_relres": float(rr.max())}
        log(f"two-material: {name}: n_sweep {1 + its.mean():.2f}, max relres {rr.max():.2e}")
    log(f"two-material: greedy sampled {out['sampled']}, rank {out['rank']}, {out['greedy_s']:.1f} s")
    return out


def sweep_leg(args):
    """Full-batch FP32 operator sweeps (every instance active) of the main
    workload for kernel traces and counter passes: `steps` applications of
    A~ = I - T Sigma_s between the region markers 1 and 2, and optionally the
    512 MiB calibration copy between markers 3 and 4."""
    import torch

    import paper_2410_08735_amd as rt
    from synth import cfg3_problem, cfg3_train_test
    _, te_mu = cfg3_train_test(n_train=args.n_train, n_test=args.n_test)
    B = rt.Batch([cfg3_problem(m, n=args.grid) for m in te_mu])
    st, ss = B.sigma()
    x = B.source()
    if args.sweep_plan:
        v, g, o, t = (int(q) for q in args.sweep_plan.split(","))
        B.set_sweep_plan("f32", v, g, t, opl=o)
    for _ in range(max(args.warmup, 1)):
        rt.apply_A(B, st, ss, x, dtype="f32")
    torch.cuda.synchronize()
    rt.prof_enable(True)
    rt.prof_mark(1)
    for _ in range(args.steps):
        rt.apply_A(B, st, ss, x, dtype="f32")
    rt.prof_mark(2)
    torch.cuda.synchronize()
    n, ms, units = rt.prof_read("sweep_f32")
    rt.prof_enable(False)
    if args.pmc_copy:
        src = torch.ones(64 * 2 ** 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        rt.prof_mark(3)
        dst.copy_(src)
        rt.prof_mark(4)
        torch.cuda.synchronize()
    avg = ms / max(n, 1)
    return {"plan": B.sweep_plan("f32"), "launches": n, "avg_launch_ms": avg,
            "cell_ordinates_per_launch": units / max(n, 1),
            "tflops_at_70": units / max(n, 1) * SWEEP_FLOPS_PER_CELL_ORD / (avg * 1e-3) / 1e12 if avg > 0 else 0.0}


def _greedy_counts(rep):
    return len(rep["sampled"]), int(rep["rank"])


def varscat_leg(args):
    """The paper's variable-scattering problem (section 5.3): [-1,1]^2, 80^2
    cells, CL(30,6), sigma_s = mu_s r^4 (2 - r^2)^2 + 0.1 inside the unit disk
    (mu_s + 0.1 outside), sigma_a = 0; 51 training values of mu_s on [49.9,
    99.9], mu_s,1 = 74.9, window 2, eps_ROM = 1e-9 (in the paper's basis
    scaling), rtol 1e-11, 10 test values, exact-solve DSA, FC and PC.  The
    paper's table: GMRES-PC-DSA 15.0, GMRES-FC-DSA 11.0, FGMRES-PC-ROMSAD 4.7,
    FGMRES-FC-ROMSAD 4.6 sweeps; 8 sampled, rank 16."""
    import numpy as np
    import torch

    import paper_2410_08735_amd as rt
    from synth import varscat_problem, varscat_sets
    tr_mu, te_mu = varscat_sets()
    h = 2.0 / 80
    Btr = rt.Batch([varscat_problem(m) for m in tr_mu])
    st, ss = Btr.sigma()
    torch.cuda.synchronize()
    t = time.perf_counter()
    rom, rep = rt.romsad_build_greedy(Btr, st, ss, Btr.source(), None, window=2, mu1_index=25, eps_rom=1e-9 / h,
                                      n_giter=25, eps_qr=1e-13, hf_rtol=1e-11, hf_dsa_tol=1e-12)
    torch.cuda.synchronize()
    out = {"greedy_s": time.perf_counter() - t, "sampled": len(rep["sampled"]), "rank": rep["rank"],
           "sampled_mu_s": [float(tr_mu[i]) for i in rep["sampled"]],
           "literal_eps": {k: v for k, v in zip(("sampled", "rank"), _greedy_counts(
               rt.romsad_build_greedy(Btr, st, ss, Btr.source(), None, window=2, mu1_index=25, eps_rom=1e-9,
                                      n_giter=25, eps_qr=1e-13, hf_rtol=1e-11, hf_dsa_tol=1e-12)[1]))},
           "paper": {"gmres_pc_dsa_nsweep": 15.0, "gmres_fc_dsa_nsweep": 11.0, "fgmres_pc_romsad_nsweep": 4.7,
                     "fgmres_fc_romsad_nsweep": 4.6, "sampled": 8, "rank": 16}}
    # the offline table's other figure: all 51 training solves with GMRES-FC-DSA (one batched solve)
    all_opts = rt.SolveOptions(precond="dsa", dsa_variant="fc", m=60, max_cycles=10, sweep_dtype="f64", rtol=1e-11,
                               dsa_inner_max=2000, dsa_restart=60, dsa_inner_tol=1e-12)
    rt.fgmres_solve(Btr, st, ss, Btr.source(), None, all_opts)
    torch.cuda.synchronize()
    t = time.perf_counter()
    rt.fgmres_solve(Btr, st, ss, Btr.source(), None, all_opts)
    torch.cuda.synchronize()
    out["all_snapshots_s"] = time.perf_counter() - t
    out["all_snapshots_over_greedy"] = out["all_snapshots_s"] / out["greedy_s"]
    out["paper"]["all_snapshots_over_greedy"] = 4.00
    del Btr, st, ss
    log(f"variable scattering: greedy sampled {out['sampled']}, rank {out['rank']}, {out['greedy_s']:.1f} s; "
        f"all 51 training solves {out['all_snapshots_s']:.2f} s")
    B = rt.Batch([varscat_problem(m) for m in te_mu])
    st, ss = B.sigma()
    G = B.source()
    exact = dict(m=60, max_cycles=10, sweep_dtype="f64", rtol=1e-11, window=2, dsa_inner_max=2000, dsa_restart=60,
                 dsa_inner_tol=1e-12)
    for name, pc, kw, var in (("gmres_pc_dsa", "dsa", {}, "pc"), ("gmres_fc_dsa", "dsa", {}, "fc"),
                              ("fgmres_pc_romsad", "romsad", dict(rom=rom), "pc"),
                              ("fgmres_fc_romsad", "romsad", dict(rom=rom), "fc")):
        dt, ok, stats = _solve_timed(rt, torch, B, st, ss, G, rt.SolveOptions(precond=pc, dsa_variant=var, **exact),
                                     reps=1, **kw)
        its = np.array([s["iterations"] for s in stats])
        rr = np.array([s["true_relres"] for s in stats])
        out[name] = {"nsweep_mean": float(1 + its.mean()), "ms": dt * 1e3, "max_true_relres": float(rr.max()),
                     "converged": int((rr <= 1e-11).sum())}
        log(f"variable scattering: {name}: n_sweep {1 + its.mean():.2f}, {dt * 1e3:.1f} ms, max relres {rr.max():.2e}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-test", type=int, default=256)
    ap.add_argument("--n-train", type=int, default=64)
    ap.add_argument("--grid", type=int, default=96)
    ap.add_argument("--n-giter", type=int, default=16)
    ap.add_argument("--dsa-inner", type=int, default=1, help="V-cycles per DSA application")
    ap.add_argument("--dsa-restart", type=int, default=0, help="0 = stationary V-cycles")
    ap.add_argument("--mlp-grid", type=int, default=128)
    ap.add_argument("--mlp-batch", type=int, default=1024)
    ap.add_argument("--mlp-snap", type=int, default=10240, help="snapshot parameters (2 rows each)")
    ap.add_argument("--mlp-test", type=int, default=1024)
    ap.add_argument("--mlp-epochs", type=int, default=60)
    ap.add_argument("--mlp-lr", type=float, default=1e-3)
    ap.add_argument("--no-mlp", action="store_true")
    ap.add_argument("--uneven-n", type=int, default=512)
    ap.add_argument("--no-uneven", action="store_true")
    ap.add_argument("--only-pincell", action="store_true", help="the paper's pin-cell problem only")
    ap.add_argument("--only-twomat", action="store_true", help="the paper's two-material problem only")
    ap.add_argument("--only-uneven", action="store_true")
    ap.add_argument("--only-varscat", action="store_true", help="the paper's variable-scattering problem only")
    ap.add_argument("--only-sweep", action="store_true",
                    help="full-batch FP32 operator sweeps of the main workload only (for traces and counters)")
    ap.add_argument("--only-mlp", action="store_true")
    ap.add_argument("--sweep-plan", type=str, default=None,
                    help="fix the FP32 sweep plan of the main workload: variant,G,opl,threads (default: autotuned)")
    ap.add_argument("--window-cycles", type=int, default=1,
                    help="restart cycles that use the ROM window (0 = every cycle)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pmc-copy", action="store_true",
                    help="after the timed region, copy 512 MiB device-to-device between markers 3 and 4 "
                         "(calibrates hardware byte counters)")
    ap.add_argument("--no-extras", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the benchmark runs on one GPU only (--gpus 1); runs on several GPUs "
              "are not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2410_08735_amd as rt
    from synth import cfg2, cfg3_problem, cfg3_train_test

    torch.cuda.set_device(0)
    common = dict(m=30, max_cycles=10, sweep_dtype="f32", rtol=1e-8, window=2,
                  dsa_inner_max=args.dsa_inner, dsa_restart=args.dsa_restart, dsa_inner_tol=1e-6,
                  window_cycles=args.window_cycles)
    if args.only_mlp:
        out = learned_leg(args, common)
        print(_json({"learned": {k: v for k, v in out.items() if not k.startswith("_")}}), flush=True)
        return
    if args.only_twomat:
        print(_json({"twomat": twomat_leg(args)}), flush=True)
        return
    if args.only_pincell:
        print(_json({"pincell": pincell_leg(args)}), flush=True)
        return
    if args.only_varscat:
        print(_json({"varscat": varscat_leg(args)}), flush=True)
        return
    if args.only_sweep:
        print(_json({"sweep": sweep_leg(args)}), flush=True)
        return
    if args.only_uneven:
        out = uneven_leg(args, common)
        print(_json({"uneven": {k: v for k, v in out.items() if not k.startswith("_")}}), flush=True)
        return
    tr_mu, te_mu = cfg3_train_test(n_train=args.n_train, n_test=args.n_test)
    n = args.grid

    # ---------------- offline: greedy ROM on the training parameters
    log(f"building training batch ({len(tr_mu)} x {n}^2 x 128)")
    Btr = rt.Batch([cfg3_problem(m, n=n) for m in tr_mu])
    st_tr, ss_tr = Btr.sigma()
    torch.cuda.synchronize()
    t = time.perf_counter()
    rom, grep = rt.romsad_build_greedy(Btr, st_tr, ss_tr, Btr.source(), None, window=2, mu1_index=0,
                                       eps_rom=1e-9, n_giter=args.n_giter, eps_qr=1e-13,
                                       hf_rtol=1e-11)
    torch.cuda.synchronize()
    offline_s = time.perf_counter() - t
    log(f"greedy: rank {grep['rank']}, sampled {len(grep['sampled'])}, {offline_s:.1f} s, "
        f"steps {[round(x, 2) for x in grep['seconds_step']]}")
    del Btr, st_tr, ss_tr

    # ---------------- test batch resident in HBM
    B = rt.Batch([cfg3_problem(m, n=n) for m in te_mu])
    st, ss = B.sigma()
    G = B.source()
    if args.sweep_plan:
        v, g, o, t = (int(x) for x in args.sweep_plan.split(","))
        B.set_sweep_plan("f32", v, g, t, opl=o)
    opts = rt.SolveOptions(precond="romsad", **common)
    for _ in range(args.warmup):
        rt.fgmres_solve(B, st, ss, G, None, opts, rom=rom)
    torch.cuda.synchronize()

    # ---------------- timed region
    rt.prof_enable(True)
    rt.prof_mark(1)  # kernel-trace boundary of the timed region
    torch.cuda.synchronize()
    t = time.perf_counter()
    ok = 0
    all_stats = []
    for _ in range(args.steps):
        phi, stats, ret = rt.fgmres_solve(B, st, ss, G, None, opts, rom=rom)
        ok += int(np.count_nonzero(stats["true_relres"] <= 1e-8))
        all_stats = stats
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    rt.prof_mark(2)
    if args.pmc_copy:
        src = torch.ones(64 * 2 ** 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        rt.prof_mark(3)
        dst.copy_(src)
        rt.prof_mark(4)
        torch.cuda.synchronize()
        del src, dst
    launches, sweep_ms, units = rt.prof_read("sweep_f32")
    rt.prof_enable(False)
    value = ok / dt
    n_err = min(16, len(te_mu))
    phis3 = {"romsad": {k: v.copy() for k, v in enumerate(B.unpack(phi)[:n_err])}}
    avg_launch_ms = sweep_ms / max(launches, 1)
    achieved = units * SWEEP_FLOPS_PER_CELL_ORD / (sweep_ms * 1e-3) if sweep_ms > 0 else 0.0
    achieved_exec = units * SWEEP_EXECUTED_FLOPS_PER_CELL_ORD / (sweep_ms * 1e-3) if sweep_ms > 0 else 0.0
    n_ord = B.n_ords[0]
    active_cells = units / n_ord  # cell-instances the timed launches swept
    hbm_alg = (active_cells * SWEEP_ALG_BYTES_PER_CELL / (sweep_ms * 1e-3)) if sweep_ms > 0 else 0.0
    its = np.array([s["iterations"] for s in all_stats])
    sw32 = np.array([s["sweeps_f32"] for s in all_stats])
    sw64 = np.array([s["sweeps_f64"] for s in all_stats])
    rr = np.array([s["true_relres"] for s in all_stats])
    log(f"ROMSAD: {value:.2f} solves/s, {dt / args.steps * 1e3:.1f} ms/step, iterations mean "
        f"{its.mean():.2f} max {its.max()}, max relres {rr.max():.2e}; sweep launches {launches}, "
        f"avg {avg_launch_ms:.3f} ms, {achieved / 1e12:.2f} TFLOP/s")

    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 sweeps / f64 Krylov",
        "data": "synthetic",
        "config": {"workload": f"checkerboard RTE family, {n}x{n} Q1 cells, CL(16,16) folded "
                               f"(128 ordinates), {len(te_mu)} test parameters batched, "
                               f"FGMRES-ROMSAD (greedy ROM r={grep['rank']} from {len(tr_mu)} "
                               f"training parameters, window 2), FP32 sweeps, FP64 Arnoldi, "
                               f"rtol 1e-8",
                   "global_batch": len(te_mu), "precond": "romsad"},
        "roofline": {"bound": "alu", "kernel": sweep_kernel_name(B.sweep_plan("f32")), "achieved": achieved / 1e12,
                     "peak": PEAK_FP32_VECTOR / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VECTOR,
                     "traffic": (SWEEP_F32_TRAFFIC_BYTES.get((SWEEP_KERNEL_VERSION,) + plan_key(B.sweep_plan("f32")))
                                 if (n == 96 and len(te_mu) == 256) else None),
                     "traffic_unit": "HBM B per full launch (256 instances active)",
                     "valu_lane_instructions_per_cell_ordinate": (
                         SWEEP_F32_VALU_LANE_INSTS.get((SWEEP_KERNEL_VERSION,) + plan_key(B.sweep_plan("f32")))
                         if (n == 96 and len(te_mu) == 256) else None),
                     "flops_per_cell_ordinate": SWEEP_FLOPS_PER_CELL_ORD,
                     "executed_flops_per_cell_ordinate": SWEEP_EXECUTED_FLOPS_PER_CELL_ORD,
                     "peak_unpacked_fp32": PEAK_FP32_ALU / 1e12,
                     "frac_unpacked_executed": achieved_exec / PEAK_FP32_ALU,
                     "hbm_algorithmic_GBps": hbm_alg / 1e9,
                     "hbm_peak_GBps": PEAK_HBM / 1e9,
                     "cell_ordinates_per_launch": units / max(launches, 1),
                     "launches": launches, "avg_launch_ms": avg_launch_ms},
        "romsad": {"iterations_mean": float(its.mean()), "iterations_max": int(its.max()),
                   "sweeps_f32_mean": float(sw32.mean()), "sweeps_f64_mean": float(sw64.mean()),
                   "max_true_relres": float(rr.max()), "converged": int((rr <= 1e-8).sum())},
        "offline": {"greedy_s": offline_s, "rank": grep["rank"], "sampled": len(grep["sampled"]),
                    "seconds_step": grep["seconds_step"]},
    }

    if not args.no_extras:
        # plain GMRES-DSA, and FGMRES-ROMSAD with FP64 sweeps throughout, on the
        # same batch and GPU, with the same warm-up and steps as the headline
        for name, pc, kw, extra in (("plain_dsa", "dsa", {}, {}),
                                    ("romsad_fp64_sweeps", "romsad", dict(rom=rom), dict(sweep_dtype="f64"))):
            o2 = rt.SolveOptions(precond=pc, **dict(common, **extra))
            for _ in range(args.warmup):
                rt.fgmres_solve(B, st, ss, G, None, o2, **kw)
            dtp, okp, stats, kept = _solve_timed(rt, torch, B, st, ss, G, o2, reps=args.steps, keep=range(n_err),
                                                 **kw)
            itp = np.array([s["iterations"] for s in stats])
            rrp = np.array([s["true_relres"] for s in stats])
            out[name] = {"value": okp / dtp, "unit": "solves/s", "iterations_mean": float(itp.mean()),
                         "iterations_max": int(itp.max()), "ms_per_step": dtp * 1e3, "converged": okp,
                         "max_true_relres": float(rrp.max())}
            phis3[name] = kept
            log(f"{name}: {okp / dtp:.2f} solves/s, iterations mean {itp.mean():.2f}")
        # why ROMSAD trails GMRES-DSA on this family: the relative residual after
        # the first correction (the metric of the section 5.2 comparison table)
        fc = {}
        for name, pc, kw in (("romsad", "romsad", dict(rom=rom)), ("dsa", "dsa", {})):
            o1 = rt.SolveOptions(precond=pc, **dict(common, m=1, max_cycles=1))
            _, s1, _ = rt.fgmres_solve(B, st, ss, G, None, o1, **kw)
            r1 = np.array([s["true_relres"] for s in s1])
            fc[name] = {"mean": float(r1.mean()), "median": float(np.median(r1)), "max": float(r1.max())}
        out["first_correction_relres"] = fc
        log(f"relative residual after the first correction: {fc}")
        # sweep throughput: batched (this workload) and single instance (64^2, 128 ordinates)
        gd = {}
        for name, batch, sig in (("batch256_96sq", B, st),):
            q = G
            for dt_name in ("f32", "f64"):
                rt.sweep(batch, sig, q, dtype=dt_name)
                torch.cuda.synchronize()
                t = time.perf_counter()
                reps = 5
                for _ in range(reps):
                    rt.sweep(batch, sig, q, dtype=dt_name)
                torch.cuda.synchronize()
                el = (time.perf_counter() - t) / reps
                dof = sum(nd * no for nd, no in zip(batch.ndofs, batch.n_ords))
                gd[f"{name}_{dt_name}"] = dof / el / 1e9
        B2 = rt.Batch([cfg2()])
        st2, _ = B2.sigma()
        q2 = B2.source()
        for dt_name in ("f32", "f64"):
            rt.sweep(B2, st2, q2, dtype=dt_name)
            torch.cuda.synchronize()
            rt.prof_enable(True)
            t = time.perf_counter()
            for _ in range(20):
                rt.sweep(B2, st2, q2, dtype=dt_name)
            torch.cuda.synchronize()
            el = (time.perf_counter() - t) / 20
            nk, msk, _ = rt.prof_read("sweep_" + dt_name)
            rt.prof_enable(False)
            # per call of rte_sweep (host, launch and reduction included), and
            # per sweep kernel launch (HIP events around the launch)
            gd[f"single64sq_{dt_name}"] = B2.ndofs[0] * B2.n_ords[0] / el / 1e9
            gd[f"single64sq_{dt_name}_kernel"] = B2.ndofs[0] * B2.n_ords[0] / (msk / max(nk, 1) * 1e-3) / 1e9
            gd[f"single64sq_{dt_name}_plan"] = B2.sweep_plan(dt_name)
        out["sweep_gdof_s"] = gd
        log(f"sweep GDoF/s: {gd}")

    jobs = [("solve", ("cfg3", k), te_mu[k], n, 16) for k in range(n_err)]
    gpu_phis = {"cfg3": phis3}
    if not args.no_mlp or not args.no_uneven:
        del B, st, ss, G, phi
        torch.cuda.empty_cache()
    if not args.no_mlp:
        out["learned"] = learned_leg(args, common)
        gpu_phis["cfg5"] = out["learned"].pop("_phis")
        jobs += out["learned"].pop("_oracle_jobs")
        torch.cuda.empty_cache()
    if not args.no_uneven:
        out["uneven"] = uneven_leg(args, common)
        gpu_phis["cfg4"] = out["uneven"].pop("_phis")
        jobs += out["uneven"].pop("_oracle_jobs")

    if not args.no_cpu_baseline:
        # the oracle on the host's cores: the CPU baseline (checkerboard 96^2
        # solves and one 64^2 sweep) and the FP64 reference fluxes the GPU's
        # results are compared with
        procs = max(1, len(os.sched_getaffinity(0)))
        jobs.append(("sweep", ("cfg2", 0), None, None, None))
        log(f"oracle: {len(jobs)} jobs on {procs} processes ({cpu_model()})")
        res, wall = run_oracle_jobs(jobs, procs)
        t3 = [r["t"] for r in res if r["kind"] == "solve" and r["key"][0] == "cfg3"]
        sw = [r for r in res if r["kind"] == "sweep"][0]
        out["cpu_baseline"] = {
            "value": procs / float(np.mean(t3)), "unit": "solves/s", "cores": procs, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{len(t3)} of the {len(te_mu)} test parameters of the same workload, each one oracle "
                      f"FGMRES-DSA solve (FP64, sparse-direct sweeps and DSA, rtol 1e-8) in its own "
                      f"single-threaded process, {procs} processes at once; value = processes / mean "
                      f"solve time ({np.mean(t3):.1f} s); the pool ran {len(jobs)} oracle jobs in {wall:.0f} s",
            "sweep_64sq_f64_gdof_s_per_process": sw["dof"] / sw["t"] / 1e9,
            "sweep_64sq_f64_gdof_s_pool": procs * sw["dof"] / sw["t"] / 1e9,
        }
        out["error_vs_oracle"] = {
            "reference": "oracle FGMRES-DSA (FP64) solved to rtol 1e-12; relative L2 error of the GPU flux",
            "cfg3_96sq": error_summary(gpu_phis["cfg3"], res, "cfg3")}
        if "cfg5" in gpu_phis:
            out["error_vs_oracle"]["cfg5_128sq"] = error_summary(gpu_phis["cfg5"], res, "cfg5")
        if "cfg4" in gpu_phis:
            out["error_vs_oracle"]["cfg4_uneven_one_per_group"] = error_summary(gpu_phis["cfg4"], res, "cfg4")
        log(f"CPU baseline: {out['cpu_baseline']['value']:.4f} solves/s; error vs oracle "
            f"{_json(out['error_vs_oracle'])}")
    else:
        out["cpu_baseline"] = None
    print(_json(out), flush=True)


if __name__ == "__main__":
    main()
