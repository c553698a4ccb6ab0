"""Writes varscat_oracle.json: the oracle's GMRES-FC-DSA and GMRES-PC-DSA
sweep counts on the variable-scattering problem of section 5.3 (80^2 cells,
CL(30, 6), the ten seeded test values of mu_s), with the DSA solved exactly
(sparse LU of the moment system) and relative residual 1e-11, as in the
paper's online table.  n_sweep = 1 + FGMRES iterations (the sweep of b~).
Calls only the oracle and the seeded input generators:

    python tests/golden/make_varscat_oracle.py      (about two minutes on 8 cores)
"""
import json
import multiprocessing as mp
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))


def _job(arg):
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle import dsa, fgmres, transport
    from synth import varscat_problem
    k, mu, variant = arg
    P = transport.Problem(varscat_problem(mu))
    b = transport.b_tilde(P)
    D = dsa.DSA(P, variant)
    r = fgmres.fgmres(lambda x: transport.A_tilde_apply(P, x), b, lambda j, v: D.apply(v), m=60, rtol=1e-11)
    return k, variant, int(r.iterations), float(r.true_relres), bool(r.converged)


def main():
    from synth import varscat_sets
    _, te = varscat_sets()
    jobs = [(k, float(m), v) for v in ("pc", "fc") for k, m in enumerate(te)]
    procs = max(1, min(len(os.sched_getaffinity(0)), 8))
    with mp.get_context("spawn").Pool(procs) as pool:
        res = pool.map(_job, jobs)
    out = {"source": "oracle FGMRES (m = 60, rtol 1e-11) with the exact FC / PC DSA, section 5.3 problem",
           "mu_s": [float(m) for m in te]}
    for v in ("fc", "pc"):
        its = [r[2] for r in sorted(res) if r[1] == v]
        assert all(r[4] for r in res if r[1] == v)
        out[v] = {"iterations": its, "nsweep_mean": 1.0 + sum(its) / len(its),
                  "max_true_relres": max(r[3] for r in res if r[1] == v)}
    with open(os.path.join(HERE, "varscat_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({v: out[v]["nsweep_mean"] for v in ("fc", "pc")}))


if __name__ == "__main__":
    main()
