"""Reference fluxes from the oracle for the full-size GPU tests: FGMRES with the
oracle's exact DSA, in separate single-threaded processes, started before the
GPU work so that they run beside it."""
import multiprocessing as mp
import os


def _solve(args):
    spec, rtol = args
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle import dsa, fgmres, transport
    P = transport.Problem(spec)
    D = dsa.DSA(P)
    r = fgmres.fgmres(lambda x: transport.A_tilde_apply(P, x), transport.b_tilde(P), lambda j, v: D.apply(v),
                      m=30, rtol=rtol, max_cycles=40)
    return r.x, r.true_relres


class OracleRefs:
    """Start oracle solves of `specs` to `rtol`; get() returns [(phi, relres)]."""

    def __init__(self, specs, rtol):
        self._pool = mp.get_context("spawn").Pool(len(specs))
        self._res = self._pool.map_async(_solve, [(s, rtol) for s in specs])

    def get(self, timeout=600):
        try:
            return self._res.get(timeout)
        finally:
            self._pool.terminate()
            self._pool.join()
