"""Python binding of the MI355X RTE / FGMRES-ROMSAD library.

Argument marshalling only: every numerical step runs in the HIP library
(librte_romsad.so, C ABI in include/rte_romsad.h).  Device arrays are torch
tensors on the current CUDA (HIP) device; their pointers and the current
stream are handed to the library.
"""
import ctypes as C

import numpy as np

from . import _lib as L
from ._lib import (RTE_BF16, RTE_F32, RTE_F64, RTE_PC_DSA, RTE_PC_MLP, RTE_PC_NONE,  # noqa: F401
                   RTE_PC_ROMSAD, RteError, check)

__all__ = ["Batch", "quadrature", "sweep", "scalar_flux", "apply_A", "rhs", "dsa_apply",
           "fgmres_solve", "SolveOptions", "Rom", "romsad_build_greedy", "romsad_apply", "Mlp",
           "mlp_snapshots"]


def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dt(dtype):
    return {"f64": RTE_F64, "f32": RTE_F32, "bf16": RTE_BF16, RTE_F64: RTE_F64, RTE_F32: RTE_F32,
            RTE_BF16: RTE_BF16}[dtype]


def quadrature(spec):
    """Ordinates of a quadrature spec ('gl', n) or ('cl', n_theta, n_z, folded),
    computed by the library."""
    lib = L.lib()
    if spec[0] == "gl":
        n = spec[1]
        ox, oy, w = (np.zeros(n) for _ in range(3))
        check(lib.rte_quadrature_gl(n, *(a.ctypes.data_as(L.pdbl) for a in (ox, oy, w))), "quadrature")
        return ox, oy, w
    nt, nz = spec[1], spec[2]
    folded = bool(spec[3]) if len(spec) > 3 else False
    n = nt * nz // (2 if folded else 1)
    ox, oy, w = (np.zeros(n) for _ in range(3))
    check(lib.rte_quadrature_cl(nt, nz, int(folded), *(a.ctypes.data_as(L.pdbl) for a in (ox, oy, w))),
          "quadrature")
    return ox, oy, w


class Batch:
    """A batch of parameter instances (problem dicts as produced by synth)."""

    def __init__(self, problems):
        lib = L.lib()
        self.problems = list(problems)
        n = len(self.problems)
        descs = (L.InstanceDesc * n)()
        self._keep = []
        for k, p in enumerate(self.problems):
            ox, oy, w = quadrature(p["quad"])
            reg = np.ascontiguousarray(p["region"], dtype=np.int32)
            self._keep += [ox, oy, w, reg]
            box = p["box"]
            d = descs[k]
            d.dim, d.nx, d.ny = p["dim"], p["nx"], p["ny"]
            d.x0, d.x1, d.y0, d.y1 = box
            d.n_ord = len(w)
            d.omega_x = ox.ctypes.data_as(L.pdbl)
            d.omega_y = oy.ctypes.data_as(L.pdbl)
            d.weight = w.ctypes.data_as(L.pdbl)
            d.region = reg.ctypes.data_as(L.pi32)
            d.n_regions = int(len(p["sigma_t"]))
        h = C.c_void_p()
        check(lib.rte_batch_create(descs, n, C.byref(h)), "rte_batch_create")
        self.h = h
        self.n = n
        self.offsets = [lib.rte_batch_offset(h, k) for k in range(n)]
        self.ndofs = [lib.rte_batch_ndof(h, k) for k in range(n)]
        self.psi_offsets = [lib.rte_batch_psi_offset(h, k) for k in range(n)]
        self.total_dof = lib.rte_batch_total_dof(h)
        self.total_psi = lib.rte_batch_total_psi(h)
        self.max_regions = lib.rte_batch_max_regions(h)
        self.n_ords = [len(self._keep[4 * k + 2]) for k in range(n)]
        fv = self.problems[0].get("field_values") if n else None
        if fv is not None:  # cross sections varying inside the cells: shape values at the Gauss points
            fv = np.ascontiguousarray(fv, dtype=np.float64)
            nq = int(round(np.sqrt(fv.shape[2])))
            check(lib.rte_batch_set_fields(h, int(fv.shape[0]), nq, fv.ctypes.data_as(L.pdbl)),
                  "rte_batch_set_fields")

    def set_sweep_plan(self, dtype, variant, G, threads, opl=1, order=0):
        check(L.lib().rte_batch_set_sweep_plan(self.h, _dt(dtype), variant, G, opl, threads),
              "rte_batch_set_sweep_plan")
        if order:
            check(L.lib().rte_batch_set_sweep_order(self.h, _dt(dtype), order), "rte_batch_set_sweep_order")

    def sweep_plan(self, dtype):
        out = (L.i32 * 6)()
        check(L.lib().rte_batch_sweep_plan(self.h, _dt(dtype), out), "rte_batch_sweep_plan")
        return {"variant": out[0], "G": out[1], "opl": out[2], "threads": out[3], "tuned": bool(out[4]),
                "order": out[5]}

    def __del__(self):
        try:
            if getattr(self, "h", None):
                L.lib().rte_batch_destroy(self.h)
                self.h = None
        except Exception:
            pass

    # ---- marshalling helpers
    def pack(self, vectors, device="cuda"):
        torch = _torch()
        return torch.from_numpy(np.concatenate([np.asarray(v, dtype=np.float64) for v in vectors])).to(device)

    def unpack(self, t):
        a = t.detach().cpu().numpy()
        return [a[o:o + n] for o, n in zip(self.offsets, self.ndofs)]

    def unpack_psi(self, t):
        a = t.detach().cpu().numpy()
        return [a[o:o + n * no].reshape(no, n) for o, n, no in zip(self.psi_offsets, self.ndofs, self.n_ords)]

    def sigma(self, device="cuda"):
        torch = _torch()
        st = np.zeros((self.n, self.max_regions))
        ss = np.zeros((self.n, self.max_regions))
        for k, p in enumerate(self.problems):
            st[k, :len(p["sigma_t"])] = p["sigma_t"]
            ss[k, :len(p["sigma_s"])] = p["sigma_s"]
        return torch.from_numpy(st).to(device), torch.from_numpy(ss).to(device)

    def inflow(self, device="cuda"):
        """[n][4] per-side inflow (left, right, bottom, top), or None if all zero.
        A problem's "inflow" is a constant (every side) or a dict keyed by
        "L", "R", "B", "T"."""
        torch = _torch()
        g = np.zeros((self.n, 4))
        for k, p in enumerate(self.problems):
            v = p.get("inflow", 0.0)
            if isinstance(v, dict):
                g[k] = [float(v.get(side, 0.0)) for side in ("L", "R", "B", "T")]
            else:
                g[k] = float(v)
        if not np.any(g):
            return None
        return torch.from_numpy(g).to(device)

    def source(self, device="cuda"):
        return self.pack([p["source"] for p in self.problems], device)

    def zeros(self, n=None):
        torch = _torch()
        return torch.zeros(self.total_dof if n is None else n, dtype=torch.float64, device="cuda")

    def empty(self, n=None):
        torch = _torch()
        return torch.empty(self.total_dof if n is None else n, dtype=torch.float64, device="cuda")


def sweep(batch, sigma_t, q, inflow=None, phi=True, psi=False, dtype="f64"):
    torch = _torch()
    phi_t = torch.empty(batch.total_dof, dtype=torch.float64, device="cuda") if phi else None
    psi_t = torch.empty(batch.total_psi, dtype=torch.float64, device="cuda") if psi else None
    check(L.lib().rte_sweep(batch.h, _ptr(sigma_t), _ptr(q), _ptr(inflow), _ptr(phi_t), _ptr(psi_t),
                            _dt(dtype), _stream()), "rte_sweep")
    return phi_t, psi_t


def sweep_noalloc(batch, sigma_t, q, phi, inflow=None, dtype="f64"):
    """rte_sweep_noalloc into the caller's phi (the library allocates nothing)."""
    check(L.lib().rte_sweep_noalloc(batch.h, _ptr(sigma_t), _ptr(q), _ptr(inflow), _ptr(phi), _dt(dtype),
                                    _stream()), "rte_sweep_noalloc")
    return phi


def scalar_flux(batch, psi):
    out = batch.zeros()
    check(L.lib().rte_scalar_flux(batch.h, _ptr(psi), _ptr(out), _stream()), "rte_scalar_flux")
    return out


def apply_A(batch, sigma_t, sigma_s, x, dtype="f64"):
    y = batch.zeros()
    check(L.lib().rte_apply_A(batch.h, _ptr(sigma_t), _ptr(sigma_s), _ptr(x), _ptr(y), _dt(dtype),
                              _stream()), "rte_apply_A")
    return y


def rhs(batch, sigma_t, G, inflow=None, dtype="f64"):
    y = batch.zeros()
    check(L.lib().rte_rhs(batch.h, _ptr(sigma_t), _ptr(G), _ptr(inflow), _ptr(y), _dt(dtype),
                          _stream()), "rte_rhs")
    return y


_DSA_VARIANTS = {"fc": 0, "pc": 1}


def dsa_apply(batch, sigma_t, sigma_s, v, inner_tol=1e-13, inner_max=2000, restart=60, variant="fc"):
    z = batch.zeros()
    iters = np.zeros(batch.n, dtype=np.int32)
    check(L.lib().rte_dsa_apply(batch.h, _ptr(sigma_t), _ptr(sigma_s), _ptr(v), _ptr(z), inner_tol,
                                inner_max, restart, _DSA_VARIANTS[variant],
                                iters.ctypes.data_as(L.pi32), _stream()),
          "rte_dsa_apply")
    return z, iters


class SolveOptions:
    def __init__(self, precond="dsa", m=30, max_cycles=20, sweep_dtype="f64", rtol=1e-8, window=2,
                 dsa_inner_max=30, dsa_restart=30, dsa_inner_tol=1e-10, window_cycles=0, use_graph=False,
                 dsa_variant="fc", breakdown_tol=0.0):
        self.precond = {"none": RTE_PC_NONE, "dsa": RTE_PC_DSA, "romsad": RTE_PC_ROMSAD,
                        "mlp": RTE_PC_MLP}[precond] if isinstance(precond, str) else precond
        self.m, self.max_cycles, self.sweep_dtype, self.rtol = m, max_cycles, sweep_dtype, rtol
        self.window = window
        self.dsa_inner_max, self.dsa_restart, self.dsa_inner_tol = dsa_inner_max, dsa_restart, dsa_inner_tol
        self.window_cycles = window_cycles
        self.use_graph = use_graph
        self.dsa_variant = dsa_variant
        self.breakdown_tol = breakdown_tol

    def c(self):
        o = L.SolveOpts()
        o.precond, o.m, o.max_cycles = self.precond, self.m, self.max_cycles
        o.sweep_dtype = _dt(self.sweep_dtype)
        o.rtol, o.window = self.rtol, self.window
        o.dsa_inner_max, o.dsa_restart, o.dsa_inner_tol = self.dsa_inner_max, self.dsa_restart, self.dsa_inner_tol
        o.keep_krylov = 0
        o.window_cycles = self.window_cycles
        o.use_graph = 1 if self.use_graph else 0
        o.dsa_variant = _DSA_VARIANTS[self.dsa_variant]
        o.breakdown_tol = self.breakdown_tol
        return o


_STATS_DTYPE = None


def _stats_array(stats):
    """Per-instance solve statistics as a numpy structured array (a view of the
    C structs, no copy): stats[k]["iterations"], stats["true_relres"], ..."""
    global _STATS_DTYPE
    if _STATS_DTYPE is None:
        T = L.SolveStats
        ct = {C.c_int32: "<i4", C.c_double: "<f8"}
        _STATS_DTYPE = np.dtype({"names": [f for f, _ in T._fields_],
                                 "formats": [ct[t] for _, t in T._fields_],
                                 "offsets": [getattr(T, f).offset for f, _ in T._fields_],
                                 "itemsize": C.sizeof(T)})
    return np.frombuffer(stats, dtype=_STATS_DTYPE)


def fgmres_solve(batch, sigma_t, sigma_s, G, inflow=None, opts=None, rom=None, mlp=None, mu=None):
    opts = opts or SolveOptions()
    phi = batch.empty()  # the library starts from phi = 0
    stats = (L.SolveStats * batch.n)()
    co = opts.c()
    mu_dim = 0 if mu is None else int(mu.shape[1])
    st = L.lib().fgmres_solve(batch.h, _ptr(sigma_t), _ptr(sigma_s), _ptr(G), _ptr(inflow), C.byref(co),
                              rom.h if rom is not None else None, mlp.h if mlp is not None else None,
                              _ptr(mu), mu_dim, _ptr(phi), stats, _stream())
    check(st, "fgmres_solve")
    return phi, _stats_array(stats), st


def si_solve(batch, sigma_t, sigma_s, G, inflow=None, opts=None, rom=None):
    """Source iteration with synthetic acceleration; opts.max_cycles bounds the iterations."""
    opts = opts or SolveOptions()
    phi = batch.empty()  # the library starts from phi = 0
    stats = (L.SolveStats * batch.n)()
    co = opts.c()
    st = L.lib().si_solve(batch.h, _ptr(sigma_t), _ptr(sigma_s), _ptr(G), _ptr(inflow), C.byref(co),
                          rom.h if rom is not None else None, _ptr(phi), stats, _stream())
    check(st, "si_solve")
    return phi, _stats_array(stats), st


class Rom:
    def __init__(self, h):
        self.h = h

    def __del__(self):
        try:
            if getattr(self, "h", None):
                L.lib().rte_rom_destroy(self.h)
                self.h = None
        except Exception:
            pass

    @property
    def rank(self):
        return L.lib().rte_rom_rank(self.h)

    @staticmethod
    def from_basis(batch, U):
        """U: device tensor holding r basis vectors of instance 0's psi-space."""
        npsi = batch.ndofs[0] * batch.n_ords[0]
        if U.numel() % npsi:
            raise ValueError("basis size is not a multiple of the psi-space size")
        h = C.c_void_p()
        check(L.lib().rte_rom_from_basis(batch.h, _ptr(U.contiguous()), int(U.numel() // npsi),
                                         C.byref(h), _stream()), "rte_rom_from_basis")
        return Rom(h)

    def export(self, nord, ndof, n_regions):
        r = self.rank
        U = np.zeros((r, nord, ndof))
        W1 = np.zeros((r, ndof))
        Ww = np.zeros((r, ndof))
        AD = np.zeros((r, r))
        G = np.zeros((n_regions, r, r))
        S = np.zeros((n_regions, r, r))
        check(L.lib().rte_rom_export(self.h, *(a.ctypes.data_as(L.pdbl) for a in (U, W1, Ww, AD, G, S))),
              "rte_rom_export")
        return dict(U=U, W1=W1, Ww=Ww, AD=AD, G=G, S=S)

    def save(self, path):
        check(L.lib().rte_rom_save(self.h, path.encode()), "rte_rom_save")

    @staticmethod
    def load(path):
        h = C.c_void_p()
        check(L.lib().rte_rom_load(path.encode(), C.byref(h)), "rte_rom_load")
        return Rom(h)

    @staticmethod
    def set(batch, roms, rom_of_instance):
        """A ROM set: instance k of `batch` uses roms[rom_of_instance[k]]."""
        arr = (C.c_void_p * len(roms))(*[r.h for r in roms])
        idx = np.ascontiguousarray(rom_of_instance, dtype=np.int32)
        h = C.c_void_p()
        check(L.lib().rte_rom_set_create(batch.h, arr, len(roms), idx.ctypes.data_as(L.pi32), C.byref(h)),
              "rte_rom_set_create")
        out = Rom(h)
        out._members = list(roms)  # the members must outlive the set
        return out


def romsad_build_greedy(batch, sigma_t, sigma_s, G, inflow=None, window=2, mu1_index=0, eps_rom=1e-9,
                        n_giter=16, eps_qr=1e-13, hf_rtol=1e-11, hf_dsa_tol=0.0):
    h = C.c_void_p()
    rep = L.GreedyReport()
    check(L.lib().romsad_build_greedy(batch.h, _ptr(sigma_t), _ptr(sigma_s), _ptr(G), _ptr(inflow),
                                      window, mu1_index, eps_rom, n_giter, eps_qr, hf_rtol, hf_dsa_tol,
                                      C.byref(h), C.byref(rep), _stream()), "romsad_build_greedy")
    report = dict(sampled=list(rep.sampled[:rep.n_sampled]),
                  max_residual=list(rep.max_residual[:max(rep.n_sampled - 1, 0) + 1]),
                  rank=rep.rank, truncated=rep.truncated, seconds_step=list(rep.seconds_step))
    return Rom(h), report


def romsad_apply(rom, batch, sigma_t, sigma_s, v):
    z = batch.zeros()
    st = L.lib().romsad_apply(rom.h, batch.h, _ptr(sigma_t), _ptr(sigma_s), _ptr(v), _ptr(z), _stream())
    check(st, "romsad_apply")
    return z


def graph_captures():
    """Operator applications captured into HIP graphs since the library loaded."""
    return int(L.lib().rte_graph_captures())


def prof_enable(on=True):
    check(L.lib().rte_prof_enable(1 if on else 0), "rte_prof_enable")


PROF_SLOTS = {"sweep_f64": 0, "sweep_f32": 1, "dsa_op": 2, "mgs": 3, "rom": 4}


def prof_mark(mark_id=0):
    """Enqueue an empty marker kernel (visible in kernel traces) on the current stream."""
    check(L.lib().rte_prof_mark(int(mark_id), _stream()), "rte_prof_mark")


def prof_read(slot):
    """(launches, total_ms, total_units) recorded for a profiler slot."""
    n, ms, u = L.i64(), L.dbl(), L.dbl()
    s = PROF_SLOTS[slot] if isinstance(slot, str) else slot
    check(L.lib().rte_prof_read(s, C.byref(n), C.byref(ms), C.byref(u)), "rte_prof_read")
    return n.value, ms.value, u.value


class Mlp:
    """GELU MLP handle (n_in -> width x depth -> n_out) living on the device."""

    def __init__(self, n_in, width=256, depth=4, n_out=32):
        h = C.c_void_p()
        check(L.lib().rte_mlp_create(n_in, width, depth, n_out, C.byref(h)), "rte_mlp_create")
        self.h = h
        self.n_in, self.width, self.depth, self.n_out = n_in, width, depth, n_out
        self.nparams = L.lib().rte_mlp_num_params(h)

    def __del__(self):
        try:
            if getattr(self, "h", None):
                L.lib().rte_mlp_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def init(self, seed=0):
        check(L.lib().rte_mlp_init(self.h, seed), "rte_mlp_init")

    def set_params(self, flat, scale=None, shift=None):
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        assert flat.size == self.nparams
        sc = None if scale is None else np.ascontiguousarray(scale, dtype=np.float32)
        sh = None if shift is None else np.ascontiguousarray(shift, dtype=np.float32)
        check(L.lib().rte_mlp_set_params(self.h, flat.ctypes.data, None if sc is None else sc.ctypes.data,
                                         None if sh is None else sh.ctypes.data), "rte_mlp_set_params")

    def get_params(self):
        p = np.zeros(self.nparams, dtype=np.float32)
        sc = np.zeros(self.n_out, dtype=np.float32)
        sh = np.zeros(self.n_out, dtype=np.float32)
        check(L.lib().rte_mlp_get_params(self.h, p.ctypes.data, sc.ctypes.data, sh.ctypes.data),
              "rte_mlp_get_params")
        return p, sc, sh

    def forward(self, X, dtype="bf16"):
        torch = _torch()
        Y = torch.empty((X.shape[0], self.n_out), dtype=torch.float32, device="cuda")
        check(L.lib().rte_mlp_forward(self.h, _ptr(X.contiguous()), _ptr(Y), int(X.shape[0]), _dt(dtype),
                                      _stream()), "rte_mlp_forward")
        return Y

    def grad(self, X, T, dtype="bf16"):
        torch = _torch()
        g = torch.empty(self.nparams, dtype=torch.float32, device="cuda")
        loss = C.c_float()
        check(L.lib().rte_mlp_grad(self.h, _ptr(X.contiguous()), _ptr(T.contiguous()), int(X.shape[0]),
                                   _dt(dtype), C.byref(loss), _ptr(g), _stream()), "rte_mlp_grad")
        return loss.value, g

    def adam_step(self, grad, lr=1e-3):
        """One Adam step with a given device gradient (FP32, num_params)."""
        check(L.lib().rte_mlp_adam_step(self.h, _ptr(grad.contiguous()), lr, _stream()), "rte_mlp_adam_step")

    def train(self, X, T, epochs=50, batch=256, lr=1e-3, seed=0, standardize=True):
        hist = np.zeros(epochs, dtype=np.float32)
        check(L.lib().rte_mlp_train(self.h, _ptr(X.contiguous()), _ptr(T.contiguous()), int(X.shape[0]),
                                    epochs, batch, lr, seed, 1 if standardize else 0, hist.ctypes.data,
                                    _stream()), "rte_mlp_train")
        return hist


def mlp_snapshots(batch, sigma_t, sigma_s, G, rom, opts, mu, inflow=None):
    """(X, T, valid) training rows from FGMRES runs on every instance of batch."""
    torch = _torch()
    w = opts.window
    r = rom.rank
    mu_dim = int(mu.shape[1])
    X = torch.zeros((batch.n * w, mu_dim + r), dtype=torch.float32, device="cuda")
    T = torch.zeros((batch.n * w, r), dtype=torch.float32, device="cuda")
    valid = torch.zeros(batch.n * w, dtype=torch.int32, device="cuda")
    co = opts.c()
    check(L.lib().rte_mlp_snapshots(batch.h, _ptr(sigma_t), _ptr(sigma_s), _ptr(G), _ptr(inflow), rom.h,
                                    C.byref(co), _ptr(mu.contiguous()), mu_dim, _ptr(X), _ptr(T), _ptr(valid),
                                    _stream()), "rte_mlp_snapshots")
    return X, T, valid
