"""ctypes declarations of the C ABI in include/rte_romsad.h.

Loading fails loudly when the built library is missing: there is no CPU
fallback for any entry point.
"""
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librte_romsad.so")

RTE_OK, RTE_EINVAL, RTE_EHIP, RTE_ENOMEM, RTE_EBREAKDOWN, RTE_ESINGULAR, RTE_EIO = 0, -1, -2, -3, -4, -5, -6
RTE_ENONFINITE = -7
RTE_WNOTCONV = 1
RTE_F64, RTE_F32, RTE_BF16 = 0, 1, 2
RTE_PC_NONE, RTE_PC_DSA, RTE_PC_ROMSAD, RTE_PC_MLP = 0, 1, 2, 3

vp = C.c_void_p
i32 = C.c_int32
i64 = C.c_int64
dbl = C.c_double
pdbl = C.POINTER(C.c_double)
pi32 = C.POINTER(C.c_int32)


class InstanceDesc(C.Structure):
    _fields_ = [("dim", i32), ("nx", i32), ("ny", i32),
                ("x0", dbl), ("x1", dbl), ("y0", dbl), ("y1", dbl),
                ("n_ord", i32), ("omega_x", pdbl), ("omega_y", pdbl), ("weight", pdbl),
                ("region", pi32), ("n_regions", i32)]


class SolveOpts(C.Structure):
    _fields_ = [("precond", i32), ("m", i32), ("max_cycles", i32), ("sweep_dtype", i32),
                ("rtol", dbl), ("window", i32), ("dsa_inner_max", i32), ("dsa_restart", i32),
                ("dsa_inner_tol", dbl), ("keep_krylov", i32), ("window_cycles", i32),
                ("use_graph", i32), ("dsa_variant", i32), ("breakdown_tol", dbl)]


class SolveStats(C.Structure):
    _fields_ = [("iterations", i32), ("cycles", i32), ("sweeps_f32", i32), ("sweeps_f64", i32),
                ("pc_rom", i32), ("pc_dsa", i32), ("pc_mlp", i32), ("pc_fallback", i32),
                ("status", i32), ("true_relres", dbl), ("est_relres", dbl), ("rom_singular", i32),
                ("pad", i32), ("mlp_rom_diff", dbl)]


class GreedyReport(C.Structure):
    _fields_ = [("n_sampled", i32), ("sampled", i32 * 256), ("max_residual", dbl * 256),
                ("rank", i32), ("truncated", i32), ("seconds_step", dbl * 5)]


# name -> (restype, argtypes)
SIGNATURES = {
    "rte_status_string": (C.c_char_p, [C.c_int]),
    "rte_quadrature_cl": (C.c_int, [C.c_int, C.c_int, C.c_int, pdbl, pdbl, pdbl]),
    "rte_quadrature_gl": (C.c_int, [C.c_int, pdbl, pdbl, pdbl]),
    "rte_batch_create": (C.c_int, [C.POINTER(InstanceDesc), C.c_int, C.POINTER(vp)]),
    "rte_batch_destroy": (None, [vp]),
    "rte_batch_size": (C.c_int, [vp]),
    "rte_batch_ndof": (i64, [vp, C.c_int]),
    "rte_batch_offset": (i64, [vp, C.c_int]),
    "rte_batch_total_dof": (i64, [vp]),
    "rte_batch_psi_offset": (i64, [vp, C.c_int]),
    "rte_batch_total_psi": (i64, [vp]),
    "rte_batch_max_regions": (C.c_int, [vp]),
    "rte_sweep": (C.c_int, [vp, vp, vp, vp, vp, vp, C.c_int, vp]),
    "rte_sweep_noalloc": (C.c_int, [vp, vp, vp, vp, vp, C.c_int, vp]),
    "rte_scalar_flux": (C.c_int, [vp, vp, vp, vp]),
    "rte_apply_A": (C.c_int, [vp, vp, vp, vp, vp, C.c_int, vp]),
    "rte_rhs": (C.c_int, [vp, vp, vp, vp, vp, C.c_int, vp]),
    "rte_dsa_apply": (C.c_int, [vp, vp, vp, vp, vp, dbl, C.c_int, C.c_int, C.c_int, pi32, vp]),
    "fgmres_solve": (C.c_int, [vp, vp, vp, vp, vp, C.POINTER(SolveOpts), vp, vp, vp, C.c_int, vp,
                               C.POINTER(SolveStats), vp]),
    "si_solve": (C.c_int, [vp, vp, vp, vp, vp, C.POINTER(SolveOpts), vp, vp, C.POINTER(SolveStats), vp]),
    "romsad_build_greedy": (C.c_int, [vp, vp, vp, vp, vp, C.c_int, C.c_int, dbl, C.c_int, dbl, dbl,
                                      dbl, C.POINTER(vp), C.POINTER(GreedyReport), vp]),
    "rte_rom_from_basis": (C.c_int, [vp, vp, C.c_int, C.POINTER(vp), vp]),
    "romsad_apply": (C.c_int, [vp, vp, vp, vp, vp, vp, vp]),
    "rte_rom_set_create": (C.c_int, [vp, C.POINTER(vp), C.c_int, pi32, C.POINTER(vp)]),
    "rte_rom_rank": (C.c_int, [vp]),
    "rte_rom_export": (C.c_int, [vp, pdbl, pdbl, pdbl, pdbl, pdbl, pdbl]),
    "rte_rom_save": (C.c_int, [vp, C.c_char_p]),
    "rte_rom_load": (C.c_int, [C.c_char_p, C.POINTER(vp)]),
    "rte_rom_destroy": (None, [vp]),
    "rte_mlp_create": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(vp)]),
    "rte_mlp_destroy": (None, [vp]),
    "rte_mlp_init": (C.c_int, [vp, C.c_uint64]),
    "rte_mlp_num_params": (i64, [vp]),
    "rte_mlp_set_params": (C.c_int, [vp, vp, vp, vp]),
    "rte_mlp_get_params": (C.c_int, [vp, vp, vp, vp]),
    "rte_mlp_forward": (C.c_int, [vp, vp, vp, C.c_int, C.c_int, vp]),
    "rte_mlp_grad": (C.c_int, [vp, vp, vp, C.c_int, C.c_int, C.POINTER(C.c_float), vp, vp]),
    "rte_mlp_adam_step": (C.c_int, [vp, vp, C.c_float, vp]),
    "rte_graph_captures": (i64, []),
    "rte_mlp_train": (C.c_int, [vp, vp, vp, C.c_int, C.c_int, C.c_int, C.c_float, C.c_uint64, C.c_int,
                                vp, vp]),
    "rte_mlp_snapshots": (C.c_int, [vp, vp, vp, vp, vp, vp, C.POINTER(SolveOpts), vp, C.c_int, vp, vp, vp,
                                    vp]),
    "rte_batch_set_sweep_plan": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]),
    "rte_batch_set_fields": (C.c_int, [vp, C.c_int, C.c_int, pdbl]),
    "rte_batch_sweep_plan": (C.c_int, [vp, C.c_int, C.POINTER(i32)]),
    "rte_batch_set_sweep_order": (C.c_int, [vp, C.c_int, C.c_int]),
    "rte_prof_enable": (C.c_int, [C.c_int]),
    "rte_prof_mark": (C.c_int, [C.c_int, vp]),
    "rte_prof_read": (C.c_int, [C.c_int, C.POINTER(i64), C.POINTER(dbl), C.POINTER(dbl)]),
}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run python -c 'import __graft_entry__; __graft_entry__.build()')")
        # torch ships its own HIP runtime (same soname); loading torch first makes
        # the library bind to that single runtime instead of a second copy.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            if hasattr(L, name):
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
        _lib = L
    return _lib


class RteError(RuntimeError):
    def __init__(self, status, where):
        msg = lib().rte_status_string(status).decode()
        super().__init__(f"{where}: {msg} ({status})")
        self.status = status


def check(status, where):
    if status < 0:
        raise RteError(status, where)
    return status
