"""rte_sweep_noalloc (the sweep for callers that cannot allocate) against
rte_sweep and the oracle: two calls in a row, the second on a smaller batch,
and the rejection of a batch whose partial fluxes exceed the static array."""
import ctypes as C

import numpy as np
import pytest

from oracle import transport as tr
from synth import tiny_2d


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


def _noalloc(B, st, q, inflow, phi, dtype):
    import torch

    from paper_2410_08735_amd import _lib
    f = _lib.lib().rte_sweep_noalloc
    f.restype = C.c_int
    f.argtypes = [C.c_void_p] * 5 + [C.c_int, C.c_void_p]
    ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())
    return f(B.h, ptr(st), ptr(q), ptr(inflow), ptr(phi), dtype,
             C.c_void_p(torch.cuda.current_stream().cuda_stream))


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sweep_noalloc_matches_rte_sweep(dtype):
    import torch

    import paper_2410_08735_amd as rt
    code = {"f64": rt.RTE_F64, "f32": rt.RTE_F32}[dtype]
    tol = 1e-12 if dtype == "f64" else 1e-5
    big = [tiny_2d(seed=1, nx=13, ny=11, quad=("cl", 8, 4, False), n_regions=3, inflow=0.3),
           tiny_2d(seed=2, nx=24, ny=20, quad=("cl", 16, 4, True), n_regions=2),
           tiny_2d(seed=3, nx=9, ny=17, quad=("cl", 6, 2, False), n_regions=2, inflow=0.5)]
    small = [tiny_2d(seed=4, nx=5, ny=3, quad=("cl", 4, 2, True), n_regions=1)]
    for specs in (big, small):  # the second call is smaller: the array keeps the first call's data
        B = rt.Batch(specs)
        st, _ = B.sigma()
        q = B.source()
        inflow = B.inflow()
        ref_gpu, _ = rt.sweep(B, st, q, inflow=inflow, dtype=dtype)
        phi = torch.full((B.total_dof,), float("nan"), dtype=torch.float64, device="cuda")
        print(f"case: rte_sweep_noalloc {dtype}, {len(specs)} instances", flush=True)
        assert _noalloc(B, st, q, inflow, phi, code) == 0
        torch.cuda.synchronize()
        # same plan, same kernels: the same result as rte_sweep, bit for bit
        assert bool((phi == ref_gpu).all())
        for k, spec in enumerate(specs):
            ref = tr.b_tilde(tr.Problem(spec))
            assert rel(B.unpack(phi)[k], ref) <= tol, (k, rel(B.unpack(phi)[k], ref))


@pytest.mark.gpu
def test_sweep_noalloc_rejects_a_batch_beyond_its_scratch():
    import torch

    import paper_2410_08735_amd as rt
    # 128 x 128 cells, 128 ordinates, FP64: the default plan (8 ordinates per
    # work item) keeps 16 partial vectors of 65,536 DoFs per instance, 8 MiB;
    # nine instances need 72 MiB, above the 64 MiB array
    specs = [tiny_2d(seed=s, nx=128, ny=128, quad=("cl", 16, 16, True), n_regions=2) for s in range(9)]
    B = rt.Batch(specs)
    st, _ = B.sigma()
    q = B.source()
    phi = torch.zeros(B.total_dof, dtype=torch.float64, device="cuda")
    print("case: rte_sweep_noalloc over its limit (expects RTE_EINVAL, no launch)", flush=True)
    assert _noalloc(B, st, q, None, phi, rt.RTE_F64) == rt._lib.RTE_EINVAL
    assert float(phi.abs().max()) == 0.0
