"""msrs_solve_global_noalloc: the online solve with its workspace in the
library's fixed device array (no device allocation in the call) against
msrs_solve_global's results on the same handle, bit for bit, on two calls in
a row (the second with fewer requests), and its refusal of a batch whose
workspace exceeds the fixed array."""
import ctypes as C

import numpy as np
import pytest

import synth
from synth import configs

pytestmark = pytest.mark.gpu


def _noalloc(lib):
    return lib.lib.msrs_solve_global_noalloc


def _solve_both(lib, pr, reqs):
    import torch
    call = _noalloc(lib)
    L = pr.layout()
    f = torch.tensor(reqs, device="cuda:0")
    ua = torch.empty((reqs.shape[0], L.n_nodes), device="cuda:0", dtype=torch.float64)
    ub = torch.full_like(ua, float("nan"))
    pr.solve_global(f, ua)
    st = call(pr.h, reqs.shape[0], C.c_void_p(f.data_ptr()), C.c_void_p(ub.data_ptr()),
              C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == lib.OK, lib.lib.msrs_last_error(pr.h)
    torch.cuda.synchronize()
    return ua.cpu().numpy(), ub.cpu().numpy()


def test_noalloc_solve_equals_the_allocating_solve(lib):
    """40 requests (two launches of the fixed workspace), then 5: the second
    call finds the first call's contents in the array and must not depend on
    them."""
    from gpu_cases import resident
    cfg = configs.small_elliptic(N=64, M=4, delta=4, s=12, k=8)
    pr = resident(cfg, lib.PREC_FP32_IR, max_batch=64)
    try:
        for n, seed0 in ((40, 0), (5, 100)):
            reqs = synth.fourier_boundary(cfg["N"], range(seed0, seed0 + n))
            ua, ub = _solve_both(lib, pr, reqs)
            assert np.array_equal(ua, ub), n
    finally:
        pr.close()


def test_noalloc_solve_kinetic_model(lib):
    from gpu_cases import resident
    from oracle import kinetic as K
    cfg = dict(name="kin", kind="kinetic", N=512, M=8, overlap=np.full(8, 32, np.int32), s=40, k=8,
               n_vel=32, eps=2.0 ** -6, coef=synth.kinetic_sigma(512, 0.05), seed=3)
    pr = resident(cfg, lib.PREC_FP32_IR, max_batch=64)
    try:
        v, _ = K.ordinates(32)
        rng = np.random.default_rng(7)
        for n in (33, 3):
            reqs = rng.standard_normal((n, 32))
            ua, ub = _solve_both(lib, pr, reqs)
            assert np.array_equal(ua, ub), n
    finally:
        pr.close()


def test_noalloc_refuses_batches_beyond_the_fixed_workspace(lib):
    """h = 1/256, 16 x 16 patches, rank 32: (boundary + coarse unknowns) x 32
    requests exceeds the 2 MiB array, 16 requests fit."""
    import torch
    from gpu_cases import resident
    N, M = 256, 16
    cfg = dict(name="wide", kind="elliptic", N=N, M=M, overlap=np.full(M * M, 4, np.int32), s=32, k=32,
               coef=synth.lognormal_coefficient(N, 0.05, 7), phi=synth.dirichlet_sin_cos(N), seed=2)
    pr = resident(cfg, lib.PREC_FP32_IR, max_batch=64)
    try:
        call = _noalloc(lib)
        L = pr.layout()
        assert (L.coarse_dim + 60 * 32) * 32 > (1 << 18) >= (L.coarse_dim + 60 * 32) * 16
        reqs = synth.fourier_boundary(N, range(32))
        f = torch.tensor(reqs, device="cuda:0")
        u = torch.empty((32, L.n_nodes), device="cuda:0", dtype=torch.float64)
        st = call(pr.h, 32, C.c_void_p(f.data_ptr()), C.c_void_p(u.data_ptr()), None)
        assert st == lib.ERR_ARG and b"fixed workspace" in lib.lib.msrs_last_error(pr.h)
        ua, ub = _solve_both(lib, pr, reqs[:16])
        assert np.array_equal(ua, ub)
    finally:
        pr.close()
