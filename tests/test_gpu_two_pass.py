"""GPU parity of the two-pass randomized SVD (MSRS_FLAG_TWO_PASS) against the
oracle's two_pass_basis: the same snapshots, the adjoint local solves through
the same factor and sweeps (FP64, and FP32 with FP64 refinement), and the
basis from the SVD of Q^T G.

Bars: snapshots as the one-pass parity tests; the singular values of Q^T G
to 1e-9 sigma_1 (they come from the Gram matrix of G^T Q, whose leading
eigenvalues are resolved to rounding); orthonormal bases; the largest
principal angle <= 1e-6 where the relative gap of Q^T G's singular values at
k is at least 1e-3; and, against the Green's matrix built by the oracle's
delta solves, a projection error no larger than the one-pass basis's (the
two-pass basis is the best rank-k subspace of span(Y) in Frobenius norm).
"""
import numpy as np
import pytest

from synth import configs
from oracle import elliptic as E
from oracle.rangefinder import sin_max_angle

from gpu_cases import rel, run

pytestmark = pytest.mark.gpu

FP64, FP32_IR = 0, 1
FLAG_TWO_PASS = 64


def _check(cfg, out, tol_y):
    ref = E.offline(cfg["coef"], cfg["N"], cfg["M"], cfg["overlap"], cfg["s"], cfg["k"], seed=cfg["seed"], two_pass=True,
                    rank_tol=cfg.get("rank_tol", 0.0))
    for p, r in enumerate(ref):
        assert rel(out["Y"][p], r["Y"]) < tol_y, p
        k = r["Q"].shape[1]
        so, sg = r["sv"], out["sv"][p]
        n = min(len(so), k + 1)
        assert np.abs(sg[:n] - so[:n]).max() <= 1e-9 * so[0], p
        Qg = out["Q"][p]
        assert Qg.shape[1] == k
        assert np.abs(Qg.T @ Qg - np.eye(k)).max() < 1e-12, p
        gap = (so[k - 1] - so[k]) / so[0] if k < len(so) else 1.0
        if gap >= 1e-3:
            assert sin_max_angle(r["Q"], Qg) <= 1e-6, p
    return ref


@pytest.mark.parametrize("prec", [FP64, FP32_IR])
def test_two_pass_small_lognormal(gpu_two_pass_cfg_small, prec):
    cfg = gpu_two_pass_cfg_small
    print(f"[two-pass] small lognormal prec={prec}", flush=True)
    out = run(cfg, prec, flags=FLAG_TWO_PASS)
    assert out["stats"].error_latched == 0
    assert out["stats"].max_rel_residual <= (1e-10 if prec == FP32_IR else 1e-12)
    _check(cfg, out, 1e-11 if prec == FP64 else 1e-8)


@pytest.mark.parametrize("prec", [FP64, FP32_IR])
def test_two_pass_periodic_128_and_projection_error(gpu, prec):
    cfg = configs.elliptic_periodic_128()
    print(f"[two-pass] periodic 128 prec={prec}", flush=True)
    out = run(cfg, prec, flags=FLAG_TWO_PASS)
    assert out["stats"].error_latched == 0
    _check(cfg, out, 1e-11 if prec == FP64 else 1e-8)
    one = run(cfg, prec)
    geo = E.patch_geometry(cfg["N"], cfg["M"], cfg["overlap"])
    for p in (0, 5):
        G = E.full_basis_patch(cfg["coef"], cfg["N"], geo[p])
        e2 = np.linalg.norm(G - out["Q"][p] @ (out["Q"][p].T @ G))
        e1 = np.linalg.norm(G - one["Q"][p] @ (one["Q"][p].T @ G))
        assert e2 <= e1 * (1 + 1e-8), (p, e2, e1)


def test_two_pass_with_a_rank_tolerance(gpu):
    """rank_tol applies to the two-pass singular values (those of Q^T G): each
    patch keeps the numerical rank of Q^T G at rank_tol sigma_1, at most k."""
    # the singular values of Q^T G of these patches fall slowly (0.33-0.40 sigma_1
    # at j = 10); 0.45 keeps 3 to 6 columns, the nearest one 2e-3 sigma_1 away
    cfg = dict(configs.small_elliptic(N=64, M=2, delta=8, s=12, k=10, coef="lognormal"), rank_tol=0.45)
    print("[two-pass] rank_tol 0.45", flush=True)
    out = run(cfg, FP64, flags=FLAG_TWO_PASS)
    ref = _check(cfg, out, 1e-11)
    ranks = [r["Q"].shape[1] for r in ref]
    assert ranks == [inf.n_cols for inf in out["infos"]]
    assert min(ranks) < cfg["k"]


def test_two_pass_flag_is_refused_where_it_does_not_apply(gpu):
    from paper_1807_08848_amd import msrs
    d = msrs.make_desc(msrs.KIND_KINETIC_DO, 256, 4, [8] * 4, 16, 4, n_vel=8, eps=1.0, flags=FLAG_TWO_PASS)
    with pytest.raises(msrs.MsrsError):
        msrs.Problem(d)
    d = msrs.make_desc(msrs.KIND_ELLIPTIC_Q1, 64, 4, [0] * 16, 16, 8, flags=FLAG_TWO_PASS | msrs.FLAG_FULL_BASIS)
    with pytest.raises(msrs.MsrsError):
        msrs.Problem(d)


@pytest.fixture
def gpu_two_pass_cfg_small(gpu):
    return configs.small_elliptic(N=64, M=2, delta=8, s=10, k=6, coef="lognormal")


@pytest.fixture(scope="module")
def gpu(lib):
    return lib


def test_two_pass_graph_replays_match_eager(gpu):
    """The captured offline step with the two-pass range finder (forward and
    adjoint refinement at fixed iteration counts) replays to the eager results."""
    import torch
    from paper_1807_08848_amd import msrs
    cfg = configs.small_elliptic(N=64, M=4, delta=4, s=12, k=6, coef="lognormal")
    print("[two-pass] graph replays", flush=True)
    st = torch.cuda.Stream()
    d = msrs.make_desc(msrs.KIND_ELLIPTIC_Q1, cfg["N"], cfg["M"], list(cfg["overlap"]), cfg["s"], cfg["k"],
                       precision=FP32_IR, seed=cfg["seed"], flags=FLAG_TWO_PASS)
    with torch.cuda.stream(st), msrs.Problem(d, stream=st) as pr:
        L = pr.layout()
        a = torch.tensor(cfg["coef"], device="cuda:0")

        def grab():
            Y = torch.empty(L.Y_total, device="cuda:0", dtype=torch.float64)
            Q = torch.empty(L.Q_total, device="cuda:0", dtype=torch.float64)
            sv = torch.empty(L.sv_total, device="cuda:0", dtype=torch.float64)
            pr.copy_results(Y, Q, sv)
            st.synchronize()
            return Y.cpu().numpy(), Q.cpu().numpy(), sv.cpu().numpy()

        pr.assemble_patch(a)
        pr.sample_local_solutions()
        pr.range_finder()
        ref = grab()
        pr.offline_graph_capture(a)
        for rep in range(3):
            x = torch.randn(4096, device="cuda:0")
            float(x.sum())
            pr.offline_graph_launch()
            got = grab()
            for g, r in zip(got, ref):
                assert np.array_equal(g, r), rep
        assert pr.stats().error_latched == 0
