"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Bars: local snapshots element by element (FP64 plain: 1e-11 of max|Y|; FP32
factor + FP64 refinement to residual 1e-10: 1e-8), relative residual of the
refined local solves <= 1e-10, bases by the sine of the largest principal
angle <= 1e-6 when the relative gap (sigma_k - sigma_{k+1})/sigma_1 >= 1e-3,
singular values to 1e-9 sigma_1, global solutions to relative L2 <= 1e-6.
"""
import numpy as np
import pytest

import synth
from synth import configs
from oracle import elliptic as E
from oracle import kinetic as K
from oracle import philox
from oracle.rangefinder import sin_max_angle

from gpu_cases import rel, run

pytestmark = pytest.mark.gpu

FP64, FP32_IR = 0, 1


@pytest.fixture(scope="module")
def gpu(lib):
    return lib


def _oracle_elliptic(cfg, omegas=None):
    return E.offline(cfg["coef"], cfg["N"], cfg["M"], cfg["overlap"], cfg["s"], cfg["k"], seed=cfg["seed"], omegas=omegas)


def _check_bases(out, ref, tol_y):
    for p, r in enumerate(ref):
        assert rel(out["Y"][p], r["Y"]) < tol_y, f"patch {p}: Y mismatch"
        sv_g, sv_o = out["sv"][p], r["sv"]
        assert np.abs(sv_g - sv_o).max() <= 1e-9 * sv_o[0], f"patch {p}: singular values"
        k = r["Q"].shape[1]
        gap = (sv_o[k - 1] - sv_o[k]) / sv_o[0] if k < len(sv_o) else 1.0
        Qg = out["Q"][p]
        assert np.abs(Qg.T @ Qg - np.eye(k)).max() < 1e-12
        if gap >= 1e-3:
            assert sin_max_angle(r["Q"], Qg) <= 1e-6, f"patch {p}: basis angle"


@pytest.mark.parametrize("prec", [FP64, FP32_IR])
def test_elliptic_small_explicit_omega(gpu, prec):
    """Several line tiles with ragged tails (b = 39, 47; s = 10 of 16)."""
    cfg = configs.small_elliptic(N=64, M=2, delta=8, s=10, k=6, coef="lognormal")
    geo = E.patch_geometry(cfg["N"], cfg["M"], cfg["overlap"])
    om = [synth.gaussian_matrix(2 * (g["cx"] + g["cy"]), cfg["s"], 100 + g["p"]) for g in geo]
    out = run(cfg, prec, omegas=om)
    for p, g in enumerate(geo):
        inf = out["infos"][p]
        assert (inf.x0, inf.y0, inf.cx, inf.cy) == (g["x0"], g["y0"], g["cx"], g["cy"])
        assert np.array_equal(out["omega"][p], om[p])
    ref = _oracle_elliptic(cfg, omegas=om)
    _check_bases(out, ref, 1e-11 if prec == FP64 else 1e-8)
    if prec == FP32_IR:
        assert out["stats"].max_rel_residual <= 1e-10
    else:
        assert out["stats"].max_rel_residual <= 1e-12


def test_device_philox_matches_oracle(gpu):
    """The device generator against the oracle's Philox4x32-10: the output
    words bit for bit, the normals to 2 ulp (the same 53-bit uniforms; the
    logarithm, square root and cosine of two math libraries)."""
    import torch
    from oracle.philox import MASK, philox4x32_10_np, normals
    seed, patch, n_node, n_sample = 0x123456789ABCDEF, 37, 300, 11
    words = torch.empty(4 * n_node * n_sample, dtype=torch.int32, device="cuda:0")
    z = torch.empty(n_node * n_sample, dtype=torch.float64, device="cuda:0")
    gpu.draw_boundary_samples(seed, patch, n_node, n_sample, words, z)
    torch.cuda.synchronize()
    w = words.cpu().numpy().view(np.uint32).reshape(n_sample, n_node, 4)
    node = np.arange(n_node, dtype=np.uint64)[None, :] * np.ones((n_sample, 1), dtype=np.uint64)
    samp = np.arange(n_sample, dtype=np.uint64)[:, None] * np.ones((1, n_node), dtype=np.uint64)
    ref = philox4x32_10_np(node, samp, np.full_like(node, patch), np.zeros_like(node), seed & MASK, seed >> 32)
    for t in range(4):
        assert np.array_equal(w[:, :, t].astype(np.uint64), ref[t]), t
    zo = normals(seed, patch, n_node, n_sample)                       # n_node x n_sample
    zg = z.cpu().numpy().reshape(n_sample, n_node).T
    ulps = np.abs(zg - zo) / np.spacing(np.maximum(np.abs(zo), np.abs(zg)))
    assert ulps.max() <= 2.0, ulps.max()
    # the sampling call draws exactly these values
    cfg = configs.small_elliptic(N=48, M=3, delta=4, s=7, k=3)
    out = run(cfg, FP64)
    geo = E.patch_geometry(cfg["N"], cfg["M"], cfg["overlap"])
    for p, g in enumerate(geo):
        o = philox.normals(cfg["seed"], p, 2 * (g["cx"] + g["cy"]), cfg["s"])
        u = np.abs(out["omega"][p] - o) / np.spacing(np.abs(o))
        assert u.max() <= 2.0, (p, u.max())


@pytest.mark.parametrize("prec", [FP64, FP32_IR])
def test_elliptic_periodic_128_full_workload(gpu, prec):
    """h=1/128, 4x4 patches, overlap 8, 10 samples, rank 6 (device Philox draws)."""
    cfg = configs.elliptic_periodic_128()
    out = run(cfg, prec, phi=cfg["phi"])
    ref = _oracle_elliptic(cfg)
    _check_bases(out, ref, 1e-11 if prec == FP64 else 1e-8)
    u_or = E.online(cfg["N"], cfg["M"], ref, cfg["coef"], cfg["phi"])
    assert E.relative_l2(out["u"][0], u_or) <= 1e-6


def test_elliptic_transposed_and_uneven_patches(gpu):
    """Per-patch overlaps give wide and tall buffered patches (line direction flips)."""
    N, M = 64, 4
    ov = np.array([0, 2, 5, 3, 7, 1, 4, 6, 2, 8, 3, 0, 5, 1, 6, 2], dtype=np.int32)
    cfg = dict(name="uneven", kind="elliptic", N=N, M=M, overlap=ov, s=9, k=4,
               coef=synth.lognormal_coefficient(N, 0.05, 7), phi=synth.dirichlet_sin_cos(N), seed=11)
    out = run(cfg, FP64, phi=cfg["phi"])
    ref = _oracle_elliptic(cfg)
    _check_bases(out, ref, 1e-11)
    u_or = E.online(N, M, ref, cfg["coef"], cfg["phi"])
    assert E.relative_l2(out["u"][0], u_or) <= 1e-6


def test_elliptic_tiny_degenerate(gpu):
    """One interior unknown per line and one line (2x2-cell patches), s = k = 1."""
    N, M = 4, 2
    cfg = dict(name="tiny", kind="elliptic", N=N, M=M, overlap=np.zeros(4, np.int32), s=1, k=1,
               coef=np.full(N * N, 1.5), phi=synth.dirichlet_sin_cos(N), seed=5)
    out = run(cfg, FP64)
    ref = _oracle_elliptic(cfg)
    for p in range(4):
        assert rel(out["Y"][p], ref[p]["Y"]) < 1e-12


def test_elliptic_global_batch_of_requests(gpu):
    cfg = configs.small_elliptic(N=64, M=4, delta=4, s=12, k=8)
    reqs = synth.fourier_boundary(cfg["N"], range(5))
    out = run(cfg, FP32_IR, phi=reqs, max_batch=8)
    ref = _oracle_elliptic(cfg)
    u_or = E.online(cfg["N"], cfg["M"], ref, cfg["coef"], reqs.T)
    for r in range(5):
        assert E.relative_l2(out["u"][r], u_or[:, r]) <= 1e-6


def _golden(name):
    import importlib.util
    import os
    spec = importlib.util.spec_from_file_location(
        "online_fixtures", os.path.join(os.path.dirname(__file__), "golden", "make_online_fixtures.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.load(name)


def _timed_form(gpu, cfg, phi=None):
    """The offline step as the benchmark times it (factor share 2, the captured
    step replayed on its own stream), then the online solve for phi."""
    import torch
    from gpu_cases import _unpack
    st = torch.cuda.Stream()
    d = gpu.make_desc(gpu.KIND_ELLIPTIC_Q1, cfg["N"], cfg["M"], list(cfg["overlap"]), cfg["s"], cfg["k"],
                      precision=FP32_IR, seed=cfg["seed"])
    a = torch.tensor(cfg["coef"], device="cuda:0")
    with torch.cuda.stream(st), gpu.Problem(d, stream=st) as pr:
        pr.set_tuning(gpu.TUNE_FACTOR_SHARE, 2)
        pr.assemble_patch(a)
        pr.sample_local_solutions()
        pr.range_finder()
        pr.offline_graph_capture(a)
        for _ in range(2):
            pr.offline_graph_launch()
        L = pr.layout()
        Y = torch.empty(L.Y_total, device="cuda:0", dtype=torch.float64)
        Q = torch.empty(L.Q_total, device="cuda:0", dtype=torch.float64)
        sv = torch.empty(L.sv_total, device="cuda:0", dtype=torch.float64)
        pr.copy_results(Y, Q, sv)
        torch.cuda.synchronize()
        stats = pr.stats()
        infos = [pr.patch(p) for p in range(L.n_patches)]
        u = None
        if phi is not None:
            pr.assemble_coarse()
            f = torch.tensor(np.atleast_2d(phi), device="cuda:0")
            ut = torch.empty((f.shape[0], L.n_nodes), device="cuda:0", dtype=torch.float64)
            pr.solve_global(f, ut)
            torch.cuda.synchronize()
            u = ut.cpu().numpy()
    Yh, Qh, svh = Y.cpu().numpy(), Q.cpu().numpy(), sv.cpu().numpy()
    per = [dict(Y=_unpack(Yh, i.Y_off, i.n_rows, i.n_samples), Q=_unpack(Qh, i.Q_off, i.n_rows, i.n_cols),
                sv=svh[i.sv_off:i.sv_off + i.n_samples]) for i in infos]
    return stats, infos, per, u


def gram_sv_bar(Yg, Yo, svo):
    """Bar of the device's singular values against the oracle's: Weyl's bound
    ||Y_g - Y_o||_2 for the snapshots' own difference, plus the resolution of
    a Gram-matrix range finder.  Its eigenvalues sigma_i^2 carry absolute
    errors up to about 4 s u sigma_1^2 (u = 2^-53; rounding of Y^T Y and of the
    rotations), so sigma_i moves by at most min(4 s u sigma_1^2 / (2 sigma_i),
    sqrt(4 s u) sigma_1): ~1e-15 sigma_1 at the top of the spectrum, up to
    ~3e-7 sigma_1 below sqrt(s u) sigma_1."""
    s = Yo.shape[1]
    d = 4 * s * 2.0 ** -53 * svo[0] ** 2
    gram = np.minimum(d / (2 * np.maximum(svo, 1e-300)), np.sqrt(d))
    return np.linalg.norm(Yg - Yo, 2) + gram + 1e-12 * svo[0]


def _check_patch_against_oracle(cfg, g, got):
    """Snapshots to 1e-8, singular values within Weyl's bound ||Y_g - Y_o||_2
    plus the Gram resolution (gram_sv_bar), orthonormal bases, and the
    largest principal angle <= 1e-6 where the gap (sigma_k - sigma_{k+1}) /
    sigma_1 is at least 1e-3."""
    from oracle.rangefinder import range_finder
    k = cfg["k"]
    Yo = E.sample_patch(cfg["coef"], cfg["N"], g, E.patch_omega(cfg["seed"], g, cfg["s"]))
    Qo, svo = range_finder(Yo, k)
    assert rel(got["Y"], Yo) < 1e-8, g["p"]
    bar = gram_sv_bar(got["Y"], Yo, svo)
    assert np.all(np.abs(got["sv"] - svo) <= bar), g["p"]
    Qg = got["Q"]
    assert np.abs(Qg.T @ Qg - np.eye(k)).max() < 1e-12, g["p"]
    if (svo[k - 1] - svo[k]) / svo[0] >= 1e-3:
        assert sin_max_angle(Qo, Qg) <= 1e-6, g["p"]


def test_elliptic_lognormal_1024_timed_form(gpu):
    """The h=1/1024 workload (16x16 patches, buffers of 16 or 32 cells, 64
    samples, rank 16) in the form the benchmark times.  The oracle recomputes
    one patch of every buffered-patch shape: 128x128 cells (line tiles of 8),
    96x128 and 128x96 (6, both line orientations), 96x96 (6), 80x96 and 96x80
    (5, both orientations) and 80x80 (5); the global solution for the
    workload's Dirichlet data is compared with the oracle's stored solution at
    every 32nd node in each direction (tests/golden/make_online_fixtures.py)."""
    cfg = configs.elliptic_lognormal_1024()
    stats, infos, per, u = _timed_form(gpu, cfg, cfg["phi"])
    assert stats.error_latched == 0 and stats.max_rel_residual <= 1e-10
    geo = E.patch_geometry(cfg["N"], cfg["M"], cfg["overlap"])
    shapes = {}
    for g in geo:
        shapes.setdefault((g["cx"], g["cy"]), g["p"])
    assert {(128, 128), (96, 128), (128, 96), (96, 96), (80, 96), (96, 80), (80, 80)} <= set(shapes)
    assert {infos[p].line_len for p in shapes.values()} == {79, 95, 127}
    for p in shapes.values():
        _check_patch_against_oracle(cfg, geo[p], per[p])
    nodes, U, norms = _golden("elliptic_lognormal_1024")
    ug = u[0]
    assert np.linalg.norm(ug[nodes] - U[:, 0]) <= 1e-6 * np.linalg.norm(U[:, 0])
    assert abs(np.linalg.norm(ug) - norms[0]) <= 1e-6 * norms[0]


def _kin_cfg(Nx=512, M=8, delta=32, s=40, k=8, eps=2.0 ** -6):
    return dict(name="kin_small", kind="kinetic", N=Nx, M=M, overlap=np.full(M, delta, np.int32), s=s, k=k,
                n_vel=32, eps=eps, coef=synth.kinetic_sigma(Nx, 0.05), seed=3)


@pytest.mark.parametrize("prec", [FP64, FP32_IR])
def test_kinetic_small(gpu, prec):
    cfg = _kin_cfg()
    v, _ = K.ordinates(32)
    phi = np.concatenate([3 + np.sin(2 * np.pi * v[v > 0]), 2 + np.sin(2 * np.pi * v[v < 0])])
    out = run(cfg, prec, phi=phi)
    ref = K.offline(cfg["coef"], cfg["eps"], cfg["N"], cfg["M"], cfg["overlap"], 32, cfg["s"], cfg["k"], seed=cfg["seed"])
    for p, r in enumerate(ref):
        assert rel(out["Y"][p], r["Y"]) < (1e-11 if prec == FP64 else 1e-8), f"patch {p}"
        if not r["full"]:
            k = cfg["k"]
            sv = r["sv"]
            if (sv[k - 1] - sv[k]) / sv[0] >= 1e-3:
                assert sin_max_angle(r["Q"], out["Q"][p]) <= 1e-6
    f_or = K.online(cfg["M"], 32, ref, phi)
    assert np.linalg.norm(out["u"][0] - f_or) / np.linalg.norm(f_or) <= 1e-6


def test_kinetic_slab_4096_full_workload(gpu):
    cfg = configs.kinetic_slab_4096()
    v, _ = K.ordinates(32)
    phi = np.concatenate([3 + np.sin(2 * np.pi * v[v > 0]), 2 + np.sin(2 * np.pi * v[v < 0])])
    out = run(cfg, FP32_IR, phi=phi)
    assert out["stats"].max_rel_residual <= 1e-10
    ref = K.offline(cfg["coef"], cfg["eps"], cfg["N"], cfg["M"], cfg["overlap"], 32, cfg["s"], cfg["k"], seed=cfg["seed"])
    for p in (0, 1, 15, 31):
        assert rel(out["Y"][p], ref[p]["Y"]) < 1e-8, f"patch {p}"
    f_or = K.online(cfg["M"], 32, ref, phi)
    assert np.linalg.norm(out["u"][0] - f_or) / np.linalg.norm(f_or) <= 1e-6


def test_non_positive_coefficient_is_reported(gpu):
    from paper_1807_08848_amd import msrs
    cfg = configs.small_elliptic(N=32, M=2, delta=2, s=4, k=2)
    a = cfg["coef"].copy()
    a[37] = -1.0
    cfg["coef"] = a
    with pytest.raises(msrs.MsrsError) as e:
        run(cfg, FP64)
    assert e.value.status == msrs.ERR_NOT_SPD


def test_single_hip_runtime_shared_with_torch(gpu):
    """libmsrs.so and torch use one HIP runtime instance (torch streams are valid handles)."""
    import torch
    maps = open("/proc/self/maps").read().splitlines()
    hip = {l.split()[-1] for l in maps if "libamdhip64" in l}
    assert len(hip) == 1, hip
    # a non-default torch stream drives the library and orders with torch's own work
    cfg = configs.small_elliptic(N=32, M=2, delta=4, s=6, k=3)
    from paper_1807_08848_amd import msrs
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        a = torch.tensor(cfg["coef"], device="cuda")
        d = msrs.make_desc(msrs.KIND_ELLIPTIC_Q1, cfg["N"], cfg["M"], list(cfg["overlap"]), cfg["s"], cfg["k"], seed=cfg["seed"])
        with msrs.Problem(d) as pr:
            L = pr.layout()
            Y = torch.zeros(L.Y_total, device="cuda", dtype=torch.float64)
            pr.assemble_patch(a)
            pr.sample_local_solutions(None, Y)
            ysum = Y.abs().sum()          # torch work on the same stream, ordered after the kernels
        st.synchronize()
    ref = E.offline(cfg["coef"], cfg["N"], cfg["M"], cfg["overlap"], cfg["s"], cfg["k"], seed=cfg["seed"])
    assert abs(float(ysum) - sum(np.abs(r["Y"]).sum() for r in ref)) < 1e-9 * float(ysum)


def test_sweep_width_and_offline_autotune_keep_results(gpu):
    """Snapshots do not depend on the sweep workgroup width; the offline autotuner
    times the three widths and keeps one."""
    import torch
    from paper_1807_08848_amd import msrs
    cfg = configs.small_elliptic(N=64, M=2, delta=8, s=40, k=6, coef="lognormal")
    d = msrs.make_desc(msrs.KIND_ELLIPTIC_Q1, cfg["N"], cfg["M"], list(cfg["overlap"]), cfg["s"], cfg["k"],
                       precision=FP32_IR, seed=cfg["seed"])
    with msrs.Problem(d) as pr:
        L = pr.layout()
        pr.assemble_patch(torch.tensor(cfg["coef"], device="cuda:0"))
        Ys = []
        for sc in (16, 32, 64):
            pr.set_tuning(msrs.TUNE_SWEEP_COLS, sc)
            Y = torch.empty(L.Y_total, device="cuda:0", dtype=torch.float64)
            pr.sample_local_solutions(None, Y)
            Ys.append(Y.cpu().numpy())
        for Y in Ys[1:]:
            assert np.abs(Y - Ys[0]).max() <= 1e-13 * np.abs(Ys[0]).max()
        trials = pr.autotune(msrs.TUNE_STAGE_OFFLINE, reps=1)
        assert [t[1] for t in trials] == [16, 32, 64]
        assert pr.get_tuning(msrs.TUNE_SWEEP_COLS) == min(trials, key=lambda t: t[2])[1]
        pr.range_finder()        # the tuner left the handle sampled


def test_seven_tile_lines_at_every_sweep_width(gpu):
    """Line-tile count 7 (the 112 x 112 centre patch of a 3 x 3 layout with
    24-cell buffers; the others have 6) at 64 samples, through each sweep width
    (16, 32 and 64 samples per workgroup, the last one the register-coupled
    FP32 sweeps): snapshots, singular values and bases against the oracle, and
    the global solution at the widest."""
    from paper_1807_08848_amd import msrs
    cfg = configs.small_elliptic(N=192, M=3, delta=24, s=64, k=8, coef="lognormal")
    ref = _oracle_elliptic(cfg)
    u_or = E.online(cfg["N"], cfg["M"], ref, cfg["coef"], cfg["phi"])
    k = cfg["k"]
    for sc in (16, 32, 64):
        out = run(cfg, FP32_IR, phi=cfg["phi"] if sc == 64 else None, tuning={msrs.TUNE_SWEEP_COLS: sc})
        assert max(-(-inf.line_len // 16) for inf in out["infos"]) == 7
        assert out["stats"].max_rel_residual <= 1e-10
        for p, r in enumerate(ref):
            # 64 samples reach sigma_64 ~ 1e-9 sigma_1 here: the singular values
            # within Weyl's bound plus the Gram resolution (gram_sv_bar)
            assert rel(out["Y"][p], r["Y"]) < 1e-8, (sc, p)
            assert np.all(np.abs(out["sv"][p] - r["sv"]) <= gram_sv_bar(out["Y"][p], r["Y"], r["sv"])), (sc, p)
            Qg = out["Q"][p]
            assert np.abs(Qg.T @ Qg - np.eye(k)).max() < 1e-12, (sc, p)
            if (r["sv"][k - 1] - r["sv"][k]) / r["sv"][0] >= 1e-3:
                assert sin_max_angle(r["Q"], Qg) <= 1e-6, (sc, p)
        if sc == 64:
            assert E.relative_l2(out["u"][0], u_or) <= 1e-6


def test_offline_graph_replays_match_eager(gpu):
    """The captured offline step replays to the eager results (every replay, with
    eager torch work and synchronisations between replays) and reads the current
    coefficient values."""
    import torch
    from paper_1807_08848_amd import msrs
    cfg = configs.small_elliptic(N=64, M=4, delta=4, s=12, k=8, coef="lognormal")
    st = torch.cuda.Stream()
    d = msrs.make_desc(msrs.KIND_ELLIPTIC_Q1, cfg["N"], cfg["M"], list(cfg["overlap"]), cfg["s"], cfg["k"],
                       precision=FP32_IR, seed=cfg["seed"])
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
            x = torch.randn(4096, device="cuda:0")          # eager work between replays
            float(x.sum())
            pr.offline_graph_launch()
            got = grab()
            for g, r in zip(got, ref):
                assert np.array_equal(g, r), rep
        assert pr.stats().error_latched == 0
        # a replay reads the coefficient buffer's current contents
        a.mul_(torch.tensor(1.0 + 0.2 * np.sin(np.arange(a.numel())), device="cuda:0"))
        pr.offline_graph_launch()
        got = grab()
        pr.assemble_patch(a)
        pr.sample_local_solutions()
        pr.range_finder()
        ref2 = grab()
        assert np.abs(got[0] - ref2[0]).max() <= 1e-12 * np.abs(ref2[0]).max()
        assert not np.allclose(got[0], ref[0])


@pytest.mark.parametrize("k", [8, 16])
def test_elliptic_full_basis_on_boundary_patches(gpu, k):
    """Boundary patches with the full delta basis and no buffer, interior
    patches sampled (MSRS_FLAG_FULL_BASIS_BOUNDARY): parity with the oracle's
    option, and the reduced solution close to the fine solve, falling with k
    (oracle: 0.107 at k=8, 0.0041 at k=16 on this workload)."""
    N, M = 64, 4
    cfg = dict(name="full_basis_boundary", kind="elliptic", N=N, M=M, overlap=np.full(M * M, 8, dtype=np.int32),
               s=k, k=k, coef=synth.periodic_coefficient(N, 1.0 / 8.0), phi=synth.dirichlet_sin_cos(N), seed=2)
    out = run(cfg, FP32_IR, phi=cfg["phi"], flags=gpu.FLAG_FULL_BASIS_BOUNDARY)
    ref = E.offline(cfg["coef"], N, M, cfg["overlap"], k, k, seed=2, full_basis_boundary=True)
    for p, inf in enumerate(out["infos"]):
        on_bd = (p % M) in (0, M - 1) or (p // M) in (0, M - 1)
        assert inf.full_basis == int(on_bd) and inf.n_cols == (4 * (N // M) if on_bd else k)
    _check_bases(out, ref, 1e-8)
    u_or = E.online(N, M, ref, cfg["coef"], cfg["phi"])
    assert E.relative_l2(out["u"][0], u_or) <= 1e-6
    err = E.relative_l2(out["u"][0], E.global_solve(cfg["coef"], N, cfg["phi"]))
    assert err < (0.15 if k == 8 else 1e-2)


@pytest.mark.parametrize("ov,counts", [
    # line-tile counts {2, 3}: one factor launch for both
    ([6, 12, 12, 6, 12, 6, 12, 12, 6, 12, 6, 12, 12, 12, 6, 6], {2, 3}),
    # {1, 2, 3}: one launch of the any-count kernel, patches costliest first
    ([0, 6, 12, 0, 12, 0, 12, 6, 6, 12, 0, 12, 0, 6, 12, 0], {1, 2, 3}),
])
def test_elliptic_mixed_line_tile_counts_fp32(gpu, ov, counts):
    """Patches of different line lengths in one FP32-IR batch: parity of the
    snapshots, bases and global solution with the oracle for both ways the
    factor stage launches them."""
    N, M = 64, 4
    cfg = dict(name="mixed", kind="elliptic", N=N, M=M, overlap=np.asarray(ov, dtype=np.int32), s=10, k=6,
               coef=synth.lognormal_coefficient(N, 0.05, 7), phi=synth.dirichlet_sin_cos(N), seed=13)
    out = run(cfg, FP32_IR, phi=cfg["phi"])
    assert {inf.line_len // 16 + (inf.line_len % 16 > 0) for inf in out["infos"]} == counts
    ref = _oracle_elliptic(cfg)
    _check_bases(out, ref, 1e-8)
    assert out["stats"].max_rel_residual <= 1e-10
    u_or = E.online(N, M, ref, cfg["coef"], cfg["phi"])
    assert E.relative_l2(out["u"][0], u_or) <= 1e-6


@pytest.mark.parametrize("prec,tol", [(FP64, 1e-9), (FP32_IR, 1e-6)])
def test_full_basis_everywhere_reproduces_the_fine_solution(gpu, prec, tol):
    """MSRS_FLAG_FULL_BASIS: DetLocalSolu on every patch (no buffer, Kronecker-
    delta boundary data).  The bases then span every restriction of a fine
    solution, and the online solve returns the fine discrete solution, for the
    elliptic and the kinetic problem (brute force: the oracle's global solve)."""
    N, M = 64, 4
    cfg = dict(name="full", kind="elliptic", N=N, M=M, overlap=np.full(M * M, 8, dtype=np.int32), s=8, k=8,
               coef=synth.lognormal_coefficient(N, 0.05, 7), phi=synth.dirichlet_sin_cos(N), seed=2)
    out = run(cfg, prec, phi=cfg["phi"], flags=gpu.FLAG_FULL_BASIS)
    assert all(inf.full_basis == 1 and inf.n_cols == 4 * (N // M) for inf in out["infos"])
    u_ref = E.global_solve(cfg["coef"], N, cfg["phi"])
    assert E.relative_l2(out["u"][0], u_ref) <= tol
    kcfg = configs.kinetic_hg_100(1.0, 10, n_vel=16)
    v, _ = K.ordinates(16)
    phi = np.concatenate([3 + np.sin(2 * np.pi * v[v > 0]), 2 + np.sin(2 * np.pi * v[v < 0])])
    kout = run(kcfg, prec, phi=phi, flags=gpu.FLAG_FULL_BASIS)
    assert all(inf.full_basis == 1 for inf in kout["infos"])
    f_ref = K.global_solve(kcfg["coef"], kcfg["eps"], 16, phi, hg=kcfg["hg"])
    assert np.linalg.norm(kout["u"][0] - f_ref) / np.linalg.norm(f_ref) <= tol


def test_elliptic_lognormal_512_benchmarked_form(gpu):
    """The h=1/512 workload (8x8 patches of two line lengths, 32 samples, rank
    12) in the form the benchmark times.  The oracle checks the snapshots,
    singular values and bases of patches of both line lengths one by one, and
    the global solution against its own least-squares gluing of all 64
    patches."""
    cfg = configs.elliptic_lognormal_512()
    stats, infos, per, u = _timed_form(gpu, cfg, cfg["phi"])
    assert stats.error_latched == 0 and stats.max_rel_residual <= 1e-10
    geo = E.patch_geometry(cfg["N"], cfg["M"], cfg["overlap"])
    lens = {}
    for p, inf in enumerate(infos):
        lens.setdefault(inf.line_len, p)
    assert len(lens) >= 2
    for p in sorted(set(lens.values()) | {0, 27, 63}):
        _check_patch_against_oracle(cfg, geo[p], per[p])
    ref = _oracle_elliptic(cfg)
    u_or = E.online(cfg["N"], cfg["M"], ref, cfg["coef"], cfg["phi"])
    assert E.relative_l2(u[0], u_or) <= 1e-6


def test_refinement_that_cannot_converge_is_reported(gpu):
    """One refinement iteration cannot reach ir_tol = 1e-10 from the FP32
    factor: MSRS_ERR_NOCONV is latched (eager form)."""
    import torch
    cfg = configs.small_elliptic(N=64, M=2, delta=8, s=10, k=6, coef="lognormal")
    d = gpu.make_desc(gpu.KIND_ELLIPTIC_Q1, cfg["N"], cfg["M"], list(cfg["overlap"]), cfg["s"], cfg["k"],
                      precision=FP32_IR, seed=cfg["seed"], ir_max_iters=1)
    with gpu.Problem(d) as pr:
        pr.assemble_patch(torch.tensor(cfg["coef"], device="cuda:0"))
        pr.sample_local_solutions()
        st = pr.stats(check=False)
        assert st.error_latched == gpu.ERR_NOCONV and st.max_rel_residual > 1e-10


@pytest.mark.parametrize("prec", [FP64, FP32_IR])
def test_non_finite_boundary_data_is_reported(gpu, prec):
    """A NaN in one column of user Omega: MSRS_ERR_NONFINITE, not a silent
    convergence (the refinement's norms treat non-finite ratios as infinite)."""
    cfg = configs.small_elliptic(N=64, M=2, delta=8, s=10, k=6, coef="lognormal")
    geo = E.patch_geometry(cfg["N"], cfg["M"], cfg["overlap"])
    om = [synth.gaussian_matrix(2 * (g["cx"] + g["cy"]), cfg["s"], 100 + g["p"]) for g in geo]
    om[1][5, 3] = np.nan
    with pytest.raises(gpu.MsrsError) as e:
        run(cfg, prec, omegas=om)
    assert e.value.status == gpu.ERR_NONFINITE


def test_online_workspaces_exhausted_is_busy(gpu):
    """Four msrs_solve_global calls on four streams hold the four online
    workspaces while their streams are busy; a fifth call on another stream
    finds none free and returns MSRS_ERR_BUSY (a bounded sleep kernel keeps
    the streams busy)."""
    import torch
    from gpu_cases import resident
    cfg = configs.small_elliptic(N=64, M=4, delta=4, s=12, k=8)
    pr = resident(cfg, FP32_IR)
    try:
        L = pr.layout()
        f = torch.tensor(synth.fourier_boundary(cfg["N"], range(1)), device="cuda:0")
        us = [torch.empty((1, L.n_nodes), device="cuda:0", dtype=torch.float64) for _ in range(5)]
        streams = [torch.cuda.Stream() for _ in range(5)]
        torch.cuda.synchronize()
        for i in range(4):
            with torch.cuda.stream(streams[i]):
                torch.cuda._sleep(200_000_000)
                pr.solve_global(f, us[i], stream=streams[i])
        with pytest.raises(gpu.MsrsError) as e:
            pr.solve_global(f, us[4], stream=streams[4])
        assert e.value.status == gpu.ERR_BUSY
        torch.cuda.synchronize()
        pr.solve_global(f, us[4], stream=streams[4])         # free again once the streams drained
        torch.cuda.synchronize()
        for i in range(4):
            assert torch.equal(us[i], us[4])
    finally:
        pr.close()


@pytest.mark.parametrize("ov", [
    [6, 12, 12, 6, 12, 6, 12, 12, 6, 12, 6, 12, 12, 12, 6, 6],     # two lengths, one launch
    [8] * 16,                                                      # one length
    [0, 6, 12, 0, 12, 0, 12, 6, 6, 12, 0, 12, 0, 6, 12, 0],        # three lengths, the any-count kernel
])
def test_factor_share_keeps_results(gpu, ov):
    """MSRS_TUNE_FACTOR_SHARE = 2 compiles the FP32 factor for two resident
    workgroups per compute unit: a register budget, not arithmetic.
    Snapshots, bases and the global solution are those of the default."""
    N, M = 64, 4
    ov = np.asarray(ov, dtype=np.int32)
    cfg = dict(name="share", kind="elliptic", N=N, M=M, overlap=ov, s=10, k=6,
               coef=synth.lognormal_coefficient(N, 0.05, 7), phi=synth.dirichlet_sin_cos(N), seed=13)
    outs = []
    for share in (1, 2):
        outs.append(run(cfg, FP32_IR, phi=cfg["phi"], tuning={gpu.TUNE_FACTOR_SHARE: share}))
    a, b = outs
    for p in range(M * M):
        assert np.array_equal(a["Y"][p], b["Y"][p]) and np.array_equal(a["Q"][p], b["Q"][p]), p
    assert np.array_equal(a["u"], b["u"])


@pytest.mark.parametrize("make", [configs.elliptic_periodic_128, configs.elliptic_lognormal_512])
def test_coarse_condition_estimate(gpu, make):
    """msrs_coarse_condition: the 1-norm condition estimate of the normal
    equations P~^T P~ (Hager-Higham on the resident band factor) against the
    exact kappa_1 of the oracle's own P~^T P~ (a lower bound, within a small
    factor), and the estimate of kappa(P~) against the 2-norm condition of the
    oracle's P~ (within the factor sqrt(Np) that separates the norms)."""
    from gpu_cases import resident
    cfg = make()
    pr = resident(cfg, FP64)
    try:
        kn, kl = pr.coarse_condition()
        Np = pr.layout().coarse_dim
    finally:
        pr.close()
    ref = _oracle_elliptic(cfg)
    P, _, _, _ = E.coarse_rows(cfg["N"], cfg["M"], ref, cfg["coef"])
    K = P.T @ P
    exact = np.linalg.cond(K, 1)
    assert exact / 10 <= kn <= exact * (1 + 1e-6), (kn, exact)
    k2 = np.linalg.cond(P)
    assert k2 / np.sqrt(Np) <= kl <= k2 * np.sqrt(Np), (kl, k2)
    assert abs(kl - np.sqrt(kn)) <= 1e-12 * kl
