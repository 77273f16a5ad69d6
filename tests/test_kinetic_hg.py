"""Anisotropic (Henyey-Greenstein) scattering, the paper's transport test
(Sec. 4: eq. RTE with the kernel of eq. HG, g = 1/2; Sec. 4.3 setup).

CPU: the discrete collision operator against what the continuous one fixes
(mass conservation, constants as equilibria, the loss integral in closed
form, the isotropic limit g -> 0), and the trends of the paper's global test
(error falls as k_m grows, and is smaller for small eps).  GPU: the HIP path
against the oracle on the paper's setup (parity bars).
"""
import numpy as np
import pytest

from synth import configs
from oracle import kinetic as K
from oracle.rangefinder import sin_max_angle

FP32_IR = 1


def _phi(nv):
    v, _ = K.ordinates(nv)
    return np.concatenate([3 + np.sin(2 * np.pi * v[v > 0]), 2 + np.sin(2 * np.pi * v[v < 0])])


def test_hg_collision_operator():
    v, w = K.ordinates(64)
    g = 0.5
    A, _ = K.assemble(np.ones(1), 1.0, 1e300, v, w, hg=g)       # one cell, streaming negligible
    C = A.toarray()
    assert np.abs(w @ C).max() < 1e-15                          # gain and loss carry the same mass
    assert np.abs(C @ np.ones(64)).max() < 1e-14                # symmetric kernel: constants are equilibria
    lam = (K.hg_kernel(v, g) * w[:, None]).sum(0)
    closed = (1 - g * g) / (4 * g * v) * np.log((1 + g * g + 2 * g * v) / (1 + g * g - 2 * g * v))
    assert np.abs(lam - closed).max() < 1e-13                   # int_{-1}^{1} k(v', v) dv' in closed form
    A0, _ = K.assemble(np.ones(3), 0.5, 0.01, v, w)
    A1, _ = K.assemble(np.ones(3), 0.5, 0.01, v, w, hg=1e-9)
    assert abs(A0 - A1).max() < 1e-8                            # g -> 0: the isotropic operator


def test_hg_global_error_trends():
    """Global test of the paper: relative error of the reduced solution against
    the fine solve falls as k_m grows, and is smaller for eps = 2^-6 than for
    eps = 1 at the same k_m."""
    nv, phi = 64, _phi(64)
    errs = {}
    for eps in (1.0, 2.0 ** -6):
        cfg = configs.kinetic_hg_100(eps, 10)
        ref = K.global_solve(cfg["coef"], eps, nv, phi, hg=cfg["hg"])
        for k in (10, 40):
            pt = K.offline(cfg["coef"], eps, cfg["N"], cfg["M"], cfg["overlap"], nv, k, k, seed=2, hg=cfg["hg"])
            f = K.online(cfg["M"], nv, pt, phi)
            errs[eps, k] = np.linalg.norm(f - ref) / np.linalg.norm(ref)
    for eps in (1.0, 2.0 ** -6):
        assert errs[eps, 40] < errs[eps, 10]
    for k in (10, 40):
        assert errs[2.0 ** -6, k] < errs[1.0, k]


@pytest.mark.gpu
@pytest.mark.parametrize("eps", [1.0, 2.0 ** -6])
def test_hg_parity(lib, eps):
    from gpu_cases import rel, run
    cfg = configs.kinetic_hg_100(eps, 10)
    nv, phi = cfg["n_vel"], _phi(cfg["n_vel"])
    out = run(cfg, FP32_IR, phi=phi)
    assert out["stats"].max_rel_residual <= 1e-10
    ref = K.offline(cfg["coef"], eps, cfg["N"], cfg["M"], cfg["overlap"], nv, cfg["s"], cfg["k"], seed=cfg["seed"],
                    hg=cfg["hg"])
    for p, r in enumerate(ref):
        assert rel(out["Y"][p], r["Y"]) < 1e-8, p
        if not r["full"]:
            assert sin_max_angle(r["Q"], out["Q"][p]) <= 1e-6, p       # s = k: the span of Y
    f_or = K.online(cfg["M"], nv, ref, phi)
    assert np.linalg.norm(out["u"][0] - f_or) / np.linalg.norm(f_or) <= 1e-6


# ------------------------------------------------------------------ local test
# The paper's local transport test (Sec. 4.3): the second patch K_2 of the
# M = 10 decomposition, its buffered patch twice as large, g = 1/2, and the
# Green's matrices G_2 (unbuffered) and G~_2 (buffered) from the patch's
# inflow data to its cells and ghost cells.  No printed values: the trends of
# its three local figures.
EPS_LOCAL = (1.0, 2.0 ** -2, 2.0 ** -4, 2.0 ** -6)


def _local_setup(eps, nv=64):
    cfg = configs.kinetic_hg_100(eps, 10, n_vel=nv)
    g = K.patch_geometry(cfg["N"], cfg["M"], cfg["overlap"])[1]
    g0 = K.patch_geometry(cfg["N"], cfg["M"], 0)[1]
    green = lambda gg: K.sample_patch(cfg["coef"], eps, cfg["N"], nv, gg, np.eye(nv), hg=cfg["hg"])
    return cfg, g, green(g0), green(g)


def test_rte_local_buffer_speeds_up_singular_value_decay():
    """Fig. rte_local: the normalized singular values of G~_2 fall faster than
    those of G_2 (at every eps; by a factor of about 9 at sigma_11 for
    eps = 2^-6)."""
    for eps in EPS_LOCAL:
        _, _, G0, Gt = _local_setup(eps)
        s0 = np.linalg.svd(G0, compute_uv=False)
        st = np.linalg.svd(Gt, compute_uv=False)
        assert st[10] / st[0] < s0[10] / s0[0], eps
        if eps == 2.0 ** -6:
            assert st[10] / st[0] < 0.2 * s0[10] / s0[0]


def test_rte_local_sampling_error_trends():
    """Fig. RTE_LocalError: ||G~_2 - Q Q^T G~_2||_2 / ||G~_2||_2 with Q from a QR
    of k_m random solutions (nested: the first k_m columns of one draw) falls
    as k_m grows, and at every k_m is smaller for smaller eps."""
    from oracle.rangefinder import projection_error, range_finder
    ks = (5, 10, 20, 40, 60)
    errs = {}
    for eps in EPS_LOCAL:
        cfg, g, _, Gt = _local_setup(eps)
        om = K.patch_omega(cfg["seed"], g, 64, max(ks))
        for k in ks:
            Y = K.sample_patch(cfg["coef"], eps, cfg["N"], 64, g, om[:, :k], hg=cfg["hg"])
            errs[eps, k] = projection_error(Gt, range_finder(Y, k)[0])
    for eps in EPS_LOCAL:
        assert all(errs[eps, a] >= errs[eps, b] for a, b in zip(ks, ks[1:])), eps
    for k in ks:
        assert all(errs[a, k] > errs[b, k] for a, b in zip(EPS_LOCAL, EPS_LOCAL[1:])), k
    assert errs[2.0 ** -6, 20] < 0.1 and errs[1.0, 20] > 0.9


def test_rte_local_leading_modes_captured():
    """Fig. rte_local_mode: at eps = 2^-6 the span of k_2 = 50 random
    solutions captures the first three left singular vectors of G_2 on the
    cells of K_2 (projection residuals below 0.1), and at eps = 1 it does not
    (above 0.3).  The ghost rows are left out: for the unbuffered patch they
    hold the inflow data itself, which no buffered solution reproduces."""
    from oracle.rangefinder import range_finder
    res = {}
    for eps in (1.0, 2.0 ** -6):
        cfg, g, G0, _ = _local_setup(eps)
        Y = K.sample_patch(cfg["coef"], eps, cfg["N"], 64, g, K.patch_omega(cfg["seed"], g, 64, 50), hg=cfg["hg"])
        U = np.linalg.svd(G0[64:-64])[0][:, :3]
        Q, _ = range_finder(Y[64:-64], 50)
        res[eps] = np.linalg.norm(U - Q @ (Q.T @ U), axis=0)
    assert res[2.0 ** -6].max() < 0.1 and res[1.0].min() > 0.3


@pytest.mark.gpu
@pytest.mark.parametrize("eps", EPS_LOCAL)
def test_rte_local_parity(lib, eps):
    """The local test on the device at every eps: the buffered Green's matrix
    G~_2 (DetLocalSolu as 64 Kronecker-delta inflow columns through the
    explicit-Omega entry, FP64) and its singular values against the oracle's,
    and the sampling error of the device's bases from k_m = 10, 20, 40 device
    Philox samples against the oracle's on the same draws."""
    from gpu_cases import run
    from oracle.rangefinder import projection_error, range_finder
    cfg, g, _, Gt = _local_setup(eps)
    nv = 64
    full = dict(cfg, s=nv, k=nv)
    out = run(full, 0, omegas=[np.eye(nv)] * cfg["M"])
    Gd = out["Y"][1]
    assert np.abs(Gd - Gt).max() <= 1e-10 * np.abs(Gt).max()
    st = np.linalg.svd(Gt, compute_uv=False)
    assert np.abs(out["sv"][1] - st).max() <= 1e-10 * st[0]
    for k in (10, 20, 40):
        o = run(dict(cfg, s=k, k=k), FP32_IR)
        Y = K.sample_patch(cfg["coef"], eps, cfg["N"], nv, g, K.patch_omega(cfg["seed"], g, nv, k), hg=cfg["hg"])
        e_or = projection_error(Gt, range_finder(Y, k)[0])
        e_dev = projection_error(Gt, o["Q"][1])
        assert abs(e_dev - e_or) <= 1e-6 * max(1.0, e_or), (k, e_dev, e_or)
