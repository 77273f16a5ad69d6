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
