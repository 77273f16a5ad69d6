"""Pins of the kinetic oracle: equilibrium, conservation, maximum principle, free streaming, symmetry."""
import numpy as np
import pytest

import synth
from oracle import kinetic as K


def test_gauss_legendre_ordinates():
    v, w = K.ordinates(32)
    assert abs(w.sum() - 2.0) < 1e-14
    assert np.allclose(v, -v[::-1]) and np.allclose(w, w[::-1])
    for d in range(0, 63, 2):
        assert abs(np.sum(w * v ** d) - 2.0 / (d + 1)) < 1e-13
    assert np.all(v != 0)


def test_constant_inflow_gives_constant_solution():
    """M(v) = 1: an isotropic constant is an exact equilibrium of the scheme."""
    sig = synth.kinetic_sigma(256)
    f = K.global_solve(sig, 2.0 ** -6, 32, np.full(32, 1.75))
    assert np.abs(f - 1.75).max() < 1e-11


def test_current_is_conserved():
    v, w = K.ordinates(16)
    sig = synth.kinetic_sigma(200, 0.05)
    rng = np.random.default_rng(0)
    f = K.global_solve(sig, 0.05, 16, rng.standard_normal(16)).reshape(200, 16)
    J = K.current(f, v, w)
    assert J.max() - J.min() < 1e-12 * max(1.0, np.abs(J).max())


def test_maximum_principle():
    rng = np.random.default_rng(1)
    phi = rng.uniform(-1, 2, 32)
    f = K.global_solve(synth.kinetic_sigma(128), 0.01, 32, phi)
    assert f.min() >= phi.min() - 1e-12 and f.max() <= phi.max() + 1e-12


def test_free_streaming_without_scattering():
    v, _ = K.ordinates(8)
    rng = np.random.default_rng(2)
    phi = rng.standard_normal(8)
    f = K.global_solve(np.zeros(40), 1.0, 8, phi).reshape(40, 8)
    assert np.allclose(f[:, v > 0], phi[None, :4], atol=1e-14)
    assert np.allclose(f[:, v < 0], phi[None, 4:], atol=1e-14)


def test_mirror_symmetry():
    """x -> 1-x, v -> -v with mirrored cross section and swapped inflow."""
    rng = np.random.default_rng(3)
    sig = 1.0 + rng.uniform(0, 1, 64)
    phi = rng.standard_normal(16)
    f = K.global_solve(sig, 0.1, 16, phi).reshape(64, 16)
    # left inflow (v>0 ascending) <-> right inflow (v<0 ascending) under v -> -v reverses order
    phim = np.concatenate([phi[8:][::-1], phi[:8][::-1]])
    g = K.global_solve(sig[::-1], 0.1, 16, phim).reshape(64, 16)
    assert np.allclose(f, g[::-1, ::-1], atol=1e-12)


def test_banded_equals_dense():
    v, w = K.ordinates(8)
    rng = np.random.default_rng(4)
    sig = 1 + rng.uniform(0, 1, 12)
    A, L = K.assemble(sig, 0.2, 1 / 12, v, w)
    om = rng.standard_normal((8, 3))
    x = np.linalg.solve(A.toarray(), L @ om)
    ext = K.local_solve(sig, 0.2, 1 / 12, v, w, om)
    assert np.allclose(ext[1:13].reshape(-1, 3), x, atol=1e-12)


@pytest.mark.parametrize("Nx,M", [(256, 4), (512, 8)])
def test_full_basis_gluing_equals_global_solve(Nx, M):
    sig = synth.kinetic_sigma(Nx, 0.05)
    v, _ = K.ordinates(32)
    phi = np.concatenate([3 + np.sin(2 * np.pi * v[v > 0]), 2 + np.sin(2 * np.pi * v[v < 0])])
    pts = K.offline(sig, 2.0 ** -6, Nx, M, Nx // M // 2, 32, 0, 0, full_basis=True)
    f = K.online(M, 32, pts, phi)
    ref = K.global_solve(sig, 2.0 ** -6, 32, phi)
    assert np.linalg.norm(f - ref) / np.linalg.norm(ref) < 1e-11


def test_snapshots_have_rank_of_inflow_dimension():
    """s = 48 samples of a 32-dimensional inflow space: sigma_33 of Y at roundoff (rank <= 32)."""
    sig = synth.kinetic_sigma(512)
    g = K.patch_geometry(512, 8, 32)[3]
    Y = K.sample_patch(sig, 2.0 ** -6, 512, 32, g, K.patch_omega(2, g, 32, 48))
    s = np.linalg.svd(Y, compute_uv=False)
    assert s[1] / s[0] > 1e-3 and s[32] / s[0] < 1e-13


@pytest.mark.parametrize("Nx,M,delta,seed", [(512, 8, 32, 2), (256, 4, 20, 5)])
def test_sampled_buffered_patches_at_full_inflow_rank_glue_exactly(Nx, M, delta, seed):
    """Buffered patches sampled with as many random inflow columns as the
    inflow space has dimensions (s = k = 32): each basis spans every solution
    of its patch, so the least-squares gluing must return the fine solve.  This
    pins the restriction of a buffered patch (the cells of K_m and one ghost
    each side, offset by the buffer): a one-cell shift breaks the interface
    rows."""
    sig = synth.kinetic_sigma(Nx, 0.05)
    v, _ = K.ordinates(32)
    phi = np.concatenate([3 + np.sin(2 * np.pi * v[v > 0]), 2 + np.sin(2 * np.pi * v[v < 0])])
    pts = K.offline(sig, 2.0 ** -6, Nx, M, delta, 32, 32, 32, seed=seed)
    assert any(not p["full"] and p["geo"]["x0"] < p["geo"]["k0"] for p in pts)
    f = K.online(M, 32, pts, phi)
    ref = K.global_solve(sig, 2.0 ** -6, 32, phi)
    assert np.linalg.norm(f - ref) / np.linalg.norm(ref) < 1e-11
