"""Pins of the oracle's range finder: library SVD, orthonormality, the HMT bound."""
import numpy as np

import synth
from oracle import elliptic as E
from oracle.rangefinder import projection_error, range_finder, sign_fix, sin_max_angle


def test_truncation_is_leading_left_singular_subspace():
    rng = np.random.default_rng(0)
    Y = rng.standard_normal((300, 20)) @ np.diag(0.7 ** np.arange(20)) @ rng.standard_normal((20, 20))
    Q, S = range_finder(Y, 6)
    U, S2, _ = np.linalg.svd(Y, full_matrices=False)
    assert np.allclose(S, S2, rtol=1e-12)
    assert np.abs(Q.T @ Q - np.eye(6)).max() < 1e-14
    assert sin_max_angle(U[:, :6], Q) < 1e-10


def test_sign_fix_makes_largest_entry_positive():
    rng = np.random.default_rng(1)
    Q = sign_fix(rng.standard_normal((50, 4)))
    idx = np.argmax(np.abs(Q), axis=0)
    assert np.all(Q[idx, np.arange(4)] > 0)


def test_sin_max_angle_of_subspaces_at_known_angles():
    """Two k-dimensional subspaces whose principal angles are set by
    construction: span{u_i} and span{cos t_i u_i + sin t_i u_{k+i}} with
    orthonormal u_1..u_2k.  The largest principal angle is max t_i, whatever
    orthonormal bases represent the two spans, in either argument order."""
    rng = np.random.default_rng(5)
    n, k = 80, 5
    U, _ = np.linalg.qr(rng.standard_normal((n, 2 * k)))
    for t in ([0.3, 0.1, 0.2, 0.05, 0.0], [1e-7, 2e-7, 0.0, 0.0, 5e-8], [1.2, 0.4, 0.0, 0.9, 0.1]):
        t = np.asarray(t)
        Qa = U[:, :k]
        Qb = U[:, :k] * np.cos(t) + U[:, k:] * np.sin(t)
        Ra, _ = np.linalg.qr(rng.standard_normal((k, k)))
        Rb, _ = np.linalg.qr(rng.standard_normal((k, k)))
        for a, b in ((Qa @ Ra, Qb @ Rb), (Qb @ Rb, Qa @ Ra)):
            assert abs(sin_max_angle(a, b) - np.sin(t.max())) <= 1e-14 + 1e-12 * np.sin(t.max())
    # a subspace against one of its own supersets' k-dimensional parts
    assert sin_max_angle(U[:, :k], U[:, :k] @ Ra) < 1e-14
    assert abs(sin_max_angle(U[:, :k], U[:, k:2 * k]) - 1.0) < 1e-14


def test_hmt_average_spectral_error_bound():
    """Theorem average_spectral (a): mean over draws of ||A - P_Y A|| below the
    stated bound, with the oracle's range finder forming the basis of the
    sketch (k + p columns kept)."""
    rng = np.random.default_rng(2)
    m, n, k, p = 200, 120, 6, 4
    sig = np.concatenate([np.ones(k), 0.05 * 0.8 ** np.arange(n - k)])
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = U @ np.diag(sig) @ V.T
    errs = []
    for t in range(100):
        Om = rng.standard_normal((n, k + p))
        Q, _ = range_finder(A @ Om, k + p)
        errs.append(projection_error(A, Q) * np.linalg.norm(A, 2))
    bound = (1 + k / (p - 1)) * sig[k] + np.e * np.sqrt(k + p) / p * np.sqrt(np.sum(sig[k:] ** 2))
    assert np.mean(errs) <= bound
    assert min(errs) >= sig[k + p] * (1 - 1e-9)  # never better than the optimal rank-(k+p) error


def test_local_error_decays_with_samples_on_a_buffered_patch():
    """Local test: ||G~ - QQ^T G~|| / ||G~|| falls as k grows (Q from QR of G^r)."""
    N, M = 48, 3
    a = synth.periodic_coefficient(N, 1.0 / 8.0)
    g = E.patch_geometry(N, M, 8)[4]
    G = E.full_basis_patch(a, N, g)
    errs = []
    for k in (2, 6, 12, 24):
        Y = E.sample_patch(a, N, g, E.patch_omega(2, g, k))
        Q, _ = np.linalg.qr(Y)
        errs.append(projection_error(G, Q))
    assert all(x > y for x, y in zip(errs, errs[1:]))


def test_buffer_speeds_up_singular_value_decay():
    """Singular values of the buffered Green's matrix decay faster than the unbuffered one."""
    N, M = 48, 3
    a = synth.periodic_coefficient(N, 1.0 / 8.0)
    s0 = np.linalg.svd(E.full_basis_patch(a, N, E.patch_geometry(N, M, 0)[4]), compute_uv=False)
    s1 = np.linalg.svd(E.full_basis_patch(a, N, E.patch_geometry(N, M, 8)[4]), compute_uv=False)
    assert s1[10] / s1[0] < 0.5 * s0[10] / s0[0]
