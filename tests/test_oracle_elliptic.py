"""Pins of the elliptic oracle against closed forms, invariants and brute force."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import elliptic as E
from oracle.rangefinder import range_finder


def _bilinear_grads(x, y):
    # SW, SE, NE, NW on the unit square
    return np.array([[-(1 - y), -(1 - x)], [(1 - y), -x], [y, x], [-y, (1 - x)]])


def test_element_matrix_equals_quadrature():
    """K_REF is the integral of grad phi_a . grad phi_b over the unit square (2x2 Gauss is exact)."""
    g = np.array([0.5 - 0.5 / np.sqrt(3), 0.5 + 0.5 / np.sqrt(3)])
    K = np.zeros((4, 4))
    for x in g:
        for y in g:
            G = _bilinear_grads(x, y)
            K += 0.25 * G @ G.T
    assert np.allclose(K, E.K_REF, atol=1e-15)


def test_stiffness_symmetric_rowsum_zero_mmatrix():
    rng = np.random.default_rng(1)
    a = np.exp(rng.standard_normal((6, 7)))
    A = E.assemble_stiffness(a).toarray()
    assert np.allclose(A, A.T)
    assert np.allclose(A.sum(1), 0.0, atol=1e-13)
    off = A - np.diag(np.diag(A))
    assert np.all(off <= 1e-15)


def test_stencil_matches_hand_derived_nine_point_form():
    """Assembly reproduces the 9-point Q1 stencil at an interior node (scatter/indexing check)."""
    rng = np.random.default_rng(2)
    nx, ny = 5, 4
    a = np.exp(rng.standard_normal((ny, nx)))
    A = E.assemble_stiffness(a).toarray()
    W = nx + 1
    i, j = 2, 2
    r = j * W + i
    NE, NW, SW, SE = a[j, i], a[j, i - 1], a[j - 1, i - 1], a[j - 1, i]
    assert np.isclose(A[r, r], 2.0 / 3.0 * (NE + NW + SW + SE))
    assert np.isclose(A[r, r + 1], -(NE + SE) / 6.0)
    assert np.isclose(A[r, r - 1], -(NW + SW) / 6.0)
    assert np.isclose(A[r, r + W], -(NE + NW) / 6.0)
    assert np.isclose(A[r, r - W], -(SE + SW) / 6.0)
    assert np.isclose(A[r, r + W + 1], -NE / 3.0)
    assert np.isclose(A[r, r + W - 1], -NW / 3.0)
    assert np.isclose(A[r, r - W - 1], -SW / 3.0)
    assert np.isclose(A[r, r - W + 1], -SE / 3.0)


def _perimeter_walk(cx, cy):
    """Boundary nodes by walking the perimeter explicitly (independent of the oracle's ordering)."""
    pts = []
    x, y = 0, 0
    for dx, dy, n in ((1, 0, cx), (0, 1, cy), (-1, 0, cx), (0, -1, cy)):
        for _ in range(n):
            pts.append((x, y))
            x, y = x + dx, y + dy
    return np.asarray(pts)


@pytest.mark.parametrize("cx,cy", [(5, 5), (7, 4), (3, 9)])
def test_boundary_ordering(cx, cy):
    assert np.array_equal(E.boundary_nodes_ccw(cx, cy), _perimeter_walk(cx, cy))


@pytest.mark.parametrize("cx,cy", [(6, 6), (9, 5), (4, 11)])
def test_constant_coefficient_reproduces_linear_data(cx, cy):
    a = np.full((cy, cx), 2.7)
    b = _perimeter_walk(cx, cy)
    om = 0.3 + 1.7 * b[:, 0] - 0.9 * b[:, 1]
    U = E.local_solve(a, om)[:, :, 0]
    jj, ii = np.meshgrid(np.arange(cy + 1), np.arange(cx + 1), indexing="ij")
    assert np.abs(U - (0.3 + 1.7 * ii - 0.9 * jj)).max() < 1e-12


@pytest.mark.parametrize("axis", [0, 1])
def test_layered_coefficient_harmonic_mean_closed_form(axis):
    """a layered in one direction, data U on that axis: U_i = sum_{e<i} 1/a_e / sum_e 1/a_e (exact)."""
    rng = np.random.default_rng(3)
    n = 12
    lay = np.exp(2.0 * rng.standard_normal(n))
    a = np.tile(lay[None, :], (n, 1)) if axis == 0 else np.tile(lay[:, None], (1, n))
    cum = np.concatenate([[0.0], np.cumsum(1.0 / lay)]) / np.sum(1.0 / lay)
    b = _perimeter_walk(n, n)
    om = cum[b[:, axis]]
    U = E.local_solve(a, om)[:, :, 0]
    exact = np.tile(cum[None, :], (n + 1, 1)) if axis == 0 else np.tile(cum[:, None], (1, n + 1))
    assert np.abs(U - exact).max() < 1e-12


def test_discrete_maximum_principle_and_spd():
    rng = np.random.default_rng(4)
    a = np.exp(rng.standard_normal((10, 13)))
    om = rng.standard_normal((2 * 23, 5))
    U = E.local_solve(a, om)
    assert np.all(U.min(axis=(0, 1)) >= om.min(0) - 1e-12)
    assert np.all(U.max(axis=(0, 1)) <= om.max(0) + 1e-12)
    A = E.assemble_stiffness(a).toarray()
    W = 14
    inner = [j * W + i for j in range(1, 10) for i in range(1, 13)]
    ev = np.linalg.eigvalsh(A[np.ix_(inner, inner)])
    assert ev.min() > 0


def test_banded_solve_equals_dense_solve():
    rng = np.random.default_rng(5)
    cx, cy = 7, 9
    a = np.exp(rng.standard_normal((cy, cx)))
    om = rng.standard_normal((2 * (cx + cy), 3))
    U = E.local_solve(a, om).reshape(-1, 3)
    A = E.assemble_stiffness(a).toarray()
    b = E.boundary_nodes_ccw(cx, cy)
    bidx = b[:, 1] * (cx + 1) + b[:, 0]
    inner = np.setdiff1d(np.arange(A.shape[0]), bidx)
    x = np.linalg.solve(A[np.ix_(inner, inner)], -A[np.ix_(inner, bidx)] @ om)
    assert np.abs(U[inner] - x).max() < 1e-12
    assert np.array_equal(U[bidx], om)


def test_patch_sizes_of_the_periodic_128_workload():
    geo = E.patch_geometry(128, 4, 8)
    sizes = sorted((g["cx"], g["cy"]) for g in geo)
    assert sizes.count((48, 48)) == 4
    assert sizes.count((40, 48)) + sizes.count((48, 40)) == 8
    assert sizes.count((40, 40)) == 4


def test_snapshots_equal_green_matrix_times_omega():
    """G^r = G~ Omega: the sampled snapshots equal the delta-solve Green's matrix times Omega."""
    N, M = 24, 3
    a = synth.lognormal_coefficient(N, 0.2, 1)
    g = E.patch_geometry(N, M, 3)[4]
    Gt = E.full_basis_patch(a, N, g)
    om = E.patch_omega(9, g, 7)
    Y = E.sample_patch(a, N, g, om)
    assert np.abs(Y - Gt @ om).max() < 1e-12 * np.abs(Y).max()


def test_restriction_keeps_boundary_values_where_clipped():
    N, M = 16, 2
    a = synth.periodic_coefficient(N, 0.25)
    g = E.patch_geometry(N, M, 2)[0]          # corner patch: clipped at x=0 and y=0
    om = E.patch_omega(2, g, 3)
    Y = E.sample_patch(a, N, g, om)
    # node (0,0) of K_m is boundary node 0 of K~_m
    assert np.array_equal(Y[0], om[0])


@pytest.mark.parametrize("N,M", [(16, 2), (24, 3), (32, 4)])
def test_full_basis_gluing_equals_global_solve(N, M):
    """With the full basis (DetLocalSolu on K_m) the least-squares gluing is the fine-grid solution."""
    a = synth.lognormal_coefficient(N, 0.1, 1)
    phi = synth.dirichlet_sin_cos(N)
    pts = E.offline(a, N, M, 0, 0, 0, full_basis=True)
    u = E.online(N, M, pts, a, phi)
    ref = E.global_solve(a, N, phi)
    assert E.relative_l2(u, ref) < 1e-12


def test_global_solve_reproduces_linear_function():
    N = 16
    a = np.full(N * N, 3.0)
    b = synth.global_boundary_nodes(N) / N
    phi = 1.0 + 2.0 * b[:, 0] - b[:, 1]
    u = E.global_solve(a, N, phi).reshape(N + 1, N + 1)
    jj, ii = np.meshgrid(np.arange(N + 1) / N, np.arange(N + 1) / N, indexing="ij")
    assert np.abs(u - (1 + 2 * ii - jj)).max() < 1e-12


def test_partition_of_unity():
    for N, M in [(16, 2), (32, 4), (64, 8)]:
        w = E.pou_weights(N, M)
        # the weights of all patches containing a node sum to one: add each
        # patch's weights over its own closed node block
        nH = N // M
        total = np.zeros((N + 1, N + 1))
        for g in E.patch_geometry(N, M, 0):
            total[g["ky0"]:g["ky0"] + nH + 1, g["kx0"]:g["kx0"] + nH + 1] += w[g["ky0"]:g["ky0"] + nH + 1,
                                                                             g["kx0"]:g["kx0"] + nH + 1]
        assert np.abs(total - 1.0).max() < 1e-15
        assert w[nH, nH] == 0.25 and w[0, nH] == 0.5 and w[1, 1] == 1.0


def test_normal_equations_equal_qr_least_squares():
    N, M = 16, 2
    a = synth.periodic_coefficient(N, 0.25)
    pts = E.offline(a, N, M, 2, 6, 6, seed=2)
    P, n_cont, drows, off = E.coarse_rows(N, M, pts, a)
    phi = synth.dirichlet_sin_cos(N)
    Qf, Rf = E.coarse_factor(P)
    c = E.coarse_solve(Qf, Rf, n_cont, drows, phi)[:, 0]
    d = np.zeros(P.shape[0])
    d[n_cont:] = phi[drows]
    c2 = np.linalg.solve(P.T @ P, P.T @ d)
    assert np.allclose(c, c2, rtol=1e-8, atol=1e-10)


def _boundary_full_offline(a, N, M, delta, s, k, seed=2):
    geo, geo0 = E.patch_geometry(N, M, delta), E.patch_geometry(N, M, 0)
    pts = []
    for g, g0 in zip(geo, geo0):
        if g["m1"] in (0, M - 1) or g["m2"] in (0, M - 1):
            Q, _ = np.linalg.qr(E.full_basis_patch(a, N, g0))
            pts.append(dict(geo=g0, Q=Q))
        else:
            Q, _ = range_finder(E.sample_patch(a, N, g, E.patch_omega(seed, g, s)), k)
            pts.append(dict(geo=g, Q=Q))
    return pts


def test_reduced_global_error_decreases_with_rank():
    """Trend of the global test: error falls as the number of random samples per patch grows."""
    N, M = 48, 3
    a = synth.periodic_coefficient(N, 1.0 / 8.0)
    phi = synth.dirichlet_sin_cos(N)
    ref = E.global_solve(a, N, phi)
    errs = []
    for k in (4, 10, 24):
        e = np.mean([E.relative_l2(E.online(N, M, _boundary_full_offline(a, N, M, 8, k, k, seed=sd), a, phi), ref)
                     for sd in (2, 3, 4)])
        errs.append(e)
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-2


def test_full_basis_boundary_option_matches_independent_construction():
    """The oracle's full_basis_boundary option (delta bases on the boundary
    patches, range finder at full rank) gives the reduced solution of the
    construction above (numpy QR of the same Green's matrices)."""
    N, M = 48, 3
    a = synth.periodic_coefficient(N, 1.0 / 8.0)
    phi = synth.dirichlet_sin_cos(N)
    for k in (4, 10):
        u1 = E.online(N, M, _boundary_full_offline(a, N, M, 8, k, k, seed=3), a, phi)
        u2 = E.online(N, M, E.offline(a, N, M, 8, k, k, seed=3, full_basis_boundary=True), a, phi)
        assert E.relative_l2(u2, u1) < 1e-10
