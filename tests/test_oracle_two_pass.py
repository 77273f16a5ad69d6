"""Pins of the oracle's adjoint local solve and two-pass randomized SVD.

The adjoint is pinned to the forward local solve (the defining identity of a
transpose) and to the transpose of the Green's matrix built independently by
DetLocalSolu (Kronecker-delta data); the two-pass basis is pinned to a dense
library SVD of that Green's matrix where the sampling spans its range, and to
the optimality that defines it otherwise.
"""
import numpy as np
import pytest

import synth
from oracle import elliptic as E
from oracle.rangefinder import range_finder, sin_max_angle

N, M = 32, 2
OVERLAP = 4


def _patch(p):
    a = synth.lognormal_coefficient(N, 0.1, 5)
    return a, E.patch_geometry(N, M, OVERLAP)[p]


@pytest.mark.parametrize("p", [0, 3])
def test_adjoint_identity_with_the_forward_solve(p):
    """<G omega, q> = <omega, G^T q> for random omega and q."""
    a, g = _patch(p)
    nb = 2 * (g["cx"] + g["cy"])
    nk = (g["nH"] + 1) ** 2
    om = synth.gaussian_matrix(nb, 3, 11)
    q = synth.gaussian_matrix(nk, 3, 12)
    lhs = q.T @ E.sample_patch(a, N, g, om)
    rhs = E.adjoint_patch(a, N, g, q).T @ om
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(lhs).max()


@pytest.mark.parametrize("p", [0, 1, 3])
def test_adjoint_equals_transpose_of_the_delta_solve_green_matrix(p):
    a, g = _patch(p)
    G = E.full_basis_patch(a, N, g)                 # n_K x n_b, DetLocalSolu
    q = synth.gaussian_matrix(G.shape[0], 4, 13)
    ref = G.T @ q
    got = E.adjoint_patch(a, N, g, q)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_adjoint_of_a_node_of_k_on_the_boundary_is_its_delta():
    """A node of K_m that lies on the buffered patch's boundary (a corner patch
    clipped to the domain) keeps its boundary value: G^T e_node has the unit
    entry at that boundary node."""
    a, g = _patch(0)
    nk = (g["nH"] + 1) ** 2
    e = np.zeros((nk, 1))
    e[0, 0] = 1.0                                   # node (0,0) of K_m = boundary node 0 of K~_m
    G = E.full_basis_patch(a, N, g)
    col = E.adjoint_patch(a, N, g, e)[:, 0]
    assert np.allclose(col, G[0], atol=1e-13)
    assert col[0] == pytest.approx(1.0, abs=1e-13)


@pytest.mark.parametrize("p", [0, 3])
def test_two_pass_with_spanning_samples_is_the_svd_of_g(p):
    """With as many samples as boundary nodes span(Y) = range(G): the two-pass
    basis is the k leading left singular vectors of G and its singular values
    are G's."""
    a, g = _patch(p)
    G = E.full_basis_patch(a, N, g)
    nb = G.shape[1]
    om = synth.gaussian_matrix(nb, nb, 21)
    Y = E.sample_patch(a, N, g, om)
    k = 8
    U, sB = E.two_pass_basis(a, N, g, Y, k)
    Ug, Sg, _ = np.linalg.svd(G, full_matrices=False)
    assert np.abs(sB[:k] - Sg[:k]).max() <= 1e-10 * Sg[0]
    gap = (Sg[k - 1] - Sg[k]) / Sg[0]
    assert gap > 1e-6
    assert sin_max_angle(Ug[:, :k], U) <= 1e-12 / gap
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-13


@pytest.mark.parametrize("s", [12, 20])
def test_two_pass_is_the_best_rank_k_projection_within_span_y(s):
    """||G - U U^T G||_F over k-dimensional U inside span(Y) is smallest for
    the two-pass basis, so it is at most the one-pass error, and at least the
    optimal rank-k error (the tail of G's singular values)."""
    a, g = _patch(3)
    G = E.full_basis_patch(a, N, g)
    k = 8
    om = synth.gaussian_matrix(G.shape[1], s, 31)
    Y = E.sample_patch(a, N, g, om)
    U2, _ = E.two_pass_basis(a, N, g, Y, k)
    U1, _ = range_finder(Y, k)
    e2 = np.linalg.norm(G - U2 @ (U2.T @ G))
    e1 = np.linalg.norm(G - U1 @ (U1.T @ G))
    Sg = np.linalg.svd(G, compute_uv=False)
    eopt = np.sqrt(np.sum(Sg[k:] ** 2))
    assert e2 <= e1 * (1 + 1e-12)
    assert e2 >= eopt * (1 - 1e-12)
    # and strictly better than one pass here (s well above k)
    assert e2 < 0.99 * e1


def test_offline_two_pass_option_matches_two_pass_basis():
    a = synth.lognormal_coefficient(N, 0.1, 5)
    ref = E.offline(a, N, M, OVERLAP, 12, 6, seed=3, two_pass=True)
    for pr in ref:
        g = pr["geo"]
        U, sB = E.two_pass_basis(a, N, g, pr["Y"], 6)
        assert np.array_equal(U, pr["Q"]) and np.array_equal(sB, pr["sv"])
