"""Seeded synthetic inputs shared by the HIP path (tests, bench) and the CPU oracle.

This module holds input generators only: coefficient fields, overlap draws,
global boundary data and Gaussian test matrices.  It contains none of the
multiscale method's arithmetic (no stiffness, no solve, no range finder), so
both sides can draw identical inputs without sharing any of the computation.

Layout conventions used throughout:

* Elliptic coefficients are element-constant on an N x N cell grid of
  [0,1]^2, evaluated at element centroids, stored row-major by cell row:
  ``a[j*N + i]`` is the cell [i h,(i+1) h] x [j h,(j+1) h], h = 1/N.
* Global elliptic boundary data has 4N values, ordered counter-clockwise
  from the node (0,0): bottom i=0..N-1, right j=0..N-1, top i=N..1,
  left j=N..1.
* Kinetic cross sections are given at the N_x cell centres of [0,1].
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "cell_centres", "periodic_coefficient", "lognormal_coefficient",
    "overlap_draw", "global_boundary_nodes", "dirichlet_sin_cos",
    "fourier_boundary", "kinetic_sigma", "gaussian_matrix", "layered_coefficient",
    "two_scale_coefficient", "high_contrast_coefficient", "dirichlet_sine",
]


def cell_centres(n: int) -> np.ndarray:
    """Centres (i + 1/2)/n of the n cells of [0,1]."""
    return (np.arange(n, dtype=np.float64) + 0.5) / n


def periodic_coefficient(N: int, eps: float = 1.0 / 16.0) -> np.ndarray:
    """a(x,y) = 1.1 + sin(2 pi x/eps) sin(2 pi y/eps) at the N*N element centroids (flat, j-major)."""
    xc = cell_centres(N)
    a = 1.1 + np.sin(2 * np.pi * xc[None, :] / eps) * np.sin(2 * np.pi * xc[:, None] / eps)
    return np.ascontiguousarray(a.reshape(-1))


def two_scale_coefficient(N: int, eps: float = 2.0 ** -4) -> np.ndarray:
    """The two-scale medium of the paper's elliptic test (Sec. 5.1, media
    equation) at the N*N element centroids (flat, j-major): a smooth O(1)
    part 2 + sin(2 pi x) cos(2 pi y) plus two quotients of eps-periodic
    trigonometric terms, each bounded away from zero and infinity."""
    xc = cell_centres(N)
    x, y = xc[None, :], xc[:, None]
    k = 2 * np.pi / eps
    a = (2 + np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
         + (2 + 1.8 * np.sin(k * x)) / (2 + 1.8 * np.cos(k * y))
         + (2 + np.sin(k * y)) / (2 + 1.8 * np.cos(k * x)))
    return np.ascontiguousarray(a.reshape(-1))


def high_contrast_coefficient(N: int, contrast: float = 1000.0) -> np.ndarray:
    """The high-contrast medium of the paper's comparison test (Sec. 5.2):
    1 everywhere plus `contrast` on the set where
    x cos(100 r) <= y - 1/2, r the distance to (1/2, 1/2), at the N*N element
    centroids (flat, j-major)."""
    xc = cell_centres(N)
    x, y = xc[None, :], xc[:, None]
    r = np.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2)
    a = 1.0 + contrast * (x * np.cos(100.0 * r) <= y - 0.5)
    return np.ascontiguousarray(a.reshape(-1))


def layered_coefficient(N: int, values_per_column: np.ndarray, axis: int = 0) -> np.ndarray:
    """Coefficient that depends on one coordinate only (axis 0: x, axis 1: y)."""
    v = np.asarray(values_per_column, dtype=np.float64)
    assert v.shape == (N,)
    a = np.tile(v[None, :], (N, 1)) if axis == 0 else np.tile(v[:, None], (1, N))
    return np.ascontiguousarray(a.reshape(-1))


def lognormal_coefficient(N: int, ell: float, seed: int) -> np.ndarray:
    """a = exp(g) at the N*N element centroids, g a zero-mean unit-variance Gaussian field.

    g has exponential covariance exp(-r/ell) and is sampled by circulant
    embedding on a 2N x 2N periodic grid of spacing 1/N (eigenvalues clipped
    at zero), then cropped to the N x N cells.  PCG64(seed) drives it.
    """
    P = 2 * N
    d = np.minimum(np.arange(P), P - np.arange(P)) / N
    r = np.sqrt(d[None, :] ** 2 + d[:, None] ** 2)
    c = np.exp(-r / ell)
    lam = np.real(np.fft.fft2(c))
    lam = np.clip(lam, 0.0, None)
    rng = np.random.Generator(np.random.PCG64(seed))
    xi = rng.standard_normal((P, P)) + 1j * rng.standard_normal((P, P))
    z = np.fft.fft2(np.sqrt(lam / (P * P)) * xi)
    g = np.real(z)[:N, :N]
    return np.ascontiguousarray(np.exp(g).reshape(-1))


def overlap_draw(M: int, choices=(16, 32), seed: int = 3) -> np.ndarray:
    """Per-patch buffer width in cells, drawn by a seeded fair coin (M*M int32, patch p = m2*M + m1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pick = rng.integers(0, len(choices), size=M * M)
    return np.asarray(choices, dtype=np.int32)[pick]


def global_boundary_nodes(N: int) -> np.ndarray:
    """(4N, 2) int array of boundary node (i, j), counter-clockwise from (0,0)."""
    out = []
    out += [(i, 0) for i in range(0, N)]
    out += [(N, j) for j in range(0, N)]
    out += [(i, N) for i in range(N, 0, -1)]
    out += [(0, j) for j in range(N, 0, -1)]
    return np.asarray(out, dtype=np.int64)


def dirichlet_sin_cos(N: int) -> np.ndarray:
    """phi = sin(2 pi x) + cos(2 pi y) on the 4N global boundary nodes."""
    b = global_boundary_nodes(N) / N
    return np.sin(2 * np.pi * b[:, 0]) + np.cos(2 * np.pi * b[:, 1])


def dirichlet_sine(N: int) -> np.ndarray:
    """A sine over the boundary, phi = sin(pi t / 2) in the perimeter
    arclength t in [0, 4) (counter-clockwise from (0,0)), on the 4N global
    boundary nodes: one smooth period around the square (the paper's global
    elliptic test specifies sine boundary data and nothing more)."""
    t = np.arange(4 * N, dtype=np.float64) / N
    return np.sin(np.pi * t / 2)


def fourier_boundary(N: int, request_ids, seed: int = 4, n_modes: int = 16) -> np.ndarray:
    """Boundary data of serving requests: (len(ids), 4N).

    f(t) on perimeter arclength t in [0,4):
    sum_{k=1..16} k^-2 (alpha_k cos(pi k t/2) + beta_k sin(pi k t/2)),
    alpha, beta ~ N(0,1) drawn from PCG64 seeded by (seed, request id).
    """
    b = global_boundary_nodes(N)
    i, j = b[:, 0] / N, b[:, 1] / N
    # arclength from (0,0) counter-clockwise
    t = np.where(b[:, 1] == 0, i, 0.0)
    t = np.where((b[:, 0] == N) & (b[:, 1] < N), 1.0 + j, t)
    t = np.where((b[:, 1] == N) & (b[:, 0] > 0), 2.0 + (1.0 - i), t)
    t = np.where((b[:, 0] == 0) & (b[:, 1] > 0), 3.0 + (1.0 - j), t)
    k = np.arange(1, n_modes + 1, dtype=np.float64)
    rows = []
    for rid in request_ids:
        rng = np.random.Generator(np.random.PCG64([seed, int(rid)]))
        al = rng.standard_normal(n_modes)
        be = rng.standard_normal(n_modes)
        ph = np.pi * k[None, :] * t[:, None] / 2.0
        rows.append((np.cos(ph) * al + np.sin(ph) * be) @ (k ** -2.0))
    return np.asarray(rows, dtype=np.float64)


def kinetic_sigma(Nx: int, period: float = 0.01) -> np.ndarray:
    """sigma(x) = 1 + 0.5 sin(2 pi x / period) at the Nx cell centres."""
    return 1.0 + 0.5 * np.sin(2 * np.pi * cell_centres(Nx) / period)


def gaussian_matrix(rows: int, cols: int, seed: int) -> np.ndarray:
    """i.i.d. N(0,1) matrix from PCG64(seed), column-major semantics left to the caller."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((rows, cols))
