"""Kinetic oracle: 1D slab linear transport with isotropic scattering (Section 4).

Test infrastructure only (see :mod:`oracle`).  The equation is
v d_x f = (sigma(x)/eps) (<f> - f) on x in [0,1], v in [-1,1], with
<f> = (1/2) int f dv, which is eq. RTE with the homogeneous collision kernel
k = sigma/2 of eq. def.LL.hom.  Inflow data on Gamma_- (x=0, v>0 and x=1, v<0).

Discretization (the paper leaves the scheme open): discrete ordinates at the
Gauss-Legendre nodes v_j with weights w_j (sum 2), cell-centred unknowns
f_{i,j} on cells of width dx, first-order upwind differences:
  v_j > 0:  v_j (f_{i,j} - f_{i-1,j}) / dx + (sigma_i/eps)(f_{i,j} - rho_i) = 0
  v_j < 0:  v_j (f_{i+1,j} - f_{i,j}) / dx + (sigma_i/eps)(f_{i,j} - rho_i) = 0
with rho_i = (1/2) sum_j w_j f_{i,j}, and the inflow values standing in for the
ghost cells f_{-1,j} (v>0) and f_{n,j} (v<0).

Domain decomposition, buffered patches, random inflow sampling
(eq. rte_random), restriction to K_m, full basis at the two end patches
(reduced-basis approach, last paragraph before eq. gb2) and the
least-squares gluing of eqs. gb2, gb3, rte_cond_reduced.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import philox
from .rangefinder import adaptive_rank, range_finder


def ordinates(nv: int = 32):
    """Gauss-Legendre nodes (ascending) and weights on [-1, 1]."""
    v, w = np.polynomial.legendre.leggauss(nv)
    return v, w


def hg_kernel(v: np.ndarray, g: float) -> np.ndarray:
    """The Henyey-Greenstein scattering kernel of eq. HG on the ordinates:
    k(v_i, v_j) = (1/2) (1 - g^2) / (1 + g^2 + 2 g v_i v_j)."""
    return 0.5 * (1 - g * g) / (1 + g * g + 2 * g * np.outer(v, v))


def assemble(sigma: np.ndarray, eps: float, dx: float, v: np.ndarray, w: np.ndarray, hg: float = 0.0):
    """Upwind discrete-ordinates operator on n cells; unknown (i,j) -> i*nv + j.

    Returns (A, L) with A the n*nv square matrix and L the n*nv x nv lifting
    of the inflow vector [left inflow for v>0 (ascending), right inflow for
    v<0 (ascending)], so that A f = L omega.

    hg != 0 replaces the isotropic collision term by the one of eq. RTE with
    the kernel of eq. HG, by quadrature on the ordinates: gain
    sum_j k(v_i, v_j) w_j f_j, loss (sum_j k(v_j, v_i) w_j) f_i, both scaled by
    sigma_i / eps.
    """
    if hg != 0.0:
        return _assemble_hg(sigma, eps, dx, v, w, hg)
    n, nv = sigma.size, v.size
    pos = np.where(v > 0)[0]
    neg = np.where(v < 0)[0]
    s = sigma / eps                                   # (n,)
    I, J = np.meshgrid(np.arange(n), np.arange(nv), indexing="ij")
    r = (I * nv + J).ravel()
    # diagonal: |v_j|/dx + sigma_i/eps
    rows, cols, vals = [r], [r], [(np.abs(v)[None, :] / dx + s[:, None]).ravel()]
    # scattering gain: -(sigma_i/eps) (1/2) w_j' f_{i,j'}
    I3, J3, K3 = np.meshgrid(np.arange(n), np.arange(nv), np.arange(nv), indexing="ij")
    rows.append((I3 * nv + J3).ravel())
    cols.append((I3 * nv + K3).ravel())
    vals.append((-s[:, None, None] * 0.5 * w[None, None, :] * np.ones((n, nv, nv))).ravel())
    # upwind neighbours
    up = (v[None, :] > 0) & (I > 0)
    rows.append(r[up.ravel()]); cols.append((r - nv)[up.ravel()]); vals.append((-v[None, :] / dx * np.ones((n, 1)))[up])
    dn = (v[None, :] < 0) & (I < n - 1)
    rows.append(r[dn.ravel()]); cols.append((r + nv)[dn.ravel()]); vals.append((v[None, :] / dx * np.ones((n, 1)))[dn])
    rows, cols, vals = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n * nv, n * nv)).tocsr()
    L = np.zeros((n * nv, nv))
    for t, j in enumerate(pos):
        L[0 * nv + j, t] = v[j] / dx
    for t, j in enumerate(neg):
        L[(n - 1) * nv + j, len(pos) + t] = -v[j] / dx
    return A, L


def _assemble_hg(sigma, eps, dx, v, w, g):
    n, nv = sigma.size, v.size
    k = hg_kernel(v, g)
    gain = k * w[None, :]                    # gain_ij = k(v_i, v_j) w_j
    loss = (k * w[:, None]).sum(axis=0)      # loss_i = sum_j k(v_j, v_i) w_j
    s = sigma / eps
    blocks = []
    for i in range(n):
        D = np.diag(np.abs(v) / dx + s[i] * loss) - s[i] * gain
        blocks.append(D)
    A = sp.block_diag(blocks, format="lil")
    for i in range(n):
        for j in range(nv):
            if v[j] > 0 and i > 0:
                A[i * nv + j, (i - 1) * nv + j] = -v[j] / dx
            if v[j] < 0 and i < n - 1:
                A[i * nv + j, (i + 1) * nv + j] = v[j] / dx
    A = A.tocsr()
    pos = np.where(v > 0)[0]
    neg = np.where(v < 0)[0]
    L = np.zeros((n * nv, nv))
    for t, j in enumerate(pos):
        L[0 * nv + j, t] = v[j] / dx
    for t, j in enumerate(neg):
        L[(n - 1) * nv + j, len(pos) + t] = -v[j] / dx
    return A, L


def banded(A: sp.spmatrix, l: int, u: int) -> np.ndarray:
    C = A.tocoo()
    ab = np.zeros((l + u + 1, A.shape[0]))
    assert np.all(C.row - C.col <= l) and np.all(C.col - C.row <= u)
    ab[u + C.row - C.col, C.col] = C.data
    return ab


def local_solve(sigma: np.ndarray, eps: float, dx: float, v, w, omega: np.ndarray, hg: float = 0.0) -> np.ndarray:
    """LocalPDESolver for the slab: banded LU solve of A f = L omega for all columns.

    Returns the extended solution (n+2, nv, s): cells 0..n-1 in the middle,
    the left ghost (v>0 entries = left inflow, others 0) first and the right
    ghost (v<0 entries = right inflow, others 0) last.
    """
    omega = np.asarray(omega, dtype=np.float64)
    if omega.ndim == 1:
        omega = omega[:, None]
    n, nv = sigma.size, v.size
    A, L = assemble(sigma, eps, dx, v, w, hg)
    f = sla.solve_banded((nv, nv), banded(A, nv, nv), L @ omega)
    s = omega.shape[1]
    ext = np.zeros((n + 2, nv, s))
    ext[1:n + 1] = f.reshape(n, nv, s)
    pos = np.where(v > 0)[0]
    neg = np.where(v < 0)[0]
    ext[0, pos, :] = omega[:len(pos), :]
    ext[n + 1, neg, :] = omega[len(pos):, :]
    return ext


def patch_geometry(Nx: int, M: int, overlap) -> list[dict]:
    """K_m = cells [m nH, (m+1) nH); K~_m grows it by overlap[m] cells per side, clipped to [0, Nx)."""
    assert Nx % M == 0
    nH = Nx // M
    ov = np.broadcast_to(np.asarray(overlap, dtype=np.int64).ravel(), (M,))
    out = []
    for m in range(M):
        d = int(ov[m])
        x0, x1 = max(0, m * nH - d), min(Nx, (m + 1) * nH + d)
        out.append(dict(p=m, nH=nH, x0=x0, cx=x1 - x0, k0=m * nH))
    return out


def restrict(ext: np.ndarray, g: dict) -> np.ndarray:
    """Cells of K_m plus one ghost cell on each side, all ordinates: ((nH+2)*nv) x s."""
    a = g["k0"] - 1 - (g["x0"] - 1)
    blk = ext[a:a + g["nH"] + 2]
    return blk.reshape(-1, ext.shape[2])


def sample_patch(sigma_all, eps, Nx, nv, g, omega, hg: float = 0.0) -> np.ndarray:
    v, w = ordinates(nv)
    sig = sigma_all[g["x0"]:g["x0"] + g["cx"]]
    return restrict(local_solve(sig, eps, 1.0 / Nx, v, w, omega, hg), g)


def patch_omega(seed: int, g: dict, nv: int, s: int) -> np.ndarray:
    return philox.normals(seed, g["p"], nv, s)


def offline(sigma_all, eps, Nx, M, overlap, nv, s, k, seed=2, omegas=None, full_basis=False,
            full_basis_ends=True, hg: float = 0.0, rank_tol: float = 0.0):
    """Offline stage: snapshots and bases per patch.

    End patches (m = 0 and m = M-1) use the full basis on the unbuffered
    patch (inflow deltas), as the paper does to capture the global inflow
    data; full_basis=True does so for every patch.  rank_tol > 0 keeps, per
    sampled patch, the numerical rank of Y_m at tau = rank_tol sigma_1(Y_m)
    (Def. num_rank), at most k, instead of k.
    """
    geo = patch_geometry(Nx, M, overlap)
    geo0 = patch_geometry(Nx, M, 0)
    out = []
    for g, g0 in zip(geo, geo0):
        end = g["p"] in (0, M - 1)
        if full_basis or (full_basis_ends and end):
            Y = sample_patch(sigma_all, eps, Nx, nv, g0, np.eye(nv), hg)
            out.append(dict(geo=g0, Y=Y, Q=Y, sv=None, full=True))
        else:
            om = omegas[g["p"]] if omegas is not None else patch_omega(seed, g, nv, s)
            Y = sample_patch(sigma_all, eps, Nx, nv, g, om, hg)
            Q, sv = range_finder(Y, k)
            kt = adaptive_rank(sv, k, rank_tol)
            if kt < k:
                Q, sv = range_finder(Y, kt)
            out.append(dict(geo=g, Y=Y, Q=Q, sv=sv, full=False))
    return out


def coarse_rows(M, nv, patches):
    """Interface and inflow rows of P~ (eq. gb3), in the cell-centred upwind reading.

    At the interface between patches m and m+1: for v>0 the last cell of K_m
    equals the left ghost of K_{m+1}; for v<0 the right ghost of K_m equals
    the first cell of K_{m+1}.  Inflow rows: left ghost of patch 0 (v>0) and
    right ghost of patch M-1 (v<0) equal the global inflow data.
    """
    v, _ = ordinates(nv)
    pos = np.where(v > 0)[0]
    neg = np.where(v < 0)[0]
    ks = [p["Q"].shape[1] for p in patches]
    off = np.concatenate([[0], np.cumsum(ks)])
    nH = patches[0]["geo"]["nH"]
    cell = lambda c, j: c * nv + j     # row of (restricted cell index c in 0..nH+1, ordinate j)
    rows = []

    def row(parts):
        r = np.zeros(off[-1])
        for pi, vec in parts:
            r[off[pi]:off[pi + 1]] += vec
        return r

    Q = [p["Q"] for p in patches]
    for j in pos:
        rows.append(row([(0, Q[0][cell(0, j)])]))
    for m in range(M - 1):
        for j in pos:
            rows.append(row([(m, Q[m][cell(nH, j)]), (m + 1, -Q[m + 1][cell(0, j)])]))
        for j in neg:
            rows.append(row([(m, Q[m][cell(nH + 1, j)]), (m + 1, -Q[m + 1][cell(1, j)])]))
    for j in neg:
        rows.append(row([(M - 1, Q[M - 1][cell(nH + 1, j)])]))
    return np.asarray(rows), off


def online(M, nv, patches, phi):
    """Least-squares coefficients (eq. rte_cond_reduced, via Householder QR) and the glued solution.

    phi: 2*npos values (left inflow v>0 ascending, right inflow v<0 ascending)
    or (2*npos, B).  Returns f on all Nx cells: (Nx*nv,) or (Nx*nv, B).
    """
    phi = np.asarray(phi, dtype=np.float64)
    one = phi.ndim == 1
    if one:
        phi = phi[:, None]
    P, off = coarse_rows(M, nv, patches)
    half = phi.shape[0] // 2
    d = np.zeros((P.shape[0], phi.shape[1]))
    d[:half] = phi[:half]
    d[-half:] = phi[half:]
    Qf, Rf = np.linalg.qr(P, mode="reduced")
    c = sla.solve_triangular(Rf, Qf.T @ d)
    nH = patches[0]["geo"]["nH"]
    outs = []
    for pi, p in enumerate(patches):
        full = p["Q"] @ c[off[pi]:off[pi + 1]]
        outs.append(full[nv:(nH + 1) * nv])
    f = np.concatenate(outs, axis=0)
    return f[:, 0] if one else f


def global_solve(sigma_all, eps, nv, phi, hg: float = 0.0) -> np.ndarray:
    """Brute-force fine solve on all cells with the global inflow data (Nx*nv,)."""
    v, w = ordinates(nv)
    Nx = sigma_all.size
    ext = local_solve(sigma_all, eps, 1.0 / Nx, v, w, phi, hg)
    return ext[1:Nx + 1].reshape(Nx * nv, -1)[:, 0] if np.ndim(phi) == 1 else ext[1:Nx + 1].reshape(Nx * nv, -1)


def current(f_cells: np.ndarray, v, w) -> np.ndarray:
    """Discrete flux J_{i+1/2} = sum_{v>0} w v f_i + sum_{v<0} w v f_{i+1} on interior faces."""
    pos = v > 0
    neg = v < 0
    return (f_cells[:-1, pos] * (w * v)[pos]).sum(1) + (f_cells[1:, neg] * (w * v)[neg]).sum(1)
