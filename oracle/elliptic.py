"""Elliptic oracle: -div(a grad u) = 0 on [0,1]^2, Dirichlet data (Section 5, eqs. Elliptic, elliptic_bdy).

Test infrastructure only (see :mod:`oracle`).  Plain FP64 NumPy/SciPy, written
step by step from the paper:

* fine discretization: bilinear (Q1) finite elements on a uniform grid of
  N x N square cells, element-constant coefficient at the centroid
  (Section 5.3 uses a bilinear nodal basis);
* domain decomposition into M x M coarse patches K_m (eq. after "We solve ...
  on a coarse mesh"), buffered patches K~_m that grow K_m by a buffer and are
  clipped to the domain (Section 3, buffer zone; Section 5.2);
* offline RanLocalSolu: for each patch, solve the local problem on K~_m with
  i.i.d. N(0,1) Dirichlet values at every boundary grid point (eq.
  elliptic_random) with a banded Cholesky factor, restrict to K_m (the reduced
  Green's matrix G^{eps,r}_m);
* DetLocalSolu (full basis): the same local solver with Kronecker-delta data
  (eq. elliptic_b);
* online: value and conormal-flux continuity across shared edges and the
  Dirichlet condition (eqs. elliptic_cont_cond, elliptic_bdy_cond,
  elliptic_cond_tilde), solved in the least-squares sense (eq.
  elliptic_cond_reduced) by Householder QR, then u = sum_m G_m c_m with
  nodal partition-of-unity weights at shared nodes;
* brute force: the global fine-grid FE solve.

Where the paper is silent, each function's docstring states the reading it takes.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import philox
from .rangefinder import adaptive_rank, range_finder, sign_fix

# Bilinear element stiffness of the unit square for -div(grad u), local node
# order SW, SE, NE, NW (counter-clockwise).  Scale-free in 2D: the element
# matrix of a cell of side h with coefficient a_e is a_e * K_REF.
K_REF = np.array([[4.0, -1.0, -2.0, -1.0],
                  [-1.0, 4.0, -1.0, -2.0],
                  [-2.0, -1.0, 4.0, -1.0],
                  [-1.0, -2.0, -1.0, 4.0]]) / 6.0


# --------------------------------------------------------------------------- grid
def assemble_stiffness(a_cells: np.ndarray) -> sp.csr_matrix:
    """Q1 stiffness of an nx x ny cell block, node (i,j) -> j*(nx+1)+i.

    a_cells has shape (ny, nx); element (i,j) has corners SW=(i,j), SE=(i+1,j),
    NE=(i+1,j+1), NW=(i,j+1).  Standard element-by-element assembly.
    """
    ny, nx = a_cells.shape
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()
    W = nx + 1
    corners = np.stack([jj * W + ii, jj * W + ii + 1, (jj + 1) * W + ii + 1, (jj + 1) * W + ii], axis=1)
    ae = a_cells.ravel()
    rows, cols, vals = [], [], []
    for al in range(4):
        for be in range(4):
            rows.append(corners[:, al])
            cols.append(corners[:, be])
            vals.append(ae * K_REF[al, be])
    n = (nx + 1) * (ny + 1)
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return A.tocsr()


def boundary_nodes_ccw(nx: int, ny: int) -> np.ndarray:
    """Boundary nodes (i,j) of an nx x ny cell block, counter-clockwise from (0,0)."""
    out = [(i, 0) for i in range(0, nx)]
    out += [(nx, j) for j in range(0, ny)]
    out += [(i, ny) for i in range(nx, 0, -1)]
    out += [(0, j) for j in range(ny, 0, -1)]
    return np.asarray(out, dtype=np.int64)


def to_banded_upper(A: sp.spmatrix, u: int) -> np.ndarray:
    """Upper banded storage ab[u + r - c, c] = A[r, c] (c >= r) for LAPACK pbtrf."""
    C = sp.triu(A).tocoo()
    n = A.shape[0]
    assert np.all(C.col - C.row <= u)
    ab = np.zeros((u + 1, n))
    ab[u + C.row - C.col, C.col] = C.data
    return ab


# ---------------------------------------------------------------- geometry
def patch_geometry(N: int, M: int, overlap) -> list[dict]:
    """Patches K_m and buffered patches K~_m in cell units.

    K_m = [m1 nH, (m1+1) nH] x [m2 nH, (m2+1) nH], nH = N/M, patch index
    p = m2*M + m1.  K~_m grows K_m by overlap[p] cells on each side and is
    clipped to [0, N]^2.
    """
    assert N % M == 0
    nH = N // M
    ov = np.broadcast_to(np.asarray(overlap, dtype=np.int64).ravel(), (M * M,))
    out = []
    for m2 in range(M):
        for m1 in range(M):
            p = m2 * M + m1
            d = int(ov[p])
            x0, x1 = max(0, m1 * nH - d), min(N, (m1 + 1) * nH + d)
            y0, y1 = max(0, m2 * nH - d), min(N, (m2 + 1) * nH + d)
            out.append(dict(p=p, m1=m1, m2=m2, nH=nH, x0=x0, y0=y0, cx=x1 - x0, cy=y1 - y0,
                            kx0=m1 * nH, ky0=m2 * nH))
    return out


def patch_coefficient(a_flat: np.ndarray, N: int, g: dict) -> np.ndarray:
    a = a_flat.reshape(N, N)
    return a[g["y0"]:g["y0"] + g["cy"], g["x0"]:g["x0"] + g["cx"]]


# ---------------------------------------------------------------- local solve
def local_solve(a_patch: np.ndarray, omega: np.ndarray) -> np.ndarray:
    """LocalPDESolver on one (buffered) patch: nodal solution with boundary values omega.

    a_patch: (cy, cx) element coefficients; omega: (n_b, s) boundary values in
    counter-clockwise order.  Solves A_II u_I = -A_IB omega with one banded
    Cholesky factor (LAPACK pbtrf/pbtrs) and s triangular solve pairs.
    Returns U with shape (cy+1, cx+1, s).
    """
    cy, cx = a_patch.shape
    omega = np.asarray(omega, dtype=np.float64)
    if omega.ndim == 1:
        omega = omega[:, None]
    s = omega.shape[1]
    A = assemble_stiffness(a_patch)
    W = cx + 1
    bn = boundary_nodes_ccw(cx, cy)
    bidx = bn[:, 1] * W + bn[:, 0]
    assert omega.shape[0] == bidx.size
    # interior nodes, ordered so that the shorter side runs fastest (narrow band)
    if cx <= cy:
        jj, ii = np.meshgrid(np.arange(1, cy), np.arange(1, cx), indexing="ij")
        band = cx
    else:
        ii, jj = np.meshgrid(np.arange(1, cx), np.arange(1, cy), indexing="ij")
        band = cy
    iidx = (jj * W + ii).ravel()
    U = np.zeros(((cx + 1) * (cy + 1), s))
    U[bidx, :] = omega
    if iidx.size:
        A_II = A[iidx][:, iidx]
        A_IB = A[iidx][:, bidx]
        rhs = -(A_IB @ omega)
        ab = to_banded_upper(A_II, band)
        cb = sla.cholesky_banded(ab, lower=False)
        U[iidx, :] = sla.cho_solve_banded((cb, False), rhs)
    return U.reshape(cy + 1, cx + 1, s)


def restrict_to_patch(U: np.ndarray, g: dict) -> np.ndarray:
    """Restriction of a buffered-patch solution to the nodes of K_m (closed), row-major: (nH+1)^2 x s."""
    nH = g["nH"]
    i0, j0 = g["kx0"] - g["x0"], g["ky0"] - g["y0"]
    blk = U[j0:j0 + nH + 1, i0:i0 + nH + 1, :]
    return blk.reshape((nH + 1) * (nH + 1), -1)


def patch_omega(seed: int, g: dict, s: int) -> np.ndarray:
    """Random boundary samples of a buffered patch, drawn by Philox (node, sample, patch)."""
    return philox.normals(seed, g["p"], 2 * (g["cx"] + g["cy"]), s)


def sample_patch(a_flat, N, g, omega) -> np.ndarray:
    """RanLocalSolu on one patch: Y_m = [r_{m,1..s}] = restricted solutions (n_K x s)."""
    U = local_solve(patch_coefficient(a_flat, N, g), omega)
    return restrict_to_patch(U, g)


def full_basis_patch(a_flat, N, g) -> np.ndarray:
    """DetLocalSolu on the patch geometry g: Kronecker-delta boundary data at every boundary node."""
    nb = 2 * (g["cx"] + g["cy"])
    return sample_patch(a_flat, N, g, np.eye(nb))


def adjoint_patch(a_flat, N, g, q) -> np.ndarray:
    """Transpose of the reduced Green's matrix of a buffered patch applied to q (n_K x r).

    The forward map (RanLocalSolu on one patch) is G omega = R_K u with u_B =
    omega and A_II u_I = -A_IB omega.  Written out, its transpose is
    G^T q = f_B - A_BI A_II^{-1} f_I, where f = R_K^T q is q placed at the nodes
    of K_m and zero elsewhere; A_II is symmetric, so the interior solve is the
    forward one with the source f_I in place of -A_IB omega.  Returns the
    n_b x r boundary values in counter-clockwise order.
    """
    a_patch = patch_coefficient(a_flat, N, g)
    cy, cx = a_patch.shape
    q = np.asarray(q, dtype=np.float64)
    if q.ndim == 1:
        q = q[:, None]
    A = assemble_stiffness(a_patch)
    W = cx + 1
    bn = boundary_nodes_ccw(cx, cy)
    bidx = bn[:, 1] * W + bn[:, 0]
    if cx <= cy:
        jj, ii = np.meshgrid(np.arange(1, cy), np.arange(1, cx), indexing="ij")
        band = cx
    else:
        ii, jj = np.meshgrid(np.arange(1, cx), np.arange(1, cy), indexing="ij")
        band = cy
    iidx = (jj * W + ii).ravel()
    # f = R_K^T q: the rows of q are the nodes of K_m, row-major (as restrict_to_patch)
    nH = g["nH"]
    i0, j0 = g["kx0"] - g["x0"], g["ky0"] - g["y0"]
    kj, ki = np.meshgrid(np.arange(nH + 1), np.arange(nH + 1), indexing="ij")
    knodes = ((j0 + kj) * W + (i0 + ki)).ravel()
    assert q.shape[0] == knodes.size
    f = np.zeros(((cx + 1) * (cy + 1), q.shape[1]))
    f[knodes, :] = q
    out = f[bidx, :].copy()
    if iidx.size:
        A_II = A[iidx][:, iidx]
        A_BI = A[bidx][:, iidx]
        cb = sla.cholesky_banded(to_banded_upper(A_II, band), lower=False)
        z = sla.cho_solve_banded((cb, False), f[iidx, :])
        out -= A_BI @ z
    return out


def two_pass_basis(a_flat, N, g, Y, k, rank_rtol=1e-12):
    """Two-pass randomized SVD of a patch's reduced Green's matrix from its snapshots.

    The randomized SVD recalled in Section 2.3 (Theorem average_spectral,
    after Halko, Martinsson and Tropp) projects G onto span(Y), Y = G Omega;
    its direct-SVD form reads G a second time through its transpose: Q = an
    orthonormal basis of span(Y) (Householder QR and the SVD of R, kept at the
    numerical rank sigma_j(Y) > rank_rtol sigma_1(Y)), B = Q^T G = (G^T Q)^T
    by adjoint local solves, B = U_B S V^T, and the basis Q U_B[:, :k] (the k
    leading left singular vectors of Q Q^T G, sign-fixed).  Returns (basis,
    singular values of B).
    """
    Qh, R = np.linalg.qr(Y, mode="reduced")
    U, S, _ = np.linalg.svd(R)
    r = int(np.count_nonzero(S > rank_rtol * S[0]))
    Q = Qh @ U[:, :r]
    C = adjoint_patch(a_flat, N, g, Q)
    UB, SB, _ = np.linalg.svd(C.T, full_matrices=False)
    return sign_fix(Q @ UB[:, :k]), SB


def offline(a_flat, N, M, overlap, s, k, seed=2, omegas=None, full_basis=False, full_basis_boundary=False,
            rank_tol=0.0, two_pass=False):
    """Offline stage over all patches: snapshots Y_m, rank-k bases Q_m and singular values.

    omegas: optional list of explicit boundary sample matrices (one per patch);
    default draws them with Philox(seed).  full_basis=True runs DetLocalSolu
    on the unbuffered patches instead and keeps the full Green's matrix.
    full_basis_boundary=True does so only for the patches that touch the
    domain boundary (no buffer, Kronecker-delta data at all 4 N/M boundary
    nodes), with the basis orthonormalized by the range finder at full rank;
    the interior patches are sampled as usual.  rank_tol > 0 keeps, per
    sampled patch, the numerical rank of Y_m at tau = rank_tol sigma_1(Y_m)
    (Def. num_rank), at most k, instead of k.  two_pass=True builds each
    sampled patch's basis by the two-pass randomized SVD (two_pass_basis; sv
    are then the singular values of Q^T G, and rank_tol applies to them).
    """
    geo = patch_geometry(N, M, 0 if full_basis else overlap)
    geo0 = patch_geometry(N, M, 0) if full_basis_boundary else None
    out = []
    for g in geo:
        on_boundary = g["m1"] in (0, M - 1) or g["m2"] in (0, M - 1)
        if full_basis:
            Y = full_basis_patch(a_flat, N, g)
            Q, sv = Y, None
        elif full_basis_boundary and on_boundary:
            g = geo0[g["p"]]
            Y = full_basis_patch(a_flat, N, g)
            Q, sv = range_finder(Y, Y.shape[1])
        else:
            om = omegas[g["p"]] if omegas is not None else patch_omega(seed, g, s)
            Y = sample_patch(a_flat, N, g, om)
            basis = (lambda kk: two_pass_basis(a_flat, N, g, Y, kk)) if two_pass else (lambda kk: range_finder(Y, kk))
            Q, sv = basis(k)
            kt = adaptive_rank(sv, k, rank_tol)
            if kt < k:
                Q, sv = basis(kt)
        out.append(dict(geo=g, Y=Y, Q=Q, sv=sv))
    return out


# ---------------------------------------------------------------- online stage
def patch_boundary_local(nH: int) -> np.ndarray:
    return boundary_nodes_ccw(nH, nH)


def traces(a_flat, N, g, Q) -> tuple[np.ndarray, np.ndarray]:
    """Values and conormal fluxes of the basis on the nodes of dK_m (all (nH+1)^2 rows kept).

    The flux of q at a node x of dK_m is (A^{K_m} q)(x) / h, with A^{K_m}
    assembled from the elements of K_m only: the discrete a d_n q of the
    continuity condition (eq. elliptic_cont_cond).  Returned arrays are
    (nH+1)^2 x k; rows of interior nodes of the flux are not used.
    """
    nH = g["nH"]
    aK = a_flat.reshape(N, N)[g["ky0"]:g["ky0"] + nH, g["kx0"]:g["kx0"] + nH]
    AK = assemble_stiffness(aK)
    h = 1.0 / N
    return Q, (AK @ Q) / h


def coarse_rows(N, M, patches, a_flat, phi=None):
    """Rows of the least-squares system P~ c = d (eqs. elliptic_cond_tilde, elliptic_bdy_cond).

    Returns (P, d, col_offsets) with P dense.  Rows, in this order:
      value continuity at every node of each interior coarse edge (endpoints included);
      flux continuity at the nH-1 nodes strictly inside each interior edge;
      a four-patch flux balance at each interior coarse vertex;
      Dirichlet rows q_m(x) c_m = phi(x) for each patch m and node x of dK_m on dOmega.
    phi: (4N,) or (4N, B) global boundary data in counter-clockwise order.
    """
    nH = N // M
    W = nH + 1
    ks = [p["Q"].shape[1] for p in patches]
    off = np.concatenate([[0], np.cumsum(ks)])
    vals, flux = [], []
    for p in patches:
        v, f = traces(a_flat, N, p["geo"], p["Q"])
        vals.append(v)
        flux.append(f)
    rows = []

    def row(parts):
        r = np.zeros(off[-1])
        for (pi, vec) in parts:
            r[off[pi]:off[pi + 1]] += vec
        return r

    pid = lambda m1, m2: m2 * M + m1
    loc = lambda i, j: j * W + i
    # vertical edges between (m1,m2) and (m1+1,m2)
    for m2 in range(M):
        for m1 in range(M - 1):
            L, R = pid(m1, m2), pid(m1 + 1, m2)
            for t in range(nH + 1):
                rows.append(row([(L, vals[L][loc(nH, t)]), (R, -vals[R][loc(0, t)])]))
            for t in range(1, nH):
                rows.append(row([(L, flux[L][loc(nH, t)]), (R, flux[R][loc(0, t)])]))
    # horizontal edges between (m1,m2) and (m1,m2+1)
    for m2 in range(M - 1):
        for m1 in range(M):
            B, T = pid(m1, m2), pid(m1, m2 + 1)
            for t in range(nH + 1):
                rows.append(row([(B, vals[B][loc(t, nH)]), (T, -vals[T][loc(t, 0)])]))
            for t in range(1, nH):
                rows.append(row([(B, flux[B][loc(t, nH)]), (T, flux[T][loc(t, 0)])]))
    # interior coarse vertices
    for v2 in range(1, M):
        for v1 in range(1, M):
            rows.append(row([(pid(v1 - 1, v2 - 1), flux[pid(v1 - 1, v2 - 1)][loc(nH, nH)]),
                             (pid(v1, v2 - 1), flux[pid(v1, v2 - 1)][loc(0, nH)]),
                             (pid(v1 - 1, v2), flux[pid(v1 - 1, v2)][loc(nH, 0)]),
                             (pid(v1, v2), flux[pid(v1, v2)][loc(0, 0)])]))
    n_cont = len(rows)
    # Dirichlet rows
    bmap = global_boundary_index(N)
    drows = []
    for p in patches:
        g = p["geo"]
        for jj in range(nH + 1):
            for ii in range(nH + 1):
                gx, gy = g["kx0"] + ii, g["ky0"] + jj
                if gx in (0, N) or gy in (0, N):
                    rows.append(row([(g["p"], vals[g["p"]][loc(ii, jj)])]))
                    drows.append(bmap[(gx, gy)])
    P = np.asarray(rows)
    return P, n_cont, np.asarray(drows, dtype=np.int64), off


def global_boundary_index(N: int) -> dict:
    out = {}
    for t, (i, j) in enumerate(boundary_nodes_ccw(N, N)):
        out[(int(i), int(j))] = t
    return out


def coarse_factor(P):
    """Householder QR of P~ (the least-squares solver of eq. elliptic_cond_reduced)."""
    Qf, Rf = np.linalg.qr(P, mode="reduced")
    return Qf, Rf


def coarse_solve(Qf, Rf, n_cont, drows, phi):
    """c = argmin ||P~ c - d||_2 with d = [0 (continuity), phi at the Dirichlet rows]."""
    phi = np.asarray(phi, dtype=np.float64)
    if phi.ndim == 1:
        phi = phi[:, None]
    d = np.zeros((Qf.shape[0], phi.shape[1]))
    d[n_cont:, :] = phi[drows, :]
    return sla.solve_triangular(Rf, Qf.T @ d)


def reconstruct(N, M, patches, off, c):
    """u = sum_m w_m (G_m c_m) on the (N+1)^2 nodes, w_m = 1/#{patches containing the node}."""
    c = np.asarray(c)
    if c.ndim == 1:
        c = c[:, None]
    nH = N // M
    B = c.shape[1]
    u = np.zeros(((N + 1) * (N + 1), B))
    cnt = np.zeros((N + 1) * (N + 1))
    for pi, p in enumerate(patches):
        g = p["geo"]
        jj, ii = np.meshgrid(np.arange(nH + 1), np.arange(nH + 1), indexing="ij")
        gidx = ((g["ky0"] + jj) * (N + 1) + g["kx0"] + ii).ravel()
        cnt[gidx] += 1
    for pi, p in enumerate(patches):
        g = p["geo"]
        jj, ii = np.meshgrid(np.arange(nH + 1), np.arange(nH + 1), indexing="ij")
        gidx = ((g["ky0"] + jj) * (N + 1) + g["kx0"] + ii).ravel()
        u[gidx, :] += (p["Q"] @ c[off[pi]:off[pi + 1], :]) / cnt[gidx][:, None]
    return u


def pou_weights(N, M) -> np.ndarray:
    nH = N // M
    cnt = np.zeros((N + 1, N + 1))
    for m2 in range(M):
        for m1 in range(M):
            cnt[m2 * nH:(m2 + 1) * nH + 1, m1 * nH:(m1 + 1) * nH + 1] += 1
    return 1.0 / cnt


def online(N, M, patches, a_flat, phi):
    P, n_cont, drows, off = coarse_rows(N, M, patches, a_flat)
    Qf, Rf = coarse_factor(P)
    c = coarse_solve(Qf, Rf, n_cont, drows, phi)
    return reconstruct(N, M, patches, off, c)[:, 0] if np.ndim(phi) == 1 else reconstruct(N, M, patches, off, c)


def coarse_solve_constrained(P, n_cont, drows, phi):
    """The constrained least-squares alternative of Sec. 5.2 (after eq.
    elliptic_cond_reduced): minimize the continuity rows ||A c||_2 (value and
    flux mismatch) subject to the Dirichlet rows B c = phi holding exactly.

    Null-space method: a particular solution c_0 of B c = phi (minimum norm),
    an orthonormal basis Z of null(B), and c = c_0 + Z y with
    y = argmin ||A (c_0 + Z y)||_2.  The constraint must be satisfiable for
    every phi: B needs full row rank, which holds when the patches touching
    the boundary keep their full bases; otherwise ValueError.
    """
    phi = np.asarray(phi, dtype=np.float64)
    if phi.ndim == 1:
        phi = phi[:, None]
    A, B = P[:n_cont], P[n_cont:]
    sv = np.linalg.svd(B, compute_uv=False)
    if sv.size < B.shape[0] or sv[-1] <= 1e-10 * sv[0]:
        raise ValueError("Dirichlet rows are rank deficient: the boundary condition cannot hold exactly")
    rhs = phi[drows, :]
    c0 = np.linalg.lstsq(B, rhs, rcond=None)[0]
    Z = sla.null_space(B)
    y = np.linalg.lstsq(A @ Z, -(A @ c0), rcond=None)[0]
    return c0 + Z @ y


def online_constrained(N, M, patches, a_flat, phi):
    """Global solution from the constrained least-squares coefficients."""
    P, n_cont, drows, off = coarse_rows(N, M, patches, a_flat)
    c = coarse_solve_constrained(P, n_cont, drows, phi)
    u = reconstruct(N, M, patches, off, c)
    return u[:, 0] if np.ndim(phi) == 1 else u


# ---------------------------------------------------------------- brute force
def global_solve(a_flat, N, phi) -> np.ndarray:
    """Fine-grid FE solution on all (N+1)^2 nodes with Dirichlet phi (the reference solution)."""
    a = a_flat.reshape(N, N)
    phi = np.asarray(phi, dtype=np.float64)
    U = local_solve(a, phi[:, None] if phi.ndim == 1 else phi)
    U = U.reshape((N + 1) * (N + 1), -1)
    return U[:, 0] if phi.ndim == 1 else U


def relative_l2(u, ref) -> float:
    return float(np.linalg.norm(u - ref) / np.linalg.norm(ref))
