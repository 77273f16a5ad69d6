// Online stage (beside the hot path): least-squares gluing of the local bases.
//
// Elliptic (eqs. elliptic_cond_tilde, elliptic_cond_reduced): rows of P~ are
// value continuity at every node of each interior coarse edge, conormal-flux
// continuity at the edge's inner nodes, a four-patch flux balance at each
// interior coarse vertex, and Dirichlet rows on dOmega.  The discrete
// conormal flux of a basis function q at a node of dK_m is
// (A^{K_m} q)(x) / h with A^{K_m} the stiffness of K_m's own elements.
// Kinetic (eqs. gb3, rte_cond_reduced): per interface, v>0 values of the last
// cell of K_m equal the left ghost of K_{m+1}, v<0 values of K_m's right
// ghost equal the first cell of K_{m+1}; inflow rows at x = 0 and x = 1.
//
// The normal equations P~^T P~ c = P~^T d are block banded (patch order);
// they are formed in lower band storage band[j*(bw+1) + d] = A[j+d][j] and
// factored once by a band Cholesky.  A request's coefficients are either two
// band triangular solves (banded path) or one product with the precomputed
// solution operator (batched path), then the reconstruction
// u = sum_m w_m Q_m c_m (nodal partition of unity w_m = 1/#patches at shared
// elliptic nodes).
#include <algorithm>
#include <cmath>
#include <vector>

#include "device_common.h"

namespace msrs {

// element matrix of the bilinear element (times 6), local order SW SE NE NW
__device__ __constant__ double kKref6[16] = {4, -1, -2, -1, -1, 4, -1, -2, -2, -1, 4, -1, -1, -2, -1, 4};

__host__ __device__ __forceinline__ void kbnode(int t, int nH, int& ii, int& jj) {
    if (t < nH) { ii = t; jj = 0; }
    else if (t < 2 * nH) { ii = nH; jj = t - nH; }
    else if (t < 3 * nH) { ii = 3 * nH - t; jj = nH; }
    else { ii = 0; jj = 4 * nH - t; }
}

__host__ __device__ __forceinline__ int kb_index(int ii, int jj, int nH) {
    if (jj == 0 && ii < nH) return ii;
    if (ii == nH && jj < nH) return nH + jj;
    if (jj == nH && ii > 0) return 2 * nH + (nH - ii);
    return 3 * nH + (nH - jj);
}

// global boundary index (counter-clockwise from (0,0)) of node (gx, gy) on dOmega
__host__ __device__ __forceinline__ int gb_index(int gx, int gy, int N) { return kb_index(gx, gy, N); }

// ------------------------------------------------------------ elliptic traces
// tr layout per patch: [values 4nH x ncols][fluxes 4nH x ncols], row-major (t, col).
__global__ __launch_bounds__(kThreads) void traces_elliptic_kernel(const PatchDesc* pd, const CoarseDesc* cd, const double* __restrict__ a,
                                                                   int N, const double* __restrict__ Q_all, double* __restrict__ tr,
                                                                   int64_t tr_stride) {
    const int p = blockIdx.x;
    const PatchDesc P = pd[p];
    const int nH = P.nH, W = nH + 1, nc = cd[p].ncols;
    const double* Q = Q_all + P.Q_off;
    double* T = tr + (int64_t)p * tr_stride;
    const double invh = (double)N;
    for (int o = threadIdx.x; o < 4 * nH * nc; o += kThreads) {
        const int t = o % (4 * nH), col = o / (4 * nH);
        int ii, jj;
        kbnode(t, nH, ii, jj);
        const double* q = Q + (int64_t)col * P.nrows;
        double flux = 0.0;
        // elements around the node: NE (node is SW corner), NW (SE), SW (NE), SE (NW)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int ei = (e == 0 || e == 3) ? ii : ii - 1;
            const int ej = (e == 0 || e == 1) ? jj : jj - 1;
            if (ei < 0 || ej < 0 || ei >= nH || ej >= nH) continue;
            const int alpha = (e == 0) ? 0 : (e == 1) ? 1 : (e == 2) ? 2 : 3;
            const double ae = a[(size_t)(P.ky0 + ej) * N + P.kx0 + ei];
            const double cq[4] = {q[ej * W + ei], q[ej * W + ei + 1], q[(ej + 1) * W + ei + 1], q[(ej + 1) * W + ei]};
            double s = 0.0;
#pragma unroll
            for (int bb = 0; bb < 4; ++bb) s += kKref6[alpha * 4 + bb] * cq[bb];
            flux += ae * s / 6.0;
        }
        T[t * nc + col] = q[jj * W + ii];
        T[4 * nH * nc + t * nc + col] = flux * invh;
    }
}

// ------------------------------------------------------------ normal matrix
__global__ void fill_kernel(double* a, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) a[i] = v;
}

struct ElTr {
    const double* T;
    int nH, nc;
    __device__ double val(int ii, int jj, int c) const { return T[kb_index(ii, jj, nH) * nc + c]; }
    __device__ double flx(int ii, int jj, int c) const { return T[4 * nH * nc + kb_index(ii, jj, nH) * nc + c]; }
};

__device__ __forceinline__ void band_add(double* band, int bw, int row, int col, double v) {
    // lower storage; caller guarantees row >= col
    band[(int64_t)col * (bw + 1) + (row - col)] += v;
}

// One workgroup per patch m: B_mm and the blocks with the neighbours n > m.
__global__ __launch_bounds__(kThreads) void normal_elliptic_kernel(const PatchDesc* pd, const CoarseDesc* cd, const double* __restrict__ tr,
                                                                   int64_t tr_stride, int M, int N, double* __restrict__ band, int bw) {
    const int m = blockIdx.x;
    const int m1 = m % M, m2 = m / M;
    const int nH = pd[m].nH;
    auto TR = [&](int p) { return ElTr{tr + (int64_t)p * tr_stride, nH, cd[p].ncols}; };
    const ElTr Tm = TR(m);
    const int km = cd[m].ncols, om = cd[m].col_off;
    // ---- B_mm
    for (int o = threadIdx.x; o < km * km; o += kThreads) {
        const int a = o / km, b = o % km;
        if (b < a) continue;      // lower storage: row (b) >= col (a)
        double s = 0.0;
        // edges: right, left, top, bottom
        if (m1 < M - 1) { for (int t = 0; t <= nH; ++t) s += Tm.val(nH, t, a) * Tm.val(nH, t, b);
                          for (int t = 1; t < nH; ++t) s += Tm.flx(nH, t, a) * Tm.flx(nH, t, b); }
        if (m1 > 0)     { for (int t = 0; t <= nH; ++t) s += Tm.val(0, t, a) * Tm.val(0, t, b);
                          for (int t = 1; t < nH; ++t) s += Tm.flx(0, t, a) * Tm.flx(0, t, b); }
        if (m2 < M - 1) { for (int t = 0; t <= nH; ++t) s += Tm.val(t, nH, a) * Tm.val(t, nH, b);
                          for (int t = 1; t < nH; ++t) s += Tm.flx(t, nH, a) * Tm.flx(t, nH, b); }
        if (m2 > 0)     { for (int t = 0; t <= nH; ++t) s += Tm.val(t, 0, a) * Tm.val(t, 0, b);
                          for (int t = 1; t < nH; ++t) s += Tm.flx(t, 0, a) * Tm.flx(t, 0, b); }
        // interior vertices at the four corners
        const int cx[4] = {0, nH, nH, 0}, cy[4] = {0, 0, nH, nH};
        const int vx[4] = {m1, m1 + 1, m1 + 1, m1}, vy[4] = {m2, m2, m2 + 1, m2 + 1};
        for (int cn = 0; cn < 4; ++cn)
            if (vx[cn] > 0 && vx[cn] < M && vy[cn] > 0 && vy[cn] < M) s += Tm.flx(cx[cn], cy[cn], a) * Tm.flx(cx[cn], cy[cn], b);
        // Dirichlet rows
        for (int t = 0; t < 4 * nH; ++t) {
            int ii, jj;
            kbnode(t, nH, ii, jj);
            const int gx = m1 * nH + ii, gy = m2 * nH + jj;
            if (gx == 0 || gx == N || gy == 0 || gy == N) s += Tm.val(ii, jj, a) * Tm.val(ii, jj, b);
        }
        band_add(band, bw, om + b, om + a, s);
    }
    // ---- off-diagonal blocks B_{m,n}, n > m
    const int nbrs[4] = {(m1 < M - 1) ? m + 1 : -1, (m1 > 0 && m2 < M - 1) ? m + M - 1 : -1,
                         (m2 < M - 1) ? m + M : -1, (m1 < M - 1 && m2 < M - 1) ? m + M + 1 : -1};
    for (int which = 0; which < 4; ++which) {
        const int n = nbrs[which];
        if (n < 0) continue;
        const ElTr Tn = TR(n);
        const int kn = cd[n].ncols, on = cd[n].col_off;
        for (int o = threadIdx.x; o < km * kn; o += kThreads) {
            const int a = o / kn, b = o % kn;
            double s = 0.0;
            if (which == 0) {   // right neighbour
                for (int t = 0; t <= nH; ++t) s -= Tm.val(nH, t, a) * Tn.val(0, t, b);
                for (int t = 1; t < nH; ++t) s += Tm.flx(nH, t, a) * Tn.flx(0, t, b);
                if (m2 > 0) s += Tm.flx(nH, 0, a) * Tn.flx(0, 0, b);          // bottom-right vertex
                if (m2 < M - 1) s += Tm.flx(nH, nH, a) * Tn.flx(0, nH, b);    // top-right vertex
            } else if (which == 1) {   // top-left diagonal neighbour: vertex at m's top-left
                s += Tm.flx(0, nH, a) * Tn.flx(nH, 0, b);
            } else if (which == 2) {   // top neighbour
                for (int t = 0; t <= nH; ++t) s -= Tm.val(t, nH, a) * Tn.val(t, 0, b);
                for (int t = 1; t < nH; ++t) s += Tm.flx(t, nH, a) * Tn.flx(t, 0, b);
                if (m1 > 0) s += Tm.flx(0, nH, a) * Tn.flx(0, 0, b);          // top-left vertex
                if (m1 < M - 1) s += Tm.flx(nH, nH, a) * Tn.flx(nH, 0, b);    // top-right vertex
            } else {                   // top-right diagonal neighbour
                s += Tm.flx(nH, nH, a) * Tn.flx(0, 0, b);
            }
            band_add(band, bw, on + b, om + a, s);
        }
    }
}

// kinetic rows read Q directly (restricted layout: cell c in [0, nH+2), ordinate j)
__global__ __launch_bounds__(kThreads) void normal_kinetic_kernel(const PatchDesc* pd, const CoarseDesc* cd, const double* __restrict__ Q_all,
                                                                  const double* __restrict__ vw, int M, int nv,
                                                                  double* __restrict__ band, int bw) {
    const int m = blockIdx.x;
    const PatchDesc P = pd[m];
    const int nH = P.nH, km = cd[m].ncols, om = cd[m].col_off;
    const double* Qm = Q_all + P.Q_off;
    const int nr = P.nrows;
    auto q = [&](const double* Qb, int nrw, int cell, int j, int col) { return Qb[(int64_t)col * nrw + cell * nv + j]; };
    for (int o = threadIdx.x; o < km * km; o += kThreads) {
        const int a = o / km, b = o % km;
        if (b < a) continue;
        double s = 0.0;
        for (int j = 0; j < nv; ++j) {
            const bool pos = vw[j] > 0;
            if (m == 0 && pos) s += q(Qm, nr, 0, j, a) * q(Qm, nr, 0, j, b);
            if (m == M - 1 && !pos) s += q(Qm, nr, nH + 1, j, a) * q(Qm, nr, nH + 1, j, b);
            if (m < M - 1) { const int cc = pos ? nH : nH + 1; s += q(Qm, nr, cc, j, a) * q(Qm, nr, cc, j, b); }
            if (m > 0) { const int cc = pos ? 0 : 1; s += q(Qm, nr, cc, j, a) * q(Qm, nr, cc, j, b); }
        }
        band_add(band, bw, om + b, om + a, s);
    }
    if (m < M - 1) {
        const PatchDesc Pn = pd[m + 1];
        const double* Qn = Q_all + Pn.Q_off;
        const int kn = cd[m + 1].ncols, on = cd[m + 1].col_off;
        for (int o = threadIdx.x; o < km * kn; o += kThreads) {
            const int a = o / kn, b = o % kn;
            double s = 0.0;
            for (int j = 0; j < nv; ++j) {
                const bool pos = vw[j] > 0;
                s -= pos ? q(Qm, nr, nH, j, a) * q(Qn, Pn.nrows, 0, j, b) : q(Qm, nr, nH + 1, j, a) * q(Qn, Pn.nrows, 1, j, b);
            }
            band_add(band, bw, on + b, om + a, s);
        }
    }
}

// ------------------------------------------------------------ band Cholesky
__global__ __launch_bounds__(1024) void band_cholesky_kernel(double* __restrict__ band, int n, int bw, int32_t* flags) {
    __shared__ double col[1024];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int ld = bw + 1;
    for (int j = 0; j < n; ++j) {
        double* Lj = band + (int64_t)j * ld;
        const int m = min(bw, n - 1 - j);
        const double d = Lj[0];
        if (!(d > 0.0) || !isfinite(d)) {
            if (tid == 0) raise_flag(flags, 0);
        }
        const double sd = d > 0.0 ? sqrt(d) : 1.0;
        __syncthreads();
        for (int i = tid; i <= m; i += nt) {
            const double v = (i == 0) ? sd : Lj[i] / sd;
            col[i] = v;
        }
        __syncthreads();
        for (int i = tid; i <= m; i += nt) Lj[i] = col[i];
        // trailing update A[j+b][j+a] -= L[j+b][j] L[j+a][j], 1 <= a <= b <= m
        const int64_t tot = (int64_t)m * m;
        for (int64_t o = tid; o < tot; o += nt) {
            const int a = (int)(o / m) + 1, b = (int)(o % m) + 1;
            if (b < a) continue;
            band[(int64_t)(j + a) * ld + (b - a)] -= col[b] * col[a];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ band solves
// L L^T X = B for the columns of B (column-major, n rows, ncols columns), in
// place; workgroup x solves columns [64 x, 64 x + 64).
__global__ __launch_bounds__(1024) void band_solve_kernel(const double* __restrict__ band, int n, int bw, double* __restrict__ xall,
                                                          int ncols) {
    __shared__ double piv[64];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int ld = bw + 1;
    const int c0 = blockIdx.x * 64;
    const int n_req = min(64, ncols - c0);
    double* x = xall + (int64_t)c0 * n;
    // forward: L y = b (column oriented)
    for (int j = 0; j < n; ++j) {
        const double* Lj = band + (int64_t)j * ld;
        const int m = min(bw, n - 1 - j);
        if (tid < n_req) {
            const double y = x[(int64_t)tid * n + j] / Lj[0];
            x[(int64_t)tid * n + j] = y;
            piv[tid] = y;
        }
        __syncthreads();
        for (int o = tid; o < m * n_req; o += nt) {
            const int d = o % m + 1, r = o / m;
            x[(int64_t)r * n + j + d] -= Lj[d] * piv[r];
        }
        __syncthreads();
    }
    // back: L^T c = y (column oriented on L^T)
    for (int j = n - 1; j >= 0; --j) {
        const double* Lj = band + (int64_t)j * ld;
        if (tid < n_req) {
            const double c = x[(int64_t)tid * n + j] / Lj[0];
            x[(int64_t)tid * n + j] = c;
            piv[tid] = c;
        }
        __syncthreads();
        const int m = min(bw, j);
        for (int o = tid; o < m * n_req; o += nt) {
            const int d = o % m + 1, r = o / m;
            const int i = j - d;
            x[(int64_t)r * n + i] -= band[(int64_t)i * ld + d] * piv[r];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ G_B set-up
// GB (Np x nB, column-major) = unit columns e_{bmap[i]}; the band solves then
// turn it into (P~^T P~)^{-1} restricted to the boundary-patch unknowns.
__global__ void unit_cols_kernel(double* __restrict__ GB, int Np, int nB, const int32_t* __restrict__ bmap) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nB) GB[(int64_t)i * Np + bmap[i]] = 1.0;
}

// ------------------------------------------------------------ per-request rhs (banded path)
// d~ = P~^T d for one request: only the Dirichlet rows of d are non-zero.
__global__ __launch_bounds__(kThreads) void rhs_elliptic_kernel(const PatchDesc* pd, const CoarseDesc* cd, const double* __restrict__ tr,
                                                                int64_t tr_stride, int M, int N, const double* __restrict__ f,
                                                                double* __restrict__ rhs) {
    const int m = blockIdx.x;
    const int m1 = m % M, m2 = m / M;
    const int nH = pd[m].nH;
    const ElTr Tm{tr + (int64_t)m * tr_stride, nH, cd[m].ncols};
    const int km = cd[m].ncols, om = cd[m].col_off;
    const bool edge = (m1 == 0 || m1 == M - 1 || m2 == 0 || m2 == M - 1);
    for (int a = threadIdx.x; a < km; a += kThreads) {
        double s = 0.0;
        if (edge)
            for (int t = 0; t < 4 * nH; ++t) {
                int ii, jj;
                kbnode(t, nH, ii, jj);
                const int gx = m1 * nH + ii, gy = m2 * nH + jj;
                if (gx == 0 || gx == N || gy == 0 || gy == N) s += Tm.val(ii, jj, a) * f[gb_index(gx, gy, N)];
            }
        rhs[om + a] = s;
    }
}

__global__ __launch_bounds__(kThreads) void rhs_kinetic_kernel(const PatchDesc* pd, const CoarseDesc* cd, const double* __restrict__ Q_all,
                                                               const double* __restrict__ vw, int M, int nv,
                                                               const double* __restrict__ f, double* __restrict__ rhs) {
    const int m = blockIdx.x;
    const PatchDesc P = pd[m];
    const int km = cd[m].ncols, om = cd[m].col_off, h = nv / 2;
    const double* Q = Q_all + P.Q_off;
    for (int a = threadIdx.x; a < km; a += kThreads) {
        double s = 0.0;
        for (int j = 0; j < nv; ++j) {
            if (m == 0 && vw[j] > 0) s += Q[(int64_t)a * P.nrows + 0 * nv + j] * f[j - h];
            if (m == M - 1 && vw[j] < 0) s += Q[(int64_t)a * P.nrows + (P.nH + 1) * nv + j] * f[h + j];
        }
        rhs[om + a] = s;
    }
}

// ------------------------------------------------------------ batched path
// g = P~_D^T d for the requests of one launch: only the unknowns of patches
// with Dirichlet rows are non-zero; g[r*nB + b_off(m) + a].  Grid (boundary
// patch, request).  The boundary data are read where the caller holds them
// (device memory, or the server's mapped pinned staging: each value crosses
// the bus once per patch that touches it).
__device__ __forceinline__ double wave_sum(double v) {
    // butterfly over the 64 lanes: a fixed order, so a sum does not depend on
    // which other requests share the launch
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Waves take every fourth basis column (KW at a time), lanes the boundary
// nodes of K_m; each lane reads its node's datum once for all its columns.
__global__ __launch_bounds__(kThreads) void bdry_rhs_elliptic_kernel(const PatchDesc* pd, const CoarseDesc* cd, const double* __restrict__ tr,
                                                                     int64_t tr_stride, const int32_t* __restrict__ bpatch, int M, int N,
                                                                     InPtrs in, int nB, double* __restrict__ g) {
    constexpr int KW = 4;
    const int m = bpatch[blockIdx.x], r = blockIdx.y;
    const int m1 = m % M, m2 = m / M;
    const int nH = pd[m].nH;
    const int km = cd[m].ncols, bo = cd[m].b_off, nc = cd[m].ncols;
    const double* T = tr + (int64_t)m * tr_stride;
    const double* fr = in.f[r];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int a0 = w * KW; a0 < km; a0 += 4 * KW) {
        double acc[KW] = {};
        for (int t = lane; t < 4 * nH; t += 64) {
            int ii, jj;
            kbnode(t, nH, ii, jj);
            const int gx = m1 * nH + ii, gy = m2 * nH + jj;
            if (!(gx == 0 || gx == N || gy == 0 || gy == N)) continue;
            const double fv = fr[gb_index(gx, gy, N)];
#pragma unroll
            for (int q = 0; q < KW; ++q)
                if (a0 + q < km) acc[q] = fma(T[t * nc + a0 + q], fv, acc[q]);
        }
#pragma unroll
        for (int q = 0; q < KW; ++q) {
            const double v = wave_sum(acc[q]);
            if (lane == 0 && a0 + q < km) g[(int64_t)r * nB + bo + a0 + q] = v;
        }
    }
}

__global__ __launch_bounds__(kThreads) void bdry_rhs_kinetic_kernel(const PatchDesc* pd, const CoarseDesc* cd, const double* __restrict__ Q_all,
                                                                    const double* __restrict__ vw, const int32_t* __restrict__ bpatch, int M,
                                                                    int nv, InPtrs in, int nB, double* __restrict__ g) {
    const int m = bpatch[blockIdx.x], r = blockIdx.y;
    const PatchDesc P = pd[m];
    const int km = cd[m].ncols, bo = cd[m].b_off, h = nv / 2;
    const double* Q = Q_all + P.Q_off;
    const double* fr = in.f[r];
    for (int a = threadIdx.x; a < km; a += kThreads) {
        double s = 0.0;
        for (int j = 0; j < nv; ++j) {
            if (m == 0 && vw[j] > 0) s += Q[(int64_t)a * P.nrows + 0 * nv + j] * fr[j - h];
            if (m == M - 1 && vw[j] < 0) s += Q[(int64_t)a * P.nrows + (P.nH + 1) * nv + j] * fr[h + j];
        }
        g[(int64_t)r * nB + bo + a] = s;
    }
}

// GT (Np x nB, row-major) = transpose of GB, through 64 x 64 LDS tiles.
__global__ __launch_bounds__(kThreads) void transpose_kernel(const double* __restrict__ A, int rows, int cols, double* __restrict__ B) {
    // A: rows x cols column-major (A[c*rows + r]); B: B[r*cols + c]
    __shared__ double t[64][65];
    const int r0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
    for (int o = threadIdx.x; o < 64 * 64; o += kThreads) {
        const int rr = o & 63, cc = o >> 6;
        if (r0 + rr < rows && c0 + cc < cols) t[cc][rr] = A[(int64_t)(c0 + cc) * rows + r0 + rr];
    }
    __syncthreads();
    for (int o = threadIdx.x; o < 64 * 64; o += kThreads) {
        const int cc = o & 63, rr = o >> 6;
        if (r0 + rr < rows && c0 + cc < cols) B[(int64_t)(r0 + rr) * cols + c0 + cc] = t[cc][rr];
    }
}

// c[r*Np + j] = sum_i GT[j*nB + i] g[r*nB + i] for the requests of one launch.
// A workgroup owns kGRows rows (two per wave) and RB requests.  Lanes stride
// the columns, so every row streams as independent 512-byte loads (16 in
// flight per wave); g is staged in LDS in column chunks; each row's lane
// sums meet in a fixed butterfly.
constexpr int kGRows = 8, kGChunk = 512;
template <int RB>
__global__ __launch_bounds__(kThreads) void apply_G_kernel(const double* __restrict__ GT, int Np, int nB,
                                                           const double* __restrict__ g, int n_req, double* __restrict__ c) {
    __shared__ double gs[RB][kGChunk];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r0 = blockIdx.y * RB;
    const int nr = min(RB, n_req - r0);
    const int j0 = blockIdx.x * kGRows + 2 * w;
    const int ja = min(j0, Np - 1), jb = min(j0 + 1, Np - 1);
    double acc0[RB] = {}, acc1[RB] = {};
    for (int i0 = 0; i0 < nB; i0 += kGChunk) {
        const int ni = min(kGChunk, nB - i0);
        __syncthreads();
        for (int o = threadIdx.x; o < RB * kGChunk; o += kThreads) {
            const int r = o / kGChunk, i = o % kGChunk;
            gs[r][i] = (r < nr && i < ni) ? g[(int64_t)(r0 + r) * nB + i0 + i] : 0.0;
        }
        __syncthreads();
        double ga[kGChunk / 64], gb[kGChunk / 64];
#pragma unroll
        for (int t = 0; t < kGChunk / 64; ++t) {
            const int i = t * 64 + lane;
            ga[t] = i < ni ? GT[(int64_t)ja * nB + i0 + i] : 0.0;
            gb[t] = i < ni ? GT[(int64_t)jb * nB + i0 + i] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < kGChunk / 64; ++t) {
            const int i = t * 64 + lane;
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const double gv = gs[r][i];
                acc0[r] = fma(ga[t], gv, acc0[r]);
                acc1[r] = fma(gb[t], gv, acc1[r]);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        const double s0 = wave_sum(acc0[r]), s1 = wave_sum(acc1[r]);
        if (lane == 0 && r < nr) {
            if (j0 < Np) c[(int64_t)(r0 + r) * Np + j0] = s0;
            if (j0 + 1 < Np) c[(int64_t)(r0 + r) * Np + j0 + 1] = s1;
        }
    }
}

// ------------------------------------------------------------ reconstruction
// u_r(x) = sum_m w_m(x) (Q_m c_{r,m})(x) for the requests of one launch; the
// output of request r is out.u[r] (requests need not be contiguous).
//
// Tiled form (nH >= 16): a workgroup owns a 16 x 16 tile of nodes, which
// touches at most 2 x 2 patches.  The loop over those patches is uniform
// across the workgroup, so a patch's coefficients c_{r,m} are wave-uniform
// (scalar loads) while each thread streams its node's basis rows once and
// accumulates every request of the launch in registers; nodes outside the
// patch add zeros.  Q is read once per launch and u written once.
constexpr int kTile = 16;
template <int NR>
__global__ __launch_bounds__(kThreads) void recon_tiled_kernel(const PatchDesc* pd, const CoarseDesc* cd, const double* __restrict__ Q_all,
                                                               int M, int N, int Np, const double* __restrict__ c, int n_req,
                                                               OutPtrs out) {
    // Requests go in passes of NR (the second pass re-reads the tile's basis
    // rows from cache); within a pass all NR are computed (rows of c past
    // n_req are workspace: their sums are discarded), so the request loop
    // has no branches and each request's coefficients arrive as wide scalar
    // loads.  Past km, q = 0 and the coefficient index is clamped inside the
    // patch, so a partial chunk adds exact zeros.
    constexpr int QC = 16;
    const int nH = N / M, W = nH + 1;
    const int X0 = blockIdx.x * kTile, Y0 = blockIdx.y * kTile;
    const int pxa = X0 > 0 ? (X0 - 1) / nH : 0, pya = Y0 > 0 ? (Y0 - 1) / nH : 0;
    const int gx = X0 + (threadIdx.x & (kTile - 1)), gy = Y0 + threadIdx.x / kTile;
    const bool valid = gx <= N && gy <= N;
    const int nx = ((gx % nH == 0 && gx > 0) ? 1 : 0) + (gx / nH < M ? 1 : 0);
    const int ny = ((gy % nH == 0 && gy > 0) ? 1 : 0) + (gy / nH < M ? 1 : 0);
    const double w = 1.0 / (nx * ny);
    const int64_t node = (int64_t)gy * (N + 1) + gx;
    for (int rb = 0; rb < n_req; rb += NR) {
        double acc[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r] = 0.0;
        for (int sl = 0; sl < 4; ++sl) {
            const int px = pxa + (sl & 1), py = pya + (sl >> 1);
            if (px >= M || py >= M) continue;
            if (X0 > (px + 1) * nH || X0 + kTile - 1 < px * nH || Y0 > (py + 1) * nH || Y0 + kTile - 1 < py * nH) continue;
            const int m = py * M + px;
            const PatchDesc& P = pd[m];
            const int km = cd[m].ncols, om = cd[m].col_off;
            const bool member = valid && gx >= px * nH && gx <= (px + 1) * nH && gy >= py * nH && gy <= (py + 1) * nH;
            const double* Q = Q_all + P.Q_off + (member ? (gy - py * nH) * W + (gx - px * nH) : 0);
            for (int c0 = 0; c0 < km; c0 += QC) {
                double q[QC];
#pragma unroll
                for (int t = 0; t < QC; ++t) q[t] = (member && c0 + t < km) ? Q[(int64_t)(c0 + t) * P.nrows] : 0.0;
                const int kc = min(QC, km - c0);
                if (kc == QC) {
#pragma unroll
                    for (int r = 0; r < NR; ++r) {
                        const double* cr = c + (int64_t)(rb + r) * Np + om + c0;
#pragma unroll
                        for (int t = 0; t < QC; ++t) acc[r] = fma(q[t], cr[t], acc[r]);
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < NR; ++r) {
                        const double* cr = c + (int64_t)(rb + r) * Np + om + c0;
#pragma unroll
                        for (int t = 0; t < QC; ++t) acc[r] = fma(q[t], cr[min(t, kc - 1)], acc[r]);
                    }
                }
            }
        }
        if (valid) {
#pragma unroll
            for (int r = 0; r < NR; ++r)
                if (rb + r < n_req) out.u[rb + r][node] = w * acc[r];
        }
    }
}

// Generic form (any nH): a thread per node, coefficients from global memory.
__global__ __launch_bounds__(kThreads) void recon_elliptic_kernel(const PatchDesc* pd, const CoarseDesc* cd, const double* __restrict__ Q_all,
                                                                  int M, int N, int Np, const double* __restrict__ c, int n_req,
                                                                  OutPtrs out) {
    constexpr int RB = 8;
    const int64_t nn = (int64_t)(N + 1) * (N + 1);
    const int nH = N / M, W = nH + 1;
    for (int64_t node = blockIdx.x * (int64_t)kThreads + threadIdx.x; node < nn; node += (int64_t)gridDim.x * kThreads) {
        const int gx = (int)(node % (N + 1)), gy = (int)(node / (N + 1));
        int xs[2], ys[2], nx = 0, ny = 0;
        if (gx % nH == 0 && gx > 0) xs[nx++] = gx / nH - 1;
        if (gx / nH < M) xs[nx++] = gx / nH;
        if (gy % nH == 0 && gy > 0) ys[ny++] = gy / nH - 1;
        if (gy / nH < M) ys[ny++] = gy / nH;
        const double w = 1.0 / (nx * ny);
        for (int r0 = 0; r0 < n_req; r0 += RB) {
            const int nr = min(RB, n_req - r0);
            double acc[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) acc[r] = 0.0;
            for (int a = 0; a < nx; ++a)
                for (int b = 0; b < ny; ++b) {
                    const int m = ys[b] * M + xs[a];
                    const PatchDesc& P = pd[m];
                    const int row = (gy - ys[b] * nH) * W + (gx - xs[a] * nH);
                    const int km = cd[m].ncols, om = cd[m].col_off;
                    const double* Q = Q_all + P.Q_off + row;
                    const double* cm = c + (int64_t)r0 * Np + om;
                    for (int cc = 0; cc < km; ++cc) {
                        const double q = Q[(int64_t)cc * P.nrows];
#pragma unroll
                        for (int r = 0; r < RB; ++r)
                            if (r < nr) acc[r] = fma(q, cm[(int64_t)r * Np + cc], acc[r]);
                    }
                }
#pragma unroll
            for (int r = 0; r < RB; ++r)
                if (r < nr) out.u[r0 + r][node] = w * acc[r];
        }
    }
}

__global__ __launch_bounds__(kThreads) void recon_kinetic_kernel(const PatchDesc* pd, const CoarseDesc* cd, const double* __restrict__ Q_all,
                                                                 int M, int Nx, int nv, int Np, const double* __restrict__ c, int n_req,
                                                                 OutPtrs out) {
    const int64_t nn = (int64_t)Nx * nv;
    const int nH = Nx / M;
    for (int64_t idx = blockIdx.x * (int64_t)kThreads + threadIdx.x; idx < nn; idx += (int64_t)gridDim.x * kThreads) {
        const int cell = (int)(idx / nv), j = (int)(idx % nv);
        const int m = cell / nH;
        const PatchDesc& P = pd[m];
        const int row = (cell - m * nH + 1) * nv + j;
        const int km = cd[m].ncols, om = cd[m].col_off;
        const double* Q = Q_all + P.Q_off + row;
        for (int r = 0; r < n_req; ++r) {
            double s = 0.0;
            for (int cc = 0; cc < km; ++cc) s += Q[(int64_t)cc * P.nrows] * c[(int64_t)r * Np + om + cc];
            out.u[r][idx] = s;
        }
    }
}

// ------------------------------------------------------------ host side
// Set-up: traces, normal matrix, band Cholesky, then G_B: the columns of
// (P~^T P~)^{-1} at the unknowns of patches with Dirichlet (inflow) rows
// (Np x nB, column-major).  The right-hand side d of the least-squares system
// vanishes outside those rows, so P~^T d lives on the same unknowns and every
// request's coefficients are c = G_B (P~_D^T f): a short sparse product and
// one dense pass instead of two sequential band solves per request.
void coarse_setup(Ctx& c) {
    StageTimer t(c, MSRS_K_COARSE);
    const int64_t nband = (int64_t)c.Np * (c.bw + 1);
    hipLaunchKernelGGL(fill_kernel, dim3(256), dim3(256), 0, c.stream, c.band, nband, 0.0);
    hipLaunchKernelGGL(fill_kernel, dim3(1024), dim3(256), 0, c.stream, c.GB, (int64_t)c.Np * c.nB, 0.0);
    hipLaunchKernelGGL(unit_cols_kernel, dim3((c.nB + 255) / 256), dim3(256), 0, c.stream, c.GB, c.Np, c.nB, c.bmap);
    if (c.kind == kElliptic) {
        hipLaunchKernelGGL(traces_elliptic_kernel, dim3(c.n_patches), dim3(kThreads), 0, c.stream, c.dp, c.dc, c.coef_copy, c.N, c.Q, c.tr, c.tr_stride);
        hipLaunchKernelGGL(normal_elliptic_kernel, dim3(c.n_patches), dim3(kThreads), 0, c.stream, c.dp, c.dc, c.tr, c.tr_stride, c.M, c.N, c.band, c.bw);
    } else {
        hipLaunchKernelGGL(normal_kinetic_kernel, dim3(c.n_patches), dim3(kThreads), 0, c.stream, c.dp, c.dc, c.Q, c.vw, c.M, c.nv, c.band, c.bw);
    }
    // the 1-norm of P~^T P~ (symmetric band, lower storage), before the factor overwrites it
    {
        std::vector<double> h((size_t)c.Np * (c.bw + 1));
        MSRS_HIP_CHECK(hipMemcpyAsync(h.data(), c.band, h.size() * sizeof(double), hipMemcpyDeviceToHost, c.stream));
        MSRS_HIP_CHECK(hipStreamSynchronize(c.stream));
        std::vector<double> colsum(c.Np, 0.0);
        const int ld = c.bw + 1;
        for (int j = 0; j < c.Np; ++j)
            for (int d = 0; d <= c.bw && j + d < c.Np; ++d) {
                const double v = std::fabs(h[(size_t)j * ld + d]);
                colsum[j] += v;
                if (d) colsum[j + d] += v;
            }
        c.norm1_normal = *std::max_element(colsum.begin(), colsum.end());
    }
    hipLaunchKernelGGL(band_cholesky_kernel, dim3(1), dim3(1024), 0, c.stream, c.band, c.Np, c.bw, c.dflags);
    hipLaunchKernelGGL(band_solve_kernel, dim3((c.nB + 63) / 64), dim3(1024), 0, c.stream, c.band, c.Np, c.bw, c.GB, c.nB);
    hipLaunchKernelGGL(transpose_kernel, dim3((c.Np + 63) / 64, (c.nB + 63) / 64), dim3(kThreads), 0, c.stream, c.GB, c.Np, c.nB, c.GT);
}

// Condition of the normal equations, the LAPACK way for a factored SPD band
// matrix: ||K||_1 (kept by coarse_setup) times an estimate of ||K^{-1}||_1 by
// Hager's method with Higham's refinements (the iteration that maximizes
// ||K^{-1} x||_1 over the unit 1-norm ball, restarted from the vertex of the
// largest gradient entry, at most five rounds, and the alternating-sign test
// vector), each solve two band triangular sweeps with the resident factor.
// The estimate is a lower bound of kappa_1(K), in practice within a small
// factor; kappa_2(P~)^2 = kappa_2(K) lies within a factor Np of it.
double coarse_condition(Ctx& c, double* work) {
    const int n = c.Np;
    std::vector<double> x(n), y(n), z(n);
    auto solve = [&](const std::vector<double>& b, std::vector<double>& out) {
        MSRS_HIP_CHECK(hipMemcpyAsync(work, b.data(), n * sizeof(double), hipMemcpyHostToDevice, c.stream));
        hipLaunchKernelGGL(band_solve_kernel, dim3(1), dim3(1024), 0, c.stream, c.band, n, c.bw, work, 1);
        MSRS_HIP_CHECK(hipMemcpyAsync(out.data(), work, n * sizeof(double), hipMemcpyDeviceToHost, c.stream));
        MSRS_HIP_CHECK(hipStreamSynchronize(c.stream));
    };
    auto norm1 = [](const std::vector<double>& v) {
        double s = 0.0;
        for (double a : v) s += std::fabs(a);
        return s;
    };
    std::fill(x.begin(), x.end(), 1.0 / n);
    double est = 0.0;
    int last = -1;
    for (int it = 0; it < 5; ++it) {
        solve(x, y);
        const double e = norm1(y);
        if (it > 0 && e <= est) break;
        est = e;
        for (int i = 0; i < n; ++i) x[i] = y[i] >= 0.0 ? 1.0 : -1.0;
        solve(x, z);                       // K symmetric: K^{-T} = K^{-1}
        int j = 0;
        double zx = 0.0;
        for (int i = 0; i < n; ++i) {
            if (std::fabs(z[i]) > std::fabs(z[j])) j = i;
            zx += z[i] * (it == 0 ? 1.0 / n : (i == last ? 1.0 : 0.0));
        }
        if (std::fabs(z[j]) <= zx || j == last) break;
        last = j;
        std::fill(x.begin(), x.end(), 0.0);
        x[j] = 1.0;
    }
    // alternating-sign vector: catches matrices the iteration underestimates
    for (int i = 0; i < n; ++i) x[i] = (i % 2 ? -1.0 : 1.0) * (1.0 + (n > 1 ? (double)i / (n - 1) : 0.0));
    solve(x, y);
    est = std::max(est, 2.0 * norm1(y) / (3.0 * n));
    return c.norm1_normal * est;
}

// ------------------------------------------------------------ constrained least squares (elliptic)
// Dirichlet rows held exactly, continuity rows minimized (the constrained
// alternative of Sec. 5.2, after eq. elliptic_cond_reduced).  With
// K = P~^T P~ (factored above), A the continuity rows and B the Dirichlet
// rows, the Lagrangian's stationarity A^T A c + B^T l = 0 plus
// B^T B c = B^T phi on both sides gives K c = B^T (phi - l); the constraint
// then fixes nu = phi - l by S nu = phi_B, S = B K^{-1} B^T (SPD when B has
// full row rank).  So c = G_B B_B^T S^{-1} E f =: G_C f, with B_B the
// Dirichlet rows on the boundary-patch unknowns and E the gather of the
// boundary data at the rows' nodes: one dense pass per request, as in the
// least-squares path.  The set-up products are small (at most 1024 rows) and
// run once per model.

// Dirichlet rows: (patch m, node t of dK_m in kbnode order, global boundary
// index of the node) for every boundary patch and node of it on dOmega.
std::vector<int32_t> constrained_rows(const Ctx& c) {
    std::vector<int32_t> rows;
    for (int m : c.bpatch) {
        const int m1 = m % c.M, m2 = m / c.M, nH = c.hp[m].nH;
        for (int t = 0; t < 4 * nH; ++t) {
            int ii, jj;
            kbnode(t, nH, ii, jj);
            const int gx = m1 * nH + ii, gy = m2 * nH + jj;
            if (gx == 0 || gx == c.N || gy == 0 || gy == c.N) {
                rows.push_back(m);
                rows.push_back(t);
                rows.push_back(gb_index(gx, gy, c.N));
            }
        }
    }
    return rows;
}

// BB (nC x nB, column-major, zeroed): row rho holds the values at its node of
// its patch's basis functions, in that patch's boundary columns.
__global__ __launch_bounds__(kThreads) void cons_bb_kernel(const CoarseDesc* __restrict__ cd, const double* __restrict__ tr,
                                                           int64_t tr_stride, const int32_t* __restrict__ rows, int nC,
                                                           double* __restrict__ BB) {
    const int rho = blockIdx.x;
    const int m = rows[3 * rho], t = rows[3 * rho + 1];
    const int km = cd[m].ncols, bo = cd[m].b_off;
    const double* T = tr + (int64_t)m * tr_stride;
    for (int a = threadIdx.x; a < km; a += kThreads) BB[(int64_t)(bo + a) * nC + rho] = T[(int64_t)t * km + a];
}

// H (nB x nB, column-major) = the rows bmap of G_B.
__global__ __launch_bounds__(kThreads) void gather_rows_kernel(const double* __restrict__ GB, int Np, const int32_t* __restrict__ bmap,
                                                               int nB, double* __restrict__ H) {
    const int64_t n = (int64_t)nB * nB;
    for (int64_t o = blockIdx.x * (int64_t)kThreads + threadIdx.x; o < n; o += (int64_t)gridDim.x * kThreads) {
        const int i = (int)(o % nB), j = (int)(o / nB);
        H[o] = GB[(int64_t)j * Np + bmap[i]];
    }
}

// C (m x n, column-major) = op(A) op(B), op(X) = X (ta / tb = 0) or X^T;
// A and B column-major with leading dimensions lda, ldb.  One thread per
// output: set-up sized products only.
__global__ __launch_bounds__(kThreads) void gemm_small_kernel(int m, int n, int k, const double* __restrict__ A, int lda, int ta,
                                                              const double* __restrict__ B, int ldb, int tb, double* __restrict__ C) {
    const int64_t tot = (int64_t)m * n;
    for (int64_t o = blockIdx.x * (int64_t)kThreads + threadIdx.x; o < tot; o += (int64_t)gridDim.x * kThreads) {
        const int i = (int)(o % m), j = (int)(o / m);
        double s = 0.0;
        for (int p = 0; p < k; ++p) {
            const double a = ta ? A[(int64_t)i * lda + p] : A[(int64_t)p * lda + i];
            const double b = tb ? B[(int64_t)p * ldb + j] : B[(int64_t)j * ldb + p];
            s = fma(a, b, s);
        }
        C[o] = s;
    }
}

// Lower band of the dense symmetric S (n x n, column-major) with bw = n - 1:
// band[j n + d] = S[j + d, j].
__global__ __launch_bounds__(kThreads) void dense_to_band_kernel(const double* __restrict__ S, int n, double* __restrict__ band) {
    const int64_t tot = (int64_t)n * n;
    for (int64_t o = blockIdx.x * (int64_t)kThreads + threadIdx.x; o < tot; o += (int64_t)gridDim.x * kThreads) {
        const int j = (int)(o / n), d = (int)(o % n);
        band[o] = j + d < n ? S[(int64_t)j * n + j + d] : 0.0;
    }
}

// E (nC x nF, column-major, zeroed): E[rho, g(rho)] = 1.
__global__ __launch_bounds__(kThreads) void cons_gather_kernel(const int32_t* __restrict__ rows, int nC, double* __restrict__ E) {
    const int rho = blockIdx.x * kThreads + threadIdx.x;
    if (rho < nC) E[(int64_t)rows[3 * rho + 2] * nC + rho] = 1.0;
}

// Copies each request's boundary data into g (r * nF + i).
__global__ __launch_bounds__(kThreads) void copy_bdry_kernel(InPtrs in, int nF, double* __restrict__ g) {
    const int r = blockIdx.y;
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < nF; i += gridDim.x * kThreads) g[(int64_t)r * nF + i] = in.f[r][i];
}

static dim3 grid_of(int64_t n) { return dim3((unsigned)std::min<int64_t>((n + kThreads - 1) / kThreads, 4096)); }

void coarse_constrained_setup(Ctx& c, const ConsWs& w) {
    StageTimer t(c, MSRS_K_COARSE);
    const int nC = c.nC, nB = c.nB, nF = c.nF, Np = c.Np;
    hipStream_t st = c.stream;
    auto gemm = [&](int m, int n, int k, const double* A, int lda, int ta, const double* B, int ldb, int tb, double* C) {
        hipLaunchKernelGGL(gemm_small_kernel, grid_of((int64_t)m * n), dim3(kThreads), 0, st, m, n, k, A, lda, ta, B, ldb, tb, C);
    };
    hipLaunchKernelGGL(fill_kernel, grid_of((int64_t)nC * nB), dim3(kThreads), 0, st, w.BB, (int64_t)nC * nB, 0.0);
    hipLaunchKernelGGL(cons_bb_kernel, dim3(nC), dim3(kThreads), 0, st, c.dc, c.tr, c.tr_stride, w.rows, nC, w.BB);
    hipLaunchKernelGGL(gather_rows_kernel, grid_of((int64_t)nB * nB), dim3(kThreads), 0, st, c.GB, Np, c.bmap, nB, w.H);
    gemm(nC, nB, nB, w.BB, nC, 0, w.H, nB, 0, w.X);             // X = B_B H
    gemm(nC, nC, nB, w.X, nC, 0, w.BB, nC, 1, w.S);             // S = X B_B^T
    hipLaunchKernelGGL(dense_to_band_kernel, grid_of((int64_t)nC * nC), dim3(kThreads), 0, st, w.S, nC, w.band);
    hipLaunchKernelGGL(band_cholesky_kernel, dim3(1), dim3(1024), 0, st, w.band, nC, nC - 1, c.dflags);
    hipLaunchKernelGGL(fill_kernel, grid_of((int64_t)nC * nF), dim3(kThreads), 0, st, w.W, (int64_t)nC * nF, 0.0);
    hipLaunchKernelGGL(cons_gather_kernel, dim3((nC + kThreads - 1) / kThreads), dim3(kThreads), 0, st, w.rows, nC, w.W);
    hipLaunchKernelGGL(band_solve_kernel, dim3((nF + 63) / 64), dim3(1024), 0, st, w.band, nC, nC - 1, w.W, nF);   // W = S^-1 E
    gemm(nB, nF, nC, w.BB, nC, 1, w.W, nC, 0, w.V);             // V = B_B^T W
    gemm(Np, nF, nB, c.GB, Np, 0, w.V, nB, 0, c.GC);            // G_C = G_B V
    hipLaunchKernelGGL(transpose_kernel, dim3((Np + 63) / 64, (nF + 63) / 64), dim3(kThreads), 0, st, c.GC, Np, nF, c.GCT);
}

// ------------------------------------------------------------ corrected semi-normal equations
// The normal equations lose about log10 kappa(P~)^2 digits of c.  Where that
// is too many, every solve takes one step of the corrected semi-normal
// equations (Bjorck, 1987): the residual r = d - P~ c with P~ itself (rebuilt
// row by row from the traces, never stored), then P~^T P~ dc = P~^T r with the
// resident Cholesky factor, and c += dc.  The step takes the forward error
// from about kappa(P~)^2 u to about kappa(P~) u, the accuracy of a QR solve.
//
// z = P~^T (d - P~ c) on the unknowns of patch m, per request (grid: patch x
// request).  The workgroup forms the residual of every row that touches m
// (a row shared with a neighbour is formed by both patches), stages them in
// LDS, and each thread sums its column's share.  LDS, for W = nH + 1:
//   [e W + t]            value row of edge e (0 right, 1 left, 2 top, 3 bottom) at node t
//   [4 W + e W + t]      flux row of edge e at inner node t (1 <= t < nH)
//   [8 W + v]            vertex row at corner v (0 SW, 1 SE, 2 NE, 3 NW)
//   [8 W + 4 + t]        Dirichlet row at node t of dK_m (kbnode order)
// Rows that do not exist (no neighbour, a vertex on dOmega, a node off
// dOmega) hold 0.
__device__ __forceinline__ double trace_dot(const ElTr& T, bool flux, int ii, int jj, const double* __restrict__ cm, int k) {
    double s = 0.0;
    for (int b = 0; b < k; ++b) s += (flux ? T.flx(ii, jj, b) : T.val(ii, jj, b)) * cm[b];
    return s;
}

// node (ii, jj) of patch m at position t of edge e, the neighbour across e
// (-1 on dOmega) and the neighbour's node facing it
__device__ __forceinline__ int edge_nodes(int e, int t, int nH, int m, int m1, int m2, int M, int& ii, int& jj, int& ni, int& nj) {
    switch (e) {
        case 0: ii = nH; jj = t; ni = 0; nj = t; return m1 < M - 1 ? m + 1 : -1;
        case 1: ii = 0; jj = t; ni = nH; nj = t; return m1 > 0 ? m - 1 : -1;
        case 2: ii = t; jj = nH; ni = t; nj = 0; return m2 < M - 1 ? m + M : -1;
        default: ii = t; jj = 0; ni = t; nj = nH; return m2 > 0 ? m - M : -1;
    }
}

__global__ __launch_bounds__(kThreads) void lsq_correct_elliptic_kernel(const PatchDesc* pd, const CoarseDesc* cd,
                                                                        const double* __restrict__ tr, int64_t tr_stride, int M,
                                                                        int N, int Np, InPtrs in, const double* __restrict__ cbuf,
                                                                        double* __restrict__ zbuf) {
    extern __shared__ double rs[];
    const int m = blockIdx.x, r = blockIdx.y;
    const int m1 = m % M, m2 = m / M;
    const int nH = pd[m].nH, W = nH + 1;
    const double* c = cbuf + (int64_t)r * Np;
    const double* f = in.f[r];
    auto TR = [&](int p) { return ElTr{tr + (int64_t)p * tr_stride, nH, cd[p].ncols}; };
    const ElTr Tm = TR(m);
    const int km = cd[m].ncols;
    const double* cm = c + cd[m].col_off;
    const int nrow = 8 * W + 4 + 4 * nH;
    for (int i = threadIdx.x; i < nrow; i += kThreads) {
        double res = 0.0;
        if (i < 8 * W) {
            const bool flux = i >= 4 * W;
            const int e = (i - (flux ? 4 * W : 0)) / W, t = i % W;
            int ii, jj, ni, nj;
            const int n = edge_nodes(e, t, nH, m, m1, m2, M, ii, jj, ni, nj);
            if (n >= 0 && (!flux || (t > 0 && t < nH))) {
                const double sm = trace_dot(Tm, flux, ii, jj, cm, km);
                const double sn = trace_dot(TR(n), flux, ni, nj, c + cd[n].col_off, cd[n].ncols);
                // d = 0; a value row is (left or bottom patch) - (right or top
                // patch), a flux row the sum of both
                res = flux ? -(sm + sn) : ((e == 0 || e == 2) ? sn - sm : sm - sn);
            }
        } else if (i < 8 * W + 4) {
            const int v = i - 8 * W;
            const int vx = m1 + (v == 1 || v == 2), vy = m2 + (v >= 2);
            if (vx > 0 && vx < M && vy > 0 && vy < M) {
                // the patches (vx - 1 + dx, vy - 1 + dy) around the vertex, each at its corner facing it
                double s = 0.0;
                for (int q = 0; q < 4; ++q) {
                    const int dx = q & 1, dy = q >> 1;
                    const int p = (vy - 1 + dy) * M + (vx - 1 + dx);
                    s += trace_dot(TR(p), true, dx ? 0 : nH, dy ? 0 : nH, c + cd[p].col_off, cd[p].ncols);
                }
                res = -s;
            }
        } else {
            const int t = i - 8 * W - 4;
            int ii, jj;
            kbnode(t, nH, ii, jj);
            const int gx = m1 * nH + ii, gy = m2 * nH + jj;
            if (gx == 0 || gx == N || gy == 0 || gy == N) res = f[gb_index(gx, gy, N)] - trace_dot(Tm, false, ii, jj, cm, km);
        }
        rs[i] = res;
    }
    __syncthreads();
    for (int a = threadIdx.x; a < km; a += kThreads) {
        double z = 0.0;
        for (int e = 0; e < 4; ++e) {
            int ii, jj, ni, nj;
            if (edge_nodes(e, 0, nH, m, m1, m2, M, ii, jj, ni, nj) < 0) continue;
            const double sg = (e == 0 || e == 2) ? 1.0 : -1.0;   // c_m's sign in the edge's value rows
            for (int t = 0; t <= nH; ++t) {
                edge_nodes(e, t, nH, m, m1, m2, M, ii, jj, ni, nj);
                z += sg * Tm.val(ii, jj, a) * rs[e * W + t];
                if (t > 0 && t < nH) z += Tm.flx(ii, jj, a) * rs[4 * W + e * W + t];
            }
        }
        for (int v = 0; v < 4; ++v) {
            const int cx = (v == 1 || v == 2) ? nH : 0, cy = v >= 2 ? nH : 0;
            z += Tm.flx(cx, cy, a) * rs[8 * W + v];
        }
        for (int t = 0; t < 4 * nH; ++t) {
            int ii, jj;
            kbnode(t, nH, ii, jj);
            z += Tm.val(ii, jj, a) * rs[8 * W + 4 + t];
        }
        zbuf[(int64_t)r * Np + cd[m].col_off + a] = z;
    }
}

// Kinetic rows (grid: patch x request).  LDS: [j] the rows of the interface
// with patch m - 1, [nv + j] those with m + 1, [2 nv + j] the inflow rows of
// an end patch, ordinate j.
__global__ __launch_bounds__(kThreads) void lsq_correct_kinetic_kernel(const PatchDesc* pd, const CoarseDesc* cd,
                                                                       const double* __restrict__ Q_all, const double* __restrict__ vw,
                                                                       int M, int nv, int Np, InPtrs in, const double* __restrict__ cbuf,
                                                                       double* __restrict__ zbuf) {
    extern __shared__ double rs[];
    const int m = blockIdx.x, r = blockIdx.y, h = nv / 2;
    const double* c = cbuf + (int64_t)r * Np;
    const double* f = in.f[r];
    // row of basis values at (cell, ordinate j) of patch p times c_p
    auto qdot = [&](int p, int cell, int j) {
        const PatchDesc& P = pd[p];
        const double* Q = Q_all + P.Q_off;
        const double* cp = c + cd[p].col_off;
        double s = 0.0;
        for (int b = 0; b < cd[p].ncols; ++b) s += Q[(int64_t)b * P.nrows + cell * nv + j] * cp[b];
        return s;
    };
    for (int i = threadIdx.x; i < 3 * nv; i += kThreads) {
        const int side = i / nv, j = i % nv;
        const bool pos = vw[j] > 0;
        double res = 0.0;
        // an interface row is (upwind patch's outgoing value) - (downwind patch's ghost value); d = 0
        if (side == 0 && m > 0)
            res = qdot(m, pos ? 0 : 1, j) - qdot(m - 1, pos ? pd[m - 1].nH : pd[m - 1].nH + 1, j);
        else if (side == 1 && m < M - 1)
            res = qdot(m + 1, pos ? 0 : 1, j) - qdot(m, pos ? pd[m].nH : pd[m].nH + 1, j);
        else if (side == 2 && m == 0 && pos)
            res = f[j - h] - qdot(m, 0, j);
        else if (side == 2 && m == M - 1 && !pos)
            res = f[h + j] - qdot(m, pd[m].nH + 1, j);
        rs[i] = res;
    }
    __syncthreads();
    const PatchDesc P = pd[m];
    const double* Q = Q_all + P.Q_off;
    for (int a = threadIdx.x; a < cd[m].ncols; a += kThreads) {
        const double* qa = Q + (int64_t)a * P.nrows;
        double z = 0.0;
        for (int j = 0; j < nv; ++j) {
            const bool pos = vw[j] > 0;
            if (m > 0) z -= qa[(pos ? 0 : 1) * nv + j] * rs[j];
            if (m < M - 1) z += qa[(pos ? P.nH : P.nH + 1) * nv + j] * rs[nv + j];
            if ((m == 0 && pos) || (m == M - 1 && !pos)) z += qa[(pos ? 0 : P.nH + 1) * nv + j] * rs[2 * nv + j];
        }
        zbuf[(int64_t)r * Np + cd[m].col_off + a] = z;
    }
}

__global__ void add_kernel(double* __restrict__ x, const double* __restrict__ y, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) x[i] += y[i];
}

size_t lsq_correct_lds(const Ctx& c) {
    if (c.kind != kElliptic) return sizeof(double) * 3 * (size_t)c.nv;
    const int nH = c.N / c.M;
    return sizeof(double) * (size_t)(12 * nH + 12);
}

static void lsq_correct(const Ctx& c, int nr, const InPtrs& in, double* cbuf, double* zbuf, hipStream_t st) {
    const dim3 g(c.n_patches, nr);
    const size_t lds = lsq_correct_lds(c);
    if (c.kind == kElliptic)
        hipLaunchKernelGGL(lsq_correct_elliptic_kernel, g, dim3(kThreads), lds, st, c.dp, c.dc, c.tr, c.tr_stride, c.M, c.N, c.Np, in,
                           cbuf, zbuf);
    else
        hipLaunchKernelGGL(lsq_correct_kinetic_kernel, g, dim3(kThreads), lds, st, c.dp, c.dc, c.Q, c.vw, c.M, c.nv, c.Np, in, cbuf,
                           zbuf);
    hipLaunchKernelGGL(band_solve_kernel, dim3((nr + 63) / 64), dim3(1024), 0, st, c.band, c.Np, c.bw, zbuf, nr);
    hipLaunchKernelGGL(add_kernel, grid_of((int64_t)c.Np * nr), dim3(kThreads), 0, st, cbuf, zbuf, (int64_t)c.Np * nr);
}

static void launch_recon(const Ctx& c, const double* cbuf, int n_req, const OutPtrs& out, hipStream_t st) {
    if (c.kind == kElliptic && c.N / c.M >= kTile) {
        const dim3 g((c.N + kTile) / kTile, (c.N + kTile) / kTile);
#define MSRS_RECON(NR) hipLaunchKernelGGL(recon_tiled_kernel<NR>, g, dim3(kThreads), 0, st, c.dp, c.dc, c.Q, c.M, c.N, c.Np, cbuf, n_req, out)
        const int nr = std::min(n_req, c.recon_batch);
        if (nr <= 1) MSRS_RECON(1);
        else if (nr <= 2) MSRS_RECON(2);
        else if (nr <= 4) MSRS_RECON(4);
        else if (nr <= 8) MSRS_RECON(8);
        else MSRS_RECON(16);
#undef MSRS_RECON
    } else if (c.kind == kElliptic) {
        const int64_t nn = (int64_t)(c.N + 1) * (c.N + 1);
        const int blocks = (int)std::min<int64_t>((nn + kThreads - 1) / kThreads, 8192);
        hipLaunchKernelGGL(recon_elliptic_kernel, dim3(blocks), dim3(kThreads), 0, st, c.dp, c.dc, c.Q, c.M, c.N, c.Np, cbuf, n_req, out);
    } else {
        const int64_t nn = (int64_t)c.N * c.nv;
        const int blocks = (int)std::min<int64_t>((nn + kThreads - 1) / kThreads, 8192);
        hipLaunchKernelGGL(recon_kinetic_kernel, dim3(blocks), dim3(kThreads), 0, st, c.dp, c.dc, c.Q, c.M, c.N, c.nv, c.Np, cbuf, n_req, out);
    }
}

void coarse_apply(const Ctx& c, int n_req, const double* const* f, double* const* u, double* gbuf, double* cbuf,
                  double* zbuf, hipStream_t st) {
    for (int r0 = 0; r0 < n_req; r0 += kOutPerLaunch) {
        const int nr = std::min(kOutPerLaunch, n_req - r0);
        InPtrs in{};
        OutPtrs out{};
        for (int r = 0; r < nr; ++r) {
            in.f[r] = f[r0 + r];
            out.u[r] = u[r0 + r];
        }
        const dim3 gb((unsigned)c.bpatch.size(), nr);
        const int ng = c.g_len();
        const double* GT = c.constrained ? c.GCT : c.GT;
        if (c.constrained)
            hipLaunchKernelGGL(copy_bdry_kernel, dim3((ng + kThreads - 1) / kThreads, nr), dim3(kThreads), 0, st, in, ng, gbuf);
        else if (c.kind == kElliptic)
            hipLaunchKernelGGL(bdry_rhs_elliptic_kernel, gb, dim3(kThreads), 0, st, c.dp, c.dc, c.tr, c.tr_stride, c.dbpatch, c.M, c.N, in,
                               c.nB, gbuf);
        else
            hipLaunchKernelGGL(bdry_rhs_kinetic_kernel, gb, dim3(kThreads), 0, st, c.dp, c.dc, c.Q, c.vw, c.dbpatch, c.M, c.nv, in, c.nB, gbuf);
        const int rb = c.apply_batch;
        const dim3 ga((c.Np + kGRows - 1) / kGRows, (nr + rb - 1) / rb);
        if (rb == 4) hipLaunchKernelGGL(apply_G_kernel<4>, ga, dim3(kThreads), 0, st, GT, c.Np, ng, gbuf, nr, cbuf);
        else if (rb == 16) hipLaunchKernelGGL(apply_G_kernel<16>, ga, dim3(kThreads), 0, st, GT, c.Np, ng, gbuf, nr, cbuf);
        else hipLaunchKernelGGL(apply_G_kernel<8>, ga, dim3(kThreads), 0, st, GT, c.Np, ng, gbuf, nr, cbuf);
        if (c.lsq_correct) lsq_correct(c, nr, in, cbuf, zbuf, st);
        launch_recon(c, cbuf, nr, out, st);
    }
}

void coarse_banded(const Ctx& c, const double* f, double* u, double* cbuf, double* zbuf, hipStream_t st) {
    if (c.kind == kElliptic)
        hipLaunchKernelGGL(rhs_elliptic_kernel, dim3(c.n_patches), dim3(kThreads), 0, st, c.dp, c.dc, c.tr, c.tr_stride, c.M, c.N, f, cbuf);
    else
        hipLaunchKernelGGL(rhs_kinetic_kernel, dim3(c.n_patches), dim3(kThreads), 0, st, c.dp, c.dc, c.Q, c.vw, c.M, c.nv, f, cbuf);
    hipLaunchKernelGGL(band_solve_kernel, dim3(1), dim3(1024), 0, st, c.band, c.Np, c.bw, cbuf, 1);
    if (c.lsq_correct) {
        InPtrs in{};
        in.f[0] = f;
        lsq_correct(c, 1, in, cbuf, zbuf, st);
    }
    OutPtrs out{};
    out.u[0] = u;
    launch_recon(c, cbuf, 1, out, st);
}

}  // namespace msrs
