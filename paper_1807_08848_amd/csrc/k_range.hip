// Range finder of the snapshots (stage a8): the QR at the end of
// RanLocalSolu and the randomized range finder of Section 2.3, in FP64.
//
// Per patch (one workgroup): G = Y^T Y; cyclic Jacobi eigendecomposition
// G = V diag(lambda) V^T (so sigma_j(Y) = sqrt(lambda_j), left singular
// vectors Y V_j / sigma_j); the k leading ones are formed and then
// re-orthonormalised by two Cholesky-QR passes (G' = Q^T Q = R^T R,
// Q <- Q R^{-1}, twice).  This handles rank-deficient sketches (more
// samples than boundary degrees of freedom) with the same code path.  Each
// column's largest-magnitude entry is made positive (first index on ties).
#include "device_common.h"

namespace msrs {

constexpr int kRfMax = 64;     // max columns
constexpr int kRfChunk = 32;   // rows staged per Gram step

// G (ld kRfMax, LDS) = A^T A for A column-major (lda rows), ncols <= 16 TS.
// Thread (ty, tx) accumulates the TS x TS block of entries (ty + 16 r, tx + 16 c).
template <int TS>
__device__ void gram_tile(const double* __restrict__ A, int nrows, int lda, int ncols, double* G, double* stage) {
    // chunk elements per thread: kRfChunk * ncols <= 32 * 64 = 8 * kThreads
    constexpr int EPT = kRfChunk * kRfMax / kThreads;
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    double acc[TS][TS];
#pragma unroll
    for (int r = 0; r < TS; ++r)
#pragma unroll
        for (int c = 0; c < TS; ++c) acc[r][c] = 0.0;
    const int n = kRfChunk * ncols;
    double pre[EPT];
    auto fetch = [&](int r0) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int o = tid + e * kThreads;
            const int col = o / kRfChunk, row = o - col * kRfChunk;
            pre[e] = (o < n && r0 + row < nrows) ? A[(int64_t)col * lda + r0 + row] : 0.0;
        }
    };
    fetch(0);
    for (int r0 = 0; r0 < nrows; r0 += kRfChunk) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int o = tid + e * kThreads;
            if (o < n) stage[(o % kRfChunk) * kRfMax + o / kRfChunk] = pre[e];
        }
        __syncthreads();
        if (r0 + kRfChunk < nrows) fetch(r0 + kRfChunk);   // next chunk in flight during this one
        const int nr = min(kRfChunk, nrows - r0);
        for (int row = 0; row < nr; ++row) {
            double a[TS], b[TS];
#pragma unroll
            for (int r = 0; r < TS; ++r) a[r] = stage[row * kRfMax + ty + 16 * r];
#pragma unroll
            for (int c = 0; c < TS; ++c) b[c] = stage[row * kRfMax + tx + 16 * c];
#pragma unroll
            for (int r = 0; r < TS; ++r)
#pragma unroll
                for (int c = 0; c < TS; ++c) acc[r][c] = fma(a[r], b[c], acc[r][c]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < TS; ++r)
#pragma unroll
        for (int c = 0; c < TS; ++c) {
            const int i = ty + 16 * r, j = tx + 16 * c;
            if (i < ncols && j < ncols) G[i * kRfMax + j] = acc[r][c];
        }
    __syncthreads();
}

__device__ void gram_lds(const double* __restrict__ A, int nrows, int lda, int ncols, double* G, double* stage) {
    if (ncols <= 16) gram_tile<1>(A, nrows, lda, ncols, G, stage);
    else if (ncols <= 32) gram_tile<2>(A, nrows, lda, ncols, G, stage);
    else if (ncols <= 48) gram_tile<3>(A, nrows, lda, ncols, G, stage);
    else gram_tile<4>(A, nrows, lda, ncols, G, stage);
}

// Cholesky of the n x n SPD matrix G (LDS, ld kRfMax) in place (lower).
// Returns false (uniformly) on a non-positive pivot.
__device__ bool chol_lds(double* G, int n, int* okflag) {
    const int tid = threadIdx.x;
    if (tid == 0) *okflag = 1;
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        if (tid == 0) {
            const double d = G[j * kRfMax + j];
            if (!(d > 0.0) || !isfinite(d)) *okflag = 0;
            G[j * kRfMax + j] = d > 0.0 ? sqrt(d) : 1.0;
        }
        __syncthreads();
        const double ljj = G[j * kRfMax + j];
        for (int i = j + 1 + tid; i < n; i += kThreads) G[i * kRfMax + j] /= ljj;
        __syncthreads();
        const int m = n - j - 1;
        for (int o = tid; o < m * m; o += kThreads) {
            const int a = j + 1 + o / m, b = j + 1 + o % m;
            if (b <= a) G[a * kRfMax + b] -= G[a * kRfMax + j] * G[b * kRfMax + j];
        }
        __syncthreads();
    }
    const bool ok = *okflag != 0;
    __syncthreads();
    return ok;
}

// T (ld kRfMax) = L^{-T} for the lower Cholesky factor L (n x n, LDS): thread
// j forms column j of L^{-1} by forward substitution; T[i][j] = L^{-1}[j][i].
__device__ void inv_transpose_lds(const double* L, int n, double* T) {
    const int j = threadIdx.x;
    if (j < n) {
        for (int i = 0; i < n; ++i) {
            double v = (i == j) ? 1.0 : 0.0;
            for (int c = j; c < i; ++c) v -= L[i * kRfMax + c] * T[j * kRfMax + c];
            T[j * kRfMax + i] = (i < j) ? 0.0 : v / L[i * kRfMax + i];
        }
    }
    __syncthreads();
}

// out (nrows x k, column-major) = A (nrows x m, column-major) * B (m x k, LDS ld kRfMax).
// A thread owns one row and a block of 8 columns, so each A element is read
// once per 8 outputs (coalesced across threads); B is broadcast from LDS.
__device__ void gemm_rows(const double* __restrict__ A, int nrows, int m, const double* B, int k, double* __restrict__ out) {
    constexpr int CB = 8;
    const int nblk = (k + CB - 1) / CB;
    for (int o = threadIdx.x; o < nrows * nblk; o += kThreads) {
        const int jb = o / nrows, r = o - jb * nrows;
        const int j0 = jb * CB;
        double acc[CB];
#pragma unroll
        for (int c = 0; c < CB; ++c) acc[c] = 0.0;
#pragma unroll 8
        for (int i = 0; i < m; ++i) {
            const double a = A[(int64_t)i * nrows + r];
#pragma unroll
            for (int c = 0; c < CB; ++c) acc[c] = fma(a, B[i * kRfMax + min(j0 + c, kRfMax - 1)], acc[c]);
        }
#pragma unroll
        for (int c = 0; c < CB; ++c)
            if (j0 + c < k) out[(int64_t)(j0 + c) * nrows + r] = acc[c];
    }
    __syncthreads();
}

__global__ __launch_bounds__(kThreads) void range_kernel(const PatchDesc* pd, int p0, const double* __restrict__ Y_all,
                                                         double* __restrict__ Q_all, double* __restrict__ ws_all,
                                                         double* __restrict__ sv_all, double* __restrict__ gap, int32_t* flags) {
    __shared__ double G[kRfMax * kRfMax];
    __shared__ double V[kRfMax * kRfMax];
    __shared__ double stage[kRfChunk * kRfMax];
    __shared__ double cs[kRfMax / 2], sn[kRfMax / 2];
    __shared__ int pu[kRfMax / 2], pv[kRfMax / 2];
    __shared__ int perm[kRfMax];
    __shared__ double lam[kRfMax];
    __shared__ int okflag;
    __shared__ double red_v[kThreads];
    __shared__ int red_i[kThreads];
    __shared__ double offn;

    const int p = p0 + blockIdx.x;
    const PatchDesc P = pd[p];
    const int tid = threadIdx.x;
    const int s = P.s, nrows = P.nrows;
    const int k = P.ncols;
    const double* Y = Y_all + P.Y_off;
    double* Q = Q_all + P.Q_off;
    double* W = ws_all + P.Q_off;   // workspace of the same shape as Q

    // 1. Gram matrix
    gram_lds(Y, nrows, nrows, s, G, stage);
    // 2. cyclic Jacobi with round-robin pairs, n even
    const int n = s + (s & 1);
    for (int o = tid; o < kRfMax * kRfMax; o += kThreads) {
        const int i = o / kRfMax, j = o % kRfMax;
        V[o] = (i == j) ? 1.0 : 0.0;
        if (i >= s || j >= s) G[o] = 0.0;
    }
    __syncthreads();
    double fro = 0.0;
    for (int o = 0; o < s; ++o) fro += G[o * kRfMax + o] * G[o * kRfMax + o];
    for (int sweep = 0; sweep < 30; ++sweep) {
        for (int st = 0; st < n - 1; ++st) {
            if (tid < n / 2) {
                const int i = tid;
                const int u = (i == 0) ? 0 : ((i - 1 + st) % (n - 1)) + 1;
                const int v = ((n - 2 - i + st) % (n - 1)) + 1;
                const int a = min(u, v), b = max(u, v);
                pu[i] = a;
                pv[i] = b;
                double c = 1.0, t = 0.0;
                const double apq = G[a * kRfMax + b];
                if (b < s && apq != 0.0) {
                    const double tau = (G[b * kRfMax + b] - G[a * kRfMax + a]) / (2.0 * apq);
                    t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                }
                cs[i] = c;
                sn[i] = t * c;
            }
            __syncthreads();
            // G <- J^T G J on 2x2 blocks (pairs i, i2): rows rotate by pair i,
            // columns by pair i2; V <- V J on (row j, pair i)
            const int np2 = n / 2;
            for (int o = tid; o < np2 * np2; o += kThreads) {
                const int i = o / np2, i2 = o % np2;
                const int a = pu[i], b = pv[i], a2 = pu[i2], b2 = pv[i2];
                const double c = cs[i], sv = sn[i], c2 = cs[i2], s2 = sn[i2];
                const double g00 = G[a * kRfMax + a2], g01 = G[a * kRfMax + b2];
                const double g10 = G[b * kRfMax + a2], g11 = G[b * kRfMax + b2];
                // rows
                const double r00 = c * g00 - sv * g10, r01 = c * g01 - sv * g11;
                const double r10 = sv * g00 + c * g10, r11 = sv * g01 + c * g11;
                // columns
                G[a * kRfMax + a2] = c2 * r00 - s2 * r01;
                G[a * kRfMax + b2] = s2 * r00 + c2 * r01;
                G[b * kRfMax + a2] = c2 * r10 - s2 * r11;
                G[b * kRfMax + b2] = s2 * r10 + c2 * r11;
            }
            for (int o = tid; o < np2 * n; o += kThreads) {
                const int i = o / n, j = o % n;
                const int a = pu[i], b = pv[i];
                const double c = cs[i], sv = sn[i];
                const double va = V[j * kRfMax + a], vb = V[j * kRfMax + b];
                V[j * kRfMax + a] = c * va - sv * vb;
                V[j * kRfMax + b] = sv * va + c * vb;
            }
            __syncthreads();
        }
        // off-diagonal norm
        double loc = 0.0;
        for (int o = tid; o < s * s; o += kThreads) {
            const int i = o / s, j = o % s;
            if (i != j) loc += G[i * kRfMax + j] * G[i * kRfMax + j];
        }
        red_v[tid] = loc;
        __syncthreads();
        for (int w = kThreads / 2; w > 0; w >>= 1) {
            if (tid < w) red_v[tid] += red_v[tid + w];
            __syncthreads();
        }
        if (tid == 0) offn = red_v[0];
        __syncthreads();
        if (offn <= 1e-32 * fro) break;
    }
    // 3. sort eigenvalues descending (stable selection on thread 0)
    if (tid == 0) {
        for (int i = 0; i < s; ++i) { perm[i] = i; lam[i] = G[i * kRfMax + i]; }
        for (int i = 0; i < s; ++i) {
            int best = i;
            for (int j = i + 1; j < s; ++j)
                if (lam[perm[j]] > lam[perm[best]]) best = j;
            const int t = perm[i]; perm[i] = perm[best]; perm[best] = t;
        }
        double* svp = sv_all + P.sv_off;
        for (int i = 0; i < s; ++i) svp[i] = sqrt(fmax(lam[perm[i]], 0.0));
        const double s1 = svp[0];
        const double sk = svp[k - 1];
        if (!(sk > 1e-13 * s1)) raise_flag(flags, 2);
        gap[p] = (k < s) ? (sk - svp[k]) / s1 : 1.0;
    }
    __syncthreads();
    // 4. B = V[:, perm[:k]] / sigma (s x k, in G, free after the sort); W = Y B
    for (int o = tid; o < s * k; o += kThreads) {
        const int i = o / k, j = o % k;
        const double sg = sqrt(fmax(lam[perm[j]], 0.0));
        G[i * kRfMax + j] = sg > 0 ? V[i * kRfMax + perm[j]] / sg : 0.0;
    }
    __syncthreads();
    gemm_rows(Y, nrows, s, G, k, W);
    // 5. two Cholesky-QR passes on the k columns: W -> Q -> W
    for (int pass = 0; pass < 2; ++pass) {
        const double* src = pass == 0 ? W : Q;
        double* dst = pass == 0 ? Q : W;
        gram_lds(src, nrows, nrows, k, G, stage);
        if (!chol_lds(G, k, &okflag)) {
            if (tid == 0) raise_flag(flags, 2);
            return;
        }
        inv_transpose_lds(G, k, V);
        gemm_rows(src, nrows, k, V, k, dst);
    }
    // 6. sign fix (largest |entry| of each column positive, lowest index on ties), W -> Q
    for (int j = 0; j < k; ++j) {
        double bv = -1.0;
        int bi = 0;
        for (int row = tid; row < nrows; row += kThreads) {
            const double a = fabs(W[(int64_t)j * nrows + row]);
            if (a > bv || (a == bv && row < bi)) { bv = a; bi = row; }
        }
        red_v[tid] = bv;
        red_i[tid] = bi;
        __syncthreads();
        for (int w = kThreads / 2; w > 0; w >>= 1) {
            if (tid < w) {
                const double ov = red_v[tid + w];
                const int oi = red_i[tid + w];
                if (ov > red_v[tid] || (ov == red_v[tid] && oi < red_i[tid])) { red_v[tid] = ov; red_i[tid] = oi; }
            }
            __syncthreads();
        }
        const int at = min(max(red_i[0], 0), nrows - 1);
        const double sg = W[(int64_t)j * nrows + at] < 0.0 ? -1.0 : 1.0;
        __syncthreads();
        for (int row = tid; row < nrows; row += kThreads) Q[(int64_t)j * nrows + row] = sg * W[(int64_t)j * nrows + row];
    }
}

void launch_range(Ctx& c, int p0, int p1) {
    StageTimer t(c, MSRS_K_RANGE);
    hipLaunchKernelGGL(range_kernel, dim3(p1 - p0), dim3(kThreads), 0, c.stream, c.dp, p0, c.Y, c.Q, c.rf_ws, c.sv, c.gap, c.dflags);
}

}  // namespace msrs
