// Range finder of the snapshots (stage a8): the QR at the end of
// RanLocalSolu and the randomized range finder of Section 2.3, in FP64.
//
// Per patch: G = Y^T Y; eigendecomposition G = V diag(lambda) V^T (Householder
// tridiagonalisation and implicit QL), so sigma_j(Y) = sqrt(lambda_j) and Y V_j / sigma_j are the left
// singular vectors; the k leading ones are formed and re-orthonormalised by
// up to two Cholesky-QR passes (G' = W^T W = L L^T, Q = W L^{-T}; the second
// only where the first one's G' was not already within 1e-4 of I).  This
// handles rank-deficient sketches (more samples than boundary degrees of
// freedom) with the same code path.  Each column's largest-magnitude entry is
// made positive (first index on ties).
//
// The eigenvalues of the rounded Y^T Y carry absolute errors of about
// s u sigma_1^2, so this resolves sigma_j only down to about sqrt(s u) sigma_1.
// A patch whose sigma_{k+1} (sigma_k when k = s) lies below kResolve sigma_1
// takes a second pass on the rotated snapshots Z = Y V: Z^T Z is graded and
// nearly diagonal (its entries carry errors of u |z_i| |z_j|, relative to its
// own scale), so a Jacobi sweep with a purely relative stopping test resolves
// its eigenvalues to high relative accuracy, and Z V2 / sigma are the left
// singular vectors with column errors of order u, down to sigma_j ~ u sigma_1.
//
// Tall work (Gram matrices, products with the small s x k / k x k factors,
// the column argmax) runs over (patch, chunk of kRowChunk rows) workgroups with
// per-chunk partials reduced per patch in a fixed order, on FP64 MFMA; the
// small dense work (eigensolvers, Cholesky) runs one workgroup per patch.
#include "device_common.h"

namespace msrs {

constexpr int kRfMax = 64;          // max columns
constexpr int kRfStage = 32;        // rows staged in LDS per Gram step
constexpr int kRowChunk = 512;      // rows per workgroup of the tall kernels
constexpr int kSmall = kRfMax * kRfMax;
constexpr double kResolve = 1e-4;   // below this sigma_{k+1} / sigma_1 a patch takes the second pass

// columns and base of the tall matrix a kernel works on
struct Tall {
    const double* base;
    int ncols;
};
// kZ: the rotated snapshots Z = Y V1 (shape of Y); kYZ: Z for the patches
// that took the second pass, Y for the others
enum Which { kY = 0, kQ = 1, kW = 2, kZ = 3, kYZ = 4 };

__device__ __forceinline__ Tall tall_of(const PatchDesc& P, int which, const double* Y, const double* Q, const double* W,
                                        const double* Z = nullptr, bool second = false) {
    if (which == kY || (which == kYZ && !second)) return Tall{Y + P.Y_off, P.s};
    if (which == kZ || which == kYZ) return Tall{Z + P.Y_off, P.s};
    return Tall{(which == kQ ? Q : W) + P.Q_off, P.ncols};
}

// ---------------------------------------------------------------- Gram partials
// FP64 MFMA (16x16x4): the chunk's rows pass through LDS in blocks of
// kRfStage rows (coalesced along the column-major tall matrix), and the
// upper-triangle 16x16 tiles of A^T A (ti <= tj) go round-robin over the
// waves; each tile's k-steps read A^T[ti][4 rows] and A[4 rows][tj] from the
// staged block, lanes along the columns.  A tile's transpose is written with
// it, so out holds the full symmetric matrix.
constexpr int kStageLd = kRfMax + 1;   // odd leading dimension of the staged block

template <int NT>
__device__ void gram_rows_mfma(const double* __restrict__ A, int nrows, int r0, int r1, int ncols, double* stage, double* out) {
    typedef Mfma<double>::acc Acc;
    constexpr int NTILE = NT * (NT + 1) / 2;
    constexpr int NWAVE = kThreads / 64;
    constexpr int PER = (NTILE + NWAVE - 1) / NWAVE;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
    int tiA[PER], tiB[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        int t = q * NWAVE + w, a = 0;
        if (t >= NTILE) { tiA[q] = -1; tiB[q] = -1; continue; }
        while (t >= NT - a) { t -= NT - a; ++a; }
        tiA[q] = a;
        tiB[q] = a + t;
    }
    Acc acc[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) acc[q] = Mfma<double>::zero();
    for (int q0 = r0; q0 < r1; q0 += kRfStage) {
        const int nr = min(kRfStage, r1 - q0);
        __syncthreads();
        for (int o = tid; o < kRfStage * 16 * NT; o += kThreads) {
            const int col = o / kRfStage, row = o - col * kRfStage;
            stage[row * kStageLd + col] = (row < nr && col < ncols) ? A[(int64_t)col * nrows + q0 + row] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < kRfStage / 4; ++kk) {
            const double* srow = stage + (4 * kk + lk) * kStageLd + li;
#pragma unroll
            for (int q = 0; q < PER; ++q)
                if (tiA[q] >= 0) acc[q] = Mfma<double>::step(srow[16 * tiA[q]], srow[16 * tiB[q]], acc[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        if (tiA[q] < 0) continue;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int i = 16 * tiA[q] + Mfma<double>::row(lane, t), j = 16 * tiB[q] + li;
            if (i < ncols && j < ncols) {
                out[i * kRfMax + j] = acc[q][t];
                if (tiA[q] != tiB[q]) out[j * kRfMax + i] = acc[q][t];   // a diagonal tile holds both halves
            }
        }
    }
}

// grid (patch, row chunk): partial Gram of the chunk's rows -> part[(p * maxrc + chunk) * 4096]
// (skip: patches whose flag is set have nothing to do)
// (only: patches whose entry is zero have nothing to do)
__global__ __launch_bounds__(kThreads) void gram_partial_kernel(const PatchDesc* pd, int p0, int which, const double* __restrict__ Y,
                                                                const double* __restrict__ Q, const double* __restrict__ W,
                                                                double* __restrict__ part, int maxrc, const int32_t* __restrict__ skip,
                                                                const double* __restrict__ Z = nullptr,
                                                                const int32_t* __restrict__ only = nullptr) {
    __shared__ double stage[kRfStage * kStageLd];
    const int p = p0 + blockIdx.x;
    if ((skip && skip[p]) || (only && !only[p])) return;
    const PatchDesc P = pd[p];
    const int r0 = blockIdx.y * kRowChunk;
    if (r0 >= P.nrows) return;
    const int r1 = min(P.nrows, r0 + kRowChunk);
    const Tall T = tall_of(P, which, Y, Q, W, Z, only && only[p]);
    double* out = part + ((int64_t)p * maxrc + blockIdx.y) * kSmall;
    if (T.ncols <= 16) gram_rows_mfma<1>(T.base, P.nrows, r0, r1, T.ncols, stage, out);
    else if (T.ncols <= 32) gram_rows_mfma<2>(T.base, P.nrows, r0, r1, T.ncols, stage, out);
    else if (T.ncols <= 48) gram_rows_mfma<3>(T.base, P.nrows, r0, r1, T.ncols, stage, out);
    else gram_rows_mfma<4>(T.base, P.nrows, r0, r1, T.ncols, stage, out);
}

// sum of the chunk partials of patch p into G (LDS, leading dimension ld), fixed order
__device__ void sum_partials(const double* __restrict__ part, int p, int maxrc, int nch, int n, double* G, int ld = kRfMax) {
    for (int o = threadIdx.x; o < n * n; o += blockDim.x) {
        const int i = o / n, j = o % n;
        double s = 0.0;
        for (int ch = 0; ch < nch; ++ch) s += part[((int64_t)p * maxrc + ch) * kSmall + i * kRfMax + j];
        G[i * ld + j] = s;
    }
    __syncthreads();
}

// ---------------------------------------------------------------- eigendecomposition
// Pair i of round st in the round-robin ordering of n = nm1 + 1 indices: index 0
// stays, the others rotate one place per round, and pair i joins the i-th
// positions from both ends; after nm1 rounds every pair has met once.
__device__ __forceinline__ void rr_pair(int i, int st, int nm1, int& a, int& b) {
    int u = 0;
    if (i > 0) { u = i - 1 + st; if (u >= nm1) u -= nm1; u += 1; }
    int v = nm1 - 1 - i + st; if (v >= nm1) v -= nm1; v += 1;
    a = min(u, v);
    b = max(u, v);
}

// Which patches take the tridiagonal eigensolver (eig_ql_kernel; Jacobi, eig_kernel, the others): sampled ones
// with at least kQlMinCols samples.
// Full-basis patches have Gram matrices that are not graded, on which Jacobi
// needs few sweeps while the QL chases run their full length (the kinetic
// test workload's full-basis end patches: 1.05 ms in QL, 0.30 in Jacobi).
// On sampled patches QL wins from 32 samples on (h=1/512, 32 samples: 0.31
// against 0.34 ms; h=1/1024, 64 samples: 1.00 against 1.90 ms); the small
// sampled patches below 32 samples keep Jacobi (not timed against QL there).
constexpr int kQlMinCols = 32;
__device__ __forceinline__ bool ql_patch(const PatchDesc& P) { return P.sampled && P.s >= kQlMinCols; }

// The tail of both eigensolvers, from the eigenvalues on G's diagonal and the
// eigenvectors in V's columns (leading dimension ldg): descending order,
// singular values, rank, the second-pass decision, relative gap, and B -> small
// (pass 0: V[:, :k] / sigma; pass 2: V[:, :k]) or V -> small2 (all s columns,
// for Z = Y V).  Every thread of the workgroup calls it.
__device__ void eig_finish(PatchDesc* pd, int p, const PatchDesc& P, const double* G, const double* V, int LDG, int* perm,
                           double* lam, int* kshared_p, int* second_sp, double* __restrict__ small, double* __restrict__ sv_all,
                           double* __restrict__ gap, int32_t* flags, double rank_tol, int pass, double* __restrict__ small2,
                           int32_t* __restrict__ second) {
    const int tid = threadIdx.x, nth = blockDim.x;
    const int s = P.s, kreq = P.kreq;
    int& kshared = *kshared_p;
    int& second_s = *second_sp;
    // descending order by rank: eigenvalue i goes to the number of eigenvalues
    // above it, ties by index (a NaN ranks as -inf, so the ranks stay a
    // permutation)
    if (tid < s) {
        const double gi = G[tid * LDG + tid];
        const double li = (gi == gi) ? gi : -INFINITY;
        int r = 0;
        for (int j = 0; j < s; ++j) {
            const double gj = G[j * LDG + j];
            const double lj = (gj == gj) ? gj : -INFINITY;
            r += (lj > li) || (lj == li && j < tid);
        }
        perm[r] = tid;
        lam[tid] = gi;
    }
    __syncthreads();
    if (tid == 0) {
        double* svp = sv_all + P.sv_off;
        for (int i = 0; i < s; ++i) svp[i] = sqrt(fmax(lam[perm[i]], 0.0));
        const double s1 = svp[0];
        // rank: the requested one, or the numerical rank at rank_tol (the count of
        // singular values above rank_tol sigma_1), between 1 and the requested one;
        // the later kernels of the range finder read it from the descriptor
        int kk = kreq;
        if (rank_tol > 0.0 && P.sampled) {
            kk = 0;
            while (kk < kreq && svp[kk] > rank_tol * s1) ++kk;
            kk = max(kk, 1);
        }
        if (kk != P.ncols) pd[p].ncols = kk;
        kshared = kk;
        const double sk = svp[kk - 1];
        const double next = svp[min(kk, s - 1)];
        const bool again = pass == 0 && P.sampled && isfinite(s1) && s1 > 0.0 &&
                           (!(next >= kResolve * s1) || (rank_tol > 0.0 && rank_tol < kResolve));
        second_s = again ? 1 : 0;
        if (pass == 0) second[p] = again ? 1 : 0;
        // the k-th direction must be resolved: a rank deficiency of the
        // snapshots themselves (sigma_k at rounding level) after the second pass
        if (!again && !(sk > 1e-13 * s1)) raise_flag(flags, 2);
        if (!isfinite(s1)) raise_flag(flags, 4);
        gap[p] = (kk < s) ? (sk - svp[kk]) / s1 : 1.0;
    }
    __syncthreads();
    const int k = kshared;
    if (second_s) {
        // V in descending order for Z = Y V (all s columns)
        double* V1 = small2 + (int64_t)p * kSmall;
        for (int o = tid; o < kSmall; o += nth) {
            const int i = o / kRfMax, j = o % kRfMax;
            V1[o] = (i < s && j < s) ? V[i * LDG + perm[j]] : 0.0;
        }
        return;
    }
    // pass 2 (two-pass range finder, G = (G^T Q)^T (G^T Q)): the eigenvectors
    // themselves, the basis being Q V[:, :k]
    double* B = small + (int64_t)p * kSmall;
    for (int o = tid; o < kSmall; o += nth) {
        const int i = o / kRfMax, j = o % kRfMax;
        double v = 0.0;
        if (i < s && j < k) {
            const double sg = pass == 2 ? 1.0 : sqrt(fmax(lam[perm[j]], 0.0));
            v = sg > 0 ? V[i * LDG + perm[j]] / sg : 0.0;
        }
        B[o] = v;
    }
}

// The second pass's eigensolver (Z^T Z is graded: Jacobi keeps its small
// eigenvalues to high relative accuracy).  One workgroup per patch: G = sum of
// partials, cyclic Jacobi (round-robin pairs, two-sided updates on 2x2
// blocks), then the shared tail (eig_finish).
// A round has two phases.  First the threads of pair ip (ip < n/2, one wave)
// form that pair's rotation from its 2x2 diagonal block and publish it.  Then
// thread (i, i2) (pairs i, i2 < n/2, i2 padded to a power of two P2 <= 32)
// applies the rotations of pairs i (rows) and i2 (columns) to the 2x2 block
// (pair i, pair i2) of G and pair i's rotation to rows i2 and i2 + n/2 of V in
// the columns of pair i.  Every entry of G and V belongs to exactly one
// thread's block in a round, so both are updated in place.
constexpr int kEigMaxThreads = (kRfMax / 2) * 32;

int eig_threads(int max_s) {
    const int np2 = (max_s + (max_s & 1)) / 2;
    int p2 = 1;
    while (p2 < np2) p2 *= 2;
    return std::max(64, (np2 * p2 + 63) / 64 * 64);
}

// pass 0: Y^T Y.  Patches whose sigma_{k+1} (sigma_k when k = s) falls below
// kResolve sigma_1, or whose rank is chosen at a tolerance below it, are
// marked in second[p] and leave V (all s columns, in descending order) in
// small2[p] for Z = Y V; the others finish here.  pass 1 (marked patches
// only): Z^T Z, with the relative stopping test alone; its singular values,
// gap, rank and B replace pass 0's.
__global__ __launch_bounds__(kEigMaxThreads) void eig_kernel(PatchDesc* pd, int p0, const double* __restrict__ part, int maxrc,
                                                             double* __restrict__ small, double* __restrict__ sv_all,
                                                             double* __restrict__ gap, int32_t* flags, double rank_tol, int pass,
                                                             double* __restrict__ small2, int32_t* __restrict__ second,
                                                             int only_rest) {
    // G and V with an odd leading dimension: a wave's column accesses
    // (V[j][a] over rows j) fall on distinct LDS banks
    constexpr int LDG = kRfMax + 1;
    __shared__ double G[kRfMax * LDG];
    __shared__ double V[kRfMax * LDG];
    __shared__ double rc[kRfMax / 2], rs[kRfMax / 2], rt[kRfMax / 2];   // rotation of each pair this round
    __shared__ int perm[kRfMax];
    __shared__ double lam[kRfMax];
    __shared__ int rot;
    const int p = p0 + blockIdx.x;
    if (pass == 1 && !second[p]) return;
    const PatchDesc P = pd[p];
    if (only_rest && ql_patch(P)) return;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int s = P.s;
    __shared__ int kshared, second_s;
    const int nch = (P.nrows + kRowChunk - 1) / kRowChunk;
    for (int o = tid; o < kRfMax * LDG; o += nth) {
        G[o] = 0.0;
        V[o] = (o / LDG == o % LDG) ? 1.0 : 0.0;
    }
    __syncthreads();
    sum_partials(part, p, maxrc, nch, s, G, LDG);
    const int n = s + (s & 1), np2 = n / 2, nm1 = n - 1;
    int sh = 0;
    while ((1 << sh) < np2) ++sh;
    const int i = tid >> sh, i2 = tid & ((1 << sh) - 1);
    const bool act = i < np2 && i2 < np2;
    // Sweeps until every rotation of a sweep finds |g_pq| <= 1e-13 sqrt(g_pp g_qq)
    // (relative off-diagonal criterion; the rotation it leaves is below 1e-13
    // over the relative gap, and the convergence is quadratic by then) or
    // |g_pq| <= 1e-16 trace(G) (the level of
    // the rounding in forming G = Y^T Y, below which the relative test cannot be
    // met between widely separated eigenvalues), at most 30.  The trace is
    // invariant under the rotations.
    // (pass 1: Z^T Z is graded; the relative test alone)
    double gtr = 0.0;
    for (int x = 0; x < s; ++x) gtr += G[x * LDG + x];
    const double floor_abs = pass != 1 ? 1e-16 * gtr : 0.0;
    if (tid == 0) rot = 0;
    __syncthreads();
    for (int sweep = 0; sweep < 30; ++sweep) {
        for (int st = 0; st < nm1; ++st) {
            // phase 1: the rotation of pair tid (tid < n/2)
            if (tid < np2) {
                int a, b;
                rr_pair(tid, st, nm1, a, b);
                const double apq = G[a * LDG + b], app = G[a * LDG + a], aqq = G[b * LDG + b];
                double c = 1.0, sn = 0.0, t = 0.0;
                bool big = false;
                if (b < s && apq != 0.0) {
                    // |g_pq| > 1e-13 sqrt|g_pp g_qq| compared in squares
                    big = apq * apq > 1e-26 * fabs(app * aqq) && fabs(apq) > floor_abs;
                    // the smaller root of t^2 + 2 tau t - 1 = 0, tau = d / (2 g_pq),
                    // d = g_qq - g_pp, with numerator and denominator scaled by 2|g_pq|
                    const double d = aqq - app;
                    t = (d < 0 ? -2.0 * apq : 2.0 * apq) / (fabs(d) + sqrt(d * d + 4.0 * apq * apq));
                    c = rsqrt(1.0 + t * t);
                    sn = t * c;
                }
                rc[tid] = c;
                rs[tid] = sn;
                rt[tid] = t;
                if (big) rot = 1;
            }
            __syncthreads();
            // phase 2: the 2x2 block (pair i, pair i2) of G and pair i's columns of V
            if (act) {
                int a, b, a2, b2;
                rr_pair(i, st, nm1, a, b);
                rr_pair(i2, st, nm1, a2, b2);
                const double c = rc[i], sv = rs[i], t = rt[i], c2 = rc[i2], s2 = rs[i2];
                const double g00 = G[a * LDG + a2], g01 = G[a * LDG + b2];
                const double g10 = G[b * LDG + a2], g11 = G[b * LDG + b2];
                const double va0 = V[i2 * LDG + a], vb0 = V[i2 * LDG + b];
                const double va1 = V[(i2 + np2) * LDG + a], vb1 = V[(i2 + np2) * LDG + b];
                if (i == i2) {
                    // the rotated pair's own block: diagonal by the tangent update,
                    // the annihilated entry exactly zero (no rounding residue left
                    // to stall the relative test on widely separated eigenvalues)
                    G[a * LDG + a] = g00 - t * g01;
                    G[b * LDG + b] = g11 + t * g01;
                    G[a * LDG + b] = 0.0;
                    G[b * LDG + a] = 0.0;
                } else {
                    const double r00 = c * g00 - sv * g10, r01 = c * g01 - sv * g11;
                    const double r10 = sv * g00 + c * g10, r11 = sv * g01 + c * g11;
                    G[a * LDG + a2] = c2 * r00 - s2 * r01;
                    G[a * LDG + b2] = s2 * r00 + c2 * r01;
                    G[b * LDG + a2] = c2 * r10 - s2 * r11;
                    G[b * LDG + b2] = s2 * r10 + c2 * r11;
                }
                V[i2 * LDG + a] = c * va0 - sv * vb0;
                V[i2 * LDG + b] = sv * va0 + c * vb0;
                V[(i2 + np2) * LDG + a] = c * va1 - sv * vb1;
                V[(i2 + np2) * LDG + b] = sv * va1 + c * vb1;
            }
            __syncthreads();
        }
        // uniform decision: every thread reads the flag before it is reset
        const int r = rot;
        __syncthreads();
        if (tid == 0) rot = 0;
        __syncthreads();
        if (!r) break;
    }
    eig_finish(pd, p, P, G, V, LDG, perm, lam, &kshared, &second_s, small, sv_all, gap, flags, rank_tol, pass, small2,
               second);
}

// ---------------------------------------------------------------- tridiagonal eigensolver
// One wave per patch (the range finder's first pass and the two-pass basis):
// Householder reduction G = Q T Q^T, then the implicit QL iteration with
// shifts on T (the tql2 procedure of Bowdler, Martin, Reinsch and Wilkinson,
// restated), its rotations accumulated into Q, which ends as the eigenvectors.
// Fixed cost (no sweep count): the Householder steps are wave-parallel over a
// row each, the QL recurrence runs on wave-uniform values (the diagonal and
// off-diagonal of T held one entry per lane, read with readlane) while every
// lane rotates its row of the eigenvector matrix.  Its eigenvalues carry
// absolute errors of a small multiple of u ||G||, as the Gram matrix's own.
__device__ __forceinline__ double lane_value(double x, int i) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), i);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), i);
    return __hiloint2double(hi, lo);
}

// 1/sqrt(x) for finite x > 0: the hardware estimate y, then one step of the
// series (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + ... with e = 1 - x y^2, which
// multiplies the estimate's number of correct bits by three (no special-value
// handling, which rsqrt() adds for 0, infinities and NaN)
__device__ __forceinline__ double rsqrt_pos(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// LDS visibility between the lanes of the one wave (in-order LDS, and no
// compiler reordering across it)
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

__global__ __launch_bounds__(64) void eig_ql_kernel(PatchDesc* pd, int p0, const double* __restrict__ part, int maxrc,
                                                    double* __restrict__ small, double* __restrict__ sv_all,
                                                    double* __restrict__ gap, int32_t* flags, double rank_tol, int pass,
                                                    double* __restrict__ small2, int32_t* __restrict__ second) {
    constexpr int LDG = kRfMax + 1;
    __shared__ double G[kRfMax * LDG];   // the matrix, reduced in place; T's diagonals at the end
    __shared__ double V[kRfMax * LDG];   // Q, then the eigenvectors (columns)
    __shared__ double hv[kRfMax], hq[kRfMax];
    // a QL chase's rotations and the entries of T it rewrites (lane 0's
    // values; the other lanes store theirs past the end, see the chase)
    __shared__ double rot_c[kRfMax + 64], rot_s[kRfMax + 64];
    __shared__ double new_e[kRfMax + 65], new_d[kRfMax + 65];
    __shared__ int perm[kRfMax];
    __shared__ double lam[kRfMax];
    __shared__ int kshared, second_s;
    const int p = p0 + blockIdx.x;
    const PatchDesc P = pd[p];
    if (!ql_patch(P)) return;
    const int lane = threadIdx.x;
    const int n = P.s;
    const int nch = (P.nrows + kRowChunk - 1) / kRowChunk;
    for (int o = lane; o < kRfMax * LDG; o += 64) {
        G[o] = 0.0;
        V[o] = (o / LDG == o % LDG) ? 1.0 : 0.0;
    }
    __syncthreads();
    sum_partials(part, p, maxrc, nch, n, G, LDG);
    // Householder step k: x = G[k+1.., k] -> (alpha, 0, .., 0) by H = I - tau v v^T
    // on indices k+1 .. n-1: A <- H A H = A - v q^T - q v^T with p = tau A v,
    // q = p - (tau / 2) (v^T p) v; Q <- Q H.  Lane j holds entry j of the
    // vectors and works on row k+1+j of A (row j of Q).
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1, o = k + 1;
        const double x = lane < m ? G[(o + lane) * LDG + k] : 0.0;
        const double x0 = lane_value(x, 0);
        const double tail = wave_sum64(lane >= 1 ? x * x : 0.0);
        if (!(tail > 0.0)) continue;   // already reduced (or not finite: left to the checks downstream)
        const double alpha = x0 > 0.0 ? -sqrt(x0 * x0 + tail) : sqrt(x0 * x0 + tail);
        const double v0 = x0 - alpha;
        const double v = lane == 0 ? v0 : x;
        const double tau = 2.0 / (v0 * v0 + tail);
        hv[lane] = v;
        wave_lds_sync();
        double pj = 0.0;
        if (lane < m) {
            const double* row = G + (o + lane) * LDG + o;
            for (int i = 0; i < m; ++i) pj += row[i] * hv[i];
            pj *= tau;
        }
        const double K = 0.5 * tau * wave_sum64(lane < m ? v * pj : 0.0);
        const double q = pj - K * v;
        hq[lane] = q;
        wave_lds_sync();
        if (lane < m) {
            double* row = G + (o + lane) * LDG + o;
            for (int i = 0; i < m; ++i) row[i] -= v * hq[i] + q * hv[i];
            const double xr = lane == 0 ? alpha : 0.0;
            G[(o + lane) * LDG + k] = xr;
            G[k * LDG + o + lane] = xr;
        }
        if (lane < n) {
            double* row = V + lane * LDG + o;
            double t = 0.0;
            for (int i = 0; i < m; ++i) t += row[i] * hv[i];
            t *= tau;
            for (int i = 0; i < m; ++i) row[i] -= t * hv[i];
        }
        wave_lds_sync();
    }
    // T in reversed order, so that QL (which deflates from the top) meets the
    // small end of the graded T first (the reduction leaves the large entries
    // at the top; reversed, the chases on these Gram matrices take 1.1-3x fewer
    // rotations): diagonal d_j = T[n-1-j][n-1-j] on lane j, off-diagonal
    // e_j = T[n-1-j][n-2-j] (e_{n-1} = 0), and the columns of Q reversed with it
    const int jr = n - 1 - lane;
    double d = lane < n ? G[jr * LDG + jr] : 0.0;
    double e = lane + 1 < n ? G[jr * LDG + jr - 1] : 0.0;
    if (lane < n) {
        double* row = V + lane * LDG;
        for (int j = 0; j < n / 2; ++j) {
            const double a = row[j], b = row[n - 1 - j];
            row[j] = b;
            row[n - 1 - j] = a;
        }
    }
    wave_lds_sync();
    // implicit QL: for each l, chase the shifted rotation from the first
    // negligible off-diagonal below l up to l until e_l is negligible, here
    // against the norm of T (|e_j| <= u max_i (|d_i| + |e_i|)): absolute
    // accuracy, which is what the Gram matrix's own rounding leaves
    constexpr double kEps = 2.220446049250313e-16;
    double tn = fabs(d) + fabs(e);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) tn = fmax(tn, __shfl_xor(tn, o, 64));
    const double tol = kEps * tn;
    bool stalled = false;
    for (int l = 0; l < n; ++l) {
        for (int iter = 0;; ++iter) {
            // first mm >= l with a negligible e_mm, else n - 1
            const bool neg = lane >= l && lane < n - 1 && fabs(e) <= tol;
            const uint64_t bal = __ballot(neg);
            const int mm = bal ? (int)__builtin_ctzll(bal) : n - 1;
            if (mm == l) break;
            if (iter == 60) { stalled = true; break; }
            const double dl = lane_value(d, l), el = lane_value(e, l);
            double g = (lane_value(d, l + 1) - dl) / (2.0 * el);
            double r = hypot(g, 1.0);
            g = lane_value(d, mm) - dl + el / (g + (g >= 0.0 ? r : -r));
            double sn = 1.0, c = 1.0, pp = 0.0;
            bool zero = false;
            int lo = l;   // the last rotation applied (a split stops the chase early)
            // rotation i reads d_i, d_{i+1} and e_i; rotation j writes only d_{j+1}
            // and e_{j+1}, after its own reads, so no rotation before i (j > i)
            // has written them: read them from copies taken at the chase's start,
            // so that the reads do not wait on the writes of the rotations before
            const double dch = d, ech = e;
            // The chase as straight-line code: no test inside (a rotation with
            // f = g = 0, the split case, is detected afterwards and the chase
            // redone below with the test), the rewritten d_{i+1}, e_{i+1} and
            // the rotation go to LDS (every lane holds the same values; lane 0's
            // copies are the ones read), and d_{i+1} of rotation i is d_i of
            // rotation i + 1.
            bool redo;
            {
                bool hit = false;
                double sf = 1.0, cf = 1.0, pf = 0.0, gf = g, di1 = lane_value(dch, mm);
                for (int i = mm - 1; i >= l; --i) {
                    const double ei = lane_value(ech, i), di = lane_value(dch, i);
                    const double f = sf * ei, bb = cf * ei;
                    const double r2 = f * f + gf * gf;
                    hit |= r2 == 0.0;
                    const double rinv = rsqrt_pos(r2);   // r2 = 0 gives non-finite values, and the redo
                    sf = f * rinv;
                    cf = gf * rinv;
                    const double gi = di1 - pf;
                    const double rr = (di - gi) * sf + 2.0 * cf * bb;
                    pf = sf * rr;
                    gf = cf * rr - bb;
                    // every lane stores (the same values; lanes 1..63 to slots
                    // past the end): no exec-mask branch in the loop
                    const int slot = lane == 0 ? i : kRfMax + lane;
                    rot_c[slot] = cf;
                    rot_s[slot] = sf;
                    new_e[slot + 1] = r2 * rinv;
                    new_d[slot + 1] = gi + pf;
                    di1 = di;
                }
                if (!hit) {
                    wave_lds_sync();
                    if (lane > l && lane <= mm) {
                        e = new_e[lane];
                        d = new_d[lane];
                    }
                    sn = sf;
                    c = cf;
                    pp = pf;
                    g = gf;
                }
                redo = hit;   // d, e and g untouched: the chase again, with the test
            }
            for (int i = mm - 1; redo && i >= l; --i) {
                const double ei = lane_value(ech, i);
                const double f = sn * ei, bb = c * ei;
                // |f|, |g| stay far from the overflow and underflow thresholds
                // here (entries of a Gram matrix of unit-variance samples), so
                // r = sqrt(f^2 + g^2) and the ratios come from one reciprocal root
                const double r2 = f * f + g * g;
                if (r2 == 0.0) {
                    // split: d_{i+1} takes the accumulated shift, e_{i+1} = 0, e_mm = 0
                    if (lane == i + 1) {
                        d -= pp;
                        e = 0.0;
                    }
                    if (lane == mm) e = 0.0;
                    zero = true;
                    lo = i + 1;
                    break;
                }
                const double rinv = rsqrt(r2);
                r = r2 * rinv;
                if (lane == i + 1) e = r;
                sn = f * rinv;
                c = g * rinv;
                const double gi = lane_value(dch, i + 1) - pp;
                r = (lane_value(dch, i) - gi) * sn + 2.0 * c * bb;
                pp = sn * r;
                if (lane == i + 1) d = gi + pp;
                g = c * r - bb;
                if (lane == 0) {
                    rot_c[i] = c;
                    rot_s[i] = sn;
                }
            }
            // the chase's rotations on every row of the eigenvector matrix
            // (lane = row): rotation i mixes columns i and i + 1, and after it
            // column i + 1 is final for this chase, so a row is one pass down
            // from column mm with the running column in a register
            wave_lds_sync();
            if (lane < n && lo < mm) {
                double* row = V + lane * LDG;
                double carry = row[mm];
#pragma unroll 4
                for (int i = mm - 1; i >= lo; --i) {
                    const double zi = row[i], ci = rot_c[i], si = rot_s[i];
                    row[i + 1] = si * zi + ci * carry;
                    carry = ci * zi - si * carry;
                }
                row[lo] = carry;
            }
            wave_lds_sync();
            if (zero) continue;
            if (lane == l) {
                d -= pp;
                e = g;
            }
            if (lane == mm) e = 0.0;
        }
        if (stalled) break;
    }
    if (stalled && lane == 0) raise_flag(flags, 4);
    wave_lds_sync();
    // eigenvalues on G's diagonal for the shared tail
    if (lane < n) G[lane * LDG + lane] = d;
    __syncthreads();
    eig_finish(pd, p, P, G, V, LDG, perm, lam, &kshared, &second_s, small, sv_all, gap, flags, rank_tol, pass, small2,
               second);
}

// Two-pass range finder: H = C^T C for C = G^T Q (nb x s per patch, Omega's
// layout), one workgroup per patch, into the partials of row chunk 0 (the
// other chunks of the patch zeroed), where the eigensolver sums them.
__global__ __launch_bounds__(kThreads) void adj_gram_kernel(const PatchDesc* pd, int p0, const double* __restrict__ C_all,
                                                            double* __restrict__ part, int maxrc) {
    const int p = p0 + blockIdx.x;
    const PatchDesc P = pd[p];
    const int s = P.s, nb = P.nb, nch = (P.nrows + kRowChunk - 1) / kRowChunk;
    const double* C = C_all + P.om_off;
    double* out = part + (int64_t)p * maxrc * kSmall;
    for (int o = threadIdx.x; o < s * s; o += kThreads) {
        const int a = o / s, b = o - a * s;
        if (b < a) continue;
        double h = 0.0;
        for (int t = 0; t < nb; ++t) h += C[(int64_t)a * nb + t] * C[(int64_t)b * nb + t];
        out[a * kRfMax + b] = h;
        out[b * kRfMax + a] = h;
    }
    for (int ch = 1; ch < nch; ++ch)
        for (int o = threadIdx.x; o < s * s; o += kThreads) out[(int64_t)ch * kSmall + (o / s) * kRfMax + o % s] = 0.0;
}

// ---------------------------------------------------------------- Cholesky factor
// One workgroup per patch: G' = sum of partials (k x k), G' = L L^T,
// T = L^{-T} -> small[p].  A non-positive pivot latches ERR_RANK.
// Pass 0 also decides whether pass 1 is needed: when the Gram matrix of its
// input is within kCholQRSkip of the identity entrywise (so its condition
// number is within 1 + 2 n kCholQRSkip of 1), one pass already leaves the
// columns orthonormal to rounding, and pass 1 applies the identity (its Gram
// matrix is not formed).
constexpr double kCholQRSkip = 1e-4;
__global__ __launch_bounds__(kThreads) void chol_kernel(const PatchDesc* pd, int p0, const double* __restrict__ part, int maxrc,
                                                        double* __restrict__ small, int32_t* flags, int32_t* __restrict__ skip,
                                                        int pass) {
    __shared__ double G[kSmall];
    __shared__ double dev[kThreads];
    __shared__ int bad;
    const int p = p0 + blockIdx.x;
    const PatchDesc P = pd[p];
    const int tid = threadIdx.x, n = P.ncols;
    double* T = small + (int64_t)p * kSmall;
    if (pass == 1 && skip[p]) {
        for (int o = tid; o < kSmall; o += kThreads) T[o] = (o / kRfMax == o % kRfMax && o % kRfMax < n) ? 1.0 : 0.0;
        return;
    }
    const int nch = (P.nrows + kRowChunk - 1) / kRowChunk;
    if (tid == 0) bad = 0;
    sum_partials(part, p, maxrc, nch, n, G);
    if (pass == 0) {
        double d = 0.0;
        for (int o = tid; o < n * n; o += kThreads) {
            const int i = o / n, j = o % n;
            d = fmax(d, fabs(G[i * kRfMax + j] - (i == j ? 1.0 : 0.0)));
        }
        dev[tid] = d;
        __syncthreads();
        if (tid == 0) {
            double m = 0.0;
            for (int t = 0; t < kThreads; ++t) m = fmax(m, dev[t]);
            skip[p] = m <= kCholQRSkip ? 1 : 0;     // a NaN never skips
        }
        __syncthreads();
    }
    for (int j = 0; j < n; ++j) {
        if (tid == 0) {
            const double d = G[j * kRfMax + j];
            if (!(d > 0.0) || !isfinite(d)) bad = 1;
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
    // column c of L^{-1} by forward substitution (thread c); T[i][c] ... stored as T[c][i] = L^{-1}[i][c]
    if (tid < kRfMax) {
        const int c = tid;
        for (int i = 0; i < kRfMax; ++i) {
            double v = 0.0;
            if (c < n && i < n && i >= c) {
                v = (i == c) ? 1.0 : 0.0;
                for (int q = c; q < i; ++q) v -= G[i * kRfMax + q] * T[c * kRfMax + q];
                v /= G[i * kRfMax + i];
            }
            T[c * kRfMax + i] = v;
        }
    }
    if (tid == 0 && bad) raise_flag(flags, 2);
}

// ---------------------------------------------------------------- tall products
// grid (patch, row chunk): dst = src * small[p] (m x k), src / dst tall
// matrices of the patch (skip: patches whose flag is set keep src as it is).
// FP64 MFMA on the transposed product dst^T = small^T src^T, so that a tile's
// accumulator holds 16 consecutive rows of one dst column per lane group
// (coalesced column-major stores) and the src operand is 16 consecutive rows
// of one src column (coalesced loads); small sits in LDS.  Each wave walks
// the chunk's 16-row tiles with every column tile of dst.
template <int NTJ>
__device__ void tall_rows_mfma(const double* __restrict__ S, int nrows, int m, int k, int r0, int r1, const double* B,
                               double* __restrict__ D) {
    typedef Mfma<double>::acc Acc;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
    const int nks = (m + 3) / 4;
    for (int rt = r0 + 16 * w; rt < r1; rt += 16 * (kThreads / 64)) {
        const int row = rt + li;
        const bool rin = row < r1;
        Acc acc[NTJ];
#pragma unroll
        for (int c = 0; c < NTJ; ++c) acc[c] = Mfma<double>::zero();
#pragma unroll 4
        for (int kk = 0; kk < nks; ++kk) {
            const int mi = 4 * kk + lk;
            const double sv = (rin && mi < m) ? S[(int64_t)mi * nrows + row] : 0.0;
            const double* brow = B + (4 * kk + lk) * kRfMax + li;
#pragma unroll
            for (int c = 0; c < NTJ; ++c) acc[c] = Mfma<double>::step(brow[16 * c], sv, acc[c]);
        }
#pragma unroll
        for (int c = 0; c < NTJ; ++c)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int j = 16 * c + Mfma<double>::row(lane, t);
                if (j < k && rin) D[(int64_t)j * nrows + row] = acc[c][t];
            }
    }
}

// (only: patches whose entry is zero have nothing to do; dst_which = kZ
// writes Z = src small with all s columns)
__global__ __launch_bounds__(kThreads) void tall_gemm_kernel(const PatchDesc* pd, int p0, int src_which, int dst_which,
                                                             const double* __restrict__ Y, double* __restrict__ Q,
                                                             double* __restrict__ W, const double* __restrict__ small,
                                                             const int32_t* __restrict__ skip, double* __restrict__ Z = nullptr,
                                                             const int32_t* __restrict__ only = nullptr,
                                                             const int32_t* __restrict__ second = nullptr) {
    __shared__ double B[kSmall];
    const int p = p0 + blockIdx.x;
    if ((skip && skip[p]) || (only && !only[p])) return;
    const PatchDesc P = pd[p];
    const int r0 = blockIdx.y * kRowChunk;
    if (r0 >= P.nrows) return;
    const int r1 = min(P.nrows, r0 + kRowChunk);
    const Tall S = tall_of(P, src_which, Y, Q, W, Z, second && second[p]);
    double* D = dst_which == kZ ? Z + P.Y_off : (dst_which == kQ ? Q : W) + P.Q_off;
    const int m = S.ncols, k = dst_which == kZ ? P.s : P.ncols, nrows = P.nrows;
    // rows of small past m and columns past k are zero in the operand
    for (int o = threadIdx.x; o < kSmall; o += kThreads) {
        const int i = o / kRfMax, j = o % kRfMax;
        B[o] = (i < m && j < k) ? small[(int64_t)p * kSmall + o] : 0.0;
    }
    __syncthreads();
    if (k <= 16) tall_rows_mfma<1>(S.base, nrows, m, k, r0, r1, B, D);
    else if (k <= 32) tall_rows_mfma<2>(S.base, nrows, m, k, r0, r1, B, D);
    else if (k <= 48) tall_rows_mfma<3>(S.base, nrows, m, k, r0, r1, B, D);
    else tall_rows_mfma<4>(S.base, nrows, m, k, r0, r1, B, D);
}

// ---------------------------------------------------------------- sign fix
// The orthonormal columns are in W after two Cholesky-QR passes, in Q where
// the second pass was skipped (skip[p]).
// grid (patch, row chunk): per column, the largest |W| of the chunk and its
// first row -> parts (value, index).
__global__ __launch_bounds__(kThreads) void sign_partial_kernel(const PatchDesc* pd, int p0, const double* __restrict__ W,
                                                                const double* __restrict__ Qs, const int32_t* __restrict__ skip,
                                                                double* __restrict__ pval, int32_t* __restrict__ pidx, int maxrc) {
    __shared__ double rv[kThreads];
    __shared__ int ri[kThreads];
    const int p = p0 + blockIdx.x;
    const PatchDesc P = pd[p];
    const int r0 = blockIdx.y * kRowChunk;
    if (r0 >= P.nrows) return;
    const int r1 = min(P.nrows, r0 + kRowChunk);
    const double* A = (skip[p] ? Qs : W) + P.Q_off;
    const int tid = threadIdx.x;
    for (int j = 0; j < P.ncols; ++j) {
        double bv = -1.0;
        int bi = r0;
        for (int r = r0 + tid; r < r1; r += kThreads) {
            const double a = fabs(A[(int64_t)j * P.nrows + r]);
            if (a > bv) { bv = a; bi = r; }
        }
        rv[tid] = bv;
        ri[tid] = bi;
        __syncthreads();
        for (int w = kThreads / 2; w > 0; w >>= 1) {
            if (tid < w) {
                const double ov = rv[tid + w];
                const int oi = ri[tid + w];
                if (ov > rv[tid] || (ov == rv[tid] && oi < ri[tid])) { rv[tid] = ov; ri[tid] = oi; }
            }
            __syncthreads();
        }
        if (tid == 0) {
            pval[((int64_t)p * maxrc + blockIdx.y) * kRfMax + j] = rv[0];
            pidx[((int64_t)p * maxrc + blockIdx.y) * kRfMax + j] = ri[0];
        }
        __syncthreads();
    }
}

// one workgroup per patch: combine the chunk maxima (first index on ties) -> sign per column in small[p][0..k)
__global__ __launch_bounds__(kRfMax) void sign_final_kernel(const PatchDesc* pd, int p0, const double* __restrict__ W,
                                                           const double* __restrict__ Qs, const int32_t* __restrict__ skip,
                                                           const double* __restrict__ pval, const int32_t* __restrict__ pidx,
                                                           int maxrc, double* __restrict__ small) {
    const int p = p0 + blockIdx.x;
    const PatchDesc P = pd[p];
    const int j = threadIdx.x;
    if (j >= P.ncols) return;
    const int nch = (P.nrows + kRowChunk - 1) / kRowChunk;
    double bv = -1.0;
    int bi = 0;
    for (int ch = 0; ch < nch; ++ch) {
        const double v = pval[((int64_t)p * maxrc + ch) * kRfMax + j];
        const int i = pidx[((int64_t)p * maxrc + ch) * kRfMax + j];
        if (v > bv || (v == bv && i < bi)) { bv = v; bi = i; }
    }
    bi = min(max(bi, 0), P.nrows - 1);
    const double* A = skip[p] ? Qs : W;
    small[(int64_t)p * kSmall + j] = A[P.Q_off + (int64_t)j * P.nrows + bi] < 0.0 ? -1.0 : 1.0;
}

// grid (patch, row chunk): Q = W * sign(column), or Q *= sign(column) in place
// (no restrict: source and destination are one array where skip[p])
__global__ __launch_bounds__(kThreads) void sign_apply_kernel(const PatchDesc* pd, int p0, const double* W, double* Q,
                                                              const int32_t* __restrict__ skip, const double* __restrict__ small) {
    const int p = p0 + blockIdx.x;
    const PatchDesc P = pd[p];
    const int r0 = blockIdx.y * kRowChunk;
    if (r0 >= P.nrows) return;
    const int r1 = min(P.nrows, r0 + kRowChunk), nr = r1 - r0;
    const double* src = skip[p] ? Q : W;
    // columns past a tolerance-chosen rank are zero
    for (int o = threadIdx.x; o < nr * P.kreq; o += kThreads) {
        const int j = o / nr, r = r0 + (o - j * nr);
        const int64_t idx = P.Q_off + (int64_t)j * P.nrows + r;
        Q[idx] = j < P.ncols ? small[(int64_t)p * kSmall + j] * src[idx] : 0.0;
    }
}

// Cholesky-QR passes on W (-> Q, -> W where the second pass is needed) and
// the sign fix into Q, over descriptors pd and buffers Q, W.
static void range_tail(Ctx& c, int p0, int p1, PatchDesc* pd, double* Q, double* W) {
    int maxrows = 0;
    for (int p = p0; p < p1; ++p) maxrows = std::max(maxrows, c.hp[p].nrows);
    const int np = p1 - p0;
    const dim3 tall(np, (maxrows + kRowChunk - 1) / kRowChunk), one(np);
    const int mrc = c.rf_maxrc;
    hipStream_t st = c.stream;
    for (int pass = 0; pass < 2; ++pass) {
        const int src = pass == 0 ? kW : kQ, dst = pass == 0 ? kQ : kW;
        hipLaunchKernelGGL(gram_partial_kernel, tall, dim3(kThreads), 0, st, pd, p0, src, c.Y, Q, W, c.rf_part, mrc,
                           pass == 1 ? (const int32_t*)c.rf_skip : nullptr);
        hipLaunchKernelGGL(chol_kernel, one, dim3(kThreads), 0, st, pd, p0, c.rf_part, mrc, c.rf_small, c.dflags, c.rf_skip, pass);
        hipLaunchKernelGGL(tall_gemm_kernel, tall, dim3(kThreads), 0, st, pd, p0, src, dst, c.Y, Q, W, c.rf_small,
                           pass == 1 ? (const int32_t*)c.rf_skip : nullptr);
    }
    // sign fix: W -> Q
    hipLaunchKernelGGL(sign_partial_kernel, tall, dim3(kThreads), 0, st, pd, p0, W, Q, c.rf_skip, c.rf_pval, c.rf_pidx, mrc);
    hipLaunchKernelGGL(sign_final_kernel, one, dim3(kRfMax), 0, st, pd, p0, W, Q, c.rf_skip, c.rf_pval, c.rf_pidx, mrc,
                       c.rf_small);
    hipLaunchKernelGGL(sign_apply_kernel, tall, dim3(kThreads), 0, st, pd, p0, W, Q, c.rf_skip, c.rf_small);
}

// The range finder over descriptors pd, into basis Q with workspace W, at
// rank tolerance rank_tol.
static void range_core(Ctx& c, int p0, int p1, PatchDesc* pd, double* Q, double* W, double rank_tol) {
    int maxrows = 0;
    for (int p = p0; p < p1; ++p) maxrows = std::max(maxrows, c.hp[p].nrows);
    const int np = p1 - p0;
    const dim3 tall(np, (maxrows + kRowChunk - 1) / kRowChunk), one(np);
    const int mrc = c.rf_maxrc;
    hipStream_t st = c.stream;
    // snapshots: Gram, eigendecomposition, W = Y B
    hipLaunchKernelGGL(gram_partial_kernel, tall, dim3(kThreads), 0, st, pd, p0, (int)kY, c.Y, Q, W, c.rf_part, mrc,
                       (const int32_t*)nullptr);
    int maxs = 0;
    for (int p = p0; p < p1; ++p) maxs = std::max(maxs, c.hp[p].s);
    hipLaunchKernelGGL(eig_ql_kernel, one, dim3(64), 0, st, pd, p0, c.rf_part, mrc, c.rf_small, c.sv, c.gap, c.dflags,
                       rank_tol, 0, c.rf_small2, c.rf_second);
    // the other patches (full-basis ones, and those with fewer than kQlMinCols samples): the Jacobi solver,
    // which returns at once for the patches of the tridiagonal one
    hipLaunchKernelGGL(eig_kernel, one, dim3(eig_threads(maxs)), 0, st, pd, p0, c.rf_part, mrc, c.rf_small, c.sv, c.gap,
                       c.dflags, rank_tol, 0, c.rf_small2, c.rf_second, 1);
    // second pass where Y^T Y does not resolve sigma_{k+1}: Z = Y V, Z^T Z, Jacobi
    hipLaunchKernelGGL(tall_gemm_kernel, tall, dim3(kThreads), 0, st, pd, p0, (int)kY, (int)kZ, c.Y, Q, W, c.rf_small2,
                       (const int32_t*)nullptr, c.rf_Z, (const int32_t*)c.rf_second, (const int32_t*)nullptr);
    hipLaunchKernelGGL(gram_partial_kernel, tall, dim3(kThreads), 0, st, pd, p0, (int)kZ, c.Y, Q, W, c.rf_part, mrc,
                       (const int32_t*)nullptr, (const double*)c.rf_Z, (const int32_t*)c.rf_second);
    hipLaunchKernelGGL(eig_kernel, one, dim3(eig_threads(maxs)), 0, st, pd, p0, c.rf_part, mrc, c.rf_small, c.sv, c.gap,
                       c.dflags, rank_tol, 1, c.rf_small2, c.rf_second, 0);
    // W = Y B (first pass) or Z B (second pass)
    hipLaunchKernelGGL(tall_gemm_kernel, tall, dim3(kThreads), 0, st, pd, p0, (int)kYZ, (int)kW, c.Y, Q, W, c.rf_small,
                       (const int32_t*)nullptr, c.rf_Z, (const int32_t*)nullptr, (const int32_t*)c.rf_second);
    range_tail(c, p0, p1, pd, Q, W);
}

void launch_range(Ctx& c, int p0, int p1) {
    StageTimer t(c, MSRS_K_RANGE);
    range_core(c, p0, p1, c.dp, c.Q, c.rf_ws, c.rank_tol);
}

// Wide pass: every patch at s columns (the wide descriptors place the basis
// at Y's offsets), at the numerical rank sigma_j(Y) > 1e-12 sigma_1(Y) (the
// handle's rank tolerance applies to the two-pass singular values instead);
// the columns past the rank are zero.
void launch_range_wide(Ctx& c, int p0, int p1) {
    StageTimer t(c, MSRS_K_RANGE);
    range_core(c, p0, p1, c.dp_wide, c.tp_Q, c.tp_W, 1e-12);
}

// H = (G^T Q)^T (G^T Q), its eigenvectors V (descending), the basis
// Q V[:, :k] -> W, then Cholesky-QR and the sign fix into the handle's basis;
// the singular values are those of Q^T G.
void launch_range_two_pass(Ctx& c, int p0, int p1) {
    StageTimer t(c, MSRS_K_RANGE);
    int maxrows = 0, maxs = 0;
    for (int p = p0; p < p1; ++p) maxrows = std::max(maxrows, c.hp[p].nrows), maxs = std::max(maxs, c.hp[p].s);
    const int np = p1 - p0;
    const dim3 tall(np, (maxrows + kRowChunk - 1) / kRowChunk), one(np);
    const int mrc = c.rf_maxrc;
    hipStream_t st = c.stream;
    hipLaunchKernelGGL(adj_gram_kernel, one, dim3(kThreads), 0, st, c.dp, p0, c.tp_C, c.rf_part, mrc);
    hipLaunchKernelGGL(eig_ql_kernel, one, dim3(64), 0, st, c.dp, p0, c.rf_part, mrc, c.rf_small, c.sv, c.gap, c.dflags,
                       c.rank_tol, 2, c.rf_small2, c.rf_second);
    hipLaunchKernelGGL(eig_kernel, one, dim3(eig_threads(maxs)), 0, st, c.dp, p0, c.rf_part, mrc, c.rf_small, c.sv, c.gap,
                       c.dflags, c.rank_tol, 2, c.rf_small2, c.rf_second, 1);
    hipLaunchKernelGGL(tall_gemm_kernel, tall, dim3(kThreads), 0, st, c.dp, p0, (int)kZ, (int)kW, c.Y, c.Q, c.rf_ws, c.rf_small,
                       (const int32_t*)nullptr, c.tp_Q, (const int32_t*)nullptr, (const int32_t*)nullptr);
    range_tail(c, p0, p1, c.dp, c.Q, c.rf_ws);
}

}  // namespace msrs
