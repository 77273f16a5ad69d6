// Local fine-scale solves of the offline stage (LocalPDESolver inside
// RanLocalSolu, Section 3): coefficient gather, boundary samples, lifting of
// the boundary data, block-row factorization, multi-RHS sweeps on MFMA, FP64
// residuals for iterative refinement, and restriction to K_m.
//
// Both operators are block tridiagonal in the line ordering of PatchDesc:
//   A = tridiag(Low_l, Dg_l, Up_l), lines l = 0..nl-1, blocks b x b.
// Elliptic (bilinear elements, eq. Elliptic): Dg_l = T_l tridiagonal,
//   Up_l = Low_{l+1} = U_l symmetric tridiagonal (coupling of node lines
//   l+1 and l+2 through cell row l+1).
// Kinetic (upwind ordinates, eq. RTE with isotropic scattering):
//   Dg_l = diag(|v|/dx + sigma_l/eps) - (sigma_l/eps) 1 (w/2)^T,
//   Low_l = -diag(v+/dx), Up_l = -diag(v-/dx).
// Block elimination: D_0 = Dg_0, D_{l+1} = Dg_{l+1} - Low_{l+1} D_l^{-1} Up_l;
// the inverses E_l = D_l^{-1} are formed explicitly (Gauss-Jordan, no
// pivoting: D_l is SPD (elliptic) or a row-diagonally-dominant M-matrix
// (kinetic)), so that both sweeps are dense products on MFMA:
//   forward  y_0 = r_0,  w_l = E_l y_l,  y_{l+1} = r_{l+1} - Low_{l+1} w_l
//   back     x_{nl-1} = w_{nl-1},  x_l = E_l (y_l - Up_l x_{l+1}).
#include "device_common.h"

namespace msrs {

// ------------------------------------------------------------ small helpers
// Counter-clockwise boundary index of local physical node (i, j) of a cx x cy
// cell block (caller guarantees the node is on the boundary).
__device__ __forceinline__ int bidx_ccw(int i, int j, int cx, int cy) {
    if (j == 0 && i < cx) return i;
    if (i == cx && j < cy) return cx + j;
    if (j == cy && i > 0) return cx + cy + (cx - i);
    return 2 * cx + cy + (cy - j);
}

// physical local node of line coordinates (p, q)
__device__ __forceinline__ void line_to_phys(const PatchDesc& P, int p, int q, int& i, int& j) {
    if (P.trans) { i = q; j = p; } else { i = p; j = q; }
}

__device__ __forceinline__ double a_cell(const double* aL, int L, int cr, int cp) { return aL[cr * L + cp]; }

// Q1 stencil coefficient between node (p,q) and (p+dp, q+dq) of a buffered
// patch, from the four elements around (p,q): NE=(p,q) NW=(p-1,q)
// SW=(p-1,q-1) SE=(p,q-1) (cell column, cell row).
__device__ __forceinline__ double q1_coef(const double* aL, int L, int p, int q, int dp, int dq) {
    const double NE = a_cell(aL, L, q, p), NW = a_cell(aL, L, q, p - 1);
    const double SW = a_cell(aL, L, q - 1, p - 1), SE = a_cell(aL, L, q - 1, p);
    if (dp == 0 && dq == 0) return (2.0 / 3.0) * (NE + NW + SW + SE);
    if (dq == 0) return dp > 0 ? -(NE + SE) / 6.0 : -(NW + SW) / 6.0;
    if (dp == 0) return dq > 0 ? -(NE + NW) / 6.0 : -(SE + SW) / 6.0;
    if (dp > 0) return dq > 0 ? -NE / 3.0 : -SE / 3.0;
    return dq > 0 ? -NW / 3.0 : -SW / 3.0;
}

// ------------------------------------------------------------ gather (a2)
__global__ __launch_bounds__(kThreads) void gather_elliptic_kernel(const PatchDesc* pd, int p0, const double* __restrict__ a,
                                                                   int N, double* __restrict__ aL_all, int32_t* flags) {
    const PatchDesc P = pd[p0 + blockIdx.x];
    double* aL = aL_all + P.a_off;
    const int n = P.L * P.Qn;
    for (int idx = threadIdx.x; idx < n; idx += kThreads) {
        const int cr = idx / P.L, cp = idx - cr * P.L;
        const int ci = P.trans ? P.x0 + cr : P.x0 + cp;
        const int cj = P.trans ? P.y0 + cp : P.y0 + cr;
        const double v = a[(size_t)cj * N + ci];
        if (!(v > 0.0) || !isfinite(v)) raise_flag(flags, 0);
        aL[idx] = v;
    }
}

__global__ __launch_bounds__(kThreads) void gather_kinetic_kernel(const PatchDesc* pd, int p0, const double* __restrict__ sigma,
                                                                  double* __restrict__ aL_all, int32_t* flags) {
    const PatchDesc P = pd[p0 + blockIdx.x];
    for (int i = threadIdx.x; i < P.cx; i += kThreads) {
        const double v = sigma[P.x0 + i];
        if (!(v >= 0.0) || !isfinite(v)) raise_flag(flags, 0);
        aL_all[P.a_off + i] = v;
    }
}

// ------------------------------------------------------------ Omega (a3)
// grid (patch, 16-column group); Omega is nb x s column-major.
__global__ __launch_bounds__(kThreads) void omega_kernel(const PatchDesc* pd, int p0, const double* __restrict__ user,
                                                         double* __restrict__ om, uint64_t seed) {
    const int p = p0 + blockIdx.x;
    const PatchDesc P = pd[p];
    const int cs0 = blockIdx.y * 16;
    if (cs0 >= P.s) return;
    const int ncol = min(16, P.s - cs0);
    const int n = P.nb * ncol;
    for (int idx = threadIdx.x; idx < n; idx += kThreads) {
        const int c = cs0 + idx / P.nb, t = idx - (idx / P.nb) * P.nb;
        const int64_t o = P.om_off + (int64_t)c * P.nb + t;
        double v;
        if (P.full) v = (t == c) ? 1.0 : 0.0;
        else if (user) v = user[o];
        else v = philox_normal(seed, (uint32_t)t, (uint32_t)c, (uint32_t)p);
        om[o] = v;
    }
}

// ------------------------------------------------------------ lifting (a3)
// Lines are processed in chunks of kChunkLines per workgroup: grid (patch,
// chunk).  Per-sample sums of squares go to part[(p * maxch + chunk) * 64 + col]
// and are reduced per patch by norms_kernel (fixed order, no atomics).

// thread -> (row group, sample column) over a line of bp x sp values
struct LineMap {
    int col, row0, rows;
    bool active;
    __device__ LineMap(int sp) : col(threadIdx.x % sp), row0(threadIdx.x / sp), rows(kThreads / sp) {
        active = row0 < rows;
    }
};

__device__ __forceinline__ void partial_column_sums(double ssum, const LineMap& m, int sp, double* red, double* out) {
    __syncthreads();
    red[threadIdx.x] = m.active ? ssum : 0.0;
    __syncthreads();
    if ((int)threadIdx.x < sp) {
        double s = 0.0;
        for (int r = 0; r < m.rows; ++r) s += red[r * sp + threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// rhs = -A_IB omega into the line vectors X (FP64 or FP32), padding zeroed.
template <int KIND, typename TX>
__global__ __launch_bounds__(kThreads) void lift_kernel(const PatchDesc* pd, int p0, const double* __restrict__ aL_all,
                                                        const double* __restrict__ om, const double* __restrict__ vw, double dx,
                                                        TX* __restrict__ X, double* __restrict__ part, int maxch) {
    __shared__ double red[kThreads];
    const int p = p0 + blockIdx.x;
    const PatchDesc P = pd[p];
    const int l0 = blockIdx.y * kChunkLines;
    if (l0 >= P.nl) return;
    const int l1 = min(P.nl, l0 + kChunkLines);
    const double* aL = aL_all + P.a_off;
    const double* O = om + P.om_off;
    const int sp = P.sp, bp = P.bp, b = P.b, nl = P.nl;
    const LineMap m(sp);
    const int c = m.col;
    double ssum = 0.0;
    for (int l = l0; l < l1; ++l) {
        // only nodes next to the buffered patch's boundary (first / last line,
        // first / last row) have boundary neighbours
        const bool edge_line = l == 0 || l == nl - 1;
        for (int i = m.row0; m.active && i < bp; i += m.rows) {
            double v = 0.0;
            if (i < b && c < P.s && (edge_line || i == 0 || i == b - 1)) {
                if (KIND == kElliptic) {
                    const int pp = i + 1, q = l + 1;
#pragma unroll
                    for (int dq = -1; dq <= 1; ++dq)
#pragma unroll
                        for (int dp = -1; dp <= 1; ++dp) {
                            const int p2 = pp + dp, q2 = q + dq;
                            if (p2 == 0 || p2 == P.L || q2 == 0 || q2 == P.Qn) {
                                int ii, jj;
                                line_to_phys(P, p2, q2, ii, jj);
                                v -= q1_coef(aL, P.L, pp, q, dp, dq) * O[(int64_t)c * P.nb + bidx_ccw(ii, jj, P.cx, P.cy)];
                            }
                        }
                } else {
                    const int h = b / 2;
                    const double vi = vw[i];
                    if (l == 0 && vi > 0) v += vi / dx * O[(int64_t)c * P.nb + (i - h)];
                    if (l == nl - 1 && vi < 0) v += -vi / dx * O[(int64_t)c * P.nb + h + i];
                }
            }
            const int64_t o = P.x_off + (int64_t)l * bp * sp + (int64_t)i * sp + c;
            X[o] = (TX)v;
            ssum += v * v;
        }
    }
    partial_column_sums(ssum, m, sp, red, part + ((int64_t)p * maxch + blockIdx.y) * kMaxSamples);
}

// ------------------------------------------------------------ factorization (a4)
// Diagonal block entry of line l (i, j < b).
template <int KIND>
__device__ __forceinline__ double diag_entry(const PatchDesc& P, const double* aL, const double* vw, double dx, double inv_eps,
                                             int l, int i, int j) {
    if (KIND == kElliptic) {
        const int q = l + 1, L = P.L;
        if (i == j) {
            const int p = i + 1;
            return (2.0 / 3.0) * (a_cell(aL, L, q, p) + a_cell(aL, L, q, p - 1) + a_cell(aL, L, q - 1, p - 1) + a_cell(aL, L, q - 1, p));
        }
        if (j == i + 1) return -(a_cell(aL, L, q, i + 1) + a_cell(aL, L, q - 1, i + 1)) / 6.0;
        if (i == j + 1) return -(a_cell(aL, L, q, j + 1) + a_cell(aL, L, q - 1, j + 1)) / 6.0;
        return 0.0;
    } else {
        const int nv = P.b;
        const double s = aL[l] * inv_eps;
        if (P.hg) {
            double v = -s * vw[3 * nv + i * nv + j];
            if (i == j) v += fabs(vw[i]) / dx + s * vw[2 * nv + i];
            return v;
        }
        double v = -s * 0.5 * vw[nv + j];
        if (i == j) v += fabs(vw[i]) / dx + s;
        return v;
    }
}


// ---- blocked Gauss-Jordan on MFMA
// The block D_l (BP = 16 R) is held as R x R tiles of 16 x 16 in MFMA
// accumulator layout, spread over the waves by factor_tile.  Pivots are taken
// in panels of 16: the panel's diagonal block is inverted by one wave with
// cross-lane shuffles, then X = Dinv A_{p,*} (new row panel), -A_{*,p} Dinv
// (new column panel) and the rank-16 update A_{i,j} -= A_{i,p} X_j run on MFMA.
constexpr int kFactorWaves = 16;
constexpr int kFactorThreads = 64 * kFactorWaves;

// Tile map of the blocked factor: slot q of wave w holds tile ti R + tj, or
// nothing (-1).  Up to R = 5 tiles per side, diagonal tile d sits alone on
// wave d (so that in FP32 its owner inverts it while the other waves run the
// panel update) and the R (R - 1) off-diagonal tiles go row-major and
// round-robin over waves R .. 15; from R = 6 on (three or more slots per wave
// there, which slows the Schur build more than the inverse gains), all R^2
// tiles go round-robin over the 16 waves.
template <int R>
constexpr bool factor_diag_alone() { return R <= 5; }
template <int R>
__device__ __forceinline__ int factor_tile(int q, int w) {
    if constexpr (!factor_diag_alone<R>()) {
        const int idx = q * kFactorWaves + w;
        return idx < R * R ? idx : -1;
    } else {
        constexpr int NW = kFactorWaves - R, NOFF = R * (R - 1), RM = R > 1 ? R - 1 : 1;
        if (w < R) return q == 0 ? w * (R + 1) : -1;
        const int o = q * NW + (w - R);
        if (o >= NOFF) return -1;
        const int i = o / RM, jj = o - i * RM;
        return i * R + (jj < i ? jj : jj + 1);
    }
}
template <int R>
constexpr int factor_slots() {
    if constexpr (!factor_diag_alone<R>()) {
        return (R * R + kFactorWaves - 1) / kFactorWaves;
    } else {
        constexpr int NW = kFactorWaves - R, NOFF = R * (R - 1);
        return NOFF == 0 ? 1 : (NOFF + NW - 1) / NW;
    }
}

// Inverse of a 16 x 16 block (row-major in LDS, leading dimension LDA; the
// inverse with LDD) by one wave: lane l
// holds row l%16, columns 4(l/16)..4(l/16)+3; Gauss-Jordan without pivoting.
// FP32 pivot step K: the pivot row reaches every lane of a 16-lane row by a
// DPP row broadcast; the pivot column entry of row r sits in lane r of 16-lane
// row K/4, which two row-swap permutes (16- then 32-lane halves, each taken
// from the side that holds that row) copy to all four rows without a trip
// through LDS; the pivot itself comes by readlane, and its reciprocal is the
// hardware approximation (the FP32 factor is refined in FP64 downstream).
template <int K>
__device__ __forceinline__ void inv16_pivot_f32(float (&a)[4], int r, int cg, bool& bad) {
    constexpr int kg = K >> 2, ku = K & 3;
    float prow[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) prow[u] = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(a[u]), 0x150 + K, 0xF, 0xF, false));
    const unsigned xc = __float_as_uint(a[ku]);
    const auto s16 = __builtin_amdgcn_permlane16_swap(xc, xc, false, false);   // rows (0,0,2,2) | (1,1,3,3)
    const unsigned h = (kg & 1) ? s16[1] : s16[0];
    const auto s32 = __builtin_amdgcn_permlane32_swap(h, h, false, false);     // rows (0,1,0,1) | (2,3,2,3) of h
    const float pcol = __uint_as_float((kg & 2) ? s32[1] : s32[0]);
    const float piv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(a[ku]), K + 16 * kg));
    if (!(piv > 0.f) || !isfinite(piv)) bad = true;
    const float ip = __builtin_amdgcn_rcpf(piv);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const bool ck = (4 * cg + u) == K;
        const float gen = ck ? -pcol * ip : a[u] - pcol * ip * prow[u];
        a[u] = (r == K) ? (ck ? ip : prow[u] * ip) : gen;
    }
    if constexpr (K + 1 < 16) inv16_pivot_f32<K + 1>(a, r, cg, bad);
}

// In-register inverse of a 16 x 16 FP32 block in MFMA accumulator layout
// (lane l: column c = l % 16, rows 4 q + t in a[t], q = l / 16), Gauss-Jordan
// without pivoting.  Pivot step K: the pivot column entries of the lane's rows
// come by a DPP row broadcast from lane K of the same 16-lane row; the pivot
// row entry of its column sits in 16-lane row K/4, register K%4, copied to all
// rows by the two row-swap permutes; the pivot by readlane, its reciprocal the
// hardware approximation.
template <int K>
__device__ __forceinline__ void inv16_acc_f32(float (&a)[4], int c, int q, bool& bad) {
    constexpr int kq = K >> 2, kt = K & 3;
    float pcol[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) pcol[t] = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(a[t]), 0x150 + K, 0xF, 0xF, false));
    const unsigned xr = __float_as_uint(a[kt]);
    const auto s16 = __builtin_amdgcn_permlane16_swap(xr, xr, false, false);
    const unsigned h = (kq & 1) ? s16[1] : s16[0];
    const auto s32 = __builtin_amdgcn_permlane32_swap(h, h, false, false);
    const float prow = __uint_as_float((kq & 2) ? s32[1] : s32[0]);
    const float piv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(a[kt]), K + 16 * kq));
    if (!(piv > 0.f) || !isfinite(piv)) bad = true;
    const float ip = __builtin_amdgcn_rcpf(piv);
    const bool ck = c == K;
    const float prs = ck ? ip : prow * ip;   // the new pivot row (its own entry 1/p)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const float gen = ck ? -pcol[t] * ip : a[t] - pcol[t] * prs;
        a[t] = (t == kt && q == kq) ? prs : gen;
    }
    if constexpr (K + 1 < 16) inv16_acc_f32<K + 1>(a, c, q, bad);
}

template <typename T, int LDA, int LDD>
__device__ __forceinline__ void inv16_wave(const T* A, T* Dinv, bool& bad) {
    const int l = threadIdx.x & 63, r = l & 15, cg = l >> 4;
    T a[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] = A[r * LDA + 4 * cg + u];
    if constexpr (sizeof(T) == 4) {
        inv16_pivot_f32<0>(a, r, cg, bad);
    } else {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int kg = k >> 2, ku = k & 3;
            T prow[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) prow[u] = __shfl(a[u], k + 16 * cg, 64);
            const T pcol = __shfl(a[ku], r + 16 * kg, 64);
            const T piv = __shfl(a[ku], k + 16 * kg, 64);
            if (!(piv > T(0)) || !isfinite((double)piv)) bad = true;
            const T ip = T(1) / piv;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const bool ck = (4 * cg + u) == k;
                const T gen = ck ? -pcol * ip : a[u] - pcol * ip * prow[u];
                a[u] = (r == k) ? (ck ? ip : prow[u] * ip) : gen;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) Dinv[r * LDD + 4 * cg + u] = a[u];
}

// The block-tridiagonal elimination runs from both ends ("twisted"): the
// top half eliminates lines 0 .. m-1 downwards (D_l = A_l - Low_l E_{l-1}
// Up_{l-1}), the bottom half lines nl-1 .. m+1 upwards (D_l = A_l - Up_l
// E_{l+1} Low_{l+1}), both at once, and the middle line m = nl/2 takes both
// Schur terms.  E_l = D_l^{-1} is stored at line l in the sweep's MFMA
// operand order.  This halves the sequential chain per patch.
//
// Mode: MID = false runs one half (dir = +1 top, -1 bottom); MID = true the
// middle line, reading E_{m-1} and E_{m+1} back from HBM.
template <typename T, int KIND, int R, bool MID>
__device__ __forceinline__ void factor_mfma_body(const PatchDesc& P, const double* __restrict__ aL, const double* __restrict__ vw,
                                              double dx, double inv_eps, T* __restrict__ E, T* lds, double* cf,
                                              double* crow, int dir, int32_t* flags) {
    constexpr int BP = 16 * R, LDE = BP + 1, NSLOT = factor_slots<R>();
    constexpr int NKS = BP / 4;
    typedef typename Mfma<T>::acc Acc;
    const int tid0 = threadIdx.x, w = tid0 >> 6;
    // Lane-dependent indices are re-derived per block row and per panel from a
    // laundered thread id, so their address arithmetic is not hoisted and kept
    // live across the loops (register pressure).
    int tid = tid0, lane = tid0 & 63, li = lane & 15, lk = lane >> 4;
    auto launder = [&]() {
        int t = tid0;
        asm volatile("" : "+v"(t));
        tid = t;
        lane = t & 63;
        li = lane & 15;
        lk = lane >> 4;
    };
    const int b = P.b, nl = P.nl, L = P.L;
    const int m = nl / 2;
    // lines of this block: line0, line0 + dir, ... (nsteps of them)
    const int nsteps = MID ? 1 : (dir > 0 ? m : nl - 1 - m);
    const int line0 = MID ? m : (dir > 0 ? 0 : nl - 1);
    if (nsteps <= 0) return;   // uniform over the workgroup
    T* Es = lds;                         // E of the previously eliminated line, BP x LDE (row-major)
    // panel buffers alias Es (free once D_l is formed); odd leading dimensions
    // spread the MFMA operand reads (16 rows x 4 k, or 4 rows x 16 columns)
    // over distinct LDS banks
    constexpr int PCL = 17, PRL = BP + 1, DVL = 17;
    T* Pc = lds;                                   // [2][BP x PCL]  column panel (row i, panel column k)
    T* Pr = lds + 2 * BP * PCL;                    // [2][16 x PRL]  row panel
    T* Xs = Pr + 2 * 16 * PRL;                     // [2][16 x PRL]  new row panel
    T* Dv = Xs + 2 * 16 * PRL;                     // [2][16 x DVL]  inverse of the diagonal block
    Acc tile[NSLOT];
    bool bad = false;
    const int npan = (b + 15) / 16;
    // elliptic: cell row r lives in crow[r & 1] (ld kMaxLine + 1); a line
    // needs its two bounding cell rows, and each step brings one new row,
    // prefetched into a register one step ahead
    double rnext = 0.0;
    const int rnew0 = dir > 0 ? line0 + 2 : line0 - 1;   // the row the second step needs
    if (KIND == kElliptic) {
        if (tid < L) {
            crow[(line0 & 1) * (kMaxLine + 1) + tid] = aL[line0 * L + tid];
            crow[((line0 + 1) & 1) * (kMaxLine + 1) + tid] = aL[(line0 + 1) * L + tid];
            if (!MID && nsteps > 1) rnext = aL[rnew0 * L + tid];
        }
    } else {
        for (int a = tid; a < b; a += kFactorThreads) {
            const double v = vw[a];
            cf[a] = v > 0 ? v / dx : 0.0;
            cf[BP + a] = v < 0 ? -v / dx : 0.0;
        }
    }
    // global E block (MFMA operand order) -> Es (row-major)
    auto load_E = [&](const T* Eg) {
        for (int o = tid; o < BP * BP; o += kFactorThreads) {
            const int kk = o % NKS, t = o / NKS;
            const int ln = t & 63, rt = t >> 6;
            Es[(16 * rt + (ln & 15)) * LDE + 4 * kk + (ln >> 4)] = Eg[o];
        }
    };
    // elliptic coupling block between two adjacent lines from their shared
    // cell row cr (symmetric tridiagonal): diagonal -(c_a + c_{a+1})/6,
    // off-diagonal (a, a+1) -c_{a+1}/3
    auto set_cf = [&](const double* cr) {
        for (int a = tid; a < b; a += kFactorThreads) {
            cf[a] = (cr[a] + cr[a + 1]) * (-1.0 / 6.0);
            cf[BP + a] = cr[a + 1] * (-1.0 / 3.0);
        }
    };

    for (int l = 0; l < nsteps; ++l) {
        launder();
        const int ln = line0 + dir * l;
        const double* rA = crow + (ln & 1) * (kMaxLine + 1);          // cell row ln
        const double* rB = crow + ((ln + 1) & 1) * (kMaxLine + 1);    // cell row ln + 1
        // the Schur terms of this line: previously eliminated neighbour(s)
        const bool term1 = MID ? (m > 0) : (l > 0);
        const bool term2 = MID && (m < nl - 1);
        if (MID && term1) load_E(E + (int64_t)(m - 1) * BP * BP);
        __syncthreads();
        // coupling to the first neighbour: top / middle -> line ln-1 (cell row ln),
        // bottom -> line ln+1 (cell row ln+1)
        if (KIND == kElliptic && term1) set_cf(dir < 0 ? rB : rA);
        __syncthreads();
        // diagonal block entry (i, j < b) of line ln
        auto dg = [&](int i, int j) -> double {
            if (KIND == kElliptic) {
                if (i == j) return (2.0 / 3.0) * (rB[i + 1] + rB[i] + rA[i] + rA[i + 1]);
                if (j == i + 1) return (rB[i + 1] + rA[i + 1]) * (-1.0 / 6.0);
                if (i == j + 1) return (rB[j + 1] + rA[j + 1]) * (-1.0 / 6.0);
                return 0.0;
            } else {
                return diag_entry<KIND>(P, aL, vw, dx, inv_eps, ln, i, j);
            }
        };
        // D = (init ? Dg : D) - (term ? C^T E C : 0) straight into the owned
        // MFMA tiles from the neighbour's E (row-major in LDS): no write-back.
        // Indices past the line (outside [0, b)) carry zero coefficients;
        // their reads are clamped inside the tile (finite values times zero).
        // Past the line, D is the identity (padding).  Kinetic: the coupling
        // is diagonal, Low = v+/dx before Up = v-/dx (top) or after (bottom).
        auto schur = [&](bool init, bool term, bool kin_rev) {
#pragma unroll
            for (int q = 0; q < NSLOT; ++q) {
                const int idx = factor_tile<R>(q, w);
                if (idx < 0) continue;
                const int ti = idx / R, tj = idx - ti * R;
                const int j = 16 * tj + li;
                if constexpr (KIND == kElliptic && sizeof(T) == 4) {
                    // f32 tiles: a lane's rows ib..ib+3 are consecutive and share column j,
                    // so Z(i', j) = (E C)(i', j) is formed once for rows ib-1..ib+4
                    const int ib = 16 * ti + 4 * lk;
                    double zc[6];
                    if (term) {
                        const double c0 = (j > 0 && j < b) ? cf[BP + j - 1] : 0.0;
                        const double c1 = (j < b) ? cf[j] : 0.0;
                        const double c2 = (j < b - 1) ? cf[BP + j] : 0.0;
                        const int jm = j > 0 ? j - 1 : 0, jp = j < BP - 1 ? j + 1 : BP - 1;
#pragma unroll
                        for (int r = 0; r < 6; ++r) {
                            const int ir = ib - 1 + r;
                            const int irc = ir < 0 ? 0 : (ir > BP - 1 ? BP - 1 : ir);
                            const T* er = Es + irc * LDE;
                            const double z = c0 * (double)er[jm] + c1 * (double)er[j] + c2 * (double)er[jp];
                            zc[r] = (ir >= 0 && ir < b) ? z : 0.0;
                        }
                    }
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int i = ib + t;
                        double v = init ? ((i == j) ? 1.0 : 0.0) : (double)tile[q][t];
                        if (i < b && j < b) {
                            if (init) v = dg(i, j);
                            if (term) {
                                const double r0 = i > 0 ? cf[BP + i - 1] : 0.0;
                                const double r2 = i < b - 1 ? cf[BP + i] : 0.0;
                                v -= r0 * zc[t] + cf[i] * zc[t + 1] + r2 * zc[t + 2];
                            }
                        }
                        tile[q][t] = (T)v;
                    }
                } else {
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int i = 16 * ti + Mfma<T>::row(lane, t);
                        double v = init ? ((i == j) ? 1.0 : 0.0) : (double)tile[q][t];
                        if (i < b && j < b) {
                            if (init) v = dg(i, j);
                            if (term) {
                                if (KIND == kElliptic) {
                                    // sum over i' in {i-1, i, i+1}, j' in {j-1, j, j+1} of C(i', i) E(i', j') C(j', j)
                                    double sv = 0.0;
#pragma unroll
                                    for (int di = -1; di <= 1; ++di) {
                                        const int ir = i + di;
                                        if (ir < 0 || ir >= b) continue;
                                        const double ru = di == 0 ? cf[i] : (di < 0 ? cf[BP + i - 1] : cf[BP + i]);
                                        const T* er = Es + ir * LDE;
                                        double z = cf[j] * (double)er[j];
                                        if (j > 0) z += cf[BP + j - 1] * (double)er[j - 1];
                                        if (j < b - 1) z += cf[BP + j] * (double)er[j + 1];
                                        sv += ru * z;
                                    }
                                    v -= sv;
                                } else {
                                    v -= kin_rev ? cf[BP + i] * (double)Es[i * LDE + j] * cf[j]
                                                 : cf[i] * (double)Es[i * LDE + j] * cf[BP + j];
                                }
                            }
                        }
                        tile[q][t] = (T)v;
                    }
                }
            }
        };
        schur(true, term1, dir < 0);
        if (term2) {
            // middle line: second term from the line below (E_{m+1}, cell row m+1)
            __syncthreads();
            load_E(E + (int64_t)(m + 1) * BP * BP);
            if (KIND == kElliptic) set_cf(rB);
            __syncthreads();
            schur(false, true, true);
        }
        __syncthreads();   // Es no longer needed: panel buffers may overwrite it
        // blocked Gauss-Jordan over the panels.  Panel pn: B1 publish its column
        // and row tiles, B2 invert the diagonal block, B3a new row panel
        // X_j = Dinv A_{p,j}, B3b column panel -A_{i,p} Dinv and rank-16 update
        // A_{i,j} -= A_{i,p} X_j.  FP32 runs B1 and B2 of panel pn+1 inside B3b of
        // panel pn (look-ahead): the owner of the next diagonal tile inverts it
        // in registers while the other waves finish their updates.
        auto publish = [&](int p, T* pc, T* pr) {
#pragma unroll
            for (int q = 0; q < NSLOT; ++q) {
                const int idx = factor_tile<R>(q, w);
                if (idx < 0) continue;
                const int ti = idx / R, tj = idx - ti * R;
                if (tj != p && ti != p) continue;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int ii = Mfma<T>::row(lane, t);
                    if (tj == p) pc[(16 * ti + ii) * PCL + li] = tile[q][t];
                    if (ti == p) pr[ii * PRL + 16 * tj + li] = tile[q][t];
                }
            }
        };
        // FP32: the diagonal tile (p, p) -> its inverse, in place and in dv
        auto invert_diag = [&](int p, T* dv) {
            if constexpr (sizeof(T) == 4) {
#pragma unroll
                for (int q = 0; q < NSLOT; ++q) {
                    if (factor_tile<R>(q, w) != p * (R + 1)) continue;
                    float a4[4];
#pragma unroll
                    for (int t = 0; t < 4; ++t) a4[t] = tile[q][t];
                    inv16_acc_f32<0>(a4, li, lk, bad);
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        tile[q][t] = a4[t];
                        dv[(4 * lk + t) * DVL + li] = a4[t];
                    }
                }
            }
        };
        auto row_panel = [&](int pn, const T* pr, T* xs, const T* dv) {
#pragma unroll
            for (int q = 0; q < NSLOT; ++q) {
                const int idx = factor_tile<R>(q, w);
                if (idx < 0) continue;
                const int ti = idx / R, tj = idx - ti * R;
                if (ti != pn || tj == pn) continue;
                Acc x = Mfma<T>::zero();
#pragma unroll
                for (int st = 0; st < 4; ++st) {
                    const int k = 4 * st + lk;
                    x = Mfma<T>::step(dv[li * DVL + k], pr[k * PRL + 16 * tj + li], x);
                }
                tile[q] = x;
#pragma unroll
                for (int t = 0; t < 4; ++t) xs[Mfma<T>::row(lane, t) * PRL + 16 * tj + li] = x[t];
            }
        };
        auto update = [&](int pn, const T* pc, const T* xs, const T* dv, bool set_diag) {
#pragma unroll
            for (int q = 0; q < NSLOT; ++q) {
                const int idx = factor_tile<R>(q, w);
                if (idx < 0) continue;
                const int ti = idx / R, tj = idx - ti * R;
                if (ti == pn) {
                    if (tj == pn && set_diag) {
#pragma unroll
                        for (int t = 0; t < 4; ++t) tile[q][t] = dv[Mfma<T>::row(lane, t) * DVL + li];
                    }
                    continue;
                }
                if (tj == pn) {
                    Acc x = Mfma<T>::zero();
#pragma unroll
                    for (int st = 0; st < 4; ++st) {
                        const int k = 4 * st + lk;
                        x = Mfma<T>::step(-pc[(16 * ti + li) * PCL + k], dv[k * DVL + li], x);
                    }
                    tile[q] = x;
                } else {
                    Acc x = tile[q];
#pragma unroll
                    for (int st = 0; st < 4; ++st) {
                        const int k = 4 * st + lk;
                        x = Mfma<T>::step(-pc[(16 * ti + li) * PCL + k], xs[k * PRL + 16 * tj + li], x);
                    }
                    tile[q] = x;
                }
            }
        };
        if constexpr (sizeof(T) == 4) {
            publish(0, Pc, Pr);
            invert_diag(0, Dv);
            __syncthreads();
            for (int pn = 0; pn < npan; ++pn) {
                launder();
                const int buf = pn & 1, nb = buf ^ 1;
                row_panel(pn, Pr + buf * 16 * PRL, Xs + buf * 16 * PRL, Dv + buf * 16 * DVL);
                __syncthreads();
                update(pn, Pc + buf * BP * PCL, Xs + buf * 16 * PRL, Dv + buf * 16 * DVL, false);
                if (pn + 1 < npan) {
                    publish(pn + 1, Pc + nb * BP * PCL, Pr + nb * 16 * PRL);
                    invert_diag(pn + 1, Dv + nb * 16 * DVL);
                }
                __syncthreads();
            }
        } else {
            for (int pn = 0; pn < npan; ++pn) {
                launder();
                const int buf = pn & 1;
                T* pc = Pc + buf * BP * PCL;
                T* pr = Pr + buf * 16 * PRL;
                T* xs = Xs + buf * 16 * PRL;
                T* dv = Dv + buf * 16 * DVL;
                publish(pn, pc, pr);
                __syncthreads();
                if (w == 0) inv16_wave<T, PCL, DVL>(pc + 16 * pn * PCL, dv, bad);
                __syncthreads();
                row_panel(pn, pr, xs, dv);
                __syncthreads();
                update(pn, pc, xs, dv, true);
            }
        }
        __syncthreads();   // panel buffers done: Es may be rewritten
        launder();
        // E_ln -> Es (row-major, the next step's neighbour), then to global in
        // the sweep's MFMA operand order
#pragma unroll
        for (int q = 0; q < NSLOT; ++q) {
            const int idx = factor_tile<R>(q, w);
            if (idx < 0) continue;
            const int ti = idx / R, tj = idx - ti * R;
#pragma unroll
            for (int t = 0; t < 4; ++t) Es[(16 * ti + Mfma<T>::row(lane, t)) * LDE + 16 * tj + li] = tile[q][t];
        }
        __syncthreads();
        T* El = E + (int64_t)ln * BP * BP;
        for (int o = tid; o < BP * BP; o += kFactorThreads) {
            const int kk = o % NKS, t = o / NKS;
            const int lnn = t & 63, rt = t >> 6;
            El[o] = Es[(16 * rt + (lnn & 15)) * LDE + 4 * kk + (lnn >> 4)];
        }
        // the next line needs one new cell row: ln + 2 (top, replacing row ln)
        // or ln - 1 (bottom, replacing row ln + 1); prefetch the one after
        if (KIND == kElliptic && !MID && tid < L && l + 1 < nsteps) {
            const int rnew = dir > 0 ? ln + 2 : ln - 1;
            crow[(rnew & 1) * (kMaxLine + 1) + tid] = rnext;
            const int rfut = dir > 0 ? ln + 3 : ln - 2;
            if (l + 2 < nsteps) rnext = aL[rfut * L + tid];
        }
    }
    if (bad) raise_flag(flags, 0);
}

// One kernel per line-tile count R (each with its own register allocation);
// plist lists the patches of this R (workgroup x -> patch plist[x]).  The
// halves kernel has grid (patches, 2): y = 0 top, y = 1 bottom; the middle
// kernel one workgroup per patch, after it.
// LDS of the factor for R line tiles: E (BP x (BP+1)) and, aliased, the
// panel buffers (2 BP x 17 + 4 x 16 (BP+1) + 2 x 16 x 17)
template <int R>
constexpr int factor_lds_elems() {
    constexpr int BPR = 16 * R;
    constexpr int PANEL = 2 * BPR * 17 + 4 * 16 * (BPR + 1) + 2 * 16 * 17;
    return BPR * (BPR + 1) > PANEL ? BPR * (BPR + 1) : PANEL;
}

template <typename T, int KIND, int R, bool MID, int SHARE = 1>
__global__ __launch_bounds__(kFactorThreads, SHARE == 2 ? 8 : 1) void factor_kernel(const PatchDesc* pd, const int32_t* __restrict__ plist,
                                                                const double* __restrict__ aL_all, const double* __restrict__ vw,
                                                                double dx, double inv_eps, T* __restrict__ E_all, int32_t* flags) {
    __shared__ T lds[factor_lds_elems<R>()];
    __shared__ double cf[2 * kMaxLine];
    __shared__ double crow[2 * (kMaxLine + 1)];
    const PatchDesc P = pd[plist[blockIdx.x]];
    if (P.bp != 16 * R) {
        if (threadIdx.x == 0) raise_flag(flags, 3);
        return;
    }
    const int dir = MID ? 0 : (blockIdx.y == 0 ? 1 : -1);
    factor_mfma_body<T, KIND, R, MID>(P, aL_all + P.a_off, vw, dx, inv_eps, E_all + P.E_off, lds, cf, crow, dir, flags);
}

// Two line-tile counts in one launch, so that a batch with two adjacent
// counts needs no second stream: workgroups x < nA factor the patches of
// plistA (RA tiles), the others those of plistB (RB tiles), each with its own
// body; LDS and registers are those of the larger.  SHARE = 2 compiles for
// two resident workgroups per compute unit (8 waves per SIMD: a 64-register
// budget, at the price of a few spills).
template <typename T, int KIND, int RA, int RB, bool MID, int SHARE>
__global__ __launch_bounds__(kFactorThreads, SHARE == 2 ? 8 : 1) void factor2_kernel(const PatchDesc* pd, const int32_t* __restrict__ plistA, int nA,
                                                                 const int32_t* __restrict__ plistB, const double* __restrict__ aL_all,
                                                                 const double* __restrict__ vw, double dx, double inv_eps,
                                                                 T* __restrict__ E_all, int32_t* flags) {
    constexpr int LA = factor_lds_elems<RA>(), LB = factor_lds_elems<RB>();
    __shared__ T lds[LA > LB ? LA : LB];
    __shared__ double cf[2 * kMaxLine];
    __shared__ double crow[2 * (kMaxLine + 1)];
    const bool a = (int)blockIdx.x < nA;
    const PatchDesc P = pd[a ? plistA[blockIdx.x] : plistB[blockIdx.x - nA]];
    if (P.bp != 16 * (a ? RA : RB)) {
        if (threadIdx.x == 0) raise_flag(flags, 3);
        return;
    }
    const int dir = MID ? 0 : (blockIdx.y == 0 ? 1 : -1);
    if (a) factor_mfma_body<T, KIND, RA, MID>(P, aL_all + P.a_off, vw, dx, inv_eps, E_all + P.E_off, lds, cf, crow, dir, flags);
    else factor_mfma_body<T, KIND, RB, MID>(P, aL_all + P.a_off, vw, dx, inv_eps, E_all + P.E_off, lds, cf, crow, dir, flags);
}

// ------------------------------------------------------------ sweeps (a5)
// Twisted block sweeps, matching the twisted elimination (m = nl/2; E_l is
// the inverse of the top recursion for l < m, of the bottom recursion for
// l > m, of the two-sided Schur complement at m):
//   forward halves (one kernel, grid (patch, chunk, half)):
//     top     y_0 = r_0,        y_{l+1} = r_{l+1} - Low_{l+1} E_l y_l,  l < m-1;
//             t_top = r_m - Low_m E_{m-1} y_{m-1}
//     bottom  y_{nl-1} = r_{nl-1}, y_{l-1} = r_{l-1} - Up_{l-1} E_l y_l, l > m+1;
//             t_bot = Up_m E_{m+1} y_{m+1}
//   middle and back halves (second kernel, same grid):
//     x_m = E_m (t_top - t_bot) (both halves form it; the top stores it, and
//     nothing of the second kernel reads line m of X)
//     top     x_l = E_l (y_l - Up_l x_{l+1}),   l = m-1 .. 0
//     bottom  x_l = E_l (y_l - Low_l x_{l-1}),  l = m+1 .. nl-1
// The y_l overwrite the right-hand sides in place and the x_l the y_l; t_top
// and t_bot go through a small per-patch buffer, so no workgroup ever waits
// for another.  In FP32 refinement the solution x_l is the correction, and the
// back halves also add it to the FP64 iterate (X64, prefetched one stage
// ahead), which saves a separate accumulation pass.  The products E_l y run
// on MFMA 16x16x4 (8 waves: wave w owns row tile w of E_l and all column
// tiles of the chunk).
//
// Software pipeline: the A operands of the next E_l are loaded into registers
// while line l is processed, and the right-hand side and coupling loads of a
// line are issued before them, so that the in-order load counter never makes
// the stencil wait for the prefetch.
constexpr int kSweepThreads = 512;   // 8 waves: wave w owns row tile w of E_l

template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef float4 type; static constexpr int n = 4; };
template <> struct Vec16<double> { typedef double2 type; static constexpr int n = 2; };

// One patch x column chunk x half, with compile-time line tiles R (bp = 16 R)
// and column tiles NCT (16 NCT samples), so the MFMA loop is straight-line
// code.  TW: this chunk's [2][bp x sp] middle-line couplings (row stride sp).
template <typename T, int KIND, int R, int NCT, int PHASE>
__device__ void sweep_body(const PatchDesc& P, const double* __restrict__ aL, const double* __restrict__ vw, double dx,
                           const T* __restrict__ E, T* __restrict__ X, double* __restrict__ X64, T* __restrict__ TW, int half,
                           T* ybuf, T* wbuf, double* craw, double* cvp, double* cvm) {
    typedef typename Vec16<T>::type V;
    constexpr int VN = Vec16<T>::n;
    constexpr int BP = 16 * R, NKS = 4 * R, NSC = 16 * NCT;
    constexpr int DI = kSweepThreads / NSC;          // rows between a thread's elements
    constexpr int RPT = (BP + DI - 1) / DI;          // elements per thread
    const int tid = threadIdx.x, lane = tid & 63, rt = tid >> 6;
    const bool mf = rt < R;                          // this wave owns a row tile
    const int b = P.b, nl = P.nl, sp = P.sp, L = P.L;
    const int lstride = BP * sp;
    const int m = nl / 2;
    const int dir = half == 0 ? 1 : -1;
    typename Mfma<T>::acc acc[NCT];
    T aC[NKS];
    T rv[RPT];
    double crow = 0.0;
    const int i0 = tid / NSC, jj = tid % NSC;
    T* TWh = TW + (int64_t)half * lstride;

    if (KIND == kKinetic) {
        for (int a = tid; a < b; a += kSweepThreads) {
            const double v = vw[a];
            cvp[a] = v > 0 ? v / dx : 0.0;
            cvm[a] = v < 0 ? -v / dx : 0.0;
        }
    }
    // Per-line copies of the thread's base indices: the empty asm hides their
    // loop invariance so that per-element offsets are recomputed each line
    // instead of being hoisted and kept live.
    int li0 = i0, ljj = jj, llane = lane;
    auto launder = [&]() {
        li0 = i0; ljj = jj; llane = lane;
        asm volatile("" : "+v"(li0), "+v"(ljj), "+v"(llane));
    };
    auto load_line = [&](const T* Xl, T (&dst)[RPT]) {
#pragma unroll
        for (int e = 0; e < RPT; ++e) {
            const int i = li0 + e * DI;
            if (BP % DI == 0 || i < BP) dst[e] = Xl[(uint32_t)(i * sp + ljj)];
        }
    };
    // every wave loads (the ones past the row tiles a copy of the last tile):
    // loads outside branches keep the compiler's wait counts exact
    auto load_A = [&](const T* El) {
        const int rtc = rt < R ? rt : R - 1;
        const V* A = reinterpret_cast<const V*>(El + (uint32_t)((rtc * 64 + llane) * NKS));
#pragma unroll
        for (int q = 0; q < NKS / VN; ++q) {
            const V v = A[q];
#pragma unroll
            for (int u = 0; u < VN; ++u) aC[q * VN + u] = v[u];
        }
    };
    auto mfma = [&]() {
        const int lli = llane & 15, llk = llane >> 4;
#pragma unroll
        for (int c = 0; c < NCT; ++c) acc[c] = Mfma<T>::zero();
        if (mf) {
#pragma unroll
            for (int kk = 0; kk < NKS; ++kk) {
                const T* yb = ybuf + (4 * kk + llk) * NSC + lli;
#pragma unroll
                for (int c = 0; c < NCT; ++c) acc[c] = Mfma<T>::step(aC[kk], yb[16 * c], acc[c]);
            }
        }
    };
    // accumulators -> wbuf, and for a solution line (gdst) to global; with
    // g64 the FP64 iterate of that line (prefetched into pre64) gets += v
    auto load_64 = [&](const double* g64, double (&dst)[NCT][4]) {
        const int lli = llane & 15, rtc = rt < R ? rt : R - 1;
#pragma unroll
        for (int c = 0; c < NCT; ++c)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int i = 16 * rtc + Mfma<T>::row(llane, t), j = 16 * c + lli;
                dst[c][t] = g64[(uint32_t)(i * sp + j)];
            }
    };
    auto store_acc = [&](T* gdst, double* g64, const double (&pre64)[NCT][4]) {
        const int lli = llane & 15;
        if (mf) {
#pragma unroll
            for (int c = 0; c < NCT; ++c)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int i = 16 * rt + Mfma<T>::row(llane, t), j = 16 * c + lli;
                    const T v = acc[c][t];
                    wbuf[i * NSC + j] = v;
                    if (gdst) gdst[(uint32_t)(i * sp + j)] = v;
                    if (g64) g64[(uint32_t)(i * sp + j)] = pre64[c][t] + (double)v;
                }
        }
    };
    // coupling block between two adjacent lines applied to column j of src,
    // row i: Low (A_{l+1,l}) if low, else Up (A_{l,l+1}).  Elliptic: the
    // symmetric tridiagonal block of their shared cell row c: diagonal
    // -(c_i + c_{i+1})/6, off-diagonal (i, i+1) -c_{i+1}/3; craw holds the
    // row already scaled by -1/3
    auto couple = [&](const T* src, int i, int j, bool low) -> double {
        if (KIND == kElliptic) {
            const int im = i > 0 ? i - 1 : 0, ip = i + 1 < BP ? i + 1 : BP - 1;
            const double cm = i > 0 ? craw[i] : 0.0;
            const double cp = i < b - 1 ? craw[i + 1] : 0.0;
            return 0.5 * (craw[i] + craw[i + 1]) * (double)src[i * NSC + j] + cm * (double)src[im * NSC + j] +
                   cp * (double)src[ip * NSC + j];
        } else {
            return -(low ? cvp[i] : cvm[i]) * (double)src[i * NSC + j];
        }
    };

    // Register sets of prefetched loads alternate between consecutive steps
    // (the step body is instantiated twice per loop trip), so that no copy of
    // a register with a load in flight makes the wave wait for it early.
    double nopre[NCT][4] = {};
    if constexpr (PHASE == 0) {
        // ---- forward half: lines ln0, ln0 + dir, ...; the last one couples into m
        const int nst = half == 0 ? m : nl - 1 - m;
        const int ln0 = half == 0 ? 0 : nl - 1;
        const bool low = half == 0;   // top: Low_{l+1} (line below from above); bottom: Up_{l-1}
        T rvA[RPT], rvB[RPT];
        launder();
        if (nst <= 0) {
            // no line in this half: t_top = r_m, t_bot = 0
            if (half == 0) load_line(X + m * lstride, rvA);
#pragma unroll
            for (int e = 0; e < RPT; ++e) {
                const int i = li0 + e * DI;
                if (BP % DI == 0 || i < BP) TWh[(uint32_t)(i * sp + ljj)] = (half == 0 && i < b) ? rvA[e] : T(0);
            }
            return;
        }
        // step k works on line ln = ln0 + dir k and its successor nx = ln + dir
        // (m after the last step); the successor's right-hand side r_nx and the
        // shared cell row are loaded during the step before, after its products
        // (so that the products' operand waits never cover them), E_nx likewise
        auto sub_of = [&](int k) { return k + 1 < nst || half == 0; };   // the top's last step carries r_m
        load_line(X + ln0 * lstride, rvA);                 // y_{ln0} = r_{ln0}
#pragma unroll
        for (int e = 0; e < RPT; ++e) {
            const int i = li0 + e * DI;
            if (BP % DI == 0 || i < BP) ybuf[i * NSC + ljj] = rvA[e];
        }
        load_A(E + (int64_t)ln0 * BP * BP);
        double crA = 0.0, crB = 0.0;
        if (sub_of(0)) load_line(X + (ln0 + dir) * lstride, rvA);
        if (KIND == kElliptic) crA = aL[(dir > 0 ? ln0 + 1 : ln0) * L + min(tid, b)];
        lds_barrier();
        auto step = [&](int k, T (&rc)[RPT], T (&rn)[RPT], double& cc, double& cn) {
            launder();
            const int ln = ln0 + dir * k, nx = ln + dir;
            const bool more = k + 1 < nst;
            const bool sub = sub_of(k);
            mfma();                                                                   // w = E_ln y_ln
            // r of the next step, its cell row and E (unconditional, clamped to
            // lines that exist when there is no next step)
            load_line(X + ((more && sub_of(k + 1)) ? nx + dir : nx) * lstride, rn);
            if (KIND == kElliptic) cn = aL[(more ? (dir > 0 ? nx + 1 : nx) : (dir > 0 ? ln + 1 : ln)) * L + min(tid, b)];
            load_A(E + (int64_t)(more ? nx : ln) * BP * BP);
            store_acc(nullptr, nullptr, nopre);
            if (KIND == kElliptic && tid <= b) craw[tid] = cc * (-1.0 / 3.0);
            lds_barrier();
            T* dst = more ? X + nx * lstride : TWh;
#pragma unroll
            for (int e = 0; e < RPT; ++e) {
                const int i = li0 + e * DI;
                if (BP % DI == 0 || i < BP) {
                    const double cw = couple(wbuf, i, ljj, low);
                    const double v = sub ? (double)rc[e] - cw : cw;
                    const T y = i < b ? (T)v : T(0);
                    dst[(uint32_t)(i * sp + ljj)] = y;
                    if (more) ybuf[i * NSC + ljj] = y;
                }
            }
            lds_barrier();
        };
        for (int k = 0; k < nst; k += 2) {
            step(k, rvA, rvB, crA, crB);
            if (k + 1 < nst) step(k + 1, rvB, rvA, crB, crA);
        }
    } else {
        // ---- middle line, then the back half; step k solves line
        // ln = m - dir (k + 1) from pv = ln + dir.  Its right-hand side y_ln, the
        // shared cell row and (FP32 refinement) the FP64 iterate of the line are
        // loaded one step ahead, E_ln during the step before.
        // PHASE 2 is the first solve of a refinement: the FP64 iterate holds
        // nothing yet and is written, not accumulated (pre64 stays zero).
        launder();
        constexpr bool kAccum = PHASE == 1;
        double pre64[NCT][4] = {}, pre64n[NCT][4] = {};
        load_A(E + (int64_t)m * BP * BP);
        const bool acc64 = X64 && half == 0;   // line m's iterate is updated once, by the top half
        if (kAccum && acc64) load_64(X64 + m * lstride, pre64);
#pragma unroll
        for (int e = 0; e < RPT; ++e) {
            const int i = li0 + e * DI;
            if (BP % DI == 0 || i < BP) {
                const double v = (double)TW[(uint32_t)(i * sp + ljj)] - (double)TW[lstride + (uint32_t)(i * sp + ljj)];
                ybuf[i * NSC + ljj] = i < b ? (T)v : T(0);
            }
        }
        const int nst = half == 0 ? m : nl - 1 - m;
        const bool low = half != 0;   // top: Up_l x_{l+1}; bottom: Low_l x_{l-1}
        if (nst > 0) {
            const int l1 = m - dir;
            load_line(X + l1 * lstride, rv);
            if (KIND == kElliptic && tid <= b) crow = aL[(dir > 0 ? m : l1) * L + tid];
            if (kAccum && X64) load_64(X64 + l1 * lstride, pre64n);
        }
        lds_barrier();
        mfma();
        if (nst > 0) load_A(E + (int64_t)(m - dir) * BP * BP);        // the first back line, one step ahead
        // x_m (identical in both halves).  With an FP64 iterate (refinement) the
        // FP32 solution is not stored: the iterate takes it, and the line
        // vectors are next overwritten by the residual.
        store_acc(half == 0 && !X64 ? X + m * lstride : nullptr, acc64 ? X64 + m * lstride : nullptr, pre64);
        lds_barrier();
        for (int k = 0; k < nst; ++k) {
            launder();
            const int ln = m - dir * (k + 1);
            const bool more = k + 1 < nst;
#pragma unroll
            for (int c = 0; c < NCT; ++c)
#pragma unroll
                for (int t = 0; t < 4; ++t) pre64[c][t] = pre64n[c][t];
            T rvn[RPT];
            double crown = 0.0;
            if (more) {
                const int l2 = ln - dir;
                load_line(X + l2 * lstride, rvn);                                     // y of the next step
                if (KIND == kElliptic && tid <= b) crown = aL[(dir > 0 ? ln : l2) * L + tid];
                if (kAccum && X64) load_64(X64 + l2 * lstride, pre64n);
            }
            if (KIND == kElliptic && tid <= b) craw[tid] = crow * (-1.0 / 3.0);
            lds_barrier();
#pragma unroll
            for (int e = 0; e < RPT; ++e) {
                const int i = li0 + e * DI;
                if (BP % DI == 0 || i < BP) {
                    const double v = (double)rv[e] - couple(wbuf, i, ljj, low);
                    ybuf[i * NSC + ljj] = i < b ? (T)v : T(0);
                }
            }
            lds_barrier();
            mfma();                                                                    // x_ln = E_ln z
            if (more) load_A(E + (int64_t)(ln - dir) * BP * BP);                     // E of the next line
            store_acc(X64 ? nullptr : X + ln * lstride, X64 ? X64 + ln * lstride : nullptr, pre64);
#pragma unroll
            for (int e = 0; e < RPT; ++e) rv[e] = rvn[e];
            crow = crown;
            lds_barrier();
        }
    }
}

// grid (patch, column chunk of 16*NCT samples, half); sp of every patch is a
// multiple of the chunk.
template <typename T, int KIND, int NCT, int PHASE>
__global__ __launch_bounds__(kSweepThreads) void sweep_kernel(const PatchDesc* pd, int p0, const double* __restrict__ aL_all,
                                                              const double* __restrict__ vw, double dx, const T* __restrict__ E_all,
                                                              T* __restrict__ X_all, double* __restrict__ X64_all, T* __restrict__ TW_all,
                                                              const int32_t* __restrict__ conv, int32_t* flags) {
    __shared__ T ybuf[kMaxLine * 16 * NCT];
    __shared__ T wbuf[kMaxLine * 16 * NCT];
    __shared__ double craw[kMaxLine + 1];
    __shared__ double cvp[kMaxLine], cvm[kMaxLine];
    const int p = p0 + blockIdx.x;
    if (conv && conv[p]) return;
    const PatchDesc P = pd[p];
    const int s0 = blockIdx.y * 16 * NCT;
    if (s0 >= P.sp) return;
    const int half = blockIdx.z;
    const double* aL = aL_all + P.a_off;
    const T* E = E_all + P.E_off;
    T* X = X_all + P.x_off + s0;
    T* TW = TW_all + P.tw_off + s0;
    double* X64 = X64_all ? X64_all + P.x_off + s0 : nullptr;
#define MSRS_SWB(RR) sweep_body<T, KIND, RR, NCT, PHASE>(P, aL, vw, dx, E, X, X64, TW, half, ybuf, wbuf, craw, cvp, cvm)
    if (KIND == kKinetic) {
        switch (P.bp >> 4) {
            case 1: MSRS_SWB(1); break;
            case 2: MSRS_SWB(2); break;
            case 3: MSRS_SWB(3); break;
            case 4: MSRS_SWB(4); break;
            default: if (threadIdx.x == 0) raise_flag(flags, 3); break;
        }
        return;
    }
    switch (P.bp >> 4) {
        case 1: MSRS_SWB(1); break;
        case 2: MSRS_SWB(2); break;
        case 3: MSRS_SWB(3); break;
        case 4: MSRS_SWB(4); break;
        case 5: MSRS_SWB(5); break;
        case 6: MSRS_SWB(6); break;
        case 7: MSRS_SWB(7); break;
        case 8: MSRS_SWB(8); break;
        default: if (threadIdx.x == 0) raise_flag(flags, 3); break;
    }
#undef MSRS_SWB
}

// ------------------------------------------------------------ FP64 residual (a6)
// r = rhs - A x64 per interior unknown, grid (patch, chunk of lines); r is
// written to x32 (the next correction's right-hand side) unless x32 is null.
template <int KIND>
__global__ __launch_bounds__(kThreads) void residual_kernel(const PatchDesc* pd, int p0, const double* __restrict__ aL_all,
                                                            const double* __restrict__ om, const double* __restrict__ vw,
                                                            double dx, double inv_eps, const double* __restrict__ x64_all,
                                                            float* __restrict__ x32_all, const int32_t* __restrict__ conv,
                                                            double* __restrict__ part, int maxch) {
    __shared__ double red[kThreads];
    const int p = p0 + blockIdx.x;
    if (conv && conv[p]) return;
    const PatchDesc P = pd[p];
    const int l0 = blockIdx.y * kChunkLines;
    if (l0 >= P.nl) return;
    const int l1 = min(P.nl, l0 + kChunkLines);
    const double* aL = aL_all + P.a_off;
    const double* O = om + P.om_off;
    const int sp = P.sp, bp = P.bp, b = P.b, nl = P.nl;
    const double* X = x64_all + P.x_off;
    float* X32 = x32_all ? x32_all + P.x_off : nullptr;
    const int64_t lstride = (int64_t)bp * sp;
    const LineMap m(sp);
    const int c = m.col;
    double ssum = 0.0;
    auto xv = [&](int l, int i) -> double { return X[(int64_t)l * lstride + (int64_t)i * sp + c]; };
    if constexpr (KIND == kElliptic) {
        for (int l = l0; l < l1; ++l) {
            for (int i = m.row0; m.active && i < bp; i += m.rows) {
                double r = 0.0;
                if (i < b && c < P.s) {
                    const int pp = i + 1, q = l + 1;
#pragma unroll
                    for (int dq = -1; dq <= 1; ++dq)
#pragma unroll
                        for (int dp = -1; dp <= 1; ++dp) {
                            const int p2 = pp + dp, q2 = q + dq;
                            double u;
                            if (p2 == 0 || p2 == P.L || q2 == 0 || q2 == P.Qn) {
                                int ii, jj;
                                line_to_phys(P, p2, q2, ii, jj);
                                u = O[(int64_t)c * P.nb + bidx_ccw(ii, jj, P.cx, P.cy)];
                            } else {
                                u = xv(q2 - 1, p2 - 1);
                            }
                            r -= q1_coef(aL, P.L, pp, q, dp, dq) * u;
                        }
                }
                if (X32) X32[(int64_t)l * lstride + (int64_t)i * sp + c] = (float)r;
                ssum += r * r;
            }
        }
    } else {
        // thread (row group g, column c): cells l0 + g, l0 + g + rows, ...; all ordinates of a cell
        const int h = b / 2;
        // anisotropic scattering: the gain table K (b x b) staged in LDS once, and
        // the gain of 16 ordinates at a time, so that a cell's values are read
        // once per 16 ordinates rather than once per ordinate
        __shared__ double Ks[kMaxHgVel * kMaxHgVel];
        if (P.hg) {
            for (int o = threadIdx.x; o < b * b; o += kThreads) Ks[o] = vw[3 * b + o];
            __syncthreads();
        }
        for (int l = l0 + m.row0; m.active && l < l1; l += m.rows) {
            double rho = 0.0;
            if (c < P.s && !P.hg)
                for (int j = 0; j < b; ++j) rho += 0.5 * vw[b + j] * xv(l, j);
            const double sg = aL[l] * inv_eps;
            for (int i0 = 0; i0 < bp; i0 += 16) {
                double gain[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) gain[u] = 0.0;
                if (P.hg && c < P.s) {
                    for (int j = 0; j < b; ++j) {
                        const double xj = xv(l, j);
#pragma unroll
                        for (int u = 0; u < 16; ++u) gain[u] += Ks[min(i0 + u, b - 1) * b + j] * xj;
                    }
                }
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int i = i0 + u;
                    double r = 0.0;
                    if (i < b && c < P.s) {
                        const double vi = vw[i];
                        double acc;
                        if (P.hg) {
                            // gain sum_j K_ij f_j, loss lambda_i f_i
                            acc = (fabs(vi) / dx + sg * vw[2 * b + i]) * xv(l, i) - sg * gain[u];
                        } else {
                            acc = (fabs(vi) / dx + sg) * xv(l, i) - sg * rho;
                        }
                        if (vi > 0) acc -= vi / dx * (l > 0 ? xv(l - 1, i) : O[(int64_t)c * P.nb + (i - h)]);
                        if (vi < 0) acc -= -vi / dx * (l < nl - 1 ? xv(l + 1, i) : O[(int64_t)c * P.nb + h + i]);
                        r = -acc;
                    }
                    if (X32) X32[(int64_t)l * lstride + (int64_t)i * sp + c] = (float)r;
                    ssum += r * r;
                }
            }
        }
    }
    partial_column_sums(ssum, m, sp, red, part + ((int64_t)p * maxch + blockIdx.y) * kMaxSamples);
}

// Elliptic residual, sliding-window form: thread (segment g, line l0 + lo,
// sample c) walks down its segment of the line with the 3 x 3 stencil window
// of x in registers (three new loads per node instead of nine) and the
// coefficient cell rows of the chunk staged in LDS (two new cells per node),
// so the loads scale with the output instead of nine-fold.  A line splits
// into as many segments as the workgroup has threads to spare for its sample
// count (2 at 32 samples): shorter dependent walks, more loads in flight.
// Same arithmetic per node as the generic kernel.
constexpr int kResThreads = kChunkLines * kMaxSamples;   // 8 lines x up to 64 samples
__global__ __launch_bounds__(kResThreads) void residual_ell_kernel(const PatchDesc* pd, int p0, const double* __restrict__ aL_all,
                                                                   const double* __restrict__ om, const double* __restrict__ x64_all,
                                                                   float* __restrict__ x32_all, const int32_t* __restrict__ conv,
                                                                   double* __restrict__ part, int maxch) {
    __shared__ double cell[(kChunkLines + 1) * (kMaxLine + 1)];
    __shared__ double red[kResThreads];
    const int p = p0 + blockIdx.x;
    if (conv && conv[p]) return;
    const PatchDesc P = pd[p];
    const int l0 = blockIdx.y * kChunkLines;
    if (l0 >= P.nl) return;
    const int l1 = min(P.nl, l0 + kChunkLines);
    const double* aL = aL_all + P.a_off;
    const double* O = om + P.om_off;
    const int sp = P.sp, bp = P.bp, b = P.b, L = P.L, Qn = P.Qn;
    const double* X = x64_all + P.x_off;
    float* X32 = x32_all ? x32_all + P.x_off : nullptr;
    const int64_t lstride = (int64_t)bp * sp;
    const int tid = threadIdx.x;
    // cell rows l0 .. l1 (line l is bounded by cell rows l and l + 1)
    for (int o = tid; o < (l1 - l0 + 1) * L; o += kResThreads) cell[o] = aL[(int64_t)l0 * L + o];
    __syncthreads();
    const int nseg = max(1, kResThreads / (sp * kChunkLines));
    const int c = tid % sp, lo = (tid / sp) % kChunkLines, g = tid / (sp * kChunkLines);
    const bool active = lo < l1 - l0 && g < nseg;
    // nodes pa .. pb of the line (1-based along it)
    const int pa = 1 + (g * b) / nseg, pb = ((g + 1) * b) / nseg;
    double ssum = 0.0;
    if (active) {
        const int l = l0 + lo, q = l + 1;
        float* R32 = X32 ? X32 + (int64_t)l * lstride + c : nullptr;
        if (c < P.s) {
            // u(q2, p2): interior nodes from x, nodes on the buffered patch's boundary from Omega
            auto u = [&](int q2, int p2) -> double {
                if (p2 == 0 || p2 == L || q2 == 0 || q2 == Qn) {
                    int ii, jj;
                    line_to_phys(P, p2, q2, ii, jj);
                    return O[(int64_t)c * P.nb + bidx_ccw(ii, jj, P.cx, P.cy)];
                }
                return X[(int64_t)(q2 - 1) * lstride + (int64_t)(p2 - 1) * sp + c];
            };
            const double* cS = cell + (l - l0) * L;        // cell row q - 1
            const double* cN = cell + (l - l0 + 1) * L;    // cell row q
            // window columns p-1, p, p+1 of node rows q-1, q, q+1
            double wm[3], w0[3], wp[3];
            wm[0] = u(q - 1, pa - 1); w0[0] = u(q, pa - 1); wp[0] = u(q + 1, pa - 1);
            wm[1] = u(q - 1, pa); w0[1] = u(q, pa); wp[1] = u(q + 1, pa);
            double SW = cS[pa - 1], NW = cN[pa - 1];
            for (int pp = pa; pp <= pb; ++pp) {
                wm[2] = u(q - 1, pp + 1);
                w0[2] = u(q, pp + 1);
                wp[2] = u(q + 1, pp + 1);
                const double SE = cS[pp], NE = cN[pp];
                // the terms of q1_coef over dq, dp = -1, 0, 1, in that order; the
                // divisions by 3 and 6 as products with the rounded reciprocals
                constexpr double k3 = 1.0 / 3.0, k6 = 1.0 / 6.0;
                double r = 0.0;
                r += (SW * k3) * wm[0];
                r += ((SE + SW) * k6) * wm[1];
                r += (SE * k3) * wm[2];
                r += ((NW + SW) * k6) * w0[0];
                r -= ((2.0 / 3.0) * (NE + NW + SW + SE)) * w0[1];
                r += ((NE + SE) * k6) * w0[2];
                r += (NW * k3) * wp[0];
                r += ((NE + NW) * k6) * wp[1];
                r += (NE * k3) * wp[2];
                if (R32) R32[(int64_t)(pp - 1) * sp] = (float)r;
                ssum += r * r;
                wm[0] = wm[1]; wm[1] = wm[2];
                w0[0] = w0[1]; w0[1] = w0[2];
                wp[0] = wp[1]; wp[1] = wp[2];
                SW = SE; NW = NE;
            }
            if (R32 && g == nseg - 1)
                for (int i = b; i < bp; ++i) R32[(int64_t)i * sp] = 0.0f;
        } else if (R32 && g == 0) {
            for (int i = 0; i < bp; ++i) R32[(int64_t)i * sp] = 0.0f;
        }
    }
    // per-sample sums over the chunk's lines and segments, fixed order
    red[tid] = active ? ssum : 0.0;
    __syncthreads();
    if (tid < sp) {
        double s = 0.0;
        for (int gg = 0; gg < nseg; ++gg)
            for (int r = 0; r < l1 - l0; ++r) s += red[(gg * kChunkLines + r) * sp + tid];
        part[((int64_t)p * maxch + blockIdx.y) * kMaxSamples + tid] = s;
    }
}


// Per patch: sum the chunk partials.  which = 0: ||rhs_j||^2 -> rn[0..sp).
// which = 1: ||r_j||^2 -> rn[sp..2sp), relres[p] = max_j ||r_j||/||rhs_j||,
// and (if conv) conv[p] = 1, iters[p] = it + 1 once relres[p] <= tol.
__global__ __launch_bounds__(64) void norms_kernel(const PatchDesc* pd, int p0, const double* __restrict__ part, int maxch,
                                                   double* __restrict__ rn_all, int which, int32_t* __restrict__ conv,
                                                   double* __restrict__ relres, int32_t* __restrict__ iters, int it, double tol) {
    const int p = p0 + blockIdx.x;
    if (which == 1 && conv && conv[p]) return;
    const PatchDesc P = pd[p];
    const int nch = (P.nl + kChunkLines - 1) / kChunkLines;
    const int t = threadIdx.x;
    double* rn = rn_all + P.rn_off;
    double s2 = 0.0;
    if (t < P.sp)
        for (int ch = 0; ch < nch; ++ch) s2 += part[((int64_t)p * maxch + ch) * kMaxSamples + t];
    if (which == 0) {
        if (t < P.sp) rn[t] = s2;
        return;
    }
    double ratio = 0.0;
    if (t < P.sp) {
        rn[P.sp + t] = s2;
        const double rh = rn[t];
        if (t < P.s) ratio = rh > 0 ? sqrt(s2 / rh) : (s2 > 0 ? INFINITY : 0.0);
    }
    for (int off = 32; off > 0; off >>= 1) ratio = fmax(ratio, __shfl_xor(ratio, off, 64));
    if (t == 0) {
        relres[p] = ratio;
        if (conv && ratio <= tol) { conv[p] = 1; iters[p] = it + 1; }
    }
}

// ------------------------------------------------------------ restriction (a7)
// grid (patch, tile of kRestrictRows rows of Y), every sample column of the
// tile.  The iterate is sample-fastest and Y column-major (row-fastest), so
// the tile passes through LDS: both the gather and the store are contiguous.
constexpr int kRestrictRows = 64;
template <int KIND>
__global__ __launch_bounds__(kThreads) void restrict_kernel(const PatchDesc* pd, int p0, const double* __restrict__ x64_all,
                                                            const double* __restrict__ om, const double* __restrict__ vw,
                                                            double* __restrict__ Y_all) {
    constexpr int LDT = kMaxSamples + 1;
    __shared__ double tile[kRestrictRows * LDT];
    const PatchDesc P = pd[p0 + blockIdx.x];
    const int r0 = blockIdx.y * kRestrictRows;
    if (r0 >= P.nrows) return;
    const int nr = min(kRestrictRows, P.nrows - r0), ns = P.s;
    const double* X = x64_all + P.x_off;
    const double* O = om + P.om_off;
    double* Y = Y_all + P.Y_off;
    const int64_t lstride = (int64_t)P.bp * P.sp;
    // gather: 32 lanes along the samples, 8 rows at a time; the row's
    // position is resolved once per row, not per value
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int rr = ty; rr < nr; rr += kThreads / 32) {
        const int row = r0 + rr;
        if (KIND == kElliptic) {
            const int W = P.nH + 1;
            const int jj = row / W, ii = row - jj * W;
            const int ip = P.kx0 - P.x0 + ii, jp = P.ky0 - P.y0 + jj;
            const int pl = P.trans ? jp : ip, ql = P.trans ? ip : jp;
            const bool inner = pl >= 1 && pl <= P.L - 1 && ql >= 1 && ql <= P.Qn - 1;
            const double* src = inner ? X + (int64_t)(ql - 1) * lstride + (int64_t)(pl - 1) * P.sp : nullptr;
            const int bi = inner ? 0 : bidx_ccw(ip, jp, P.cx, P.cy);
            for (int c = tx; c < ns; c += 32) tile[rr * LDT + c] = inner ? src[c] : O[(int64_t)c * P.nb + bi];
        } else {
            const int nv = P.b, h = nv / 2;
            const int cell = row / nv, j = row - cell * nv;
            const int lc = P.kx0 - 1 + cell - P.x0;
            for (int c = tx; c < ns; c += 32) {
                double v;
                if (lc >= 0 && lc < P.cx) v = X[(int64_t)lc * lstride + (int64_t)j * P.sp + c];
                else if (lc < 0) v = vw[j] > 0 ? O[(int64_t)c * P.nb + (j - h)] : 0.0;
                else v = vw[j] < 0 ? O[(int64_t)c * P.nb + h + j] : 0.0;
                tile[rr * LDT + c] = v;
            }
        }
    }
    __syncthreads();
    // store: 64 lanes along the rows of one column, 4 columns at a time
    const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
    if (lx < nr)
        for (int c = ly; c < ns; c += kThreads / 64) Y[(int64_t)c * P.nrows + r0 + lx] = tile[lx * LDT + c];
}

__global__ void clear_kernel(int32_t* a, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) a[i] = 0;
}

// ------------------------------------------------------------ launchers
static inline double dx_of(const Ctx& c) { return 1.0 / c.N; }

void launch_gather_elliptic(Ctx& c, const double* a, int p0, int p1) {
    StageTimer t(c, MSRS_K_ASSEMBLE);
    hipLaunchKernelGGL(gather_elliptic_kernel, dim3(p1 - p0), dim3(kThreads), 0, c.stream, c.dp, p0, a, c.N, c.aL, c.dflags);
}

void launch_gather_kinetic(Ctx& c, const double* sigma, int p0, int p1) {
    StageTimer t(c, MSRS_K_ASSEMBLE);
    hipLaunchKernelGGL(gather_kinetic_kernel, dim3(p1 - p0), dim3(kThreads), 0, c.stream, c.dp, p0, sigma, c.aL, c.dflags);
}

void launch_omega(Ctx& c, const double* user, int p0, int p1) {
    StageTimer t(c, MSRS_K_OMEGA);
    int maxs = 0;
    for (int p = p0; p < p1; ++p) maxs = std::max(maxs, c.hp[p].s);
    hipLaunchKernelGGL(omega_kernel, dim3(p1 - p0, (maxs + 15) / 16), dim3(kThreads), 0, c.stream, c.dp, p0, user, c.om, c.seed);
}

static int max_chunks(const Ctx& c, int p0, int p1) {
    int m = 1;
    for (int p = p0; p < p1; ++p) m = std::max(m, (c.hp[p].nl + kChunkLines - 1) / kChunkLines);
    return m;
}

void launch_lift(Ctx& c, int p0, int p1) {
    StageTimer t(c, MSRS_K_LIFT);
    const bool ir = c.prec == MSRS_PREC_FP32_IR;
    const dim3 grid(p1 - p0, max_chunks(c, p0, p1));
    if (c.kind == kElliptic) {
        if (ir) hipLaunchKernelGGL((lift_kernel<kElliptic, float>), grid, dim3(kThreads), 0, c.stream, c.dp, p0, c.aL, c.om, c.vw, dx_of(c), c.x32, c.part, c.maxch);
        else hipLaunchKernelGGL((lift_kernel<kElliptic, double>), grid, dim3(kThreads), 0, c.stream, c.dp, p0, c.aL, c.om, c.vw, dx_of(c), c.x64, c.part, c.maxch);
    } else {
        if (ir) hipLaunchKernelGGL((lift_kernel<kKinetic, float>), grid, dim3(kThreads), 0, c.stream, c.dp, p0, c.aL, c.om, c.vw, dx_of(c), c.x32, c.part, c.maxch);
        else hipLaunchKernelGGL((lift_kernel<kKinetic, double>), grid, dim3(kThreads), 0, c.stream, c.dp, p0, c.aL, c.om, c.vw, dx_of(c), c.x64, c.part, c.maxch);
    }
    hipLaunchKernelGGL(norms_kernel, dim3(p1 - p0), dim3(64), 0, c.stream, c.dp, p0, c.part, c.maxch, c.rn, 0, (int32_t*)nullptr,
                       (double*)nullptr, (int32_t*)nullptr, 0, 0.0);
}

template <typename T, int KIND>
static void launch_factor_r(Ctx& c, int R, hipStream_t st, const int32_t* plist, int n) {
    const double inv_eps = 1.0 / c.eps;
    T* E = (T*)c.E;
    // both halves at once, then the middle lines
#define MSRS_FACTOR_SH(RR, SH)                                                                                                    \
    do {                                                                                                                        \
        hipLaunchKernelGGL((factor_kernel<T, KIND, RR, false, SH>), dim3(n, 2), dim3(kFactorThreads), 0, st, c.dp, plist, c.aL,    \
                           c.vw, dx_of(c), inv_eps, E, c.dflags);                                                               \
        hipLaunchKernelGGL((factor_kernel<T, KIND, RR, true, SH>), dim3(n), dim3(kFactorThreads), 0, st, c.dp, plist, c.aL, c.vw, \
                           dx_of(c), inv_eps, E, c.dflags);                                                                     \
    } while (0)
    // the factor share applies to the FP32 kernels
#define MSRS_FACTOR(RR)                                                           \
    do {                                                                          \
        if constexpr (sizeof(T) == 4) {                                           \
            if (c.factor_share == 2) MSRS_FACTOR_SH(RR, 2);                       \
            else MSRS_FACTOR_SH(RR, 1);                                           \
        } else {                                                                  \
            MSRS_FACTOR_SH(RR, 1);                                                \
        }                                                                         \
    } while (0)
    switch (R) {
        case 1: MSRS_FACTOR(1); break;
        case 2: MSRS_FACTOR(2); break;
        case 3: MSRS_FACTOR(3); break;
        case 4: MSRS_FACTOR(4); break;
        case 5: if constexpr (KIND == kElliptic) MSRS_FACTOR(5); break;
        case 6: if constexpr (KIND == kElliptic) MSRS_FACTOR(6); break;
        case 7: if constexpr (KIND == kElliptic) MSRS_FACTOR(7); break;
        case 8: if constexpr (KIND == kElliptic) MSRS_FACTOR(8); break;
        default: break;
    }
#undef MSRS_FACTOR
#undef MSRS_FACTOR_SH
}

static void launch_factor_group(Ctx& c, int R, hipStream_t st, const int32_t* plist, int n) {
    const bool ir = c.prec == MSRS_PREC_FP32_IR;
    if (c.kind == kElliptic) {
        if (ir) launch_factor_r<float, kElliptic>(c, R, st, plist, n);
        else launch_factor_r<double, kElliptic>(c, R, st, plist, n);
    } else {
        if (ir) launch_factor_r<float, kKinetic>(c, R, st, plist, n);
        else launch_factor_r<double, kKinetic>(c, R, st, plist, n);
    }
}

// FP32 batch with two adjacent line-tile counts ra = rb + 1: one launch for
// the halves and one for the middle lines, on the handle's stream.
template <int KIND>
static bool launch_factor_pair(Ctx& c, int ra, int rb) {
    if (c.prec != MSRS_PREC_FP32_IR || ra != rb + 1) return false;
    const int nA = c.rgroup_n[ra], nB = c.rgroup_n[rb];
    const double inv_eps = 1.0 / c.eps;
    float* E = (float*)c.E;
#define MSRS_FACTOR2_SH(RA, RB, SH)                                                                                               \
    do {                                                                                                                        \
        hipLaunchKernelGGL((factor2_kernel<float, KIND, RA, RB, false, SH>), dim3(nA + nB, 2), dim3(kFactorThreads), 0, c.stream,    \
                           c.dp, c.rgroup[RA], nA, c.rgroup[RB], c.aL, c.vw, dx_of(c), inv_eps, E, c.dflags);                   \
        hipLaunchKernelGGL((factor2_kernel<float, KIND, RA, RB, true, SH>), dim3(nA + nB), dim3(kFactorThreads), 0, c.stream,        \
                           c.dp, c.rgroup[RA], nA, c.rgroup[RB], c.aL, c.vw, dx_of(c), inv_eps, E, c.dflags);                   \
    } while (0)
#define MSRS_FACTOR2(RA, RB)                                 \
    do {                                                     \
        if (c.factor_share == 2) MSRS_FACTOR2_SH(RA, RB, 2); \
        else MSRS_FACTOR2_SH(RA, RB, 1);                     \
    } while (0)
    if constexpr (KIND == kElliptic) {
        switch (ra) {
            case 2: MSRS_FACTOR2(2, 1); return true;
            case 3: MSRS_FACTOR2(3, 2); return true;
            case 4: MSRS_FACTOR2(4, 3); return true;
            case 5: MSRS_FACTOR2(5, 4); return true;
            case 6: MSRS_FACTOR2(6, 5); return true;
            case 7: MSRS_FACTOR2(7, 6); return true;
            case 8: MSRS_FACTOR2(8, 7); return true;
            default: return false;
        }
    } else {
        switch (ra) {
            case 2: MSRS_FACTOR2(2, 1); return true;
            case 3: MSRS_FACTOR2(3, 2); return true;
            case 4: MSRS_FACTOR2(4, 3); return true;
            default: return false;
        }
    }
#undef MSRS_FACTOR2
#undef MSRS_FACTOR2_SH
}

// Patches are grouped by line-tile count R; each group runs its own kernel.
// A single patch (reference mode) launches on the handle's stream.  A batch
// with one count, or (FP32) two adjacent ones, launches on the handle's
// stream; otherwise it forks one stream per group from the handle's stream
// and joins back.
void launch_factor(Ctx& c, int p0, int p1) {
    StageTimer t(c, MSRS_K_FACTOR);
    if (p1 - p0 == 1) {
        launch_factor_group(c, c.hp[p0].bp / 16, c.stream, c.pid + p0, 1);
        return;
    }
    int ng = 0, rmax = 0, rmin = 9;
    for (int g = 0; g < 9; ++g)
        if (c.rgroup_n[g] > 0) {
            ++ng;
            rmax = std::max(rmax, g);
            rmin = std::min(rmin, g);
        }
    if (ng == 2 && (c.kind == kElliptic ? launch_factor_pair<kElliptic>(c, rmax, rmin) : launch_factor_pair<kKinetic>(c, rmax, rmin)))
        return;
    if (ng <= 1) {
        for (int g = 0; g < 9; ++g)
            if (c.rgroup_n[g]) launch_factor_group(c, g, c.stream, c.rgroup[g], c.rgroup_n[g]);
        return;
    }
    MSRS_HIP_CHECK(hipEventRecord(c.ev_fork, c.stream));
    int k = 0;
    for (int g = 0; g < 9; ++g) {
        if (!c.rgroup_n[g]) continue;
        hipStream_t st = c.aux[k];
        MSRS_HIP_CHECK(hipStreamWaitEvent(st, c.ev_fork, 0));
        launch_factor_group(c, g, st, c.rgroup[g], c.rgroup_n[g]);
        MSRS_HIP_CHECK(hipEventRecord(c.ev_join[k], st));
        if (!c.defer_factor_join) MSRS_HIP_CHECK(hipStreamWaitEvent(c.stream, c.ev_join[k], 0));
        ++k;
    }
    if (c.defer_factor_join) c.n_join = k;
}

void join_factor(Ctx& c) {
    for (int k = 0; k < c.n_join; ++k) MSRS_HIP_CHECK(hipStreamWaitEvent(c.stream, c.ev_join[k], 0));
    c.n_join = 0;
}

// samples per sweep workgroup: the largest of {64, 32, 16} (FP64 at most 32,
// a register budget) not above the requested width that divides every sp
static int sweep_chunk(const Ctx& c, int p0, int p1, bool fp32) {
    int want = fp32 ? c.sweep_cols32 : std::min(c.sweep_cols64, 32);
    for (int sc : {64, 32, 16}) {
        if (sc > want) continue;
        bool ok = true;
        for (int p = p0; p < p1; ++p) ok = ok && (c.hp[p].sp % sc == 0);
        if (ok) return sc;
    }
    return 16;
}

void launch_sweep(Ctx& c, int p0, int p1, bool fp32, bool first) {
    StageTimer t(c, MSRS_K_SWEEP);
    int maxsp = 0;
    for (int p = p0; p < p1; ++p) maxsp = std::max(maxsp, c.hp[p].sp);
    const int sc = sweep_chunk(c, p0, p1, fp32);
    const dim3 grid(p1 - p0, maxsp / sc, 2), blk(kSweepThreads);
    const int32_t* conv = fp32 ? c.conv : nullptr;
    const double dx = dx_of(c);
    // FP32 refinement: the back halves add the correction to the FP64 iterate
    double* x64acc = fp32 ? c.x64 : nullptr;
#define MSRS_SWEEP(TT, KK, NN, XX)                                                                                             \
    do {                                                                                                                      \
        hipLaunchKernelGGL((sweep_kernel<TT, KK, NN, 0>), grid, blk, 0, c.stream, c.dp, p0, c.aL, c.vw, dx, (const TT*)c.E, XX, \
                           (double*)nullptr, (TT*)c.tw, conv, c.dflags);                                                      \
        hipLaunchKernelGGL((sweep_kernel<TT, KK, NN, 1>), grid, blk, 0, c.stream, c.dp, p0, c.aL, c.vw, dx, (const TT*)c.E, XX, \
                           x64acc, (TT*)c.tw, conv, c.dflags);                                                                 \
    } while (0)
    // the first solve of a refinement writes the FP64 iterate instead of adding to it
#define MSRS_SWEEP_FIRST(KK, NN)                                                                                               \
    do {                                                                                                                      \
        hipLaunchKernelGGL((sweep_kernel<float, KK, NN, 0>), grid, blk, 0, c.stream, c.dp, p0, c.aL, c.vw, dx, (const float*)c.E, \
                           c.x32, (double*)nullptr, (float*)c.tw, conv, c.dflags);                                            \
        hipLaunchKernelGGL((sweep_kernel<float, KK, NN, 2>), grid, blk, 0, c.stream, c.dp, p0, c.aL, c.vw, dx, (const float*)c.E, \
                           c.x32, x64acc, (float*)c.tw, conv, c.dflags);                                                      \
    } while (0)
    if (c.kind == kElliptic) {
        if (fp32 && first) {
            if (sc == 64) MSRS_SWEEP_FIRST(kElliptic, 4);
            else if (sc == 32) MSRS_SWEEP_FIRST(kElliptic, 2);
            else MSRS_SWEEP_FIRST(kElliptic, 1);
        } else if (fp32) {
            if (sc == 64) MSRS_SWEEP(float, kElliptic, 4, c.x32);
            else if (sc == 32) MSRS_SWEEP(float, kElliptic, 2, c.x32);
            else MSRS_SWEEP(float, kElliptic, 1, c.x32);
        } else {
            if (sc == 32) MSRS_SWEEP(double, kElliptic, 2, c.x64);
            else MSRS_SWEEP(double, kElliptic, 1, c.x64);
        }
    } else {
        if (fp32 && first) {
            if (sc == 64) MSRS_SWEEP_FIRST(kKinetic, 4);
            else if (sc == 32) MSRS_SWEEP_FIRST(kKinetic, 2);
            else MSRS_SWEEP_FIRST(kKinetic, 1);
        } else if (fp32) {
            if (sc == 64) MSRS_SWEEP(float, kKinetic, 4, c.x32);
            else if (sc == 32) MSRS_SWEEP(float, kKinetic, 2, c.x32);
            else MSRS_SWEEP(float, kKinetic, 1, c.x32);
        } else {
            if (sc == 32) MSRS_SWEEP(double, kKinetic, 2, c.x64);
            else MSRS_SWEEP(double, kKinetic, 1, c.x64);
        }
    }
#undef MSRS_SWEEP
#undef MSRS_SWEEP_FIRST
}

void launch_residual(Ctx& c, int p0, int p1, bool stats_only, int it) {
    StageTimer t(c, MSRS_K_RESIDUAL);
    const double inv_eps = 1.0 / c.eps;
    int32_t* conv = stats_only ? nullptr : c.conv;
    float* x32 = stats_only ? nullptr : c.x32;
    const dim3 grid(p1 - p0, max_chunks(c, p0, p1));
    if (c.kind == kElliptic)
        hipLaunchKernelGGL(residual_ell_kernel, grid, dim3(kResThreads), 0, c.stream, c.dp, p0, c.aL, c.om, c.x64, x32, conv, c.part,
                           c.maxch);
    else
        hipLaunchKernelGGL((residual_kernel<kKinetic>), grid, dim3(kThreads), 0, c.stream, c.dp, p0, c.aL, c.om, c.vw, dx_of(c), inv_eps,
                           c.x64, x32, conv, c.part, c.maxch);
    hipLaunchKernelGGL(norms_kernel, dim3(p1 - p0), dim3(64), 0, c.stream, c.dp, p0, c.part, c.maxch, c.rn, 1, conv,
                       c.gap + c.n_patches, c.iters, it, c.ir_tol);
}

void launch_restrict(Ctx& c, int p0, int p1) {
    StageTimer t(c, MSRS_K_RESTRICT);
    int maxrows = 0;
    for (int p = p0; p < p1; ++p) maxrows = std::max(maxrows, c.hp[p].nrows);
    const dim3 grid(p1 - p0, (maxrows + kRestrictRows - 1) / kRestrictRows);
    if (c.kind == kElliptic)
        hipLaunchKernelGGL((restrict_kernel<kElliptic>), grid, dim3(kThreads), 0, c.stream, c.dp, p0, c.x64, c.om, c.vw, c.Y);
    else
        hipLaunchKernelGGL((restrict_kernel<kKinetic>), grid, dim3(kThreads), 0, c.stream, c.dp, p0, c.x64, c.om, c.vw, c.Y);
}

void launch_clear_conv(Ctx& c) {
    hipLaunchKernelGGL(clear_kernel, dim3(1), dim3(kThreads), 0, c.stream, c.conv, c.n_patches);
}

// NOCONV if a patch has not converged after a fixed number of refinement
// iterations (the host-free form of the convergence check).
__global__ void check_conv_kernel(const int32_t* __restrict__ conv, int n, int32_t* flags) {
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        if (!conv[i]) raise_flag(flags, 1);
}

void launch_check_conv(Ctx& c) {
    hipLaunchKernelGGL(check_conv_kernel, dim3(1), dim3(kThreads), 0, c.stream, c.conv, c.n_patches, c.dflags);
}

}  // namespace msrs
