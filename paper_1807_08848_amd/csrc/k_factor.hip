// Block-row factorization of the local operators (stage a4 of
// LocalPDESolver inside RanLocalSolu, Section 3): explicit inverses of the
// Schur blocks by blocked Gauss-Jordan on MFMA, eliminated from both ends of
// the line chain.  The operator's block structure is described in k_local.hip.
#include "local_common.h"

namespace msrs {

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

// Symmetric storage (elliptic FP32): the Schur blocks D_l are symmetric and
// only the R (R + 1) / 2 upper tiles (ti <= tj) are held, round-robin over
// the waves (slot q of wave w: upper tile q * 16 + w in row-major order).
template <int R>
constexpr int factor_sym_slots() { return (R * (R + 1) / 2 + kFactorWaves - 1) / kFactorWaves; }
template <int R>
__device__ __forceinline__ int factor_sym_tile(int q, int w) {
    int rem = q * kFactorWaves + w, ti = 0;
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (ti == r && rem >= R - r) { rem -= R - r; ++ti; }
    return ti < R ? ti * R + ti + rem : -1;
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
    // SYM: elliptic, upper tiles only (the blocks are symmetric, and
    // Gauss-Jordan keeps every block symmetric except those between pivoted
    // and unpivoted indices, which are antisymmetric: A_ji = -A_ij^T)
    constexpr bool SYM = KIND == kElliptic;
    constexpr int BP = 16 * R, LDE = BP + 1, NSLOT = SYM ? factor_sym_slots<R>() : factor_slots<R>();
    constexpr int NKS = BP / 4;
    typedef typename Mfma<T>::acc Acc;
    const int tid0 = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid0 >> 6);
    auto tile_of = [&](int q) -> int { return SYM ? factor_sym_tile<R>(q, w) : factor_tile<R>(q, w); };
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
                const int idx = tile_of(q);
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
                const int idx = tile_of(q);
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
                    if (tile_of(q) != p * (R + 1)) continue;
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
                const int idx = tile_of(q);
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
                const int idx = tile_of(q);
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
        // SYM: the pivot step pn on upper tiles.  Publish: a tile of column pn
        // (ti <= pn) gives Pc block ti and, transposed and negated, Pr block ti
        // (A_{pn,ti} = -A_{ti,pn}^T: ti pivoted, pn not); a tile of row pn
        // (tj > pn) gives Pr block tj and, transposed, Pc block tj (both
        // unpivoted).  Row panel: X_j = Dinv A_{pn,j} for every j != pn, by the
        // owner of the row tile (pn, j), j > pn (which becomes X_j), or of the
        // column tile (j, pn), j < pn.  Update: column tiles -A_{i,pn} Dinv, the
        // others A_ij -= A_{i,pn} X_j.
        auto publish_sym = [&](int p, T* pc, T* pr) {
#pragma unroll
            for (int q = 0; q < NSLOT; ++q) {
                const int idx = tile_of(q);
                if (idx < 0) continue;
                const int ti = idx / R, tj = idx - ti * R;
                if (tj != p && ti != p) continue;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int r = Mfma<T>::row(lane, t);
                    const T v = tile[q][t];
                    if (tj == p) {
                        pc[(16 * ti + r) * PCL + li] = v;
                        if (ti < p) pr[li * PRL + 16 * ti + r] = -v;
                    } else {
                        pr[r * PRL + 16 * tj + li] = v;
                        pc[(16 * tj + li) * PCL + r] = v;
                    }
                }
            }
        };
        auto row_panel_sym = [&](int pn, const T* pr, T* xs, const T* dv) {
#pragma unroll
            for (int q = 0; q < NSLOT; ++q) {
                const int idx = tile_of(q);
                if (idx < 0) continue;
                const int ti = idx / R, tj = idx - ti * R;
                const int j = ti == pn ? tj : (tj == pn ? ti : -1);
                if (j < 0 || j == pn) continue;
                Acc x = Mfma<T>::zero();
#pragma unroll
                for (int st = 0; st < 4; ++st) {
                    const int k = 4 * st + lk;
                    x = Mfma<T>::step(dv[li * DVL + k], pr[k * PRL + 16 * j + li], x);
                }
                if (ti == pn) tile[q] = x;
#pragma unroll
                for (int t = 0; t < 4; ++t) xs[Mfma<T>::row(lane, t) * PRL + 16 * j + li] = x[t];
            }
        };
        // set_diag: the owner writes Dinv into the diagonal tile (FP64, whose
        // inverse is formed in LDS; the FP32 owner inverted it in place)
        auto update_sym = [&](int pn, const T* pc, const T* xs, const T* dv, bool set_diag) {
#pragma unroll
            for (int q = 0; q < NSLOT; ++q) {
                const int idx = tile_of(q);
                if (idx < 0) continue;
                const int ti = idx / R, tj = idx - ti * R;
                if (ti == pn) {   // the new row (X) or the diagonal (Dinv)
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
        if constexpr (SYM && sizeof(T) == 8) {
            for (int pn = 0; pn < npan; ++pn) {
                launder();
                const int buf = pn & 1;
                T* pc = Pc + buf * BP * PCL;
                T* pr = Pr + buf * 16 * PRL;
                T* xs = Xs + buf * 16 * PRL;
                T* dv = Dv + buf * 16 * DVL;
                publish_sym(pn, pc, pr);
                __syncthreads();
                if (w == 0) inv16_wave<T, PCL, DVL>(pc + 16 * pn * PCL, dv, bad);
                __syncthreads();
                row_panel_sym(pn, pr, xs, dv);
                __syncthreads();
                update_sym(pn, pc, xs, dv, true);
            }
        } else if constexpr (SYM) {
            publish_sym(0, Pc, Pr);
            invert_diag(0, Dv);
            __syncthreads();
            for (int pn = 0; pn < npan; ++pn) {
                launder();
                const int buf = pn & 1, nb = buf ^ 1;
                row_panel_sym(pn, Pr + buf * 16 * PRL, Xs + buf * 16 * PRL, Dv + buf * 16 * DVL);
                __syncthreads();
                update_sym(pn, Pc + buf * BP * PCL, Xs + buf * 16 * PRL, Dv + buf * 16 * DVL, false);
                if (pn + 1 < npan) {
                    publish_sym(pn + 1, Pc + nb * BP * PCL, Pr + nb * 16 * PRL);
                    invert_diag(pn + 1, Dv + nb * 16 * DVL);
                }
                __syncthreads();
            }
        } else if constexpr (sizeof(T) == 4) {
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
            const int idx = tile_of(q);
            if (idx < 0) continue;
            const int ti = idx / R, tj = idx - ti * R;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                Es[(16 * ti + Mfma<T>::row(lane, t)) * LDE + 16 * tj + li] = tile[q][t];
                if (SYM && ti != tj) Es[(16 * tj + li) * LDE + 16 * ti + Mfma<T>::row(lane, t)] = tile[q][t];
            }
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

// Any mix of line-tile counts 1..RMAX in one launch: workgroup x factors
// patch plist[x] with the body compiled for its count; LDS and registers are
// those of the largest body.  plist is in longest-processing-time order (the
// costliest patches first), so the long chains start first and the short ones
// fill in behind them; a batch of several line lengths is then one launch on
// the handle's stream, a single chain in a captured graph.
// items (halves launch, optional): workgroup x runs the chain items[x] =
// (patch << 1 | half), half 1 the bottom one, in place of (plist[x],
// blockIdx.y); the list is sorted by cost with its second half reversed, so
// that with two resident workgroups per compute unit a long chain shares its
// unit with a short one.
template <typename T, int KIND, int RMAX, bool MID, int SHARE>
__global__ __launch_bounds__(kFactorThreads, SHARE == 2 ? 8 : 1) void factor_any_kernel(const PatchDesc* pd, const int32_t* __restrict__ plist,
                                                                    const double* __restrict__ aL_all, const double* __restrict__ vw,
                                                                    double dx, double inv_eps, T* __restrict__ E_all, int32_t* flags,
                                                                    const int32_t* __restrict__ items) {
    __shared__ T lds[factor_lds_elems<RMAX>()];
    __shared__ double cf[2 * kMaxLine];
    __shared__ double crow[2 * (kMaxLine + 1)];
    const int item = (!MID && items) ? items[blockIdx.x] : 0;
    const PatchDesc P = pd[(!MID && items) ? item >> 1 : plist[blockIdx.x]];
    const int dir = MID ? 0 : ((items ? (item & 1) : (int)blockIdx.y) == 0 ? 1 : -1);
    const double* aL = aL_all + P.a_off;
    T* E = E_all + P.E_off;
#define MSRS_FB(RR) factor_mfma_body<T, KIND, RR, MID>(P, aL, vw, dx, inv_eps, E, lds, cf, crow, dir, flags)
    const int R = P.bp >> 4;
    if (R == 1) MSRS_FB(1);
    else if (R == 2) MSRS_FB(2);
    else if (R == 3) MSRS_FB(3);
    else if (R == 4) MSRS_FB(4);
    else {
        bool done = false;
        if constexpr (RMAX >= 8) {
            done = true;
            if (R == 5) MSRS_FB(5);
            else if (R == 6) MSRS_FB(6);
            else if (R == 7) MSRS_FB(7);
            else if (R == 8) MSRS_FB(8);
            else done = false;
        }
        if (!done && threadIdx.x == 0) raise_flag(flags, 3);
    }
#undef MSRS_FB
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

// One launch for the halves and one for the middle lines over every patch
// of plist (any mix of line-tile counts).
template <typename T, int KIND>
static void launch_factor_any(Ctx& c, const int32_t* plist, int n, const int32_t* items) {
    constexpr int RMAX = KIND == kElliptic ? 8 : 4;
    const double inv_eps = 1.0 / c.eps;
    T* E = (T*)c.E;
    const dim3 halves = items ? dim3(2 * n) : dim3(n, 2);
#define MSRS_FANY(SH)                                                                                                        \
    do {                                                                                                                     \
        hipLaunchKernelGGL((factor_any_kernel<T, KIND, RMAX, false, SH>), halves, dim3(kFactorThreads), 0, c.stream, c.dp,    \
                           plist, c.aL, c.vw, dx_of(c), inv_eps, E, c.dflags, items);                                         \
        hipLaunchKernelGGL((factor_any_kernel<T, KIND, RMAX, true, SH>), dim3(n), dim3(kFactorThreads), 0, c.stream, c.dp,     \
                           plist, c.aL, c.vw, dx_of(c), inv_eps, E, c.dflags, (const int32_t*)nullptr);                       \
    } while (0)
    if constexpr (sizeof(T) == 4) {
        if (c.factor_share == 2) MSRS_FANY(2);
        else MSRS_FANY(1);
    } else {
        MSRS_FANY(1);
    }
#undef MSRS_FANY
}

// Patches are grouped by line-tile count R.  A single patch (reference mode)
// or a batch of one count runs the kernel compiled for exactly that count; a
// FP32 batch of two adjacent counts the two-count kernel; any other mix one
// launch of the any-count kernel over the patches in longest-processing-time
// order.  Everything goes to the handle's stream.
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
    if (ng <= 1) {
        for (int g = 0; g < 9; ++g)
            if (c.rgroup_n[g]) launch_factor_group(c, g, c.stream, c.rgroup[g], c.rgroup_n[g]);
        return;
    }
    if (ng == 2 && (c.kind == kElliptic ? launch_factor_pair<kElliptic>(c, rmax, rmin) : launch_factor_pair<kKinetic>(c, rmax, rmin)))
        return;
    const bool ir = c.prec == MSRS_PREC_FP32_IR;
    if (c.kind == kElliptic) {
        if (ir) launch_factor_any<float, kElliptic>(c, c.lpt, c.n_patches, c.factor_items);
        else launch_factor_any<double, kElliptic>(c, c.lpt, c.n_patches, c.factor_items);
    } else {
        if (ir) launch_factor_any<float, kKinetic>(c, c.lpt, c.n_patches, c.factor_items);
        else launch_factor_any<double, kKinetic>(c, c.lpt, c.n_patches, c.factor_items);
    }
}

}  // namespace msrs
