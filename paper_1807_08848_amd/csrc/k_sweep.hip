// Multi-RHS block sweeps of the local solves (stage a5): forward and back
// substitution through the explicit inverses E_l, products on MFMA.  The
// operator's block structure is described in k_local.hip.
#include <type_traits>
#include "local_common.h"

namespace msrs {

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
__device__ __forceinline__ void sweep_body(const PatchDesc& P, const double* __restrict__ aL, const double* __restrict__ vw, double dx,
                           const T* __restrict__ E, T* __restrict__ X, const T* __restrict__ XR, double* __restrict__ X64,
                           T* __restrict__ TW, int half, T* ybuf, T* wbuf, double* craw, double* cvp, double* cvm) {
    typedef typename Vec16<T>::type V;
    constexpr int VN = Vec16<T>::n;
    constexpr int BP = 16 * R, NKS = 4 * R, NSC = 16 * NCT;
    struct alignas(sizeof(T) * NCT) YRow { T v[NCT]; };
    // ybuf element (row i, column j of the chunk): column tiles innermost
    auto yix = [](int i, int j) { return i * NSC + (j & 15) * NCT + (j >> 4); };
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
    // B operands: the NCT column tiles of a lane's k row are adjacent in ybuf
    // (yix), one vector read per k step, issued a step ahead of its products
    auto mfma = [&]() {
        const int lli = llane & 15, llk = llane >> 4;
#pragma unroll
        for (int c = 0; c < NCT; ++c) acc[c] = Mfma<T>::zero();
        if (mf) {
            const T* yb = ybuf + llk * NSC + lli * NCT;     // k row 4 kk + llk at yb + 4 kk NSC
            YRow bc = *reinterpret_cast<const YRow*>(yb), bn;
#pragma unroll
            for (int kk = 0; kk < NKS; ++kk) {
                if (kk + 1 < NKS) bn = *reinterpret_cast<const YRow*>(yb + 4 * (kk + 1) * NSC);
#pragma unroll
                for (int c = 0; c < NCT; ++c) acc[c] = Mfma<T>::step(aC[kk], bc.v[c], acc[c]);
                bc = bn;
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
    // (each destination's test taken once, outside the element loops: tests per
    // element left the memory-counter waits at their merge points conservative)
    auto store_acc = [&](T* gdst, double* g64, const double (&pre64)[NCT][4], bool to_wbuf) {
        const int lli = llane & 15;
        if (!mf) return;
        if (to_wbuf) {
#pragma unroll
            for (int c = 0; c < NCT; ++c)
#pragma unroll
                for (int t = 0; t < 4; ++t) wbuf[(16 * rt + Mfma<T>::row(llane, t)) * NSC + 16 * c + lli] = acc[c][t];
        }
        if (gdst) {
#pragma unroll
            for (int c = 0; c < NCT; ++c)
#pragma unroll
                for (int t = 0; t < 4; ++t) gdst[(uint32_t)((16 * rt + Mfma<T>::row(llane, t)) * sp + 16 * c + lli)] = acc[c][t];
        }
        if (g64) {
#pragma unroll
            for (int c = 0; c < NCT; ++c)
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    g64[(uint32_t)((16 * rt + Mfma<T>::row(llane, t)) * sp + 16 * c + lli)] = pre64[c][t] + (double)acc[c][t];
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

    // Register-resident coupling (FP32 elliptic).  A line vector of a step
    // lives in the MFMA accumulator layout: element (c, t) of a lane is row
    // 16 rt + 4 (lane / 16) + t, column 16 c + lane % 16 of the chunk.  The
    // coupling of row i takes rows i - 1, i, i + 1 of the product: rows inside
    // the lane's four come from its registers, the rows just above and below
    // them from the edge rows (= 0 and 3 mod 4) that every lane puts into wbuf
    // (column tiles innermost, as in ybuf).
    constexpr bool RC = sizeof(T) == 4 && KIND == kElliptic;
    // (the back half with an FP64 iterate to accumulate keeps the LDS form:
    // the iterate's registers do not fit beside the accumulators)
    constexpr bool RC_BACK = PHASE != 1;
    const int rtc = rt < R ? rt : R - 1;
    // (the lane's row and column offsets come from the laundered lane index,
    // so that they are recomputed per line rather than held in registers)
    // a line in the accumulator layout (waves past the row tiles: a copy of the last tile)
    auto ld_acc_line = [&](const T* Xl, T (&dst)[NCT][4]) {
        const int q4 = 4 * (llane >> 4), lq = llane & 15;
#pragma unroll
        for (int c = 0; c < NCT; ++c)
#pragma unroll
            for (int t = 0; t < 4; ++t) dst[c][t] = Xl[(uint32_t)((16 * rtc + q4 + t) * sp + 16 * c + lq)];
    };
    auto put_halo = [&]() {
        const int q4 = 4 * (llane >> 4), lq = llane & 15;
        if (mf) {
            YRow a, z;
#pragma unroll
            for (int c = 0; c < NCT; ++c) { a.v[c] = acc[c][0]; z.v[c] = acc[c][3]; }
            *reinterpret_cast<YRow*>(wbuf + yix(16 * rt + q4, lq)) = a;
            *reinterpret_cast<YRow*>(wbuf + yix(16 * rt + q4 + 3, lq)) = z;
        }
    };
    // y over the lane's elements: r - C w with sub, else C w, C the coupling
    // block of the cell row in craw (the same expression and order as
    // couple()); rows at or past b zero.  y goes to ybuf
    // (toy: the next product's B operand) and, with glob, to gdst.
    auto couple_rc = [&](const T (&r)[NCT][4], bool sub, T* gdst, bool toy, auto glob) {
        if (!mf) return;
        const int q4 = 4 * (llane >> 4), lq = llane & 15;
        const int i0r = 16 * rt + q4;
        const YRow hm = *reinterpret_cast<const YRow*>(wbuf + yix(i0r > 0 ? i0r - 1 : 0, lq));
        const YRow hp = *reinterpret_cast<const YRow*>(wbuf + yix(i0r + 4 < BP ? i0r + 4 : BP - 1, lq));
        double cr[5];
#pragma unroll
        for (int u = 0; u < 5; ++u) cr[u] = craw[i0r + u];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int i = i0r + t;
            const double cm = i > 0 ? cr[t] : 0.0;
            const double cp = i < b - 1 ? cr[t + 1] : 0.0;
            YRow yr;
#pragma unroll
            for (int c = 0; c < NCT; ++c) {
                const double wm = (double)(t > 0 ? acc[c][t > 0 ? t - 1 : 0] : hm.v[c]);
                const double wp = (double)(t < 3 ? acc[c][t < 3 ? t + 1 : 3] : hp.v[c]);
                const double cw = 0.5 * (cr[t] + cr[t + 1]) * (double)acc[c][t] + cm * wm + cp * wp;
                const double v = sub ? (double)r[c][t] - cw : cw;
                const T y = i < b ? (T)v : T(0);
                yr.v[c] = y;
                if constexpr (decltype(glob)::value) gdst[(uint32_t)(i * sp + 16 * c + lq)] = y;
            }
            if (toy) *reinterpret_cast<YRow*>(ybuf + yix(i, lq)) = yr;
        }
    };

    // Register sets of prefetched loads alternate between consecutive steps
    // (the step body is instantiated twice per loop trip), so that no copy of
    // a register with a load in flight makes the wave wait for it early.
    double nopre[NCT][4] = {};
    if constexpr (PHASE == 0) {
        // ---- forward half: lines ln0, ln0 + dir, ...; the last one couples into m
        // (right-hand sides read from XR, results written to X: no line read here
        // is written here)
        const int nst = half == 0 ? m : nl - 1 - m;
        const int ln0 = half == 0 ? 0 : nl - 1;
        const bool low = half == 0;   // top: Low_{l+1} (line below from above); bottom: Up_{l-1}
        T rvA[RPT], rvB[RPT];
        launder();
        if (nst <= 0) {
            // no line in this half: t_top = r_m, t_bot = 0
            if (half == 0) load_line(XR + m * lstride, rvA);
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
        if constexpr (RC) {
            {
                T r0[RPT];
                load_line(XR + ln0 * lstride, r0);                 // y_{ln0} = r_{ln0}
                const bool copy = XR != X;                         // the back half reads y_{ln0} from X
#pragma unroll
                for (int e = 0; e < RPT; ++e) {
                    const int i = li0 + e * DI;
                    if (BP % DI == 0 || i < BP) {
                        ybuf[yix(i, ljj)] = r0[e];
                        if (copy) X[ln0 * lstride + (uint32_t)(i * sp + ljj)] = r0[e];
                    }
                }
            }
            T rcA[NCT][4] = {}, rcB[NCT][4] = {};
            load_A(E + (int64_t)ln0 * BP * BP);
            double crA = 0.0, crB = 0.0;
            if (sub_of(0)) ld_acc_line(XR + (ln0 + dir) * lstride, rcA);
            crA = aL[(dir > 0 ? ln0 + 1 : ln0) * L + min(tid, b)];
            lds_barrier();
            auto step = [&](int k, T (&rc)[NCT][4], T (&rn)[NCT][4], double& cc, double& cn) {
                launder();
                const int ln = ln0 + dir * k, nx = ln + dir;
                const bool more = k + 1 < nst;
                const bool sub = sub_of(k);
                mfma();                                                               // w = E_ln y_ln
                cn = aL[(more ? (dir > 0 ? nx + 1 : nx) : (dir > 0 ? ln + 1 : ln)) * L + min(tid, b)];
                load_A(E + (int64_t)(more ? nx : ln) * BP * BP);                     // E of the next step
                put_halo();
                if (tid <= b) craw[tid] = cc * (-1.0 / 3.0);
                lds_barrier();
                couple_rc(rc, sub, more ? X + nx * lstride : TWh, more, std::true_type{});
                // r of the next step, after the coupling (its registers are free
                // then), consumed after the next products
                ld_acc_line(XR + ((more && sub_of(k + 1)) ? nx + dir : nx) * lstride, rn);
                lds_barrier();
            };
            for (int k = 0; k < nst; k += 2) {
                step(k, rcA, rcB, crA, crB);
                if (k + 1 < nst) step(k + 1, rcB, rcA, crB, crA);
            }
        } else {
            load_line(XR + ln0 * lstride, rvA);                 // y_{ln0} = r_{ln0}
            const bool copy = XR != X;                          // the back half reads y_{ln0} from X
#pragma unroll
            for (int e = 0; e < RPT; ++e) {
                const int i = li0 + e * DI;
                if (BP % DI == 0 || i < BP) {
                    ybuf[yix(i, ljj)] = rvA[e];
                    if (copy) X[ln0 * lstride + (uint32_t)(i * sp + ljj)] = rvA[e];
                }
            }
            load_A(E + (int64_t)ln0 * BP * BP);
            double crA = 0.0, crB = 0.0;
            if (sub_of(0)) load_line(XR + (ln0 + dir) * lstride, rvA);
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
                load_line(XR + ((more && sub_of(k + 1)) ? nx + dir : nx) * lstride, rn);
                if (KIND == kElliptic) cn = aL[(more ? (dir > 0 ? nx + 1 : nx) : (dir > 0 ? ln + 1 : ln)) * L + min(tid, b)];
                load_A(E + (int64_t)(more ? nx : ln) * BP * BP);
                store_acc(nullptr, nullptr, nopre, true);
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
                        if (more) ybuf[yix(i, ljj)] = y;
                    }
                }
                lds_barrier();
            };
            for (int k = 0; k < nst; k += 2) {
                step(k, rvA, rvB, crA, crB);
                if (k + 1 < nst) step(k + 1, rvB, rvA, crB, crA);
            }
        }
    } else {
        // ---- middle line, then the back half; step k solves line
        // ln = m - dir (k + 1) from pv = ln + dir.  Its right-hand side y_ln, the
        // shared cell row and (FP32 refinement) the FP64 iterate of the line are
        // loaded one step ahead, E_ln during the step before.
        // PHASE 2 is the first solve of a refinement: the FP64 iterate holds
        // nothing yet and is written, not accumulated (pre64 stays zero).
        if constexpr (RC && RC_BACK) {
            launder();
            constexpr bool kAccum = PHASE == 1;
            constexpr bool kAhead = NCT <= 2;
            double pre64[NCT][4] = {}, pre64n[kAhead ? NCT : 1][4] = {};
            load_A(E + (int64_t)m * BP * BP);
            const bool acc64 = X64 && half == 0;   // line m's iterate is updated once, by the top half
            if (kAccum && acc64) load_64(X64 + m * lstride, pre64);
#pragma unroll
            for (int e = 0; e < RPT; ++e) {
                const int i = li0 + e * DI;
                if (BP % DI == 0 || i < BP) {
                    const double v = (double)TW[(uint32_t)(i * sp + ljj)] - (double)TW[lstride + (uint32_t)(i * sp + ljj)];
                    ybuf[yix(i, ljj)] = i < b ? (T)v : T(0);
                }
            }
            const int nst = half == 0 ? m : nl - 1 - m;
            T rv2[NCT][4] = {};
            double crow2 = 0.0;
            if (nst > 0) {
                const int l1 = m - dir;
                ld_acc_line(X + l1 * lstride, rv2);
                if (tid <= b) crow2 = aL[(dir > 0 ? m : l1) * L + tid];
                if constexpr (kAhead) {
                    if (kAccum && X64) load_64(X64 + l1 * lstride, pre64n);
                }
            }
            lds_barrier();
            mfma();
            if (nst > 0) load_A(E + (int64_t)(m - dir) * BP * BP);        // the first back line, one step ahead
            store_acc(half == 0 && !X64 ? X + m * lstride : nullptr, acc64 ? X64 + m * lstride : nullptr, pre64, false);
            put_halo();
            // the cell row of the first back step's coupling: every read of craw
            // comes after the barrier that follows its write
            if (tid <= b) craw[tid] = crow2 * (-1.0 / 3.0);
            lds_barrier();
            for (int k = 0; k < nst; ++k) {
                launder();
                const int ln = m - dir * (k + 1);
                const bool more = k + 1 < nst;
                couple_rc(rv2, true, nullptr, true, std::false_type{});              // z = y_ln - C x_{ln + dir}
                // after the coupling (its registers are free then): the next
                // step's y and cell row; this line's FP64 iterate (consumed after
                // the products) a step ahead where the registers allow it
                if constexpr (kAhead) {
#pragma unroll
                    for (int c = 0; c < NCT; ++c)
#pragma unroll
                        for (int t = 0; t < 4; ++t) pre64[c][t] = pre64n[c][t];
                }
                double crown = 0.0;
                if (more) {
                    const int l2 = ln - dir;
                    ld_acc_line(X + l2 * lstride, rv2);                               // y of the next step
                    if (tid <= b) crown = aL[(dir > 0 ? ln : l2) * L + tid];
                    if constexpr (kAhead) {
                        if (kAccum && X64) load_64(X64 + l2 * lstride, pre64n);
                    }
                }
                lds_barrier();
                if constexpr (!kAhead) {
                    if (kAccum && X64) load_64(X64 + ln * lstride, pre64);
                }
                mfma();                                                                // x_ln = E_ln z
                if (more) load_A(E + (int64_t)(ln - dir) * BP * BP);                 // E of the next line
                store_acc(X64 ? nullptr : X + ln * lstride, X64 ? X64 + ln * lstride : nullptr, pre64, false);
                put_halo();
                // the couplings of this step were read before the barrier above
                if (more && tid <= b) craw[tid] = crown * (-1.0 / 3.0);
                lds_barrier();
            }
        } else {
            launder();
            constexpr bool kAccum = PHASE == 1;
            // the FP64 iterate of a back line: loaded one step ahead where the
            // registers allow it (up to 32 samples), else at the top of its own step
            constexpr bool kAhead = NCT <= 2;
            double pre64[NCT][4] = {}, pre64n[kAhead ? NCT : 1][4] = {};
            load_A(E + (int64_t)m * BP * BP);
            const bool acc64 = X64 && half == 0;   // line m's iterate is updated once, by the top half
            if (kAccum && acc64) load_64(X64 + m * lstride, pre64);
#pragma unroll
            for (int e = 0; e < RPT; ++e) {
                const int i = li0 + e * DI;
                if (BP % DI == 0 || i < BP) {
                    const double v = (double)TW[(uint32_t)(i * sp + ljj)] - (double)TW[lstride + (uint32_t)(i * sp + ljj)];
                    ybuf[yix(i, ljj)] = i < b ? (T)v : T(0);
                }
            }
            const int nst = half == 0 ? m : nl - 1 - m;
            const bool low = half != 0;   // top: Up_l x_{l+1}; bottom: Low_l x_{l-1}
            if (nst > 0) {
                const int l1 = m - dir;
                load_line(X + l1 * lstride, rv);
                if (KIND == kElliptic && tid <= b) crow = aL[(dir > 0 ? m : l1) * L + tid];
                if constexpr (kAhead) {
                    if (kAccum && X64) load_64(X64 + l1 * lstride, pre64n);
                }
            }
            lds_barrier();
            mfma();
            if (nst > 0) load_A(E + (int64_t)(m - dir) * BP * BP);        // the first back line, one step ahead
            // x_m (identical in both halves).  With an FP64 iterate (refinement) the
            // FP32 solution is not stored: the iterate takes it, and the line
            // vectors are next overwritten by the residual.
            store_acc(half == 0 && !X64 ? X + m * lstride : nullptr, acc64 ? X64 + m * lstride : nullptr, pre64, true);
            lds_barrier();
            for (int k = 0; k < nst; ++k) {
                launder();
                const int ln = m - dir * (k + 1);
                const bool more = k + 1 < nst;
                if constexpr (kAhead) {
#pragma unroll
                    for (int c = 0; c < NCT; ++c)
#pragma unroll
                        for (int t = 0; t < 4; ++t) pre64[c][t] = pre64n[c][t];
                }
                if (KIND == kElliptic && tid <= b) craw[tid] = crow * (-1.0 / 3.0);
                lds_barrier();
#pragma unroll
                for (int e = 0; e < RPT; ++e) {
                    const int i = li0 + e * DI;
                    if (BP % DI == 0 || i < BP) {
                        const double v = (double)rv[e] - couple(wbuf, i, ljj, low);
                        ybuf[yix(i, ljj)] = i < b ? (T)v : T(0);
                    }
                }
                // after the coupling (fewer registers live than during it): this
                // line's FP64 iterate where it is not loaded a step ahead (the
                // products hide it; it is consumed after them), and the next step's
                // y and cell row
                if constexpr (!kAhead) {
                    if (kAccum && X64) load_64(X64 + ln * lstride, pre64);
                }
                T rvn[RPT];
                double crown = 0.0;
                if (more) {
                    const int l2 = ln - dir;
                    load_line(X + l2 * lstride, rvn);                                     // y of the next step
                    if (KIND == kElliptic && tid <= b) crown = aL[(dir > 0 ? ln : l2) * L + tid];
                    if constexpr (kAhead) {
                        if (kAccum && X64) load_64(X64 + l2 * lstride, pre64n);
                    }
                }
                lds_barrier();
                mfma();                                                                    // x_ln = E_ln z
                if (more) load_A(E + (int64_t)(ln - dir) * BP * BP);                     // E of the next line
                store_acc(X64 ? nullptr : X + ln * lstride, X64 ? X64 + ln * lstride : nullptr, pre64, true);
#pragma unroll
                for (int e = 0; e < RPT; ++e) rv[e] = rvn[e];
                crow = crown;
                lds_barrier();
            }
        }
    }
}

// grid (patch, column chunk of 16*NCT samples, half); sp of every patch is a
// multiple of the chunk.
template <typename T, int KIND, int NCT, int PHASE>
__global__ __launch_bounds__(kSweepThreads) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1))) void sweep_kernel(const PatchDesc* pd, int p0, const double* __restrict__ aL_all,
                                                              const double* __restrict__ vw, double dx, const T* __restrict__ E_all,
                                                              T* __restrict__ X_all, const T* __restrict__ XR_all,
                                                              double* __restrict__ X64_all, T* __restrict__ TW_all,
                                                              const int32_t* __restrict__ conv, const int32_t* __restrict__ items,
                                                              int32_t* flags) {
    __shared__ __align__(16) T ybuf[kMaxLine * 16 * NCT];
    __shared__ T wbuf[kMaxLine * 16 * NCT];
    __shared__ double craw[kMaxLine + 1];
    __shared__ double cvp[kMaxLine], cvm[kMaxLine];
    // items: workgroup x runs (patch, half) = (items[x] >> 1, items[x] & 1);
    // without it, patch p0 + x and half z
    const int it = items ? items[blockIdx.x] : 0;
    const int p = items ? it >> 1 : p0 + (int)blockIdx.x;
    const int half = items ? it & 1 : (int)blockIdx.z;
    if (conv && conv[p]) return;
    const PatchDesc P = pd[p];
    const int s0 = blockIdx.y * 16 * NCT;
    if (s0 >= P.sp) return;
    const double* aL = aL_all + P.a_off;
    const T* E = E_all + P.E_off;
    T* X = X_all + P.x_off + s0;
    // the forward half's right-hand sides: XR_all where given (FP32 refinement's
    // first solve: the lifted boundary data), else X itself
    const T* XR = XR_all ? XR_all + P.x_off + s0 : X;
    T* TW = TW_all + P.tw_off + s0;
    double* X64 = X64_all ? X64_all + P.x_off + s0 : nullptr;
#define MSRS_SWB(RR) sweep_body<T, KIND, RR, NCT, PHASE>(P, aL, vw, dx, E, X, XR, X64, TW, half, ybuf, wbuf, craw, cvp, cvm)
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
    // the whole batch runs in the paired cost order; a single patch as (patch, half)
    const bool all = p0 == 0 && p1 == c.n_patches && c.sweep_items;
    const int32_t* items = all ? c.sweep_items : nullptr;
    const dim3 grid(all ? 2 * c.n_patches : p1 - p0, maxsp / sc, all ? 1 : 2), blk(kSweepThreads);
    const int32_t* conv = fp32 ? c.conv : nullptr;
    const double dx = dx_of(c);
    // FP32 refinement: the back halves add the correction to the FP64 iterate
    double* x64acc = fp32 ? c.x64 : nullptr;
#define MSRS_SWEEP(TT, KK, NN, XX)                                                                                             \
    do {                                                                                                                      \
        hipLaunchKernelGGL((sweep_kernel<TT, KK, NN, 0>), grid, blk, 0, c.stream, c.dp, p0, c.aL, c.vw, dx, (const TT*)c.E, XX, \
                           (const TT*)nullptr, (double*)nullptr, (TT*)c.tw, conv, items, c.dflags);                                  \
        hipLaunchKernelGGL((sweep_kernel<TT, KK, NN, 1>), grid, blk, 0, c.stream, c.dp, p0, c.aL, c.vw, dx, (const TT*)c.E, XX, \
                           (const TT*)nullptr, x64acc, (TT*)c.tw, conv, items, c.dflags);                                             \
    } while (0)
    // the first solve of a refinement writes the FP64 iterate instead of adding to it
#define MSRS_SWEEP_FIRST(KK, NN)                                                                                               \
    do {                                                                                                                      \
        hipLaunchKernelGGL((sweep_kernel<float, KK, NN, 0>), grid, blk, 0, c.stream, c.dp, p0, c.aL, c.vw, dx, (const float*)c.E, \
                           c.x32, (const float*)(c.rhs_in_xlift ? c.xlift : nullptr), (double*)nullptr, (float*)c.tw, conv,      \
                           items, c.dflags);                                                                                         \
        hipLaunchKernelGGL((sweep_kernel<float, KK, NN, 2>), grid, blk, 0, c.stream, c.dp, p0, c.aL, c.vw, dx, (const float*)c.E, \
                           c.x32, (const float*)nullptr, x64acc, (float*)c.tw, conv, items, c.dflags);                              \
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

}  // namespace msrs
