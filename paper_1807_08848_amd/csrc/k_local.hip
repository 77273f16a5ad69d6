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
#include "local_common.h"

namespace msrs {

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

// The generator alone: the four output words and the normal of counter
// (node, sample, patch, 0) for a node x sample block of one patch, in the
// order of Omega (column-major, samples as columns).
__global__ __launch_bounds__(kThreads) void philox_draw_kernel(uint64_t seed, uint32_t patch, int n_node, int n_sample,
                                                               uint32_t* __restrict__ words, double* __restrict__ normals) {
    const int64_t n = (int64_t)n_node * n_sample;
    for (int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x; o < n; o += (int64_t)gridDim.x * kThreads) {
        const uint32_t node = (uint32_t)(o % n_node), sample = (uint32_t)(o / n_node);
        if (words) {
            const U4 r = philox4x32_10(U4{node, sample, patch, 0u}, (uint32_t)seed, (uint32_t)(seed >> 32));
            words[4 * o + 0] = r.x;
            words[4 * o + 1] = r.y;
            words[4 * o + 2] = r.z;
            words[4 * o + 3] = r.w;
        }
        if (normals) normals[o] = philox_normal(seed, node, sample, patch);
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
// SPARSE: only the entries that can be non-zero are written (the nodes next to
// the buffered patch's boundary: the first and last line whole, rows 0 and
// b - 1 of the others; kinetic: the first and last line), into a buffer that
// holds zeros everywhere else from its allocation on.  The threads of a
// sample take the chunk's list of such entries in turn.
template <int KIND>
__device__ __forceinline__ double lift_value(const PatchDesc& P, const double* __restrict__ aL, const double* __restrict__ O,
                                             const double* __restrict__ vw, double dx, int l, int i, int c) {
    double v = 0.0;
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
        const int h = P.b / 2;
        const double vi = vw[i];
        if (l == 0 && vi > 0) v += vi / dx * O[(int64_t)c * P.nb + (i - h)];
        if (l == P.nl - 1 && vi < 0) v += -vi / dx * O[(int64_t)c * P.nb + h + i];
    }
    return v;
}

template <int KIND, typename TX, bool SPARSE>
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
    if constexpr (SPARSE) {
        if (m.active && c < P.s) {
            auto put = [&](int l, int i) {
                const double v = lift_value<KIND>(P, aL, O, vw, dx, l, i, c);
                X[P.x_off + (int64_t)l * bp * sp + (int64_t)i * sp + c] = (TX)v;
                ssum += v * v;
            };
            // the chunk's lines next to the boundary, whole (independent
            // entries: unrolled so that their loads overlap)
            for (int e = 0; e < 2; ++e) {
                const int l = e == 0 ? 0 : nl - 1;
                if (l < l0 || l >= l1 || (e == 1 && nl == 1)) continue;
#pragma unroll 4
                for (int i = m.row0; i < b; i += m.rows) put(l, i);
            }
            // elliptic: rows 0 and b - 1 of the chunk's other lines
            if (KIND == kElliptic) {
                const int la = max(l0, 1), lb = min(l1, nl - 1), nper = b > 1 ? 2 : 1;
#pragma unroll 4
                for (int t = m.row0; t < nper * (lb - la); t += m.rows) put(la + t / nper, (t % nper) ? b - 1 : 0);
            }
        }
    } else {
        for (int l = l0; l < l1; ++l) {
            const bool edge_line = l == 0 || l == nl - 1;
            for (int i = m.row0; m.active && i < bp; i += m.rows) {
                // only nodes next to the buffered patch's boundary (first / last
                // line, first / last row) have boundary neighbours
                const double v = (i < b && c < P.s && (edge_line || i == 0 || i == b - 1)) ? lift_value<KIND>(P, aL, O, vw, dx, l, i, c) : 0.0;
                X[P.x_off + (int64_t)l * bp * sp + (int64_t)i * sp + c] = (TX)v;
                ssum += v * v;
            }
        }
    }
    partial_column_sums(ssum, m, sp, red, part + ((int64_t)p * maxch + blockIdx.y) * kMaxSamples);
}

// Adjoint source (two-pass range finder): f_I = R_K^T q at the interior nodes
// of K_m (zero elsewhere and in the padding), q the columns of Qs (Y's
// layout), into the line vectors X; per-sample sums of squares as lift_kernel.
template <typename TX>
__global__ __launch_bounds__(kThreads) void adj_lift_kernel(const PatchDesc* pd, int p0, const double* __restrict__ Qs,
                                                            TX* __restrict__ X, double* __restrict__ part, int maxch) {
    __shared__ double red[kThreads];
    const int p = p0 + blockIdx.x;
    const PatchDesc P = pd[p];
    const int l0 = blockIdx.y * kChunkLines;
    if (l0 >= P.nl) return;
    const int l1 = min(P.nl, l0 + kChunkLines);
    const int sp = P.sp, bp = P.bp, b = P.b;
    const LineMap m(sp);
    const int c = m.col;
    const double* Qc = Qs + P.Y_off + (int64_t)c * P.nrows;
    double ssum = 0.0;
    for (int l = l0; l < l1; ++l) {
        for (int i = m.row0; m.active && i < bp; i += m.rows) {
            double v = 0.0;
            if (i < b && c < P.s) {
                const int row = k_row_of(P, i + 1, l + 1);
                if (row >= 0) v = Qc[row];
            }
            X[P.x_off + (int64_t)l * bp * sp + (int64_t)i * sp + c] = (TX)v;
            ssum += v * v;
        }
    }
    partial_column_sums(ssum, m, sp, red, part + ((int64_t)p * maxch + blockIdx.y) * kMaxSamples);
}

// Boundary values of the adjoint (two-pass range finder): for boundary node
// t of the buffered patch and sample column c, C = f_B - A_BI z, with z the
// interior solution (x64) of A_II z = f_I and f = R_K^T q (q in Qs, Y's
// layout); C in Omega's layout.  A_BI from the stencil of each interior
// neighbour (A symmetric).  grid (patch, chunk of kThreads outputs).
__global__ __launch_bounds__(kThreads) void adj_flux_kernel(const PatchDesc* pd, int p0, const double* __restrict__ aL_all,
                                                            const double* __restrict__ x64_all, const double* __restrict__ Qs,
                                                            double* __restrict__ C_all) {
    const int p = p0 + blockIdx.x;
    const PatchDesc P = pd[p];
    const int o = blockIdx.y * kThreads + threadIdx.x;
    if (o >= P.nb * P.s) return;
    const int c = o / P.nb, t = o - c * P.nb;
    int i, j;
    phys_of_bidx(t, P.cx, P.cy, i, j);
    const int pp = P.trans ? j : i, q = P.trans ? i : j;
    const int row = k_row_of(P, pp, q);
    double v = row >= 0 ? Qs[P.Y_off + (int64_t)c * P.nrows + row] : 0.0;
    const double* aL = aL_all + P.a_off;
    const double* X = x64_all + P.x_off;
    const int64_t lstride = (int64_t)P.bp * P.sp;
#pragma unroll
    for (int dq = -1; dq <= 1; ++dq)
#pragma unroll
        for (int dp = -1; dp <= 1; ++dp) {
            const int p2 = pp + dp, q2 = q + dq;
            if (p2 < 1 || p2 > P.L - 1 || q2 < 1 || q2 > P.Qn - 1) continue;   // not an interior node
            v -= q1_coef(aL, P.L, p2, q2, -dp, -dq) * X[(int64_t)(q2 - 1) * lstride + (int64_t)(p2 - 1) * P.sp + c];
        }
    C_all[P.om_off + (int64_t)c * P.nb + t] = v;
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

// Elliptic residual, sliding-window form: a workgroup takes 16 lines of a
// patch, thread (segment g, line pair lo, sample c) walks down its segment of
// lines l0 + 2 lo and l0 + 2 lo + 1 together, with the 4 x 3 window of x
// spanning both lines' stencils in registers (four new loads per node for two
// outputs) and the coefficient cell rows of the chunk staged in LDS.  Chunks
// of 16 lines read 18 rows of x per 16 (the halo rows two chunks share)
// instead of 10 per 8.  A line splits into as many segments as the workgroup
// has threads to spare for its sample count (2 at 32 samples): shorter
// dependent walks, more loads in flight.  Same arithmetic per node as the
// generic kernel.  The per-sample sums of a chunk go to the first of its two
// 8-line partial slots, zero to the second.
// ADJ (two-pass range finder): the adjoint system A_II z = f_I, f = R_K^T q
// with q the columns of Qs: zero boundary values and the source f added.
constexpr int kResThreads = kChunkLines * kMaxSamples;   // 8 line pairs x up to 64 samples
constexpr int kResLines = 2 * kChunkLines;                // lines per workgroup
template <bool ADJ>
__global__ __launch_bounds__(kResThreads) void residual_ell_kernel(const PatchDesc* pd, int p0, const double* __restrict__ aL_all,
                                                                   const double* __restrict__ om, const double* __restrict__ x64_all,
                                                                   float* __restrict__ x32_all, const int32_t* __restrict__ conv,
                                                                   double* __restrict__ part, int maxch, const double* __restrict__ Qs,
                                                                   int np, int nch) {
    __shared__ double cell[(kResLines + 1) * (kMaxLine + 1)];
    __shared__ double red[kResThreads];
    // workgroup -> (patch, chunk) so that a patch's chunks are dispatched one
    // after another on one XCD (workgroups go round-robin over the 8 XCDs):
    // the rows two neighbouring chunks share are still in that XCD's L2 when
    // the second one reads them
    const int grp = blockIdx.x / (8 * nch), rem = blockIdx.x - grp * 8 * nch;
    const int chunk = rem >> 3, pl = grp * 8 + (rem & 7);
    if (pl >= np) return;
    const int p = p0 + pl;
    if (conv && conv[p]) return;
    const PatchDesc P = pd[p];
    const int l0 = chunk * kResLines;
    if (l0 >= P.nl) return;
    const int l1 = min(P.nl, l0 + kResLines);
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
    const int la = l0 + 2 * lo;                 // the pair's first line
    const bool active = la < l1 && g < nseg;
    const bool two = la + 1 < l1;               // the pair's second line exists
    // nodes pa .. pb of the lines (1-based along them)
    const int pa = 1 + (g * b) / nseg, pb = ((g + 1) * b) / nseg;
    double ssum = 0.0;
    if (active) {
        const int q = la + 1;                   // node row of line la
        float* Ra = X32 ? X32 + (int64_t)la * lstride + c : nullptr;
        float* Rb = X32 && two ? X32 + (int64_t)(la + 1) * lstride + c : nullptr;
        if (c < P.s) {
            // u(q2, p2): interior nodes from x, nodes on the buffered patch's boundary from Omega
            auto u = [&](int q2, int p2) -> double {
                if (p2 == 0 || p2 == L || q2 == 0 || q2 == Qn) {
                    if constexpr (ADJ) return 0.0;
                    int ii, jj;
                    line_to_phys(P, p2, q2, ii, jj);
                    return O[(int64_t)c * P.nb + bidx_ccw(ii, jj, P.cx, P.cy)];
                }
                return X[(int64_t)(q2 - 1) * lstride + (int64_t)(p2 - 1) * sp + c];
            };
            // the terms of q1_coef over dq, dp = -1, 0, 1, in that order; the
            // divisions by 3 and 6 as products with the rounded reciprocals
            auto stencil = [](const double (&wm)[3], const double (&w0)[3], const double (&wp)[3], double SW, double SE,
                              double NW, double NE) {
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
                return r;
            };
            const double* cS = cell + (la - l0) * L;   // cell row q - 1
            const double* cM = cell + (la - l0 + 1) * L;   // cell row q
            const double* cN = cell + (la - l0 + (two ? 2 : 1)) * L;   // cell row q + 1 (second line only)
            // window columns p-1, p, p+1 of node rows q-1 .. q+2 (q+2: second line only)
            double w[4][3];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                w[r][0] = (r < 3 || two) ? u(q - 1 + r, pa - 1) : 0.0;
                w[r][1] = (r < 3 || two) ? u(q - 1 + r, pa) : 0.0;
            }
            double SW = cS[pa - 1], MW = cM[pa - 1], NW = cN[pa - 1];
            for (int pp = pa; pp <= pb; ++pp) {
#pragma unroll
                for (int r = 0; r < 4; ++r) w[r][2] = (r < 3 || two) ? u(q - 1 + r, pp + 1) : 0.0;
                const double SE = cS[pp], ME = cM[pp], NE = cN[pp];
                double ra = stencil(w[0], w[1], w[2], SW, SE, MW, ME);
                double rb = stencil(w[1], w[2], w[3], MW, ME, NW, NE);
                if constexpr (ADJ) {
                    const int row = k_row_of(P, pp, q);
                    if (row >= 0) ra += Qs[P.Y_off + (int64_t)c * P.nrows + row];
                    const int row2 = two ? k_row_of(P, pp, q + 1) : -1;
                    if (row2 >= 0) rb += Qs[P.Y_off + (int64_t)c * P.nrows + row2];
                }
                if (Ra) Ra[(int64_t)(pp - 1) * sp] = (float)ra;
                if (Rb) Rb[(int64_t)(pp - 1) * sp] = (float)rb;
                ssum += ra * ra;
                if (two) ssum += rb * rb;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    w[r][0] = w[r][1];
                    w[r][1] = w[r][2];
                }
                SW = SE; MW = ME; NW = NE;
            }
            if (g == nseg - 1)
                for (int i = b; i < bp; ++i) {
                    if (Ra) Ra[(int64_t)i * sp] = 0.0f;
                    if (Rb) Rb[(int64_t)i * sp] = 0.0f;
                }
        } else if (g == 0) {
            for (int i = 0; i < bp; ++i) {
                if (Ra) Ra[(int64_t)i * sp] = 0.0f;
                if (Rb) Rb[(int64_t)i * sp] = 0.0f;
            }
        }
    }
    // per-sample sums over the chunk's line pairs and segments, fixed order
    red[tid] = active ? ssum : 0.0;
    __syncthreads();
    if (tid < sp) {
        double s = 0.0;
        const int npair = (l1 - l0 + 1) / 2;
        for (int gg = 0; gg < nseg; ++gg)
            for (int r = 0; r < npair; ++r) s += red[(gg * kChunkLines + r) * sp + tid];
        const int64_t slot = (int64_t)p * maxch + 2 * chunk;
        part[slot * kMaxSamples + tid] = s;
        if (l1 - l0 > kChunkLines) part[(slot + 1) * kMaxSamples + tid] = 0.0;
    }
}


// Per patch: sum the chunk partials.  which = 0: ||rhs_j||^2 -> rn[0..sp).
// which = 1: ||r_j||^2 -> rn[sp..2sp) and relres[p] = max_j ||r_j||/||rhs_j||.
// With conv (refinement), the patch stops (conv[p] = 1, iters[p] = it + 1)
// once relres[p] <= stop, or once relres[p] <= tol and this iteration did not
// halve it (stagnation: the FP64 residual has reached its rounding level).  A
// non-finite rhs or residual norm counts as an infinite ratio, latches flag 4
// and stops the patch.
__global__ __launch_bounds__(64) void norms_kernel(const PatchDesc* pd, int p0, const double* __restrict__ part, int maxch,
                                                   double* __restrict__ rn_all, int which, int32_t* __restrict__ conv,
                                                   double* __restrict__ relres, int32_t* __restrict__ iters, int it, double tol,
                                                   double stop, int32_t* flags) {
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
        if (__any(t < P.s && !isfinite(s2)) && t == 0) raise_flag(flags, 4);
        return;
    }
    double ratio = 0.0;
    bool nonfinite = false;
    if (t < P.sp) {
        rn[P.sp + t] = s2;
        const double rh = rn[t];
        if (t < P.s) {
            if (!isfinite(rh) || !isfinite(s2)) {
                nonfinite = true;
                ratio = INFINITY;
            } else {
                ratio = rh > 0 ? sqrt(s2 / rh) : (s2 > 0 ? INFINITY : 0.0);
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) ratio = fmax(ratio, __shfl_xor(ratio, off, 64));
    nonfinite = __any(nonfinite);
    if (t == 0) {
        const double prev = relres[p];
        relres[p] = ratio;
        if (nonfinite) raise_flag(flags, 4);
        if (conv && (nonfinite || ratio <= stop || (it > 0 && ratio <= tol && ratio > 0.5 * prev))) {
            conv[p] = 1;
            iters[p] = it + 1;
        }
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
    // gather: 32 lanes along the samples (two samples each, s <= 64), 8 rows at
    // a time; all of a thread's loads are issued before the tile is written,
    // so they are in flight together.  A row's position is resolved once.
    constexpr int RPTH = kRestrictRows / (kThreads / 32);   // rows per thread
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    double v[RPTH][2];
#pragma unroll
    for (int k = 0; k < RPTH; ++k) {
        const int rr = ty + k * (kThreads / 32), row = r0 + rr;
        v[k][0] = v[k][1] = 0.0;
        if (rr >= nr) continue;
        if (KIND == kElliptic) {
            const int W = P.nH + 1;
            const int jj = row / W, ii = row - jj * W;
            const int ip = P.kx0 - P.x0 + ii, jp = P.ky0 - P.y0 + jj;
            const int pl = P.trans ? jp : ip, ql = P.trans ? ip : jp;
            const bool inner = pl >= 1 && pl <= P.L - 1 && ql >= 1 && ql <= P.Qn - 1;
            const double* src = inner ? X + (int64_t)(ql - 1) * lstride + (int64_t)(pl - 1) * P.sp : nullptr;
            const int bi = inner ? 0 : bidx_ccw(ip, jp, P.cx, P.cy);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int c = tx + 32 * h;
                if (c < ns) v[k][h] = inner ? src[c] : O[(int64_t)c * P.nb + bi];
            }
        } else {
            const int nv = P.b, hv = nv / 2;
            const int cell = row / nv, j = row - cell * nv;
            const int lc = P.kx0 - 1 + cell - P.x0;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int c = tx + 32 * h;
                if (c >= ns) continue;
                if (lc >= 0 && lc < P.cx) v[k][h] = X[(int64_t)lc * lstride + (int64_t)j * P.sp + c];
                else if (lc < 0) v[k][h] = vw[j] > 0 ? O[(int64_t)c * P.nb + (j - hv)] : 0.0;
                else v[k][h] = vw[j] < 0 ? O[(int64_t)c * P.nb + hv + j] : 0.0;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < RPTH; ++k) {
        const int rr = ty + k * (kThreads / 32);
        if (rr >= nr) continue;
#pragma unroll
        for (int h = 0; h < 2; ++h)
            if (tx + 32 * h < ns) tile[rr * LDT + tx + 32 * h] = v[k][h];
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

void launch_philox_draw(uint64_t seed, int patch, int n_node, int n_sample, uint32_t* words, double* normals, hipStream_t st) {
    const int64_t n = (int64_t)n_node * n_sample;
    const int blocks = (int)std::min<int64_t>(4096, (n + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(philox_draw_kernel, dim3(std::max(blocks, 1)), dim3(kThreads), 0, st, seed, (uint32_t)patch, n_node, n_sample,
                       words, normals);
}

static int max_chunks(const Ctx& c, int p0, int p1) {
    int m = 1;
    for (int p = p0; p < p1; ++p) m = std::max(m, (c.hp[p].nl + kChunkLines - 1) / kChunkLines);
    return m;
}

void launch_lift(Ctx& c, int p0, int p1, const double* adjQ) {
    StageTimer t(c, MSRS_K_LIFT);
    const bool ir = c.prec == MSRS_PREC_FP32_IR;
    const dim3 grid(p1 - p0, max_chunks(c, p0, p1));
    if (adjQ) {
        if (ir) hipLaunchKernelGGL(adj_lift_kernel<float>, grid, dim3(kThreads), 0, c.stream, c.dp, p0, adjQ, c.x32, c.part, c.maxch);
        else hipLaunchKernelGGL(adj_lift_kernel<double>, grid, dim3(kThreads), 0, c.stream, c.dp, p0, adjQ, c.x64, c.part, c.maxch);
    } else if (c.kind == kElliptic) {
        if (ir) hipLaunchKernelGGL((lift_kernel<kElliptic, float, true>), grid, dim3(kThreads), 0, c.stream, c.dp, p0, c.aL, c.om, c.vw, dx_of(c), c.xlift, c.part, c.maxch);
        else hipLaunchKernelGGL((lift_kernel<kElliptic, double, false>), grid, dim3(kThreads), 0, c.stream, c.dp, p0, c.aL, c.om, c.vw, dx_of(c), c.x64, c.part, c.maxch);
    } else {
        if (ir) hipLaunchKernelGGL((lift_kernel<kKinetic, float, true>), grid, dim3(kThreads), 0, c.stream, c.dp, p0, c.aL, c.om, c.vw, dx_of(c), c.xlift, c.part, c.maxch);
        else hipLaunchKernelGGL((lift_kernel<kKinetic, double, false>), grid, dim3(kThreads), 0, c.stream, c.dp, p0, c.aL, c.om, c.vw, dx_of(c), c.x64, c.part, c.maxch);
    }
    // FP32 refinement: the first solve reads the lifted data from xlift, the
    // adjoint source (dense) from x32
    c.rhs_in_xlift = ir && !adjQ;
    hipLaunchKernelGGL(norms_kernel, dim3(p1 - p0), dim3(64), 0, c.stream, c.dp, p0, c.part, c.maxch, c.rn, 0, (int32_t*)nullptr,
                       (double*)nullptr, (int32_t*)nullptr, 0, 0.0, 0.0, c.dflags);
}

void launch_residual(Ctx& c, int p0, int p1, bool stats_only, int it, const double* adjQ) {
    StageTimer t(c, MSRS_K_RESIDUAL);
    const double inv_eps = 1.0 / c.eps;
    int32_t* conv = stats_only ? nullptr : c.conv;
    float* x32 = stats_only ? nullptr : c.x32;
    const dim3 grid(p1 - p0, max_chunks(c, p0, p1));
    const int np = p1 - p0, nch = max_chunks(c, p0, p1);
    const int nch16 = (nch + 1) / 2;                 // the elliptic kernel's chunks of 16 lines
    const dim3 grid_ell((np + 7) / 8 * 8 * nch16);   // (patch, chunk) in the XCD-aware order of the kernel
    if (c.kind == kElliptic && adjQ)
        hipLaunchKernelGGL(residual_ell_kernel<true>, grid_ell, dim3(kResThreads), 0, c.stream, c.dp, p0, c.aL, c.om, c.x64, x32,
                           conv, c.part, c.maxch, adjQ, np, nch16);
    else if (c.kind == kElliptic)
        hipLaunchKernelGGL(residual_ell_kernel<false>, grid_ell, dim3(kResThreads), 0, c.stream, c.dp, p0, c.aL, c.om, c.x64, x32,
                           conv, c.part, c.maxch, (const double*)nullptr, np, nch16);
    else
        hipLaunchKernelGGL((residual_kernel<kKinetic>), grid, dim3(kThreads), 0, c.stream, c.dp, p0, c.aL, c.om, c.vw, dx_of(c), inv_eps,
                           c.x64, x32, conv, c.part, c.maxch);
    hipLaunchKernelGGL(norms_kernel, dim3(p1 - p0), dim3(64), 0, c.stream, c.dp, p0, c.part, c.maxch, c.rn, 1, conv,
                       c.gap + c.n_patches, c.iters, it, c.ir_tol, c.ir_stop, c.dflags);
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

void launch_adj_flux(Ctx& c, int p0, int p1, const double* Qs, double* C) {
    StageTimer t(c, MSRS_K_RESTRICT);
    int maxn = 0;
    for (int p = p0; p < p1; ++p) maxn = std::max(maxn, c.hp[p].nb * c.hp[p].s);
    const dim3 grid(p1 - p0, (maxn + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(adj_flux_kernel, grid, dim3(kThreads), 0, c.stream, c.dp, p0, c.aL, c.x64, Qs, C);
}

void launch_clear_conv(Ctx& c) {
    hipLaunchKernelGGL(clear_kernel, dim3(1), dim3(kThreads), 0, c.stream, c.conv, c.n_patches);
}

// NOCONV if a patch's largest relative residual is above tol after the last
// refinement iteration (the host-free form of the convergence check; a patch
// that stopped at stagnation below tol is fine).
__global__ void check_conv_kernel(const double* __restrict__ relres, int n, double tol, int32_t* flags) {
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        if (!(relres[i] <= tol)) raise_flag(flags, 1);
}

void launch_check_conv(Ctx& c) {
    hipLaunchKernelGGL(check_conv_kernel, dim3(1), dim3(kThreads), 0, c.stream, c.gap + c.n_patches, c.n_patches, c.ir_tol, c.dflags);
}

}  // namespace msrs
