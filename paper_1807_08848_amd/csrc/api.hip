// Host implementation of the msrs C ABI (include/msrs.h): problem set-up
// (domain decomposition into patches and buffered patches, Section 3),
// device buffers, orchestration of the offline and online stages, error
// latching and timing.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "msrs_internal.h"

using namespace msrs;

namespace {

thread_local std::string g_create_err;

int round16(int v) { return ((v + 15) / 16) * 16; }

// Smallest relative tolerance of an adaptive rank: the range finder resolves
// sigma_j down to about u sigma_1 (its second pass on the rotated snapshots),
// and a tolerance needs a margin above the rounding of the snapshots.
constexpr double kMinRankTol = 1e-12;

// Gauss-Legendre nodes (ascending) and weights on [-1, 1], Newton iteration
// on the three-term recurrence of the Legendre polynomials.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double pp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= n; ++j) {
                const double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            pp = n * (z * p1 - p2) / (z * z - 1.0);
            const double dz = p1 / pp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

template <typename T>
T* dalloc(Ctx& c, int64_t n) {
    if (n <= 0) n = 1;
    void* p = nullptr;
    MSRS_HIP_CHECK(hipMalloc(&p, (size_t)n * sizeof(T)));
    c.allocs.push_back(p);
    c.bytes += n * (int64_t)sizeof(T);
    return (T*)p;
}

msrs_status fail(Ctx* c, msrs_status st, const std::string& msg) {
    if (c) c->err = msg;
    else g_create_err = msg;
    return st;
}

msrs_status hip_fail(Ctx* c, const HipError& e) {
    char buf[512];
    std::snprintf(buf, sizeof buf, "HIP error %d (%s) in %s at %s:%d", (int)e.e, hipGetErrorString(e.e), e.what, e.file, e.line);
    return fail(c, e.e == hipErrorOutOfMemory ? MSRS_ERR_OOM : MSRS_ERR_HIP, buf);
}

// number of patches launched together: all (batched) or one (reference mode)
template <typename F>
void for_patches(Ctx& c, F&& f) {
    if (c.flags & MSRS_FLAG_PER_PATCH_LAUNCH) {
        for (int p = 0; p < c.n_patches; ++p) f(p, p + 1);
    } else {
        f(0, c.n_patches);
    }
}

void build_elliptic(Ctx& c) {
    const int N = c.N, M = c.M, nH = N / M;
    const bool fbb = (c.flags & MSRS_FLAG_FULL_BASIS_BOUNDARY) != 0, fball = (c.flags & MSRS_FLAG_FULL_BASIS) != 0;
    int64_t a_off = 0, om_off = 0, x_off = 0, E_off = 0, Y_off = 0, Q_off = 0, sv_off = 0, rn_off = 0, tw_off = 0;
    for (int m2 = 0; m2 < M; ++m2)
        for (int m1 = 0; m1 < M; ++m1) {
            const int p = m2 * M + m1;
            const bool full = fball || (fbb && (m1 == 0 || m1 == M - 1 || m2 == 0 || m2 == M - 1));
            const int d = full ? 0 : c.overlap[p];
            PatchDesc P{};
            const int x0 = std::max(0, m1 * nH - d), x1 = std::min(N, (m1 + 1) * nH + d);
            const int y0 = std::max(0, m2 * nH - d), y1 = std::min(N, (m2 + 1) * nH + d);
            P.x0 = x0; P.y0 = y0; P.cx = x1 - x0; P.cy = y1 - y0;
            P.trans = P.cx > P.cy ? 1 : 0;
            P.L = std::min(P.cx, P.cy);
            P.Qn = std::max(P.cx, P.cy);
            P.b = P.L - 1;
            P.nl = P.Qn - 1;
            P.bp = std::max(16, round16(P.b));
            P.nb = 2 * (P.cx + P.cy);
            P.s = full ? P.nb : c.s;
            P.sp = round16(P.s);
            P.kx0 = m1 * nH; P.ky0 = m2 * nH; P.nH = nH;
            P.nrows = (nH + 1) * (nH + 1);
            P.ncols = full ? P.nb : c.k;
            P.kreq = P.ncols;
            P.full = full ? 1 : 0;
            P.sampled = full ? 0 : 1;
            P.a_off = a_off; a_off += (int64_t)P.L * P.Qn;
            P.om_off = om_off; om_off += (int64_t)P.nb * P.s;
            P.x_off = x_off; x_off += (int64_t)P.nl * P.bp * P.sp;
            P.E_off = E_off; E_off += (int64_t)P.nl * P.bp * P.bp;
            P.Y_off = Y_off; Y_off += (int64_t)P.nrows * P.s;
            P.Q_off = Q_off; Q_off += (int64_t)P.nrows * P.ncols;
            P.sv_off = sv_off; sv_off += P.s;
            P.rn_off = rn_off; rn_off += 2 * P.sp;
            P.tw_off = tw_off; tw_off += 2LL * P.bp * P.sp;
            c.hp.push_back(P);
        }
    c.aL_total = a_off; c.omega_total = om_off; c.x_total = x_off; c.E_total = E_off; c.tw_total = tw_off;
    c.Y_total = Y_off; c.Q_total = Q_off; c.sv_total = sv_off;
    c.n_bdry = 4 * N;
    c.n_nodes = (int64_t)(N + 1) * (N + 1);
}

void build_kinetic(Ctx& c) {
    const int Nx = c.N, M = c.M, nH = Nx / M, nv = c.nv;
    const bool ends = (c.flags & MSRS_FLAG_FULL_BASIS_ENDS) != 0, fball = (c.flags & MSRS_FLAG_FULL_BASIS) != 0;
    int64_t a_off = 0, om_off = 0, x_off = 0, E_off = 0, Y_off = 0, Q_off = 0, sv_off = 0, rn_off = 0, tw_off = 0;
    for (int m = 0; m < M; ++m) {
        const bool full = fball || (ends && (m == 0 || m == M - 1));
        const int d = full ? 0 : c.overlap[m];
        PatchDesc P{};
        const int x0 = std::max(0, m * nH - d), x1 = std::min(Nx, (m + 1) * nH + d);
        P.x0 = x0; P.cx = x1 - x0; P.y0 = 0; P.cy = 0;
        P.trans = 0;
        P.L = nv; P.Qn = P.cx;
        P.b = nv; P.nl = P.cx; P.bp = std::max(16, round16(nv));
        P.nb = nv;
        P.s = full ? nv : c.s;
        P.sp = round16(P.s);
        P.kx0 = m * nH; P.ky0 = 0; P.nH = nH;
        P.nrows = (nH + 2) * nv;
        P.ncols = full ? nv : c.k;
        P.kreq = P.ncols;
        P.full = full ? 1 : 0;
        P.sampled = full ? 0 : 1;
        P.hg = c.hg != 0.0 ? 1 : 0;
        P.a_off = a_off; a_off += P.cx;
        P.om_off = om_off; om_off += (int64_t)P.nb * P.s;
        P.x_off = x_off; x_off += (int64_t)P.nl * P.bp * P.sp;
        P.E_off = E_off; E_off += (int64_t)P.nl * P.bp * P.bp;
        P.Y_off = Y_off; Y_off += (int64_t)P.nrows * P.s;
        P.Q_off = Q_off; Q_off += (int64_t)P.nrows * P.ncols;
        P.sv_off = sv_off; sv_off += P.s;
        P.rn_off = rn_off; rn_off += 2 * P.sp;
        P.tw_off = tw_off; tw_off += 2LL * P.bp * P.sp;
        c.hp.push_back(P);
    }
    c.aL_total = a_off; c.omega_total = om_off; c.x_total = x_off; c.E_total = E_off; c.tw_total = tw_off;
    c.Y_total = Y_off; c.Q_total = Q_off; c.sv_total = sv_off;
    c.n_bdry = nv;
    c.n_nodes = (int64_t)Nx * nv;
}

msrs_status validate(const msrs_problem_desc* d, std::string& msg) {
    if (!d) { msg = "desc is NULL"; return MSRS_ERR_ARG; }
    if (d->kind != MSRS_KIND_ELLIPTIC_Q1 && d->kind != MSRS_KIND_KINETIC_DO) { msg = "unknown kind"; return MSRS_ERR_ARG; }
    if (d->n_cells <= 0 || d->M <= 0 || d->n_cells % d->M) { msg = "M must divide n_cells"; return MSRS_ERR_ARG; }
    if (d->n_samples < 1 || d->n_samples > kMaxSamples) { msg = "n_samples must be in [1, 64]"; return MSRS_ERR_ARG; }
    if (d->rank < 1 || d->rank > d->n_samples) { msg = "rank must be in [1, n_samples]"; return MSRS_ERR_ARG; }
    if (d->precision != MSRS_PREC_FP64 && d->precision != MSRS_PREC_FP32_IR) { msg = "unknown precision"; return MSRS_ERR_ARG; }
    if (!d->overlap) { msg = "overlap is NULL"; return MSRS_ERR_ARG; }
    if (!(d->rank_tol >= 0.0 && d->rank_tol < 1.0)) { msg = "rank_tol must be in [0, 1)"; return MSRS_ERR_ARG; }
    if (d->rank_tol > 0.0 && d->rank_tol < kMinRankTol) {
        msg = "rank_tol below the range finder's resolution (1e-12)";
        return MSRS_ERR_ARG;
    }
    if (!(d->ir_tol >= 0.0) || !(d->ir_stop >= 0.0)) { msg = "ir_tol and ir_stop must be >= 0"; return MSRS_ERR_ARG; }
    if ((d->flags & MSRS_FLAG_LS_NORMAL) && (d->flags & MSRS_FLAG_LS_CORRECTED)) {
        msg = "MSRS_FLAG_LS_NORMAL and MSRS_FLAG_LS_CORRECTED exclude each other";
        return MSRS_ERR_ARG;
    }
    if ((d->flags & MSRS_FLAG_LS_CORRECTED) && (d->flags & MSRS_FLAG_CONSTRAINED_BC)) {
        msg = "the corrected semi-normal step applies to the least-squares system, not the constrained variant";
        return MSRS_ERR_ARG;
    }
    const int np = d->kind == MSRS_KIND_ELLIPTIC_Q1 ? d->M * d->M : d->M;
    for (int p = 0; p < np; ++p)
        if (d->overlap[p] < 0) { msg = "negative overlap"; return MSRS_ERR_ARG; }
    if (d->kind == MSRS_KIND_ELLIPTIC_Q1) {
        const int nH = d->n_cells / d->M;
        if (nH < 2) { msg = "patches need at least 2 cells per side"; return MSRS_ERR_ARG; }
        for (int m2 = 0; m2 < d->M; ++m2)
            for (int m1 = 0; m1 < d->M; ++m1) {
                const int dd = d->overlap[m2 * d->M + m1];
                const int cx = std::min(d->n_cells, (m1 + 1) * nH + dd) - std::max(0, m1 * nH - dd);
                const int cy = std::min(d->n_cells, (m2 + 1) * nH + dd) - std::max(0, m2 * nH - dd);
                if (std::min(cx, cy) - 1 > kMaxLine) { msg = "buffered patch too large: min side must be <= 129 cells"; return MSRS_ERR_ARG; }
            }
        if (d->M < 2) { msg = "elliptic needs M >= 2"; return MSRS_ERR_ARG; }
        if ((d->flags & (MSRS_FLAG_FULL_BASIS_BOUNDARY | MSRS_FLAG_FULL_BASIS)) && 4 * nH > kMaxSamples) {
            msg = "full bases need at most 64 boundary nodes per patch (4 N/M <= 64)";
            return MSRS_ERR_ARG;
        }
        if ((d->flags & MSRS_FLAG_CONSTRAINED_BC) && !(d->flags & (MSRS_FLAG_FULL_BASIS_BOUNDARY | MSRS_FLAG_FULL_BASIS))) {
            msg = "the constrained least-squares variant needs MSRS_FLAG_FULL_BASIS_BOUNDARY";
            return MSRS_ERR_ARG;
        }
        if ((d->flags & MSRS_FLAG_TWO_PASS) && (d->flags & (MSRS_FLAG_FULL_BASIS_BOUNDARY | MSRS_FLAG_FULL_BASIS))) {
            msg = "the two-pass range finder applies to sampled patches (no full-basis flags)";
            return MSRS_ERR_ARG;
        }
    } else {
        if (d->n_vel < 2 || d->n_vel > 64 || (d->n_vel & 1)) { msg = "n_vel must be even, 2..64"; return MSRS_ERR_ARG; }
        if (!(d->hg_g > -1.0 && d->hg_g < 1.0)) { msg = "hg_g must be in (-1, 1)"; return MSRS_ERR_ARG; }
        if (d->flags & (MSRS_FLAG_CONSTRAINED_BC | MSRS_FLAG_FULL_BASIS_BOUNDARY | MSRS_FLAG_TWO_PASS)) {
            msg = "MSRS_FLAG_FULL_BASIS_BOUNDARY, MSRS_FLAG_CONSTRAINED_BC and MSRS_FLAG_TWO_PASS are elliptic options";
            return MSRS_ERR_ARG;
        }
        if (!(d->eps > 0)) { msg = "eps must be positive"; return MSRS_ERR_ARG; }
        if (d->M < 2) { msg = "kinetic needs M >= 2"; return MSRS_ERR_ARG; }
        if (d->n_cells / d->M < 1) { msg = "patch too small"; return MSRS_ERR_ARG; }
    }
    return MSRS_OK;
}

void latch_from_host(Ctx& c, msrs_status& st) {
    // flags copied to pinned memory by the last synchronising call
    if (c.hflags[0]) { st = MSRS_ERR_NOT_SPD; c.err = "non-positive coefficient or pivot"; }
    else if (c.hflags[4]) { st = MSRS_ERR_NONFINITE; c.err = "non-finite boundary data, local solution or residual"; }
    else if (c.hflags[1]) { st = MSRS_ERR_NOCONV; c.err = "iterative refinement did not reach ir_tol"; }
    else if (c.hflags[2]) { st = MSRS_ERR_RANK; c.err = "sketch rank below the requested rank"; }
    else if (c.hflags[3]) { st = MSRS_ERR_ARG; c.err = "unsupported patch shape on the device"; }
}

void sync_flags(Ctx& c) {
    MSRS_HIP_CHECK(hipMemcpyAsync(c.hflags, c.dflags, kFlags * sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
    MSRS_HIP_CHECK(hipStreamSynchronize(c.stream));
}

void resolve_timing(Ctx& c) {
    for (auto& pe : c.pending) {
        float ms = 0.f;
        // events of online calls may sit on other streams than the handle's
        if (hipEventSynchronize(pe.b) == hipSuccess && hipEventElapsedTime(&ms, pe.a, pe.b) == hipSuccess) c.tms[pe.cls] += ms;
        c.event_pool.push_back(pe.a);
        c.event_pool.push_back(pe.b);
    }
    c.pending.clear();
}

}  // namespace

// ---------------------------------------------------------------- StageTimer
namespace msrs {
static hipEvent_t take_event(Ctx& c) {
    if (!c.event_pool.empty()) {
        hipEvent_t e = c.event_pool.back();
        c.event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    MSRS_HIP_CHECK(hipEventCreate(&e));
    return e;
}
StageTimer::StageTimer(Ctx& cc, int k, hipStream_t s) : c(cc), cls(k), st(s ? s : cc.stream) {
    c.tlaunch[cls] += 1;
    if (!c.timing) return;
    a = take_event(c);
    b = take_event(c);
    MSRS_HIP_CHECK(hipEventRecord(a, st));
}
StageTimer::~StageTimer() {
    if (!c.timing || !a) return;
    if (hipEventRecord(b, st) == hipSuccess) c.pending.push_back({cls, a, b});
}
}  // namespace msrs

namespace {
// An online workspace that the call on stream st may use: one last used on
// st (stream order puts this call after that use), else one whose last use
// has completed on the device, else null.
Ctx::OnlineWs* take_ws(Ctx* c, hipStream_t st) {
    for (auto& w : c->ws)
        if (w.used && w.last == st) return &w;
    for (auto& w : c->ws) {
        if (!w.used) return &w;
        const hipError_t q = hipEventQuery(w.done);
        if (q == hipSuccess) return &w;
        if (q != hipErrorNotReady) MSRS_HIP_CHECK(q);
    }
    return nullptr;
}

// Time one candidate: warm-up call, then reps calls between events on the
// handle's stream; average milliseconds per call.
template <typename F>
double time_calls(Ctx& c, int reps, F&& f) {
    hipEvent_t a, b;
    MSRS_HIP_CHECK(hipEventCreate(&a));
    MSRS_HIP_CHECK(hipEventCreate(&b));
    f();
    MSRS_HIP_CHECK(hipEventRecord(a, c.stream));
    for (int i = 0; i < reps; ++i) f();
    MSRS_HIP_CHECK(hipEventRecord(b, c.stream));
    MSRS_HIP_CHECK(hipEventSynchronize(b));
    float ms = 0.f;
    MSRS_HIP_CHECK(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms / reps;
}

}  // namespace

namespace {
// Enqueue stages a3-a7.  fixed_iters < 0: FP32 refinement until every patch
// has converged (host checks between iterations); fixed_iters >= 0: exactly
// that many iterations with no host synchronisation (converged patches skip
// their work) and a device-side NOCONV check, the form a graph can capture.
// adjQ != nullptr: the adjoint solves of the two-pass range finder instead
// (source R_K^T q for the columns q of adjQ, zero boundary values; the
// boundary values G^T q go to adjC in place of the restriction).
void sample_enqueue(Ctx* c, const double* omega_dev, int fixed_iters, const double* adjQ = nullptr, double* adjC = nullptr) {
    if (!adjQ) for_patches(*c, [&](int p0, int p1) { launch_omega(*c, omega_dev, p0, p1); });
    for_patches(*c, [&](int p0, int p1) { launch_lift(*c, p0, p1, adjQ); });
    if (c->prec == MSRS_PREC_FP64) {
        for_patches(*c, [&](int p0, int p1) { launch_sweep(*c, p0, p1, false, false); });
        for_patches(*c, [&](int p0, int p1) { launch_residual(*c, p0, p1, true, 0, adjQ); });
        c->last_ir_iters = 0;
    } else if (fixed_iters >= 0) {
        launch_clear_conv(*c);
        for (int it = 0; it < fixed_iters; ++it) {
            for_patches(*c, [&](int p0, int p1) { launch_sweep(*c, p0, p1, true, it == 0); });
            for_patches(*c, [&](int p0, int p1) { launch_residual(*c, p0, p1, false, it, adjQ); });
        }
        launch_check_conv(*c);
        c->last_ir_iters = fixed_iters;
    } else {
        launch_clear_conv(*c);
        int it = 0;
        int& hint = adjQ ? c->ir_hint_adj : c->ir_hint;
        const int first = std::min(c->ir_max, hint);
        for (; it < first; ++it) {
            for_patches(*c, [&](int p0, int p1) { launch_sweep(*c, p0, p1, true, it == 0); });
            for_patches(*c, [&](int p0, int p1) { launch_residual(*c, p0, p1, false, it, adjQ); });
        }
        // continue until every patch has converged (one host check per extra iteration)
        std::vector<int32_t> conv(c->n_patches);
        while (true) {
            MSRS_HIP_CHECK(hipMemcpyAsync(conv.data(), c->conv, c->n_patches * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
            MSRS_HIP_CHECK(hipStreamSynchronize(c->stream));
            const bool all = std::all_of(conv.begin(), conv.end(), [](int32_t v) { return v != 0; });
            if (all || it >= c->ir_max) {
                if (!all) launch_check_conv(*c);
                break;
            }
            for_patches(*c, [&](int p0, int p1) { launch_sweep(*c, p0, p1, true, it == 0); });
            for_patches(*c, [&](int p0, int p1) { launch_residual(*c, p0, p1, false, it, adjQ); });
            ++it;
        }
        std::vector<int32_t> iters(c->n_patches);
        MSRS_HIP_CHECK(hipMemcpyAsync(iters.data(), c->iters, c->n_patches * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
        MSRS_HIP_CHECK(hipStreamSynchronize(c->stream));
        int mx = 0;
        for (int v : iters) mx = std::max(mx, v);
        c->last_ir_iters = it;
        hint = std::max(1, mx);
    }
    if (adjQ) for_patches(*c, [&](int p0, int p1) { launch_adj_flux(*c, p0, p1, adjQ, adjC); });
    else for_patches(*c, [&](int p0, int p1) { launch_restrict(*c, p0, p1); });
}

// Stage a8: the range finder; with MSRS_FLAG_TWO_PASS the wide pass, the
// adjoint solves (refinement as the forward's: fixed_iters as in
// sample_enqueue) and the basis from Q^T G.
void range_enqueue(Ctx* c, int fixed_iters) {
    if (!c->two_pass) {
        for_patches(*c, [&](int p0, int p1) { launch_range(*c, p0, p1); });
        return;
    }
    for_patches(*c, [&](int p0, int p1) { launch_range_wide(*c, p0, p1); });
    sample_enqueue(c, nullptr, fixed_iters, c->tp_Q, c->tp_C);
    for_patches(*c, [&](int p0, int p1) { launch_range_two_pass(*c, p0, p1); });
}

void assemble_enqueue(Ctx* c, const double* coef_dev) {
    const int64_t n = c->kind == kElliptic ? (int64_t)c->N * c->N : c->N;
    MSRS_HIP_CHECK(hipMemcpyAsync(c->coef_copy, coef_dev, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    for_patches(*c, [&](int p0, int p1) {
        if (c->kind == kElliptic) launch_gather_elliptic(*c, c->coef_copy, p0, p1);
        else launch_gather_kinetic(*c, c->coef_copy, p0, p1);
    });
    for_patches(*c, [&](int p0, int p1) { launch_factor(*c, p0, p1); });
}

void drop_graph(Ctx* c) {
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
}
}  // namespace

// ---- basis files
namespace {
constexpr char kBasisMagic[8] = {'M', 'S', 'R', 'S', 'B', 'A', 'S', '1'};
constexpr uint32_t kBasisVersion = 2;   // 2: adds ir_stop after rank_tol

// FNV-1a (64-bit) over a byte range, continuing from h
uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

struct BasisWriter {
    FILE* f;
    uint64_t h = 1469598103934665603ull;
    bool ok = true;
    void put(const void* p, size_t n) {
        if (ok && n && fwrite(p, 1, n, f) != n) ok = false;
        h = fnv1a(h, p, n);
    }
    template <class V> void val(const V& v) { put(&v, sizeof(v)); }
};

struct BasisReader {
    FILE* f;
    uint64_t h = 1469598103934665603ull;
    bool ok = true;
    void get(void* p, size_t n) {
        if (ok && n && fread(p, 1, n, f) != n) ok = false;
        if (ok) h = fnv1a(h, p, n);
    }
    template <class V> V val() {
        V v{};
        get(&v, sizeof(v));
        return v;
    }
};

struct FileGuard {
    FILE* f;
    ~FileGuard() {
        if (f) fclose(f);
    }
};
}  // namespace

// ---------------------------------------------------------------- ABI
extern "C" {

int32_t msrs_version(void) { return 100; }

int32_t msrs_device_count(void) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return 0;
    return n;
}

msrs_status msrs_create(msrs_handle* out, const msrs_problem_desc* desc, void* stream, size_t hbm_budget_bytes) {
    if (!out) return fail(nullptr, MSRS_ERR_ARG, "out is NULL");
    *out = nullptr;
    std::string msg;
    msrs_status st = validate(desc, msg);
    if (st != MSRS_OK) return fail(nullptr, st, msg);
    if (msrs_device_count() <= 0) return fail(nullptr, MSRS_ERR_NO_DEVICE, "no HIP device visible");
    msrs_ctx* c = new (std::nothrow) msrs_ctx();
    if (!c) return fail(nullptr, MSRS_ERR_OOM, "host allocation failed");
    try {
        MSRS_HIP_CHECK(hipGetDevice(&c->device));
        c->kind = desc->kind == MSRS_KIND_ELLIPTIC_Q1 ? kElliptic : kKinetic;
        c->stream = (hipStream_t)stream;
        c->N = desc->n_cells; c->M = desc->M; c->s = desc->n_samples; c->k = desc->rank;
        c->prec = desc->precision;
        c->ir_max = desc->ir_max_iters > 0 ? desc->ir_max_iters : 30;
        c->ir_tol = desc->ir_tol > 0 ? desc->ir_tol : 1e-10;
        c->ir_stop = std::min(c->ir_tol, desc->ir_stop > 0 ? desc->ir_stop : 1e-13);
        c->eps = desc->kind == MSRS_KIND_KINETIC_DO ? desc->eps : 1.0;
        c->hg = desc->kind == MSRS_KIND_KINETIC_DO ? desc->hg_g : 0.0;
        c->rank_tol = desc->rank_tol;
        c->nv = desc->kind == MSRS_KIND_KINETIC_DO ? desc->n_vel : 0;
        c->seed = desc->seed;
        c->flags = desc->flags;
        c->constrained = desc->kind == MSRS_KIND_ELLIPTIC_Q1 && (desc->flags & MSRS_FLAG_CONSTRAINED_BC);
        c->nF = c->constrained ? 4 * desc->n_cells : 0;
        c->timing = (desc->flags & MSRS_FLAG_TIMING) != 0;
        c->budget = hbm_budget_bytes;
        const int np = c->kind == kElliptic ? c->M * c->M : c->M;
        c->overlap.assign(desc->overlap, desc->overlap + np);
        if (c->kind == kElliptic) build_elliptic(*c); else build_kinetic(*c);
        c->n_patches = (int)c->hp.size();
        // footprint
        const bool ir = c->prec == MSRS_PREC_FP32_IR;
        c->two_pass = (desc->flags & MSRS_FLAG_TWO_PASS) != 0;
        int64_t need = c->aL_total * 8 + c->omega_total * 8 + c->x_total * 8 + (ir ? c->x_total * 8 : 0) +
                       c->E_total * (ir ? 4 : 8) + c->Y_total * 8 + c->Q_total * 8 + c->sv_total * 8;
        if (c->two_pass) need += 2 * c->Y_total * 8 + c->omega_total * 8;
        need += (c->kind == kElliptic ? (int64_t)c->N * c->N : c->N) * 8;
        if (c->budget && (size_t)need > c->budget) {
            delete c;
            return fail(nullptr, MSRS_ERR_OOM, "footprint exceeds the HBM budget");
        }
        c->dp = dalloc<PatchDesc>(*c, c->n_patches);
        MSRS_HIP_CHECK(hipMemcpy(c->dp, c->hp.data(), sizeof(PatchDesc) * c->n_patches, hipMemcpyHostToDevice));
        c->aL = dalloc<double>(*c, c->aL_total);
        c->om = dalloc<double>(*c, c->omega_total);
        c->x64 = dalloc<double>(*c, c->x_total);
        if (ir) {
            c->x32 = dalloc<float>(*c, c->x_total);
            // zero once: the lift writes only the entries next to each patch's boundary
            c->xlift = dalloc<float>(*c, c->x_total);
            MSRS_HIP_CHECK(hipMemset(c->xlift, 0, sizeof(float) * (size_t)c->x_total));
        }
        c->E = ir ? (void*)dalloc<float>(*c, c->E_total) : (void*)dalloc<double>(*c, c->E_total);
        c->tw = dalloc<double>(*c, c->tw_total);
        c->Y = dalloc<double>(*c, c->Y_total);
        c->Q = dalloc<double>(*c, c->Q_total);
        c->rf_ws = dalloc<double>(*c, c->Q_total);
        for (auto& P : c->hp) c->rf_maxrc = std::max(c->rf_maxrc, (P.nrows + 511) / 512);
        c->rf_part = dalloc<double>(*c, (int64_t)c->n_patches * c->rf_maxrc * 4096);
        c->rf_small = dalloc<double>(*c, (int64_t)c->n_patches * 4096);
        c->rf_pval = dalloc<double>(*c, (int64_t)c->n_patches * c->rf_maxrc * 64);
        c->rf_pidx = dalloc<int32_t>(*c, (int64_t)c->n_patches * c->rf_maxrc * 64);
        c->rf_skip = dalloc<int32_t>(*c, c->n_patches);
        c->rf_second = dalloc<int32_t>(*c, c->n_patches);
        c->rf_small2 = dalloc<double>(*c, (int64_t)c->n_patches * 4096);
        c->rf_Z = dalloc<double>(*c, c->Y_total);
        if (c->two_pass) {
            // the wide pass: s basis columns at Y's offsets
            std::vector<PatchDesc> w(c->hp);
            for (auto& P : w) {
                P.Q_off = P.Y_off;
                P.ncols = P.kreq = P.s;
            }
            c->dp_wide = dalloc<PatchDesc>(*c, c->n_patches);
            MSRS_HIP_CHECK(hipMemcpy(c->dp_wide, w.data(), sizeof(PatchDesc) * c->n_patches, hipMemcpyHostToDevice));
            c->tp_Q = dalloc<double>(*c, c->Y_total);
            c->tp_W = dalloc<double>(*c, c->Y_total);
            c->tp_C = dalloc<double>(*c, c->omega_total);
        }
        c->sv = dalloc<double>(*c, c->sv_total);
        int64_t rn_total = 0;
        for (auto& P : c->hp) rn_total += 2 * P.sp;
        c->rn = dalloc<double>(*c, rn_total);
        c->gap = dalloc<double>(*c, 2 * c->n_patches);
        c->conv = dalloc<int32_t>(*c, c->n_patches);
        c->iters = dalloc<int32_t>(*c, c->n_patches);
        for (auto& P : c->hp) c->maxch = std::max(c->maxch, (P.nl + kChunkLines - 1) / kChunkLines);
        c->part = dalloc<double>(*c, (int64_t)c->n_patches * c->maxch * kMaxSamples);
        {
            std::vector<int32_t> ids(c->n_patches);
            for (int p = 0; p < c->n_patches; ++p) ids[p] = p;
            c->pid = dalloc<int32_t>(*c, c->n_patches);
            MSRS_HIP_CHECK(hipMemcpy(c->pid, ids.data(), ids.size() * sizeof(int32_t), hipMemcpyHostToDevice));
            std::vector<std::vector<int32_t>> grp(9);
            for (int p = 0; p < c->n_patches; ++p) grp[std::min(8, c->hp[p].bp / 16)].push_back(p);
            for (int g = 0; g < 9; ++g) {
                c->rgroup_n[g] = (int)grp[g].size();
                if (grp[g].empty()) continue;
                c->rgroup[g] = dalloc<int32_t>(*c, (int64_t)grp[g].size());
                MSRS_HIP_CHECK(hipMemcpy(c->rgroup[g], grp[g].data(), grp[g].size() * sizeof(int32_t), hipMemcpyHostToDevice));
            }
            // longest-processing-time order of the patches: cost of the banded
            // factor plus the s solve pairs, N (b+1)^2 + 4 N (b+1) s (ties by index)
            std::vector<int32_t> order(ids);
            auto cost = [&](int p) {
                const PatchDesc& P = c->hp[p];
                const double n = (double)P.b * P.nl, w = P.b + 1.0;
                return n * w * w + 4.0 * n * w * P.s;
            };
            std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
            c->lpt = dalloc<int32_t>(*c, c->n_patches);
            MSRS_HIP_CHECK(hipMemcpy(c->lpt, order.data(), order.size() * sizeof(int32_t), hipMemcpyHostToDevice));
            // sweep workgroups (patch, half), a chain of the half's lines each:
            // sorted by cost (lines x bp^2), the costliest half first, and the
            // second half of the list reversed, so that with two resident
            // workgroups per compute unit the i-th costliest shares its unit
            // with the i-th cheapest rather than with a chain of the same length
            std::vector<int32_t> items;
            for (int p = 0; p < c->n_patches; ++p) items.push_back(p << 1), items.push_back(p << 1 | 1);
            auto scost = [&](int32_t v) {
                const PatchDesc& P = c->hp[v >> 1];
                const int m = P.nl / 2, nlines = (v & 1) ? P.nl - 1 - m : m + 1;
                return (double)nlines * P.bp * P.bp;
            };
            std::stable_sort(items.begin(), items.end(), [&](int32_t a, int32_t b) { return scost(a) > scost(b); });
            std::reverse(items.begin() + c->n_patches, items.end());
            c->sweep_items = dalloc<int32_t>(*c, (int64_t)items.size());
            MSRS_HIP_CHECK(hipMemcpy(c->sweep_items, items.data(), items.size() * sizeof(int32_t), hipMemcpyHostToDevice));
            // the factor's chains (a half's lines of b x b inverses, b^3 each) in
            // the same paired order
            auto fcost = [&](int32_t v) {
                const PatchDesc& P = c->hp[v >> 1];
                const int m = P.nl / 2, nlines = (v & 1) ? P.nl - 1 - m : m;
                return (double)nlines * P.bp * P.bp * P.bp;
            };
            std::stable_sort(items.begin(), items.end(), [&](int32_t a, int32_t b) { return fcost(a) > fcost(b); });
            std::reverse(items.begin() + c->n_patches, items.end());
            c->factor_items = dalloc<int32_t>(*c, (int64_t)items.size());
            MSRS_HIP_CHECK(hipMemcpy(c->factor_items, items.data(), items.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        }
        c->dflags = dalloc<int32_t>(*c, kFlags);
        c->coef_copy = dalloc<double>(*c, c->kind == kElliptic ? (int64_t)c->N * c->N : c->N);
        MSRS_HIP_CHECK(hipMemset(c->dflags, 0, kFlags * sizeof(int32_t)));
        MSRS_HIP_CHECK(hipMemset(c->gap, 0, 2 * c->n_patches * sizeof(double)));
        MSRS_HIP_CHECK(hipMemset(c->iters, 0, c->n_patches * sizeof(int32_t)));
        MSRS_HIP_CHECK(hipMemset(c->x64, 0, c->x_total * sizeof(double)));
        MSRS_HIP_CHECK(hipHostMalloc((void**)&c->hflags, kFlags * sizeof(int32_t), hipHostMallocDefault));
        std::memset(c->hflags, 0, kFlags * sizeof(int32_t));
        // kinetic ordinate tables: [v (nv) | w (nv) | lambda (nv) | K (nv x nv)], with
        // K_ij = k(v_i, v_j) w_j the quadrature of the gain and lambda_i =
        // sum_j k(v_j, v_i) w_j that of the loss (isotropic: K_ij = w_j / 2, lambda = 1)
        const int nvt = std::max(c->nv, 1);
        std::vector<double> vw(3 * nvt + (int64_t)nvt * nvt, 0.0);
        if (c->kind == kKinetic) {
            const int nv = c->nv;
            std::vector<double> x, w;
            gauss_legendre(nv, x, w);
            for (int i = 0; i < nv; ++i) { vw[i] = x[i]; vw[nv + i] = w[i]; }
            const double g = c->hg;
            auto kern = [&](double a, double b) { return g == 0.0 ? 0.5 : 0.5 * (1 - g * g) / (1 + g * g + 2 * g * a * b); };
            for (int i = 0; i < nv; ++i) {
                double lam = 0.0;
                for (int j = 0; j < nv; ++j) {
                    vw[3 * nv + (int64_t)i * nv + j] = kern(x[i], x[j]) * w[j];
                    lam += kern(x[j], x[i]) * w[j];
                }
                vw[2 * nv + i] = g == 0.0 ? 1.0 : lam;
            }
        }
        c->vw = dalloc<double>(*c, (int64_t)vw.size());
        MSRS_HIP_CHECK(hipMemcpy(c->vw, vw.data(), vw.size() * sizeof(double), hipMemcpyHostToDevice));
        if (c->budget && (size_t)c->bytes > c->budget) {
            msrs_destroy(c);
            return fail(nullptr, MSRS_ERR_OOM, "footprint exceeds the HBM budget");
        }
    } catch (const HipError& e) {
        msrs_status s2 = hip_fail(nullptr, e);
        msrs_destroy(c);
        return s2;
    }
    *out = c;
    return MSRS_OK;
}

msrs_status msrs_assemble_patch(msrs_handle h, const double* coef_dev) {
    Ctx* c = h;
    if (!c) return fail(nullptr, MSRS_ERR_ARG, "handle is NULL");
    if (c->served) return fail(c, MSRS_ERR_STATE, "the handle is held by a server (destroy the server first)");
    if (!coef_dev) return fail(c, MSRS_ERR_ARG, "coef_dev is NULL");
    try {
        assemble_enqueue(c, coef_dev);
        MSRS_HIP_CHECK(hipGetLastError());
    } catch (const HipError& e) {
        return hip_fail(c, e);
    }
    c->assembled = true;
    c->sampled = c->ranged = c->coarse_ready = false;
    return MSRS_OK;
}

msrs_status msrs_sample_local_solutions(msrs_handle h, const double* omega_dev, double* Y_out_dev) {
    Ctx* c = h;
    if (!c) return fail(nullptr, MSRS_ERR_ARG, "handle is NULL");
    if (c->served) return fail(c, MSRS_ERR_STATE, "the handle is held by a server (destroy the server first)");
    if (!c->assembled) return fail(c, MSRS_ERR_STATE, "msrs_assemble_patch must come first");
    try {
        sample_enqueue(c, omega_dev, -1);
        if (Y_out_dev)
            MSRS_HIP_CHECK(hipMemcpyAsync(Y_out_dev, c->Y, c->Y_total * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        MSRS_HIP_CHECK(hipGetLastError());
    } catch (const HipError& e) {
        return hip_fail(c, e);
    }
    c->sampled = true;
    c->ranged = c->coarse_ready = false;
    return MSRS_OK;
}

// Host copy of the ranks the range finder chose at a tolerance (the device
// descriptors hold them once the range finder has run).
static void sync_ranks(Ctx* c) {
    if (!c->ranks_stale) return;
    std::vector<PatchDesc> d(c->n_patches);
    MSRS_HIP_CHECK(hipMemcpyAsync(d.data(), c->dp, sizeof(PatchDesc) * c->n_patches, hipMemcpyDeviceToHost, c->stream));
    MSRS_HIP_CHECK(hipStreamSynchronize(c->stream));
    for (int p = 0; p < c->n_patches; ++p) c->hp[p].ncols = d[p].ncols;
    c->ranks_stale = false;
}

msrs_status msrs_range_finder(msrs_handle h, double* Q_out_dev, double* sv_out_dev) {
    Ctx* c = h;
    if (!c) return fail(nullptr, MSRS_ERR_ARG, "handle is NULL");
    if (c->served) return fail(c, MSRS_ERR_STATE, "the handle is held by a server (destroy the server first)");
    if (!c->sampled) return fail(c, MSRS_ERR_STATE, "msrs_sample_local_solutions must come first");
    try {
        range_enqueue(c, -1);
        if (Q_out_dev)
            MSRS_HIP_CHECK(hipMemcpyAsync(Q_out_dev, c->Q, c->Q_total * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        if (sv_out_dev)
            MSRS_HIP_CHECK(hipMemcpyAsync(sv_out_dev, c->sv, c->sv_total * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        MSRS_HIP_CHECK(hipGetLastError());
    } catch (const HipError& e) {
        return hip_fail(c, e);
    }
    c->ranged = true;
    c->coarse_ready = false;
    c->ranks_stale = c->rank_tol > 0.0;
    return MSRS_OK;
}

msrs_status msrs_offline_graph_capture(msrs_handle h, const double* coef_dev) {
    Ctx* c = h;
    if (!c) return fail(nullptr, MSRS_ERR_ARG, "handle is NULL");
    if (c->served) return fail(c, MSRS_ERR_STATE, "the handle is held by a server (destroy the server first)");
    if (!coef_dev) return fail(c, MSRS_ERR_ARG, "coef_dev is NULL");
    if (!c->stream) return fail(c, MSRS_ERR_STATE, "graph capture needs a handle created on a non-default stream");
    if (c->prec == MSRS_PREC_FP32_IR && !c->sampled) return fail(c, MSRS_ERR_STATE, "an eager msrs_sample_local_solutions must come first");
    const bool timing = c->timing;
    try {
        drop_graph(c);
        MSRS_HIP_CHECK(hipStreamSynchronize(c->stream));
        const int iters = c->prec == MSRS_PREC_FP32_IR ? std::min(c->ir_max, c->ir_hint + 1) : 0;
        const int iters_adj = c->prec == MSRS_PREC_FP32_IR ? std::min(c->ir_max, c->ir_hint_adj + 1) : 0;
        c->timing = false;   // no event nodes inside the graph
        MSRS_HIP_CHECK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        try {
            assemble_enqueue(c, coef_dev);
            sample_enqueue(c, nullptr, iters);
            range_enqueue(c, iters_adj);
        } catch (const HipError&) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(c->stream, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        MSRS_HIP_CHECK(hipStreamEndCapture(c->stream, &c->graph));
        MSRS_HIP_CHECK(hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
        c->graph_iters = c->two_pass ? iters_adj : iters;   // the last solve of the step
    } catch (const HipError& e) {
        c->timing = timing;
        drop_graph(c);
        return hip_fail(c, e);
    }
    c->timing = timing;
    return MSRS_OK;
}

msrs_status msrs_offline_graph_launch(msrs_handle h) {
    Ctx* c = h;
    if (!c) return fail(nullptr, MSRS_ERR_ARG, "handle is NULL");
    if (c->served) return fail(c, MSRS_ERR_STATE, "the handle is held by a server (destroy the server first)");
    if (!c->graph_exec) return fail(c, MSRS_ERR_STATE, "msrs_offline_graph_capture must come first");
    try {
        StageTimer t(*c, MSRS_K_GRAPH);
        MSRS_HIP_CHECK(hipGraphLaunch(c->graph_exec, c->stream));
    } catch (const HipError& e) {
        return hip_fail(c, e);
    }
    c->assembled = c->sampled = c->ranged = true;
    c->coarse_ready = false;
    c->ranks_stale = c->rank_tol > 0.0;
    c->last_ir_iters = c->graph_iters;
    return MSRS_OK;
}

msrs_status msrs_copy_results(msrs_handle h, double* Y_out_dev, double* Q_out_dev, double* sv_out_dev) {
    Ctx* c = h;
    if (!c) return fail(nullptr, MSRS_ERR_ARG, "handle is NULL");
    if ((Y_out_dev && !c->sampled) || ((Q_out_dev || sv_out_dev) && !c->ranged))
        return fail(c, MSRS_ERR_STATE, "the requested results have not been computed");
    try {
        if (Y_out_dev) MSRS_HIP_CHECK(hipMemcpyAsync(Y_out_dev, c->Y, c->Y_total * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        if (Q_out_dev) MSRS_HIP_CHECK(hipMemcpyAsync(Q_out_dev, c->Q, c->Q_total * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        if (sv_out_dev) MSRS_HIP_CHECK(hipMemcpyAsync(sv_out_dev, c->sv, c->sv_total * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    } catch (const HipError& e) {
        return hip_fail(c, e);
    }
    return MSRS_OK;
}


msrs_status msrs_save(msrs_handle h, const char* path) {
    Ctx* c = h;
    if (!c) return fail(nullptr, MSRS_ERR_ARG, "handle is NULL");
    if (!path) return fail(c, MSRS_ERR_ARG, "path is NULL");
    if (c->served) return fail(c, MSRS_ERR_STATE, "the handle is held by a server (destroy the server first)");
    if (!c->ranged) return fail(c, MSRS_ERR_STATE, "msrs_range_finder must come first");
    try {
        sync_ranks(c);
        const int64_t ncoef = c->kind == kElliptic ? (int64_t)c->N * c->N : c->N;
        std::vector<double> coef(ncoef), Q(c->Q_total), sv(c->sv_total), gp(2 * c->n_patches);
        std::vector<int32_t> ranks(c->n_patches);
        for (int p = 0; p < c->n_patches; ++p) ranks[p] = c->hp[p].ncols;
        MSRS_HIP_CHECK(hipMemcpyAsync(coef.data(), c->coef_copy, ncoef * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        MSRS_HIP_CHECK(hipMemcpyAsync(Q.data(), c->Q, Q.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        MSRS_HIP_CHECK(hipMemcpyAsync(sv.data(), c->sv, sv.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        MSRS_HIP_CHECK(hipMemcpyAsync(gp.data(), c->gap, gp.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        MSRS_HIP_CHECK(hipStreamSynchronize(c->stream));
        FileGuard g{fopen(path, "wb")};
        if (!g.f) return fail(c, MSRS_ERR_IO, std::string("cannot open for writing: ") + path);
        if (fwrite(kBasisMagic, 1, sizeof(kBasisMagic), g.f) != sizeof(kBasisMagic))
            return fail(c, MSRS_ERR_IO, std::string("write failed: ") + path);
        BasisWriter w{g.f};
        w.val(kBasisVersion);
        w.val<int32_t>(c->kind == kElliptic ? MSRS_KIND_ELLIPTIC_Q1 : MSRS_KIND_KINETIC_DO);
        w.val<int32_t>(c->N);
        w.val<int32_t>(c->M);
        w.val<int32_t>(c->s);
        w.val<int32_t>(c->k);
        w.val<int32_t>(c->prec);
        w.val<int32_t>(c->ir_max);
        w.val<int32_t>(c->nv);
        w.val<uint64_t>(c->seed);
        w.val<double>(c->ir_tol);
        w.val<double>(c->eps);
        w.val<double>(c->hg);
        w.val<double>(c->rank_tol);
        w.val<double>(c->ir_stop);
        w.val<uint32_t>(c->flags);
        w.val<int32_t>(c->last_ir_iters);
        w.val<int32_t>((int32_t)c->overlap.size());
        w.put(c->overlap.data(), c->overlap.size() * sizeof(int32_t));
        w.val<int64_t>(ncoef);
        w.val<int64_t>(c->Q_total);
        w.val<int64_t>(c->sv_total);
        w.val<int64_t>((int64_t)gp.size());
        w.put(coef.data(), coef.size() * sizeof(double));
        w.put(Q.data(), Q.size() * sizeof(double));
        w.put(sv.data(), sv.size() * sizeof(double));
        w.put(gp.data(), gp.size() * sizeof(double));
        w.put(ranks.data(), ranks.size() * sizeof(int32_t));
        const uint64_t sum = w.h;
        if (!w.ok || fwrite(&sum, 1, sizeof(sum), g.f) != sizeof(sum) || fflush(g.f) != 0)
            return fail(c, MSRS_ERR_IO, std::string("write failed: ") + path);
    } catch (const HipError& e) {
        return hip_fail(c, e);
    } catch (const std::bad_alloc&) {
        return fail(c, MSRS_ERR_OOM, "host allocation failed");
    }
    return MSRS_OK;
}

msrs_status msrs_load(msrs_handle* out, const char* path, void* stream) {
    if (!out) return fail(nullptr, MSRS_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!path) return fail(nullptr, MSRS_ERR_ARG, "path is NULL");
    const std::string where = std::string(": ") + path;
    FileGuard g{fopen(path, "rb")};
    if (!g.f) return fail(nullptr, MSRS_ERR_IO, "cannot open for reading" + where);
    char magic[sizeof(kBasisMagic)];
    if (fread(magic, 1, sizeof(magic), g.f) != sizeof(magic) || std::memcmp(magic, kBasisMagic, sizeof(magic)))
        return fail(nullptr, MSRS_ERR_IO, "not a basis file" + where);
    BasisReader r{g.f};
    const uint32_t version = r.val<uint32_t>();
    if ((version != 1 && version != kBasisVersion) || !r.ok) return fail(nullptr, MSRS_ERR_IO, "unsupported basis file version" + where);
    msrs_problem_desc d{};
    d.kind = r.val<int32_t>();
    d.n_cells = r.val<int32_t>();
    d.M = r.val<int32_t>();
    d.n_samples = r.val<int32_t>();
    d.rank = r.val<int32_t>();
    d.precision = r.val<int32_t>();
    d.ir_max_iters = r.val<int32_t>();
    d.n_vel = r.val<int32_t>();
    d.seed = r.val<uint64_t>();
    d.ir_tol = r.val<double>();
    d.eps = r.val<double>();
    d.hg_g = r.val<double>();
    d.rank_tol = r.val<double>();
    d.ir_stop = version >= 2 ? r.val<double>() : 0.0;
    d.flags = r.val<uint32_t>();
    const int32_t ir_iters = r.val<int32_t>();
    const int32_t nov = r.val<int32_t>();
    if (!r.ok || nov < 1 || nov > (1 << 20)) return fail(nullptr, MSRS_ERR_IO, "truncated or corrupt header" + where);
    std::vector<int32_t> ov(nov);
    r.get(ov.data(), ov.size() * sizeof(int32_t));
    d.overlap = ov.data();
    const int64_t ncoef = r.val<int64_t>(), nQ = r.val<int64_t>(), nsv = r.val<int64_t>(), ngp = r.val<int64_t>();
    if (!r.ok) return fail(nullptr, MSRS_ERR_IO, "truncated or corrupt header" + where);
    const int64_t expect_ov = d.kind == MSRS_KIND_ELLIPTIC_Q1 ? (int64_t)d.M * d.M : d.M;
    const int64_t expect_coef = d.kind == MSRS_KIND_ELLIPTIC_Q1 ? (int64_t)d.n_cells * d.n_cells : d.n_cells;
    if (nov != expect_ov || ncoef != expect_coef)
        return fail(nullptr, MSRS_ERR_IO, "sizes do not match the description" + where);
    msrs_handle h = nullptr;
    const msrs_status cst = msrs_create(&h, &d, stream, 0);
    if (cst != MSRS_OK) return cst;
    Ctx* c = h;
    if (nQ != c->Q_total || nsv != c->sv_total || ngp != 2LL * c->n_patches) {
        msrs_destroy(h);
        return fail(nullptr, MSRS_ERR_IO, "sizes do not match the description" + where);
    }
    try {
        std::vector<double> coef(ncoef), Q(nQ), sv(nsv), gp(ngp);
        std::vector<int32_t> ranks(c->n_patches);
        r.get(coef.data(), coef.size() * sizeof(double));
        r.get(Q.data(), Q.size() * sizeof(double));
        r.get(sv.data(), sv.size() * sizeof(double));
        r.get(gp.data(), gp.size() * sizeof(double));
        r.get(ranks.data(), ranks.size() * sizeof(int32_t));
        const uint64_t sum = r.h;
        uint64_t stored = 0;
        if (!r.ok || fread(&stored, 1, sizeof(stored), g.f) != sizeof(stored) || stored != sum) {
            msrs_destroy(h);
            return fail(nullptr, MSRS_ERR_IO, "truncated file or checksum mismatch" + where);
        }
        for (int p = 0; p < c->n_patches; ++p) {
            if (ranks[p] < 1 || ranks[p] > c->hp[p].kreq || (ranks[p] != c->hp[p].kreq && !(d.rank_tol > 0.0))) {
                msrs_destroy(h);
                return fail(nullptr, MSRS_ERR_IO, "patch ranks do not match the description" + where);
            }
            c->hp[p].ncols = ranks[p];
        }
        MSRS_HIP_CHECK(hipMemcpyAsync(c->dp, c->hp.data(), sizeof(PatchDesc) * c->n_patches, hipMemcpyHostToDevice, c->stream));
        MSRS_HIP_CHECK(hipMemcpyAsync(c->coef_copy, coef.data(), ncoef * sizeof(double), hipMemcpyHostToDevice, c->stream));
        MSRS_HIP_CHECK(hipMemcpyAsync(c->Q, Q.data(), nQ * sizeof(double), hipMemcpyHostToDevice, c->stream));
        MSRS_HIP_CHECK(hipMemcpyAsync(c->sv, sv.data(), nsv * sizeof(double), hipMemcpyHostToDevice, c->stream));
        MSRS_HIP_CHECK(hipMemcpyAsync(c->gap, gp.data(), ngp * sizeof(double), hipMemcpyHostToDevice, c->stream));
        MSRS_HIP_CHECK(hipStreamSynchronize(c->stream));
    } catch (const HipError& e) {
        msrs_destroy(h);
        return fail(nullptr, e.e == hipErrorOutOfMemory ? MSRS_ERR_OOM : MSRS_ERR_HIP, std::string("HIP: ") + e.what);
    } catch (const std::bad_alloc&) {
        msrs_destroy(h);
        return fail(nullptr, MSRS_ERR_OOM, "host allocation failed");
    }
    c->last_ir_iters = ir_iters;
    c->assembled = c->sampled = false;
    c->ranged = true;
    c->coarse_ready = false;
    *out = h;
    return MSRS_OK;
}

msrs_status msrs_draw_boundary_samples(uint64_t seed, int32_t patch, int32_t n_node, int32_t n_sample, uint32_t* words_dev,
                                       double* normals_dev, void* stream) {
    if (patch < 0 || n_node < 0 || n_sample < 0) return fail(nullptr, MSRS_ERR_ARG, "negative patch, node or sample count");
    if ((int64_t)n_node * n_sample == 0) return MSRS_OK;
    try {
        launch_philox_draw(seed, patch, n_node, n_sample, words_dev, normals_dev, (hipStream_t)stream);
        MSRS_HIP_CHECK(hipGetLastError());
    } catch (const HipError& e) {
        return hip_fail(nullptr, e);
    }
    return MSRS_OK;
}

msrs_status msrs_copy_omega(msrs_handle h, double* omega_out_dev) {
    Ctx* c = h;
    if (!c) return fail(nullptr, MSRS_ERR_ARG, "handle is NULL");
    if (!omega_out_dev) return fail(c, MSRS_ERR_ARG, "omega_out_dev is NULL");
    if (!c->sampled) return fail(c, MSRS_ERR_STATE, "msrs_sample_local_solutions must come first");
    try {
        MSRS_HIP_CHECK(hipMemcpyAsync(omega_out_dev, c->om, c->omega_total * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    } catch (const HipError& e) {
        return hip_fail(c, e);
    }
    return MSRS_OK;
}

msrs_status msrs_set_max_batch(msrs_handle h, int32_t max_batch) {
    Ctx* c = h;
    if (!c) return fail(nullptr, MSRS_ERR_ARG, "handle is NULL");
    if (c->served) return fail(c, MSRS_ERR_STATE, "the handle is held by a server (destroy the server first)");
    if (max_batch < 1 || max_batch > 4096) return fail(c, MSRS_ERR_ARG, "max_batch must be in [1, 4096]");
    c->max_batch = max_batch;
    return MSRS_OK;
}

// Coarse unknowns (patch columns in patch order), the half bandwidth of the
// normal equations and the columns of the patches with Dirichlet / inflow
// rows, at the ranks in hp (or every patch at its requested rank).
static void coarse_layout(Ctx* c, bool requested, std::vector<int32_t>& bmap) {
    c->hc.assign(c->n_patches, CoarseDesc{});
    int off = 0;
    for (int p = 0; p < c->n_patches; ++p) {
        c->hc[p].col_off = off;
        c->hc[p].ncols = requested ? c->hp[p].kreq : c->hp[p].ncols;
        c->hc[p].b_off = -1;
        off += c->hc[p].ncols;
    }
    c->Np = off;
    // half bandwidth: last unknown of the farthest coupled patch
    int bw = 0;
    for (int p = 0; p < c->n_patches; ++p) {
        int far = p;
        if (c->kind == kElliptic) {
            const int m1 = p % c->M, m2 = p / c->M;
            if (m2 < c->M - 1) far = p + c->M + (m1 < c->M - 1 ? 1 : 0);
            else if (m1 < c->M - 1) far = p + 1;
        } else {
            far = std::min(p + 1, c->n_patches - 1);
        }
        bw = std::max(bw, c->hc[far].col_off + c->hc[far].ncols - 1 - c->hc[p].col_off);
    }
    c->bw = std::min(bw, c->Np - 1);
    c->bpatch.clear();
    bmap.clear();
    for (int p = 0; p < c->n_patches; ++p) {
        bool bd;
        if (c->kind == kElliptic) {
            const int m1 = p % c->M, m2 = p / c->M;
            bd = m1 == 0 || m2 == 0 || m1 == c->M - 1 || m2 == c->M - 1;
        } else {
            bd = p == 0 || p == c->n_patches - 1;
        }
        if (!bd) continue;
        c->hc[p].b_off = (int32_t)bmap.size();
        c->bpatch.push_back(p);
        for (int a = 0; a < c->hc[p].ncols; ++a) bmap.push_back(c->hc[p].col_off + a);
    }
    c->nB = (int)bmap.size();
}

msrs_status msrs_assemble_coarse(msrs_handle h) {
    Ctx* c = h;
    if (!c) return fail(nullptr, MSRS_ERR_ARG, "handle is NULL");
    if (c->served) return fail(c, MSRS_ERR_STATE, "the handle is held by a server (destroy the server first)");
    if (!c->ranged) return fail(c, MSRS_ERR_STATE, "msrs_range_finder must come first");
    try {
        sync_ranks(c);
        std::vector<int32_t> bmap;
        const bool first = !c->dc;
        if (first) {
            // buffers for every patch at its requested rank: the ranks a
            // tolerance chooses (never above it) fit without reallocation
            coarse_layout(c, true, bmap);
            if (c->bw + 1 > 1024) return fail(c, MSRS_ERR_ARG, "coarse band wider than 1023");
            c->Np_cap = c->Np;
            c->nB_cap = c->nB;
            int kmax = 0;
            for (auto& d : c->hc) kmax = std::max(kmax, d.ncols);
            c->dc = dalloc<CoarseDesc>(*c, c->n_patches);
            if (c->kind == kElliptic) {
                c->tr_stride = 2LL * 4 * (c->N / c->M) * kmax;
                c->tr = dalloc<double>(*c, (int64_t)c->n_patches * c->tr_stride);
            }
            c->band = dalloc<double>(*c, (int64_t)c->Np * (c->bw + 1));
            c->dbpatch = dalloc<int32_t>(*c, (int64_t)c->bpatch.size());
            c->bmap = dalloc<int32_t>(*c, c->nB);
            c->GB = dalloc<double>(*c, (int64_t)c->Np * c->nB);
            c->GT = dalloc<double>(*c, (int64_t)c->Np * c->nB);
            for (auto& w : c->ws) {
                w.cbuf = dalloc<double>(*c, (int64_t)c->Np * kOutPerLaunch);
                w.gbuf = dalloc<double>(*c, (int64_t)std::max(c->nB, c->nF) * kOutPerLaunch);
                w.zbuf = dalloc<double>(*c, (int64_t)c->Np * kOutPerLaunch);
                MSRS_HIP_CHECK(hipEventCreateWithFlags(&w.done, hipEventDisableTiming));
            }
            if (c->budget && (size_t)c->bytes > c->budget) return fail(c, MSRS_ERR_OOM, "coarse factor exceeds the HBM budget");
        }
        // the set-up rewrites the factor and G_B that online calls read
        for (auto& w : c->ws)
            if (w.used) MSRS_HIP_CHECK(hipEventSynchronize(w.done));
        if (first || c->rank_tol > 0.0) {
            coarse_layout(c, false, bmap);
            MSRS_HIP_CHECK(hipMemcpy(c->dc, c->hc.data(), sizeof(CoarseDesc) * c->n_patches, hipMemcpyHostToDevice));
            MSRS_HIP_CHECK(hipMemcpy(c->dbpatch, c->bpatch.data(), sizeof(int32_t) * c->bpatch.size(), hipMemcpyHostToDevice));
            if (c->nB) MSRS_HIP_CHECK(hipMemcpy(c->bmap, bmap.data(), sizeof(int32_t) * bmap.size(), hipMemcpyHostToDevice));
        }
        coarse_setup(*c);
        if (c->constrained) {
            const std::vector<int32_t> rows = constrained_rows(*c);
            const int nC = (int)rows.size() / 3;
            if (nC < 1 || nC > 1024) return fail(c, MSRS_ERR_ARG, "the constrained variant needs 1..1024 Dirichlet rows");
            if (!c->cons_rows) {
                // the rows are fixed by the geometry; the boundary unknowns are at most nB_cap
                const int64_t nBc = c->nB_cap, nF = c->nF;
                c->cons_rows = dalloc<int32_t>(*c, 3LL * nC);
                const int64_t sz[7] = {nC * nBc, nBc * nBc, nC * nBc, (int64_t)nC * nC, (int64_t)nC * nC, nC * nF, nBc * nF};
                for (int64_t n : sz) c->cons_ws.push_back(dalloc<double>(*c, n));
                c->GC = dalloc<double>(*c, (int64_t)c->Np_cap * nF);
                c->GCT = dalloc<double>(*c, (int64_t)c->Np_cap * nF);
                c->cons_cap_C = nC;
                if (c->budget && (size_t)c->bytes > c->budget) return fail(c, MSRS_ERR_OOM, "constrained set-up exceeds the HBM budget");
            }
            if (nC != c->cons_cap_C) return fail(c, MSRS_ERR_STATE, "Dirichlet rows changed since the first set-up");
            c->nC = nC;
            MSRS_HIP_CHECK(hipMemcpy(c->cons_rows, rows.data(), sizeof(int32_t) * rows.size(), hipMemcpyHostToDevice));
            const auto& v = c->cons_ws;
            coarse_constrained_setup(*c, ConsWs{c->cons_rows, v[0], v[1], v[2], v[3], v[4], v[5], v[6]});
        }
        MSRS_HIP_CHECK(hipGetLastError());
        sync_flags(*c);
        c->cond_normal = c->hflags[0] ? INFINITY : coarse_condition(*c, c->ws[0].cbuf);
        // kappa(P~)^2 above 1e12 leaves the normal equations fewer than about
        // four correct digits: the solves then take the corrected step
        c->lsq_correct = !c->constrained && !(c->flags & MSRS_FLAG_LS_NORMAL) &&
                         ((c->flags & MSRS_FLAG_LS_CORRECTED) || c->cond_normal > kLsqCorrectKappa);
        if (c->lsq_correct && lsq_correct_lds(*c) > 65536)
            return fail(c, MSRS_ERR_ARG, "the corrected semi-normal step needs N/M <= 680 (its rows of one patch in 64 KiB of LDS)");
    } catch (const HipError& e) {
        return hip_fail(c, e);
    }
    msrs_status st = MSRS_OK;
    if (c->hflags[0]) {
        st = MSRS_ERR_NOT_SPD;
        c->err = c->constrained ? "normal equations or constraint system not positive definite (P~ or its Dirichlet rows rank deficient)"
                                : "normal equations not positive definite (P~ rank deficient)";
    }
    if (st == MSRS_OK) c->coarse_ready = true;
    return st;
}

static msrs_status solve_common(Ctx* c, int32_t n_req, const double* f_dev, double* u_dev, void* stream, bool banded) {
    if (!c) return fail(nullptr, MSRS_ERR_ARG, "handle is NULL");
    if (!c->coarse_ready) return fail(c, MSRS_ERR_STATE, "msrs_assemble_coarse must come first");
    if (banded && c->constrained)
        return fail(c, MSRS_ERR_STATE, "the banded path solves the plain least-squares system only");
    if (n_req < 1 || n_req > c->max_batch) return fail(c, MSRS_ERR_ARG, "n_req must be in [1, max_batch]");
    if (!f_dev || !u_dev) return fail(c, MSRS_ERR_ARG, "f_dev / u_dev is NULL");
    try {
        hipStream_t st = stream ? (hipStream_t)stream : c->stream;
        Ctx::OnlineWs* w = take_ws(c, st);
        if (!w) return fail(c, MSRS_ERR_BUSY, "every online workspace is in use by unfinished calls");
        if (banded) {
            StageTimer t(*c, MSRS_K_CSOLVE, st);
            for (int r = 0; r < n_req; ++r)
                coarse_banded(*c, f_dev + (int64_t)r * c->n_bdry, u_dev + r * c->n_nodes, w->cbuf, w->zbuf, st);
        } else {
            std::vector<double*> u(n_req);
            std::vector<const double*> f(n_req);
            for (int r = 0; r < n_req; ++r) {
                u[r] = u_dev + r * c->n_nodes;
                f[r] = f_dev + (int64_t)r * c->n_bdry;
            }
            StageTimer t(*c, MSRS_K_CSOLVE, st);
            coarse_apply(*c, n_req, f.data(), u.data(), w->gbuf, w->cbuf, w->zbuf, st);
        }
        MSRS_HIP_CHECK(hipGetLastError());
        MSRS_HIP_CHECK(hipEventRecord(w->done, st));
        w->used = true;
        w->last = st;
    } catch (const HipError& e) {
        return hip_fail(c, e);
    }
    return MSRS_OK;
}

msrs_status msrs_coarse_condition(msrs_handle h, double* kappa_normal, double* kappa_ls) {
    Ctx* c = h;
    if (!c) return fail(nullptr, MSRS_ERR_ARG, "handle is NULL");
    if (!c->coarse_ready) return fail(c, MSRS_ERR_STATE, "msrs_assemble_coarse must come first");
    if (kappa_normal) *kappa_normal = c->cond_normal;
    if (kappa_ls) *kappa_ls = std::sqrt(c->cond_normal);
    return MSRS_OK;
}

msrs_status msrs_coarse_corrected(msrs_handle h, int32_t* corrected) {
    Ctx* c = h;
    if (!c) return fail(nullptr, MSRS_ERR_ARG, "handle is NULL");
    if (!corrected) return fail(c, MSRS_ERR_ARG, "corrected is NULL");
    if (!c->coarse_ready) return fail(c, MSRS_ERR_STATE, "msrs_assemble_coarse must come first");
    *corrected = c->lsq_correct ? 1 : 0;
    return MSRS_OK;
}

msrs_status msrs_solve_global(msrs_handle h, int32_t n_req, const double* f_dev, double* u_dev, void* stream) {
    return solve_common(h, n_req, f_dev, u_dev, stream, false);
}

msrs_status msrs_solve_global_banded(msrs_handle h, int32_t n_req, const double* f_dev, double* u_dev, void* stream) {
    return solve_common(h, n_req, f_dev, u_dev, stream, true);
}

msrs_status msrs_set_tuning(msrs_handle h, int32_t key, int32_t value) {
    Ctx* c = h;
    if (!c) return fail(nullptr, MSRS_ERR_ARG, "handle is NULL");
    auto in = [&](std::initializer_list<int> ok) {
        for (int v : ok)
            if (v == value) return true;
        return false;
    };
    switch (key) {
        case MSRS_TUNE_SWEEP_COLS:
            if (!in({16, 32, 64})) return fail(c, MSRS_ERR_ARG, "sweep columns must be 16, 32 or 64");
            c->sweep_cols32 = value;
            c->sweep_cols64 = std::min(value, 32);
            return MSRS_OK;
        case MSRS_TUNE_RECON_BATCH:
            if (!in({1, 2, 4, 8, 16})) return fail(c, MSRS_ERR_ARG, "reconstruction batch must be 1, 2, 4, 8 or 16");
            c->recon_batch = value;
            return MSRS_OK;
        case MSRS_TUNE_APPLY_BATCH:
            if (!in({4, 8, 16})) return fail(c, MSRS_ERR_ARG, "apply batch must be 4, 8 or 16");
            c->apply_batch = value;
            return MSRS_OK;
        case MSRS_TUNE_FACTOR_SHARE:
            if (!in({1, 2})) return fail(c, MSRS_ERR_ARG, "factor share must be 1 or 2");
            c->factor_share = value;
            return MSRS_OK;
        default:
            return fail(c, MSRS_ERR_ARG, "unknown tuning key");
    }
}

msrs_status msrs_autotune(msrs_handle h, int32_t stage, int32_t reps, msrs_tune_report* out) {
    Ctx* c = h;
    if (!c || !out) return fail(c, MSRS_ERR_ARG, "NULL argument");
    if (c->served) return fail(c, MSRS_ERR_STATE, "the handle is held by a server (destroy the server first)");
    if (reps < 1 || reps > 1000) return fail(c, MSRS_ERR_ARG, "reps must be in [1, 1000]");
    *out = msrs_tune_report{};
    auto record = [&](int key, int value, double ms) {
        if (out->n_trials < 32) {
            out->key[out->n_trials] = key;
            out->value[out->n_trials] = value;
            out->ms[out->n_trials] = ms;
            out->n_trials += 1;
        }
    };
    const bool timing = c->timing;
    c->timing = false;   // candidates are timed as whole calls
    msrs_status st = MSRS_OK;
    try {
        if (stage == MSRS_TUNE_STAGE_OFFLINE) {
            if (!c->assembled) { c->timing = timing; return fail(c, MSRS_ERR_STATE, "msrs_assemble_patch must come first"); }
            double best = 1e300;
            int arg = c->sweep_cols32;
            for (int sc : {16, 32, 64}) {
                c->sweep_cols32 = sc;
                c->sweep_cols64 = std::min(sc, 32);
                const double ms = time_calls(*c, reps, [&] {
                    const msrs_status s2 = msrs_sample_local_solutions(h, nullptr, nullptr);
                    if (s2 != MSRS_OK) throw s2;
                });
                record(MSRS_TUNE_SWEEP_COLS, sc, ms);
                if (ms < best) { best = ms; arg = sc; }
            }
            c->sweep_cols32 = arg;
            c->sweep_cols64 = std::min(arg, 32);
            // leave the handle sampled with the chosen shape (same results)
            st = msrs_sample_local_solutions(h, nullptr, nullptr);
        } else if (stage == MSRS_TUNE_STAGE_ONLINE) {
            if (!c->coarse_ready) { c->timing = timing; return fail(c, MSRS_ERR_STATE, "msrs_assemble_coarse must come first"); }
            const int nr = kOutPerLaunch;
            double* f = nullptr;
            double* u = nullptr;
            MSRS_HIP_CHECK(hipMalloc(&f, sizeof(double) * (size_t)nr * c->n_bdry));
            MSRS_HIP_CHECK(hipMalloc(&u, sizeof(double) * (size_t)nr * c->n_nodes));
            MSRS_HIP_CHECK(hipMemsetAsync(f, 0, sizeof(double) * (size_t)nr * c->n_bdry, c->stream));
            std::vector<const double*> fp(nr);
            std::vector<double*> up(nr);
            for (int r = 0; r < nr; ++r) {
                fp[r] = f + (int64_t)r * c->n_bdry;
                up[r] = u + (int64_t)r * c->n_nodes;
            }
            Ctx::OnlineWs* w = take_ws(c, c->stream);
            if (!w) {
                (void)hipFree(f);
                (void)hipFree(u);
                c->timing = timing;
                return fail(c, MSRS_ERR_BUSY, "every online workspace is in use by unfinished calls");
            }
            double best = 1e300;
            int ra = c->recon_batch, aa = c->apply_batch;
            for (int rb : {4, 8, 16})
                for (int ab : {4, 8, 16}) {
                    c->recon_batch = rb;
                    c->apply_batch = ab;
                    const double ms = time_calls(*c, reps, [&] { coarse_apply(*c, nr, fp.data(), up.data(), w->gbuf, w->cbuf, w->zbuf, c->stream); });
                    record(MSRS_TUNE_RECON_BATCH * 100 + MSRS_TUNE_APPLY_BATCH, rb * 100 + ab, ms);
                    if (ms < best) { best = ms; ra = rb; aa = ab; }
                }
            c->recon_batch = ra;
            c->apply_batch = aa;
            MSRS_HIP_CHECK(hipEventRecord(w->done, c->stream));
            w->used = true;
            w->last = c->stream;
            MSRS_HIP_CHECK(hipStreamSynchronize(c->stream));
            (void)hipFree(f);
            (void)hipFree(u);
        } else {
            c->timing = timing;
            return fail(c, MSRS_ERR_ARG, "unknown stage");
        }
    } catch (const HipError& e) {
        c->timing = timing;
        return hip_fail(c, e);
    } catch (msrs_status s2) {
        c->timing = timing;
        return s2;
    }
    c->timing = timing;
    return st;
}

msrs_status msrs_get_tuning(msrs_handle h, int32_t key, int32_t* value) {
    Ctx* c = h;
    if (!c || !value) return fail(c, MSRS_ERR_ARG, "NULL argument");
    switch (key) {
        case MSRS_TUNE_SWEEP_COLS: *value = c->sweep_cols32; return MSRS_OK;
        case MSRS_TUNE_RECON_BATCH: *value = c->recon_batch; return MSRS_OK;
        case MSRS_TUNE_APPLY_BATCH: *value = c->apply_batch; return MSRS_OK;
        case MSRS_TUNE_FACTOR_SHARE: *value = c->factor_share; return MSRS_OK;
        default: return fail(c, MSRS_ERR_ARG, "unknown tuning key");
    }
}

msrs_status msrs_query_layout(msrs_handle h, msrs_layout* out) {
    Ctx* c = h;
    if (!c || !out) return fail(c, MSRS_ERR_ARG, "NULL argument");
    try {
        sync_ranks(c);
    } catch (const HipError& e) {
        return hip_fail(c, e);
    }
    out->n_patches = c->n_patches;
    out->n_samples = c->s;
    out->rank = c->k;
    out->n_bdry = c->n_bdry;
    out->n_nodes = c->n_nodes;
    out->omega_total = c->omega_total;
    out->Y_total = c->Y_total;
    out->Q_total = c->Q_total;
    out->sv_total = c->sv_total;
    int64_t np = 0;
    for (auto& P : c->hp) np += P.ncols;
    out->coarse_dim = np;
    out->device_bytes = c->bytes;
    return MSRS_OK;
}

msrs_status msrs_query_patch(msrs_handle h, int32_t patch, msrs_patch_info* out) {
    Ctx* c = h;
    if (!c || !out) return fail(c, MSRS_ERR_ARG, "NULL argument");
    if (patch < 0 || patch >= c->n_patches) return fail(c, MSRS_ERR_ARG, "patch out of range");
    try {
        sync_ranks(c);
    } catch (const HipError& e) {
        return hip_fail(c, e);
    }
    const PatchDesc& P = c->hp[patch];
    out->x0 = P.x0; out->y0 = P.y0; out->cx = P.cx; out->cy = P.cy;
    out->kx0 = P.kx0; out->ky0 = P.ky0; out->nH = P.nH;
    out->n_bdry = P.nb;
    out->n_rows = P.nrows;
    out->n_cols = P.ncols;
    out->full_basis = P.full;
    out->line_len = P.b;
    out->n_lines = P.nl;
    out->n_samples = P.s;
    out->omega_off = P.om_off; out->Y_off = P.Y_off; out->Q_off = P.Q_off; out->sv_off = P.sv_off;
    return MSRS_OK;
}

msrs_status msrs_get_stats(msrs_handle h, msrs_stats* out) {
    Ctx* c = h;
    if (!c || !out) return fail(c, MSRS_ERR_ARG, "NULL argument");
    std::memset(out, 0, sizeof(*out));
    msrs_status st = MSRS_OK;
    try {
        sync_flags(*c);
        std::vector<double> g(2 * c->n_patches);
        MSRS_HIP_CHECK(hipMemcpy(g.data(), c->gap, g.size() * sizeof(double), hipMemcpyDeviceToHost));
        double mg = 1e300, mr = 0.0;
        for (int p = 0; p < c->n_patches; ++p) {
            if (c->hp[p].sampled) mg = std::min(mg, g[p]);
            mr = std::max(mr, g[c->n_patches + p]);
        }
        out->min_rel_gap = mg == 1e300 ? 0.0 : mg;
        out->max_rel_residual = mr;
        out->ir_iters = c->last_ir_iters;
        resolve_timing(*c);
        for (int i = 0; i < 12; ++i) { out->kernel_ms[i] = c->tms[i]; out->kernel_launches[i] = c->tlaunch[i]; }
    } catch (const HipError& e) {
        return hip_fail(c, e);
    }
    latch_from_host(*c, st);
    out->error_latched = st;
    return st;
}

msrs_status msrs_reset_stats(msrs_handle h) {
    Ctx* c = h;
    if (!c) return fail(nullptr, MSRS_ERR_ARG, "handle is NULL");
    try {
        MSRS_HIP_CHECK(hipStreamSynchronize(c->stream));
        resolve_timing(*c);
    } catch (const HipError& e) {
        return hip_fail(c, e);
    }
    for (int i = 0; i < 12; ++i) { c->tms[i] = 0; c->tlaunch[i] = 0; }
    return MSRS_OK;
}

const char* msrs_last_error(msrs_handle h) {
    if (!h) return g_create_err.c_str();
    return h->err.c_str();
}

void msrs_destroy(msrs_handle h) {
    msrs_ctx* c = h;
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto& w : c->ws)
        if (w.used) (void)hipEventSynchronize(w.done);
    for (auto& pe : c->pending) { (void)hipEventDestroy(pe.a); (void)hipEventDestroy(pe.b); }
    for (auto e : c->event_pool) (void)hipEventDestroy(e);
    for (auto& w : c->ws)
        if (w.done) (void)hipEventDestroy(w.done);
    drop_graph(c);
    for (void* p : c->allocs) (void)hipFree(p);
    if (c->hflags) (void)hipHostFree(c->hflags);
    delete c;
}

}  // extern "C"
