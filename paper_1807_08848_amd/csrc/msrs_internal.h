// Internal declarations of the msrs library: per-patch descriptors, the
// handle, and the host-side launchers of the kernels in k_*.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/msrs.h"

namespace msrs {

constexpr int kMaxLine = 128;      // padded unknowns per block row (elliptic); 16 | bp
constexpr int kMaxSamples = 64;    // padded samples per patch
constexpr int kMaxHgVel = 64;      // ordinates of an anisotropic-scattering (kinetic) problem at most
constexpr int kThreads = 256;      // threads of every per-patch workgroup
constexpr int kChunkLines = 8;     // block rows per workgroup of the lifting and residual kernels
constexpr int kOutPerLaunch = 32;  // requests per reconstruction launch
constexpr double kLsqCorrectKappa = 1e12;  // condition of P~^T P~ above which solves take the corrected step
constexpr int kOnlineWs = 4;       // concurrent msrs_solve_global calls per handle
constexpr int kFlags = 8;          // device error flags (see Ctx::dflags)

// Input and output pointers of the requests of one launch, passed by value in
// the kernel arguments (no device pointer array to stage).  Inputs may be
// device memory or mapped pinned host memory.
struct InPtrs { const double* f[kOutPerLaunch]; };
struct OutPtrs { double* u[kOutPerLaunch]; };

// One buffered patch, in the block-row ("line") view of the local problem.
//
// Elliptic: the interior unknowns of the buffered patch K~_m are grouped in
// lines of constant node index q along the shorter side (trans = 1 when the
// lines run along physical y).  In line coordinates a node is (p, q), p in
// [0, L] along the line and q in [0, Qn] across; interior unknowns are p in
// [1, L-1] (b = L-1 per line) and q in [1, Qn-1] (nl = Qn-1 lines).  The
// element coefficients of K~_m are gathered to aL[cr * L + cp] (cell row cr,
// cell column cp) in the same orientation.
//
// Kinetic: a line is one cell of K~_m with its nv ordinates (b = nv), nl = cx.
struct PatchDesc {
    int32_t x0, y0, cx, cy;   // buffered patch (cells)
    int32_t trans;            // elliptic: lines along physical y
    int32_t L, Qn;            // cells along / across lines
    int32_t b, nl, bp;        // unknowns per line, lines, padded line length
    int32_t nb;               // boundary values per sample column
    int32_t s, sp;            // sample columns and their padding to 16
    int32_t kx0, ky0, nH;     // patch K_m (cells)
    int32_t nrows, ncols;     // rows of Y / Q, columns of Q
    int32_t full;             // full (delta) basis: Omega = identity
    int32_t sampled;          // Omega drawn at random (0 for full-basis patches)
    int32_t hg;               // kinetic: anisotropic (Henyey-Greenstein) scattering, tables in vw
    int32_t kreq;             // requested basis columns (ncols before a tolerance-chosen rank lowers it)
    int64_t a_off;            // aL (doubles)
    int64_t om_off;           // Omega, nb x s column-major
    int64_t x_off;            // line vectors, nl x bp x sp (samples fastest)
    int64_t E_off;            // inverse diagonal blocks, nl x bp x bp (column-major blocks)
    int64_t Y_off;            // nrows x s column-major
    int64_t Q_off;            // nrows x ncols column-major
    int64_t sv_off;           // s singular values
    int64_t rn_off;           // per-sample norms: [0,sp) ||rhs||^2, [sp,2sp) ||r||^2
    int64_t tw_off;           // sweeps: the two halves' couplings into the middle line, 2 x bp x sp
};

// Online (coarse) geometry of one patch.
struct CoarseDesc {
    int32_t col_off;          // first unknown of the patch in the least-squares system
    int32_t ncols;            // its unknowns
    int32_t nbr[8];           // elliptic: patches that share an edge or vertex (-1 if none)
    int32_t b_off;            // first column of the patch in G_B (boundary patches), else -1
    int32_t pad_[5];
};

enum Kind { kElliptic = 0, kKinetic = 1 };


struct Ctx {
    int kind = kElliptic;
    int device = 0;
    hipStream_t stream = nullptr;
    int N = 0, M = 0, s = 0, k = 0, prec = 0, nv = 0;
    int ir_max = 30;
    double ir_tol = 1e-10;
    double ir_stop = 1e-13;   // a patch stops refining at this relative residual (or at stagnation below ir_tol)
    double eps = 1.0;
    double hg = 0.0;          // kinetic: Henyey-Greenstein anisotropy g (0: isotropic)
    double rank_tol = 0.0;    // > 0: each sampled patch keeps its numerical rank at this tolerance (at most k)
    uint64_t seed = 0;
    uint32_t flags = 0;
    size_t budget = 0;
    int n_patches = 0;
    int ir_hint = 3;
    int ir_hint_adj = 3;          // the same for the adjoint solves of the two-pass range finder
    int last_ir_iters = 0;
    std::string err;

    std::vector<PatchDesc> hp;    // host copy of descriptors
    std::vector<int32_t> overlap;

    // device buffers
    PatchDesc* dp = nullptr;
    double* aL = nullptr;         // gathered coefficients (per patch)
    double* om = nullptr;         // Omega
    double* x64 = nullptr;        // FP64 line vectors (solution)
    float* x32 = nullptr;         // FP32 line vectors (FP32_IR: residual / correction)
    float* xlift = nullptr;       // FP32_IR: the lifted boundary data, zero except next to each patch's boundary
    bool rhs_in_xlift = false;    // the next first solve reads xlift (else x32: the adjoint source)
    void* E = nullptr;            // inverse blocks (float or double)
    void* tw = nullptr;           // middle-line couplings of the twisted sweeps (float or double)
    int64_t tw_total = 0;
    double* Y = nullptr;
    double* Q = nullptr;
    double* sv = nullptr;
    double* rn = nullptr;         // norms
    double* gap = nullptr;        // per patch relative gap
    int32_t* conv = nullptr;      // per patch converged flag
    // device error flags: [0] NOT_SPD, [1] NOCONV, [2] RANK, [3] unsupported patch shape, [4] non-finite values
    int32_t* dflags = nullptr;
    int32_t* hflags = nullptr;    // pinned host mirror
    double* vw = nullptr;         // kinetic ordinates and weights (2 nv)
    double* rf_ws = nullptr;      // range finder workspace (shape of Q)
    double* rf_part = nullptr;    // per (patch, row chunk) partial Gram matrices, 64 x 64 each
    double* rf_small = nullptr;   // per patch 64 x 64 factor (B, L^{-T}, signs)
    double* rf_pval = nullptr;    // per (patch, row chunk) column maxima
    int32_t* rf_pidx = nullptr;
    int32_t* rf_skip = nullptr;   // per patch: the second Cholesky-QR pass is not needed
    int32_t* rf_second = nullptr; // per patch: the range finder's second (rotated) pass is needed
    double* rf_small2 = nullptr;  // per patch 64 x 64: the first pass's eigenvectors (second pass only)
    double* rf_Z = nullptr;       // rotated snapshots Z = Y V (shape of Y; second pass only)
    int rf_maxrc = 1;             // row chunks per patch at most
    // two-pass range finder (MSRS_FLAG_TWO_PASS): the wide pass's descriptors
    // (basis at Y's offsets with s columns), its basis and workspace (shape of
    // Y), and the adjoint boundary values G^T Q (shape of Omega)
    bool two_pass = false;
    PatchDesc* dp_wide = nullptr;
    double* tp_Q = nullptr;
    double* tp_W = nullptr;
    double* tp_C = nullptr;
    double* coef_copy = nullptr;  // device copy of the coefficient field (traces)
    int32_t* iters = nullptr;     // per patch refinement iterations at convergence
    double* part = nullptr;       // per (patch, line chunk) partial column sums, 64 each
    int32_t* pid = nullptr;       // 0..n_patches-1 (single-patch launches)
    int32_t* rgroup[9] = {};      // patches with line-tile count R (device lists)
    int rgroup_n[9] = {};
    int32_t* lpt = nullptr;       // every patch, costliest first (factor launches over mixed line lengths)
    int32_t* sweep_items = nullptr;   // 2 n_patches (patch << 1 | half): sweep workgroup order, costliest paired with cheapest
    int32_t* factor_items = nullptr;  // 2 n_patches (patch << 1 | half): factor chains in the same paired order, by factor cost
    bool ranks_stale = false;     // the device descriptors hold ranks the host copy has not seen
    int maxch = 1;                // line chunks per patch at most

    int64_t omega_total = 0, Y_total = 0, Q_total = 0, sv_total = 0;
    int64_t x_total = 0, E_total = 0, aL_total = 0;
    int64_t bytes = 0;

    bool assembled = false, sampled = false, ranged = false, coarse_ready = false;

    // online
    int max_batch = 64;
    int sweep_cols32 = 64;       // samples per sweep workgroup (FP32), 16 | value
    int factor_share = 2;        // factor workgroups per compute unit the kernel's registers allow (1 or 2)
    int sweep_cols64 = 32;       // samples per sweep workgroup (FP64)
    int recon_batch = 8;         // requests per reconstruction pass (1, 2, 4, 8, 16)
    int apply_batch = 8;         // requests per G_B workgroup (4, 8, 16)
    int Np = 0, bw = 0;
    double norm1_normal = 0.0;    // ||P~^T P~||_1 of the last coarse assembly
    double cond_normal = 0.0;     // 1-norm condition estimate of P~^T P~ (0 before msrs_assemble_coarse)
    bool lsq_correct = false;     // online solves take a corrected semi-normal step
    int Np_cap = 0, nB_cap = 0;   // sizes the coarse buffers were allocated for (every patch at its requested rank)
    std::vector<CoarseDesc> hc;
    CoarseDesc* dc = nullptr;
    double* tr = nullptr;         // traces (values, fluxes)
    double* band = nullptr;       // normal matrix, then its Cholesky factor (lower band)
    double* GB = nullptr;         // (P~^T P~)^{-1} restricted to the columns of boundary-patch unknowns, Np x nB
    double* GT = nullptr;         // the same, row-major (row j contiguous): the batched solve streams its rows
    // constrained least squares (Dirichlet rows exact): G_C (Np x nF, nF = 4N)
    // maps the global boundary data to c; GCT is it row-major
    bool constrained = false;
    int nC = 0, nF = 0;           // Dirichlet rows, boundary data length
    double* GC = nullptr;
    double* GCT = nullptr;
    int g_len() const { return constrained ? nF : nB; }   // per-request length of the batched solve's input
    std::vector<double*> cons_ws;  // constrained set-up workspaces (BB, H, X, S, band, W, V)
    int32_t* cons_rows = nullptr;
    int cons_cap_C = 0;            // rows the workspaces were sized for
    int nB = 0;                   // unknowns of the patches with Dirichlet / inflow rows
    std::vector<int32_t> bpatch;  // those patches (host), and on the device:
    int32_t* dbpatch = nullptr;
    int32_t* bmap = nullptr;      // column i of G_B -> its unknown in the least-squares system
    int64_t tr_stride = 0;        // doubles per patch of tr
    // online workspaces: msrs_solve_global calls on different streams take
    // distinct ones; a workspace is free once its event has completed
    struct OnlineWs {
        double* cbuf = nullptr;
        double* gbuf = nullptr;
        double* zbuf = nullptr;      // Np x kOutPerLaunch, the corrected semi-normal step's workspace
        hipEvent_t done = nullptr;   // recorded after the last use
        hipStream_t last = nullptr;  // stream of the last use (stream order makes reuse there safe)
        bool used = false;
    };
    OnlineWs ws[kOnlineWs];
    int served = 0;               // servers holding this handle (offline and set-up calls refused)

    // captured offline step (msrs_offline_graph_capture)
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int graph_iters = 0;
    int32_t n_bdry = 0;
    int64_t n_nodes = 0;
    std::vector<void*> allocs;

    // timing (MSRS_FLAG_TIMING): events around every launcher, resolved in msrs_get_stats
    bool timing = false;
    double tms[12] = {0};
    int64_t tlaunch[12] = {0};
    struct Pending { int cls; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
};

// ---- launchers (k_*.hip) ---------------------------------------------------
// Every launcher enqueues on c.stream and takes the patch range [p0, p1).
void launch_gather_elliptic(Ctx& c, const double* a, int p0, int p1);
void launch_gather_kinetic(Ctx& c, const double* sigma, int p0, int p1);
void launch_omega(Ctx& c, const double* user, int p0, int p1);
void launch_philox_draw(uint64_t seed, int patch, int n_node, int n_sample, uint32_t* words, double* normals, hipStream_t st);
// adjQ: the adjoint source f_I = R_K^T q, q the columns of adjQ (Y's layout)
void launch_lift(Ctx& c, int p0, int p1, const double* adjQ = nullptr);
void launch_factor(Ctx& c, int p0, int p1);
void launch_sweep(Ctx& c, int p0, int p1, bool fp32, bool first);   // first: the first solve of a refinement
void launch_residual(Ctx& c, int p0, int p1, bool stats_only, int it, const double* adjQ = nullptr);
void launch_restrict(Ctx& c, int p0, int p1);
void launch_adj_flux(Ctx& c, int p0, int p1, const double* Qs, double* C);   // C = f_B - A_BI z (Omega's layout)
void launch_range(Ctx& c, int p0, int p1);
// two-pass range finder: the wide pass (orthonormal basis of span(Y) at its
// numerical rank into tp_Q), then, after the adjoint solves have written
// G^T tp_Q into tp_C, the basis from the SVD of (G^T tp_Q)^T
void launch_range_wide(Ctx& c, int p0, int p1);
void launch_range_two_pass(Ctx& c, int p0, int p1);
void launch_clear_conv(Ctx& c);
void launch_check_conv(Ctx& c);

// coarse (k_coarse.hip)
void coarse_setup(Ctx& c);     // traces, normal matrix, Cholesky (enqueued)
// 1-norm condition estimate of the factored normal matrix (host-driven band
// solves on the handle's stream; work: Np device doubles)
double coarse_condition(Ctx& c, double* work);
// Batched path: n_req requests, boundary data f[r] (device or mapped pinned
// host memory), outputs u[r] (device), workspaces gbuf (nB x kOutPerLaunch)
// and cbuf (Np x kOutPerLaunch).  Reads the handle only, so several streams
// may run it at once.
void coarse_apply(const Ctx& c, int n_req, const double* const* f, double* const* u, double* gbuf, double* cbuf,
                  double* zbuf, hipStream_t st);
// With lsq_correct set: one corrected semi-normal step per solve, zbuf
// (Np x kOutPerLaunch) its workspace (unused, may be null, otherwise).  LDS
// bytes per workgroup of its row kernel (at most 64 KiB must hold).
size_t lsq_correct_lds(const Ctx& c);
// Constrained least squares: the Dirichlet rows (3 ints each: patch, node of
// dK_m, global boundary index) and the set-up of G_C / GCT from G_B, with
// workspaces sized for nC rows and nB boundary unknowns.
struct ConsWs {
    int32_t* rows;   // 3 nC
    double* BB;      // nC x nB
    double* H;       // nB x nB
    double* X;       // nC x nB
    double* S;       // nC x nC
    double* band;    // nC x nC
    double* W;       // nC x nF
    double* V;       // nB x nF
};
std::vector<int32_t> constrained_rows(const Ctx& c);
void coarse_constrained_setup(Ctx& c, const ConsWs& w);
// Banded path: one request by P~^T d and two band triangular solves; cbuf Np.
void coarse_banded(const Ctx& c, const double* f, double* u, double* cbuf, double* zbuf, hipStream_t st);

// timing helpers (api.hip)
struct StageTimer {
    Ctx& c;
    int cls;
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t st;
    StageTimer(Ctx& cc, int k, hipStream_t s = nullptr);
    ~StageTimer();
};

}  // namespace msrs

// the opaque handle of the ABI is the library context
struct msrs_ctx : public msrs::Ctx {};

#define MSRS_HIP_CHECK(expr)                                                          \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess) throw msrs::HipError(e_, #expr, __FILE__, __LINE__);    \
    } while (0)

namespace msrs {
struct HipError {
    hipError_t e;
    const char* what;
    const char* file;
    int line;
    HipError(hipError_t ee, const char* w, const char* f, int l) : e(ee), what(w), file(f), line(l) {}
};
}  // namespace msrs
