/*
 * msrs.h -- C ABI of the multiscale random-sampling library for MI355X (gfx950).
 *
 * The library computes the offline stage of the domain-decomposition method
 * of Chen, Li, Lu and Wright, "Random sampling and efficient algorithms for
 * multiscale PDEs" (Section 3, Algorithm alg:summary): for every buffered
 * patch, local fine-scale solves with i.i.d. N(0,1) boundary data
 * (RanLocalSolu), restriction to the patch, and a range finder that keeps an
 * orthonormal rank-k basis.  The online stage (least-squares gluing and
 * reconstruction, eqs. elliptic_cond_reduced and rte_cond_reduced) reuses the
 * resident bases.  Two problems are supported:
 *
 *   MSRS_KIND_ELLIPTIC_Q1  -div(a grad u) = 0 on [0,1]^2, Dirichlet data
 *                          (Section 5), bilinear finite elements on an N x N
 *                          cell grid, M x M coarse patches;
 *   MSRS_KIND_KINETIC_DO   v d_x f = (sigma/eps)(<f> - f) on [0,1] x [-1,1],
 *                          inflow data (Section 4, isotropic scattering),
 *                          upwind discrete ordinates on N_x cells, M patches.
 *
 * Conventions shared by every call
 *  - Every function returns msrs_status; no C++ exception crosses the ABI.
 *  - "device" pointers are HIP device allocations of the caller (e.g. torch
 *    tensors); "host" pointers are ordinary host memory.  The caller owns
 *    every pointer it passes; device pointers must stay valid until the work
 *    enqueued on the handle's stream has completed.  The library owns its
 *    workspace, factors, bases and coarse factor, allocated in msrs_create /
 *    msrs_assemble_coarse and released by msrs_destroy.
 *  - All device work is enqueued on the stream given to msrs_create (or to
 *    msrs_solve_global); calls return without synchronising unless stated.
 *  - Errors the kernels detect (non-positive pivot, non-finite values,
 *    refinement that does not converge) are latched on the device and
 *    reported by msrs_get_stats (which synchronises) and by the next call
 *    that synchronises; msrs_last_error gives a message.
 *  - Floating-point data are IEEE binary64, integers are int32/int64 as typed.
 *  - One handle per host thread.
 *
 * Layouts
 *  - Elliptic coefficient a: N*N values, element (i,j) = cell
 *    [i h,(i+1)h] x [j h,(j+1)h] at index j*N + i (h = 1/N).
 *  - Kinetic cross section sigma: N_x values at the cell centres.
 *  - Patch p = m2*M + m1 (elliptic) or p = m (kinetic).
 *  - Omega (boundary samples) of patch p: n_bdry(p) x s, column-major, at
 *    offset omega_off(p) of the concatenated array.  Elliptic boundary nodes
 *    of the buffered patch are ordered counter-clockwise from its lower-left
 *    node; kinetic inflow values are [left inflow at the v>0 ordinates
 *    (ascending v), right inflow at the v<0 ordinates (ascending v)].
 *  - Y (snapshots) of patch p: n_rows(p) x s, column-major, offset Y_off(p).
 *    Elliptic rows are the (nH+1)^2 nodes of the closed patch K_m, row-major
 *    (index jj*(nH+1)+ii, nH = N/M); kinetic rows are (cell c, ordinate j) ->
 *    c*n_vel + j for the nH+2 cells [first cell of K_m - 1, last cell + 1].
 *  - Q (bases) of patch p: n_rows(p) x n_cols(p), column-major, offset Q_off(p);
 *    the space reserved is n_rows(p) x k (x n_bdry for a full-basis patch),
 *    whose columns past n_cols(p) are zero.
 *  - Global boundary data f of one request: elliptic 4N values
 *    counter-clockwise from node (0,0) (bottom i=0..N-1, right j=0..N-1, top
 *    i=N..1, left j=N..1); kinetic n_vel values laid out as Omega.
 *  - Global solution u of one request: elliptic (N+1)^2 nodal values, index
 *    j*(N+1)+i; kinetic N_x*n_vel values, index i*n_vel + j.
 */
#ifndef MSRS_H
#define MSRS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t msrs_status;

#define MSRS_OK             0
#define MSRS_ERR_ARG        1   /* invalid argument (null, out of range, inconsistent sizes) */
#define MSRS_ERR_STATE      2   /* call out of order (e.g. range_finder before sampling) */
#define MSRS_ERR_OOM        3   /* device memory exhausted or footprint above the budget */
#define MSRS_ERR_HIP        4   /* a HIP runtime call failed */
#define MSRS_ERR_NO_DEVICE  5   /* no HIP device is visible */
#define MSRS_ERR_NOT_SPD    6   /* non-positive coefficient or pivot (matrix not SPD / singular) */
#define MSRS_ERR_NOCONV     7   /* iterative refinement above tolerance after ir_max_iters */
#define MSRS_ERR_RANK       8   /* sketch rank below the requested rank k */
#define MSRS_ERR_BUSY       9   /* no free online slot */
#define MSRS_ERR_IO        10   /* a basis file could not be written or read, or is not one */
#define MSRS_ERR_NONFINITE 11   /* non-finite values in the boundary samples, local solutions or residuals */

#define MSRS_KIND_ELLIPTIC_Q1 0
#define MSRS_KIND_KINETIC_DO  1

#define MSRS_PREC_FP64     0   /* plain FP64 factor and sweeps */
#define MSRS_PREC_FP32_IR  1   /* FP32 factor and sweeps, FP64 residuals and refinement */

/* flags */
#define MSRS_FLAG_FULL_BASIS_ENDS   1u  /* kinetic: full (delta) basis on the two end patches (default on) */
#define MSRS_FLAG_PER_PATCH_LAUNCH  2u  /* launch every stage once per patch (unbatched reference mode) */
#define MSRS_FLAG_TIMING            4u  /* record HIP events around every kernel class (msrs_get_stats) */
/* elliptic: every patch that touches the domain boundary uses no buffer and the
 * full (delta) basis of its 4 N/M boundary nodes instead of random samples
 * (needs 4 N/M <= 64); interior patches are sampled as usual */
#define MSRS_FLAG_FULL_BASIS_BOUNDARY 8u
/* elliptic, with MSRS_FLAG_FULL_BASIS_BOUNDARY: the constrained alternative
 * of the online least-squares problem (Sec. 5.2, after eq.
 * elliptic_cond_reduced): the Dirichlet rows hold exactly and only the
 * continuity rows are minimized.  The full bases on the boundary patches (this
 * flag or MSRS_FLAG_FULL_BASIS) make
 * the constraint satisfiable for any boundary data.  Needs at most 1024
 * Dirichlet rows (one per boundary patch and node of it on the domain
 * boundary); msrs_solve_global_banded does not support it. */
#define MSRS_FLAG_CONSTRAINED_BC 16u
/* every patch: no buffer and the full (delta) basis of its boundary data,
 * DetLocalSolu of Alg. alg:summary (elliptic: 4 N/M <= 64 boundary nodes;
 * kinetic: the n_vel inflow ordinates).  The bases then span the fine
 * solution's restrictions, and the online solve reproduces the fine
 * discrete solution. */
#define MSRS_FLAG_FULL_BASIS 32u
/* elliptic, sampled patches (no full-basis flag): msrs_range_finder builds
 * each basis by the two-pass randomized SVD -- the direct SVD of Q^T G_m, Q an
 * orthonormal basis of span(Y_m) (the randomized SVD of Section 2.3 with
 * G_m read a second time through its transpose): adjoint local solves
 * G_m^T Q, which use the same factor (A_II is symmetric), the same sweeps
 * and refinement.  Extra device memory: two arrays of Y's size and one of
 * Omega's. */
#define MSRS_FLAG_TWO_PASS 64u
/* The online least-squares solver (eqs. elliptic_cond_reduced,
 * rte_cond_reduced through their normal equations).  By default every solve
 * takes one step of the corrected semi-normal equations (Bjorck's method:
 * r = d - P~ c with P~ itself, P~^T P~ dc = P~^T r with the resident
 * Cholesky factor, c += dc) when the condition estimate of P~^T P~ made at
 * msrs_assemble_coarse exceeds 1e12, where the normal equations alone keep
 * fewer than about four correct digits; the step brings the coefficients'
 * error from about kappa(P~)^2 u to about kappa(P~) u.  LS_NORMAL never takes
 * the step, LS_CORRECTED always does (not with MSRS_FLAG_CONSTRAINED_BC).
 * The step costs, per launch of up to 32 requests, the rows of P~ rebuilt
 * from the traces and two band triangular sweeps. */
#define MSRS_FLAG_LS_NORMAL    128u
#define MSRS_FLAG_LS_CORRECTED 256u

typedef struct msrs_ctx* msrs_handle;

/* Problem description (msrs_create).  Sizes are validated; see msrs_create. */
typedef struct msrs_problem_desc {
    int32_t kind;            /* MSRS_KIND_* */
    int32_t n_cells;         /* N (cells per side, elliptic) or N_x (kinetic) */
    int32_t M;               /* coarse patches per side (elliptic) or along x (kinetic); divides n_cells */
    int32_t n_samples;       /* s, random boundary samples per patch, 1..64 */
    int32_t rank;            /* k, basis columns kept per sampled patch, 1..s */
    int32_t precision;       /* MSRS_PREC_* */
    int32_t ir_max_iters;    /* FP32_IR: refinement iterations at most (0 -> 30) */
    int32_t n_vel;           /* kinetic: Gauss-Legendre ordinates (even, 2..64) */
    uint64_t seed;           /* Philox key of the device-drawn boundary samples */
    double ir_tol;           /* FP32_IR: every column must reach ||r_j||/||rhs_j|| <= ir_tol (0 -> 1e-10), else
                                MSRS_ERR_NOCONV after ir_max_iters refinement iterations */
    double eps;              /* kinetic: eps of the collision term */
    const int32_t* overlap;  /* host: buffer width in cells per patch (M*M elliptic, M kinetic) */
    uint32_t flags;          /* MSRS_FLAG_* */
    int32_t reserved;
    double hg_g;             /* kinetic: anisotropy g in (-1, 1) of the Henyey-Greenstein scattering kernel
                                k(v, v') = (1 - g^2) / (2 (1 + g^2 + 2 g v v')) (Sec. 4, eq. HG); 0: isotropic,
                                k = 1/2 (eq. def.LL.hom).  The collision term is int k(v,v') f(v') dv' -
                                int k(v',v) dv' f(v), by Gauss-Legendre quadrature on the ordinates. */
    double rank_tol;         /* 0: every sampled patch keeps rank k.  In (0, 1): each keeps its numerical rank at
                                this relative tolerance (Def. num_rank with tau = rank_tol sigma_1(Y_m): the number of
                                singular values of Y_m above it), at least 1 and at most k; msrs_query_patch reports
                                it as n_cols once the range finder has run, and the columns of Q past it are zero.
                                Values below 1e-12 (the range finder's resolution) are refused. */
    double ir_stop;          /* FP32_IR: refinement runs to stagnation.  A patch stops once the largest
                                ||r_j||/||rhs_j|| of its columns is <= ir_stop, or is <= ir_tol and the last
                                iteration did not halve it (0 -> 1e-13, the level of the FP64 residual's own
                                rounding; ir_stop = ir_tol stops at ir_tol). */
} msrs_problem_desc;

typedef struct msrs_layout {
    int32_t n_patches;
    int32_t n_samples;       /* s */
    int32_t rank;            /* k */
    int32_t n_bdry;          /* length of one request's global boundary data */
    int64_t n_nodes;         /* length of one request's global solution */
    int64_t omega_total;     /* elements of the concatenated Omega array */
    int64_t Y_total;         /* elements of the concatenated Y array */
    int64_t Q_total;         /* elements of the concatenated Q array */
    int64_t sv_total;        /* elements of the singular-value array (s per patch) */
    int64_t coarse_dim;      /* unknowns of the least-squares system (the sum of n_cols) */
    int64_t device_bytes;    /* device memory held by the handle */
} msrs_layout;

typedef struct msrs_patch_info {
    int32_t x0, y0, cx, cy;  /* buffered patch in cells (kinetic: x0, cx; y0 = cy = 0) */
    int32_t kx0, ky0, nH;    /* patch K_m origin and width in cells */
    int32_t n_bdry;          /* boundary samples per column of Omega */
    int32_t n_rows;          /* rows of Y and Q */
    int32_t n_cols;          /* columns of Q (k, or n_bdry for a full-basis patch, or the rank chosen at rank_tol) */
    int32_t full_basis;      /* 1 if the patch keeps its full delta basis */
    int32_t line_len;        /* unknowns per block row of the local factorization */
    int32_t n_lines;         /* block rows of the local factorization */
    int32_t n_samples;       /* columns of Omega and Y (s, or n_bdry for a full-basis patch) */
    int64_t omega_off, Y_off, Q_off, sv_off;
} msrs_patch_info;

typedef struct msrs_stats {
    int32_t ir_iters;            /* refinement iterations run by the last sampling call */
    int32_t error_latched;       /* first device-detected error (MSRS_ERR_*) or 0 */
    double max_rel_residual;     /* max over patches, samples of ||rhs - A x|| / ||rhs|| (FP64) */
    double min_rel_gap;          /* min over sampled patches of (sigma_k - sigma_{k+1}) / sigma_1 */
    double kernel_ms[12];        /* accumulated event time per kernel class (MSRS_FLAG_TIMING) */
    int64_t kernel_launches[12]; /* launches per kernel class */
} msrs_stats;

/* kernel classes of msrs_stats */
#define MSRS_K_ASSEMBLE 0
#define MSRS_K_OMEGA    1
#define MSRS_K_LIFT     2
#define MSRS_K_FACTOR   3
#define MSRS_K_SWEEP    4
#define MSRS_K_RESIDUAL 5
#define MSRS_K_RESTRICT 6
#define MSRS_K_RANGE    7
#define MSRS_K_COARSE   8
#define MSRS_K_CSOLVE   9
#define MSRS_K_RECON    10
#define MSRS_K_GRAPH    11   /* a replay of the captured offline step, as a whole */

/* Library version (major*10000 + minor*100 + patch). */
int32_t msrs_version(void);

/* Number of visible HIP devices (0 if none); never fails. */
int32_t msrs_device_count(void);

/*
 * Create a handle on the current HIP device for one problem (Section 3:
 * domain decomposition into patches K_m and buffered patches K~_m, which
 * grow K_m by overlap[p] cells per side and are clipped to the domain).
 * stream: hipStream_t (as void*) on which all offline work is enqueued; NULL
 * is the default stream.  hbm_budget_bytes: upper bound on the device memory
 * of the handle (0: no bound); MSRS_ERR_OOM if the footprint exceeds it.
 * Allocates all device buffers.  Errors: ARG, OOM, HIP, NO_DEVICE.
 */
msrs_status msrs_create(msrs_handle* out, const msrs_problem_desc* desc, void* stream,
                        size_t hbm_budget_bytes);

/*
 * Stage a2: fine-scale operator of every buffered patch (LocalPDESolver's
 * discretization: bilinear elements, eq. Elliptic; or the upwind ordinates
 * scheme of eq. RTE with isotropic scattering) and its block-row
 * factorization.  coef_dev: device, N*N (elliptic a) or N_x (kinetic
 * sigma) FP64 values, read during the call's kernels only.
 * Non-positive values or pivots latch MSRS_ERR_NOT_SPD.  Errors: ARG, STATE.
 */
msrs_status msrs_assemble_patch(msrs_handle h, const double* coef_dev);

/*
 * Stages a3-a7 (RanLocalSolu, eqs. elliptic_random / rte_random): for every
 * patch, s local solves with i.i.d. N(0,1) boundary data, then restriction
 * to K_m (the reduced Green's matrix G^{eps,r}_m = G~_m Omega_m).
 * omega_dev: device, concatenated Omega (layout above), or NULL to draw it on
 * the device with Philox4x32-10 (key = seed, counter = (node, sample,
 * patch, 0), Box-Muller on two 53-bit uniforms).  Y_out_dev: device,
 * optional copy of the concatenated Y (NULL: kept resident only).
 * FP32_IR refines each patch to stagnation (desc.ir_stop) and requires
 * ||r||/||rhs|| <= ir_tol of every column.
 * Errors: ARG, STATE; latched NOT_SPD / NOCONV / NONFINITE (a non-finite
 * boundary value, right-hand side or residual norm).
 */
msrs_status msrs_sample_local_solutions(msrs_handle h, const double* omega_dev, double* Y_out_dev);

/*
 * Stage a8: range finder of each patch's snapshots (QR at the end of
 * RanLocalSolu; randomized SVD of Section 2.3): orthonormal basis of the k
 * leading left singular vectors of Y_m, each column's largest-magnitude
 * entry made positive.  Full-basis patches keep all columns.
 * Q_out_dev: device, optional copy of the concatenated Q.  sv_out_dev:
 * device, optional s singular values of each Y_m (descending).
 * The singular values come from the Gram matrix Y_m^T Y_m (resolved down to
 * about sqrt(s u) sigma_1, u = 2^-53); a patch whose sigma_{k+1} lies below
 * 1e-4 sigma_1 takes a second pass on the rotated snapshots Y_m V, whose
 * graded Gram matrix resolves them down to about u sigma_1.
 * With MSRS_FLAG_TWO_PASS: Q = the orthonormal basis of span(Y_m) at its
 * numerical rank (sigma_j(Y_m) > 1e-12 sigma_1(Y_m), by the
 * passes above), C = G_m^T Q by adjoint local solves (refined like the
 * forward solves; msrs_get_stats then reports them), the eigenvectors V of
 * C^T C, and the basis = Q V[:, :k], re-orthonormalised and sign-fixed; the
 * singular values are those of Q^T G_m (zero past the rank), and k and
 * rank_tol apply to them.
 * Errors: STATE; latched RANK if sigma_k(Y_m) <= 1e-13 sigma_1(Y_m) (the
 * snapshots have lower rank than k; with MSRS_FLAG_TWO_PASS sigma_k(Q^T G_m))
 * or the orthonormalisation breaks down; latched NONFINITE for non-finite
 * snapshots; NOCONV from the adjoint refinement.
 */
msrs_status msrs_range_finder(msrs_handle h, double* Q_out_dev, double* sv_out_dev);

/*
 * Online set-up (eqs. elliptic_cond_tilde / gb3): boundary traces and
 * conormal fluxes of the bases, the normal-equations matrix of the
 * least-squares system and its FP64 Cholesky factor, kept resident.
 * With MSRS_FLAG_CONSTRAINED_BC also the constrained solution operator
 * G_C = K^{-1} B^T S^{-1} E (K = P~^T P~, B the Dirichlet rows,
 * S = B K^{-1} B^T, E the gather of the boundary data at the rows' nodes):
 * the stationarity condition of the Lagrangian with B^T B c = B^T phi added
 * to both sides.  Synchronises the stream.  Errors: STATE, OOM; ARG (more
 * than 1024 Dirichlet rows); NOT_SPD if P~ (or S) is rank deficient.
 */
msrs_status msrs_assemble_coarse(msrs_handle h);

/*
 * Online solve (eqs. elliptic_cond_reduced / rte_cond_reduced and the ansatz
 * u = sum_m G_m c_m): for n_req requests, least-squares coefficients from the
 * global boundary data and the reconstructed global solution.  The
 * coefficients are c = K f with the solution operator
 * K = (P~^T P~)^{-1} P~_D^T formed at msrs_assemble_coarse (the right-hand
 * side of the least-squares system is zero outside the Dirichlet / inflow
 * rows), so a batch costs one pass over K and the bases.
 * f_dev: device, n_req x n_bdry (request-major).  u_dev: device,
 * n_req x n_nodes.  stream: hipStream_t (as void*) for this call, NULL for
 * the handle's stream.  Elliptic nodes shared by several patches take the
 * partition-of-unity average.  Calls on one stream reuse one internal
 * workspace in stream order; calls on up to four different streams may
 * overlap, each taking a workspace that is no longer in use on the device,
 * and a call that finds none fails with MSRS_ERR_BUSY.  With
 * MSRS_FLAG_CONSTRAINED_BC the coefficients are c = G_C f instead (the same
 * cost).  Where the handle's solves take the corrected semi-normal step
 * (MSRS_FLAG_LS_CORRECTED, msrs_coarse_corrected) it follows c = K f.
 * Errors: ARG (n_req outside [1, max_batch]), STATE, BUSY.
 */
msrs_status msrs_solve_global(msrs_handle h, int32_t n_req, const double* f_dev, double* u_dev,
                              void* stream);

/*
 * Conditioning of the least-squares system of eq. elliptic_cond_reduced /
 * rte_cond_reduced, which the online stage solves through its normal
 * equations: *kappa_normal (nullable) receives the 1-norm condition estimate
 * of P~^T P~ made at msrs_assemble_coarse (||K||_1 times Hager and Higham's
 * estimate of ||K^{-1}||_1 from the resident band Cholesky factor, as
 * LAPACK's banded condition estimators do; a lower bound, in practice within
 * a small factor), *kappa_ls (nullable) its square root, the matching
 * estimate of kappa(P~).  The normal equations lose about
 * log10(kappa_normal) digits of the coefficients.  Errors: ARG, STATE.
 */
msrs_status msrs_coarse_condition(msrs_handle h, double* kappa_normal, double* kappa_ls);

/*
 * *corrected = 1 if the online solves of this handle take the corrected
 * semi-normal step (MSRS_FLAG_LS_CORRECTED, or a condition estimate of
 * P~^T P~ above 1e12 without MSRS_FLAG_LS_NORMAL), else 0; decided at
 * msrs_assemble_coarse, which fails with ARG where the step would need more
 * than 64 KiB of LDS (elliptic N/M > 680).  Errors: ARG (NULL), STATE.
 */
msrs_status msrs_coarse_corrected(msrs_handle h, int32_t* corrected);

/*
 * The same solve by the plain direct method, one request after another:
 * d~ = P~^T d and two band triangular solves with the Cholesky factor of
 * P~^T P~ per request, then the reconstruction.  Same arguments, layouts
 * and errors as msrs_solve_global; results agree to rounding.  STATE for a
 * handle with MSRS_FLAG_CONSTRAINED_BC.
 */
msrs_status msrs_solve_global_banded(msrs_handle h, int32_t n_req, const double* f_dev, double* u_dev,
                                     void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve
 * of msrs_solve_global with the same arguments, layouts and results (the
 * same kernels), but its per-launch workspace (the boundary right-hand sides
 * and least-squares coefficients of up to 32 requests) lives in a fixed
 * 2 MiB device array of the library, one per GPU, held until the process
 * ends, instead of the handle's online workspaces.  The call allocates no
 * device memory; the array's address on each device is looked up on that
 * device's first call.  Every call on a GPU shares its array, so calls that
 * overlap on one GPU (other streams, other handles, other threads) race:
 * order them on one stream or synchronise between them.  Errors: ARG
 * (n_req outside [1, max_batch], NULL pointers, or
 * (boundary unknowns + coarse unknowns) x min(n_req, 32) doubles above the
 * array, the coarse unknowns counted twice where the solves take the
 * corrected semi-normal step), STATE (no msrs_assemble_coarse yet), HIP.
 */
msrs_status msrs_solve_global_noalloc(msrs_handle h, int32_t n_req, const double* f_dev, double* u_dev, void* stream);

/*
 * Capture one offline step -- msrs_assemble_patch(coef_dev),
 * msrs_sample_local_solutions with device-drawn samples, msrs_range_finder
 * -- as a HIP graph of the handle's stream (which must not be the default
 * stream), and instantiate it.  Nothing runs during the capture.  coef_dev
 * is baked into the graph: it must stay valid, and a replay reads its
 * current contents.  FP32_IR: the graph runs a fixed number of refinement
 * iterations, one more than the most any patch needed in the preceding
 * eager sampling call (required first); patches that have stopped skip their
 * work, so the results equal the eager ones, and a patch still above ir_tol
 * after the last iteration latches MSRS_ERR_NOCONV.  A new capture replaces the
 * previous graph.  Synchronises.  Errors: ARG, STATE, HIP.
 */
msrs_status msrs_offline_graph_capture(msrs_handle h, const double* coef_dev);

/* Enqueue one replay of the captured offline step on the handle's stream. */
msrs_status msrs_offline_graph_launch(msrs_handle h);

/*
 * Copy the resident snapshots Y, bases Q and singular values (each
 * nullable; device buffers of Y_total, Q_total, sv_total doubles) on the
 * handle's stream, without recomputing them.  Errors: ARG, STATE (not
 * computed yet).
 */
msrs_status msrs_copy_results(msrs_handle h, double* Y_out_dev, double* Q_out_dev, double* sv_out_dev);

/*
 * Copy the resident boundary samples Omega (all patches, layout above) of
 * the last sampling call to omega_out_dev (device, omega_total doubles).
 * Full-basis patches hold the identity.  Errors: ARG, STATE.
 */
msrs_status msrs_copy_omega(msrs_handle h, double* omega_out_dev);

/*
 * The device generator of the random boundary data (Sec. 3, RanLocalSolu:
 * i.i.d. N(0,1) values at the boundary nodes), without a handle: for nodes
 * 0..n_node-1 and samples 0..n_sample-1 of patch `patch` under key `seed`,
 * the four Philox4x32-10 output words of counter (node, sample, patch, 0) go
 * to words_dev[4 (sample n_node + node) + t], t = 0..3 (device, nullable),
 * and the normal msrs_sample_local_solutions draws for that node and sample
 * to normals_dev[sample n_node + node] (device, nullable).  Enqueued on
 * stream (NULL: the default stream).  Errors: ARG (negative sizes), HIP.
 */
msrs_status msrs_draw_boundary_samples(uint64_t seed, int32_t patch, int32_t n_node, int32_t n_sample, uint32_t* words_dev,
                                       double* normals_dev, void* stream);

/*
 * Keep the product of the offline stage (the call summary of the method,
 * Alg. 1: the local bases are computed once and reused by every online
 * solve) in a file, and make a handle of it again later.
 *
 * msrs_save writes the problem description, the coefficient field, the bases
 * Q, the singular values, the per-patch gaps and residuals and the ranks of handle h
 * to path (created or truncated): a little-endian binary file with an
 * 8-byte magic, a version and a 64-bit FNV-1a checksum over everything after
 * the magic.  It synchronizes the handle's stream.  Errors: ARG (NULL
 * argument), STATE (no range finder yet, or the handle is held by a
 * server), IO (the file cannot be written), HIP.
 *
 * msrs_load reads such a file and creates a new handle on stream (as
 * msrs_create, HBM budget unbounded) that holds the bases and the coefficient
 * field: msrs_assemble_coarse and msrs_solve_global may follow at once; the
 * offline calls start over from msrs_assemble_patch.  The caller destroys
 * the handle.  Errors: ARG (NULL argument), IO (unreadable file, wrong magic
 * or version, sizes or ranks that do not match the description, checksum mismatch),
 * and those of msrs_create.  *out is NULL on failure.
 */
msrs_status msrs_save(msrs_handle h, const char* path);
msrs_status msrs_load(msrs_handle* out, const char* path, void* stream);

/* Requests per msrs_solve_global call at most (1..4096, default 64). */
msrs_status msrs_set_max_batch(msrs_handle h, int32_t max_batch);

/*
 * Launch-shape parameters (results do not depend on them beyond rounding
 * order; the batched online results of one request are the same for every
 * value).  Set any time; they apply to later calls (a captured offline graph
 * keeps the shapes it was captured with).  Errors: ARG (unknown key
 * or value not listed).
 */
#define MSRS_TUNE_SWEEP_COLS   0   /* samples per sweep workgroup: 16, 32, 64 (FP64 path: at most 32) */
#define MSRS_TUNE_RECON_BATCH  1   /* requests per reconstruction pass: 1, 2, 4, 8, 16 */
#define MSRS_TUNE_APPLY_BATCH  2   /* requests per workgroup of the G_B product: 4, 8, 16 */
/* factor workgroups a compute unit can hold (FP32 path): 2 (default: the
 * register budget of two resident workgroups, so every chain of lines of a
 * batch runs at once) or 1 (registers and scalar registers unconstrained: a
 * unit holds one workgroup, and a batch of more chains than units runs in
 * rounds) */
#define MSRS_TUNE_FACTOR_SHARE 3
msrs_status msrs_set_tuning(msrs_handle h, int32_t key, int32_t value);
msrs_status msrs_get_tuning(msrs_handle h, int32_t key, int32_t* value);

typedef struct msrs_tune_report {
    int32_t n_trials;
    int32_t key[32];     /* MSRS_TUNE_SWEEP_COLS, or 100*RECON_BATCH + APPLY_BATCH (= 102) */
    int32_t value[32];   /* the candidate (online: 100*recon_batch + apply_batch) */
    double ms[32];       /* device milliseconds per call */
} msrs_tune_report;

#define MSRS_TUNE_STAGE_OFFLINE 0   /* sweep columns, timed on msrs_sample_local_solutions */
#define MSRS_TUNE_STAGE_ONLINE  1   /* reconstruction x product batches, timed on a 32-request solve */

/*
 * Autotuner: time every candidate of a stage on this handle's own problem
 * (warm-up + reps calls between events on the handle's stream), keep the
 * fastest and report all trials.  OFFLINE needs msrs_assemble_patch and
 * leaves the handle sampled (results do not depend on the choice); ONLINE
 * needs msrs_assemble_coarse and uses zero requests in temporary device
 * buffers.  Synchronises.  Errors: ARG, STATE, BUSY, HIP, and those of the
 * timed calls.
 */
msrs_status msrs_autotune(msrs_handle h, int32_t stage, int32_t reps, msrs_tune_report* out);

/* Sizes and offsets of the concatenated arrays.  After a range finder with
 * rank_tol > 0 the first query synchronizes the handle's stream to read the
 * ranks it chose.  Errors: ARG, HIP. */
msrs_status msrs_query_layout(msrs_handle h, msrs_layout* out);
msrs_status msrs_query_patch(msrs_handle h, int32_t patch, msrs_patch_info* out);

/* Synchronise the handle's stream and report refinement, residual, gap and timing figures. */
msrs_status msrs_get_stats(msrs_handle h, msrs_stats* out);

/* Zero the accumulated kernel times and launch counts. */
msrs_status msrs_reset_stats(msrs_handle h);

/* Message of the last error on h (or of the last failed create if h is NULL). */
const char* msrs_last_error(msrs_handle h);

/*
 * Release every device buffer of the handle (synchronises its stream and
 * waits for its online calls).  Destroy every server that holds the handle
 * first: a server keeps using the handle's bases and coarse operator.
 */
void msrs_destroy(msrs_handle h);

/* ------------------------------------------------------------------------
 * Request server (the online stage as a service over resident models)
 *
 * A server holds one or more handles whose coarse problem is assembled
 * (e.g. two grids of different size).  Requests -- a model index and that
 * model's global boundary data f in host memory -- are queued in arrival
 * order and admitted when an HBM slot for their solution fits in the slot
 * budget (admission by footprint; strict arrival order, so a large request
 * is never overtaken).  Admitted requests of one model are solved in batches
 * of at most max_batch by msrs_solve_global's method on n_streams streams at
 * once; requests arriving while batches run are admitted and launched as
 * slots and streams free up.  A request's solution stays in its slot until
 * msrs_server_fetch copies it out and releases the slot.  A result does not
 * depend on the batch it ran in: every request's arithmetic is the same,
 * alone or in a mix.
 *
 * Threads: submit, wait, fetch and get_stats may be called from any host
 * threads at once; destroy must not overlap any other call on the server.
 * While a server exists its handles refuse the offline and set-up calls
 * (MSRS_ERR_STATE); msrs_solve_global stays usable.
 * ---------------------------------------------------------------------- */
typedef struct msrs_server_s* msrs_server;

typedef struct msrs_server_config {
    int32_t n_streams;       /* batches in flight at once, 1..8 (0 -> 4) */
    int32_t max_batch;       /* requests per batch, 1..256 (0 -> 32) */
    int32_t max_pending;     /* submitted and not yet fetched requests at most (0 -> 4096) */
    int32_t idle_spin_us;    /* the worker polls for this long after its last activity before
                                it sleeps (0 -> 10000; trades a host core for arrival latency) */
    size_t slot_bytes;       /* device bytes for request solutions (0 -> 1 GiB) */
    size_t staging_bytes;    /* pinned host bytes for queued boundary data (0 -> 64 MiB) */
} msrs_server_config;

typedef struct msrs_request_info {
    int32_t model;
    int32_t status;          /* MSRS_OK, or the error that failed the request */
    int32_t batch_size;      /* requests of the batch that solved it */
    int32_t stream;          /* index of the server stream that solved it */
    double t_arrival;        /* seconds on msrs_server_clock */
    double t_admit;          /* slot granted */
    double t_launch;         /* batch enqueued */
    double t_done;           /* batch observed complete (solution resident) */
} msrs_request_info;

typedef struct msrs_server_stats {
    int64_t submitted, completed, batches;
    int64_t max_in_flight;     /* requests on the device at once, at most */
    int64_t peak_slot_bytes;   /* slot memory in use, at most */
    int64_t slot_capacity;
    int64_t admission_waits;   /* requests that had to wait for slot memory */
    double mean_batch;         /* requests per batch */
} msrs_server_stats;

/* Monotonic clock of the server's timestamps, in seconds. */
double msrs_server_clock(void);

/* Message of the last failed server call of the calling thread. */
const char* msrs_server_last_error(void);

/*
 * Create a server over n_models handles (host array; every handle must have
 * passed msrs_assemble_coarse, all on one device).  cfg: host, NULL for the
 * defaults.  Allocates the slot memory, pinned staging and per-stream
 * workspaces and starts the worker thread.  Errors: ARG, STATE, OOM (a
 * model's solution or boundary data exceeds the budgets), HIP.
 */
msrs_status msrs_server_create(msrs_server* out, const msrs_handle* models, int32_t n_models,
                               const msrs_server_config* cfg);

/*
 * Queue one request: f_host (host, n_bdry of the model) is copied before the
 * call returns.  t_arrival: arrival time on msrs_server_clock (<= 0: now),
 * the origin of the request's latency.  *ticket identifies it in wait and
 * fetch.  Errors: ARG, STATE (shutting down), BUSY (max_pending unfetched
 * requests or staging full; retry later), the server's latched error.
 */
msrs_status msrs_server_submit(msrs_server s, int32_t model, const double* f_host, double t_arrival,
                               int64_t* ticket);

/*
 * Queue n requests in order under one lock (models[i], f_host[i] as in
 * msrs_server_submit; t_arrival nullable).  Stops at the first request that
 * cannot be queued and returns that request's error; *n_done requests were
 * queued, with their tickets in tickets[0 .. *n_done).
 */
msrs_status msrs_server_submit_many(msrs_server s, int32_t n, const int32_t* models, const double* const* f_host,
                                    const double* t_arrival, int64_t* tickets, int32_t* n_done);

/*
 * Replay an arrival trace (load generation and capacity measurement): queue
 * request i (models[i], f_host[i]) once msrs_server_clock reaches
 * t_arrival[i] (ascending; NULL: all at once), waiting out back-pressure, and
 * return when every queued request has finished.  Solutions are discarded:
 * a slot is released as soon as its request completes, and infos[i] (host,
 * n records) receives the request's timestamps.  The calling thread spins
 * between arrivals.  Errors: ARG, the first submission or request error.
 */
msrs_status msrs_server_replay(msrs_server s, int32_t n, const int32_t* models, const double* const* f_host,
                               const double* t_arrival, msrs_request_info* infos);

/* Wait until the request is solved (timeout_s < 0: no limit).  BUSY on time-out. */
msrs_status msrs_server_wait(msrs_server s, int64_t ticket, double timeout_s);

/*
 * Wait for the request, copy its solution (n_nodes doubles) to u_out (host
 * or device; NULL: discard), fill *info (nullable) and release the request
 * and its slot; the ticket is invalid afterwards.  Errors: ARG (unknown
 * ticket), HIP, or the error that failed the request.
 */
msrs_status msrs_server_fetch(msrs_server s, int64_t ticket, double* u_out, msrs_request_info* info);

/* Counters of the server; returns its latched error, if any. */
msrs_status msrs_server_get_stats(msrs_server s, msrs_server_stats* out);

/*
 * Stop the server: queued requests that were not launched fail with
 * MSRS_ERR_STATE, launched batches are waited for, memory and streams are
 * released and the handles accept offline calls again.
 */
void msrs_server_destroy(msrs_server s);

#ifdef __cplusplus
}
#endif

#endif /* MSRS_H */
