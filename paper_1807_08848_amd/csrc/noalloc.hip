// Online solve for callers that cannot allocate device memory: the method of
// msrs_solve_global (boundary right-hand side, the G_B product, the
// partition-of-unity reconstruction) with its per-launch workspace in a fixed
// device array of this library instead of the handle's online workspaces.
//
// The array is one per GPU (each device holds its own copy of it for the
// lifetime of the process).  Host code never uses the array's name as a
// device address: the address of each device's copy is looked up once, with
// that device current, and kept in scratch_ptr[device].
#include <algorithm>
#include <cstring>
#include <mutex>

#include "msrs_internal.h"

using namespace msrs;

namespace {

// The workspace of one launch of up to kOutPerLaunch requests: the boundary
// right-hand sides (g_len doubles per request), then the least-squares
// coefficients (Np doubles per request), then, for a handle whose solves take
// the corrected semi-normal step, that step's right-hand sides (Np doubles
// per request).
constexpr int64_t kScratchDoubles = int64_t(1) << 18;   // 2 MiB

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
double* scratch_ptr[kMaxDevices] = {};

// Address of this device's copy of the workspace, looked up on first use with
// the device current.
hipError_t device_scratch(int device, double** out) {
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    if (!scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        scratch_ptr[device] = static_cast<double*>(p);
    }
    *out = scratch_ptr[device];
    return hipSuccess;
}

msrs_status set_err(msrs_handle h, msrs_status st, const char* msg) {
    h->err = msg;
    return st;
}

}  // namespace

extern "C" msrs_status msrs_solve_global_noalloc(msrs_handle h, int32_t n_req, const double* f_dev, double* u_dev,
                                                 void* stream) {
    Ctx* c = h;
    if (!c) return MSRS_ERR_ARG;
    if (!c->coarse_ready) return set_err(h, MSRS_ERR_STATE, "msrs_assemble_coarse must come first");
    if (n_req < 1 || n_req > c->max_batch) return set_err(h, MSRS_ERR_ARG, "n_req must be in [1, max_batch]");
    if (!f_dev || !u_dev) return set_err(h, MSRS_ERR_ARG, "f_dev / u_dev is NULL");
    const int nr = std::min<int>(n_req, kOutPerLaunch);
    const int64_t ng = c->g_len();
    const int64_t per_req = ng + c->Np * (c->lsq_correct ? 2 : 1);
    if (per_req * nr > kScratchDoubles)
        return set_err(h, MSRS_ERR_ARG,
                       "the fixed workspace (2 MiB) is too small: (boundary unknowns + coarse unknowns, twice the "
                       "latter with the corrected semi-normal step) x min(n_req, 32) doubles must fit; use fewer "
                       "requests per call or msrs_solve_global");
    double* ws = nullptr;
    const hipError_t e = device_scratch(c->device, &ws);
    if (e != hipSuccess) return set_err(h, MSRS_ERR_HIP, "hipGetSymbolAddress of the fixed workspace failed");
    double* gbuf = ws;
    double* cbuf = ws + ng * nr;
    double* zbuf = c->lsq_correct ? cbuf + c->Np * nr : nullptr;
    const hipStream_t st = stream ? (hipStream_t)stream : c->stream;
    try {
        const double* fp[kOutPerLaunch];
        double* up[kOutPerLaunch];
        for (int r0 = 0; r0 < n_req; r0 += kOutPerLaunch) {
            const int m = std::min<int>(kOutPerLaunch, n_req - r0);
            for (int r = 0; r < m; ++r) {
                fp[r] = f_dev + (int64_t)(r0 + r) * c->n_bdry;
                up[r] = u_dev + (int64_t)(r0 + r) * c->n_nodes;
            }
            coarse_apply(*c, m, fp, up, gbuf, cbuf, zbuf, st);
        }
        MSRS_HIP_CHECK(hipGetLastError());
    } catch (const HipError&) {
        return set_err(h, MSRS_ERR_HIP, "kernel launch failed");
    }
    return MSRS_OK;
}
