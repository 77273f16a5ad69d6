// Request server over resident models (the online stage of Section 3 as a
// service): global boundary data f of several problems arrive as requests,
// wait for an HBM slot for their solution (admission by footprint), and are
// solved in model-homogeneous batches -- c = K f and the partition-of-unity
// reconstruction u = sum_m w_m Q_m c_m -- on several streams at once, so
// that requests arriving while batches run are admitted and launched as
// slots and streams free up (continuous batching).
//
// One worker thread per server admits, forms batches, launches them and
// polls their completion events; submit / wait / fetch are called from any
// host thread.  A request's life: waiting -> admitted (slot held) -> running
// -> done (solution resident in its slot) -> fetched (slot released).
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>

#include "msrs_internal.h"
#include "serve_core.h"

using namespace msrs;

namespace {

thread_local std::string g_server_err;

constexpr int kMaxStreams = 8;
constexpr int kMaxBatch = 256;

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

enum ReqState { kWaiting = 0, kAdmitted = 1, kRunning = 2, kDone = 3, kFailed = 4 };

struct Req {
    int model = 0;
    int state = kWaiting;
    msrs_status status = MSRS_OK;
    int64_t slot_off = -1, slot_bytes = 0;
    int64_t stage_off = -1, stage_bytes = 0;
    int batch = 0, stream = -1;
    bool stalled = false, fetching = false;
    msrs_request_info* discard_info = nullptr;   // replayed request: record here and release at completion
    int64_t* discard_count = nullptr;            // ... and count it for its replay call
    double t_arrival = 0, t_admit = 0, t_launch = 0, t_done = 0;
};

struct Lane {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    double* cbuf = nullptr;   // max Np x kOutPerLaunch
    double* gbuf = nullptr;   // max nB x kOutPerLaunch
    double* zbuf = nullptr;   // max Np x kOutPerLaunch (corrected semi-normal step)
    std::vector<int64_t> ids;
    bool busy = false;
};

}  // namespace

struct msrs_server_s {
    std::vector<Ctx*> models;
    int device = 0;
    int n_streams = 4, max_batch = 32, max_pending = 4096;
    double idle_spin_s = 0.01;
    char* dslots = nullptr;
    serve::Arena slots;
    char* hstage = nullptr;      // pinned host
    char* hstage_dev = nullptr;  // its device address
    serve::Arena stage;
    std::vector<Lane> lanes;
    hipStream_t copy = nullptr;
    std::vector<void*> dallocs;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::unordered_map<int64_t, Req> reqs;
    serve::Scheduler sched;
    int64_t next_id = 1;
    bool stop = false;
    msrs_status fatal = MSRS_OK;
    std::string fatal_msg;
    std::thread worker;

    // statistics
    int64_t n_submitted = 0, n_completed = 0, n_batches = 0, batch_reqs = 0;
    int64_t in_flight = 0, max_in_flight = 0, peak_slot = 0, stalls = 0;
};

namespace {

msrs_status sfail(msrs_status st, const std::string& msg) {
    g_server_err = msg;
    return st;
}

void fill_info(const Req& r, msrs_status st, msrs_request_info* info) {
    info->model = r.model;
    info->status = st;
    info->batch_size = r.batch;
    info->stream = r.stream;
    info->t_arrival = r.t_arrival;
    info->t_admit = r.t_admit;
    info->t_launch = r.t_launch;
    info->t_done = r.t_done;
}

// Worker side: mark every request of a failed server and stop launching.
void fail_all(msrs_server_s* s, msrs_status st, const std::string& msg) {
    if (s->fatal == MSRS_OK) {
        s->fatal = st;
        s->fatal_msg = msg;
    }
    for (auto& it : s->sched.drop_all()) {
        Req& r = s->reqs[it.id];
        r.state = kFailed;
        r.status = st;
    }
    for (auto& L : s->lanes)
        for (int64_t id : L.ids) {
            Req& r = s->reqs[id];
            r.state = kFailed;
            r.status = st;
        }
    // replayed requests report through their info records
    for (auto it = s->reqs.begin(); it != s->reqs.end();) {
        Req& r = it->second;
        if (r.discard_info && r.state == kFailed) {
            fill_info(r, r.status, r.discard_info);
            if (r.slot_off >= 0) s->slots.release(r.slot_off, r.slot_bytes);
            if (r.stage_off >= 0) s->stage.release(r.stage_off, r.stage_bytes);
            *r.discard_count += 1;
            it = s->reqs.erase(it);
        } else {
            ++it;
        }
    }
}

void launch_batch(msrs_server_s* s, int k, const std::vector<serve::Scheduler::Item>& b) {
    Lane& L = s->lanes[k];
    const Ctx& c = *s->models[b[0].model];
    const int n = (int)b.size();
    const double t = now_s();
    std::vector<double*> u(n);
    std::vector<const double*> f(n);
    L.ids.clear();
    for (int r = 0; r < n; ++r) {
        Req& q = s->reqs[b[r].id];
        f[r] = (const double*)(s->hstage_dev + q.stage_off);   // read by the kernels from pinned memory
        u[r] = (double*)(s->dslots + q.slot_off);
        q.state = kRunning;
        q.t_launch = t;
        q.batch = n;
        q.stream = k;
        L.ids.push_back(b[r].id);
    }
    coarse_apply(c, n, f.data(), u.data(), L.gbuf, L.cbuf, L.zbuf, L.st);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(L.ev, L.st);
    if (e != hipSuccess) throw HipError(e, "batch launch", __FILE__, __LINE__);
    L.busy = true;
    s->n_batches += 1;
    s->batch_reqs += n;
    s->in_flight += n;
    s->max_in_flight = std::max(s->max_in_flight, s->in_flight);
}

void worker_main(msrs_server_s* s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    double last_active = now_s();
    for (;;) {
        bool done_any = false, busy = false;
        try {
            // completions
            for (auto& L : s->lanes) {
                if (!L.busy) continue;
                const hipError_t q = hipEventQuery(L.ev);
                if (q == hipErrorNotReady) { busy = true; continue; }
                if (q != hipSuccess) throw HipError(q, "hipEventQuery", __FILE__, __LINE__);
                const double t = now_s();
                for (int64_t id : L.ids) {
                    auto rit = s->reqs.find(id);
                    Req& r = rit->second;
                    r.state = kDone;
                    r.t_done = t;
                    s->stage.release(r.stage_off, r.stage_bytes);
                    r.stage_off = -1;
                    if (r.discard_info) {
                        fill_info(r, MSRS_OK, r.discard_info);
                        s->slots.release(r.slot_off, r.slot_bytes);
                        *r.discard_count += 1;
                        s->reqs.erase(rit);
                    }
                }
                s->n_completed += (int64_t)L.ids.size();
                s->in_flight -= (int64_t)L.ids.size();
                L.ids.clear();
                L.busy = false;
                done_any = true;
            }
            if (done_any) s->cv_done.notify_all();
            if (s->fatal == MSRS_OK && !s->stop) {
                // admission by footprint, arrival order
                const double t = now_s();
                for (auto& it : s->sched.admit([&](const serve::Scheduler::Item& it) {
                         Req& r = s->reqs[it.id];
                         const int64_t off = s->slots.alloc(it.bytes);
                         if (off < 0) {
                             if (!r.stalled) s->stalls += 1;   // waits for slot memory
                             r.stalled = true;
                             return false;
                         }
                         r.slot_off = off;
                         return true;
                     })) {
                    Req& r = s->reqs[it.id];
                    r.state = kAdmitted;
                    r.t_admit = t;
                }
                s->peak_slot = std::max(s->peak_slot, s->slots.used());
                // batches on free lanes
                for (int k = 0; k < (int)s->lanes.size(); ++k) {
                    if (s->lanes[k].busy) continue;
                    auto b = s->sched.form(s->max_batch);
                    if (b.empty()) break;
                    launch_batch(s, k, b);
                    busy = true;
                }
            }
        } catch (const HipError& e) {
            char buf[512];
            std::snprintf(buf, sizeof buf, "HIP error %d (%s) in %s", (int)e.e, hipGetErrorString(e.e), e.what);
            fail_all(s, e.e == hipErrorOutOfMemory ? MSRS_ERR_OOM : MSRS_ERR_HIP, buf);
            s->cv_done.notify_all();
            for (auto& L : s->lanes) { L.busy = false; L.ids.clear(); }
            busy = false;
        }
        if (s->stop && !busy) break;
        const double tn = now_s();
        if (busy || done_any) last_active = tn;
        if (busy || tn - last_active < s->idle_spin_s) {
            // batches in flight, or recently active: poll (a timed or
            // notified wait would add the scheduler's wake-up latency to
            // every completion and arrival)
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        } else {
            s->cv_work.wait(lk);
            last_active = now_s();
        }
    }
}

bool valid(msrs_server s) { return s != nullptr; }

}  // namespace

extern "C" {

double msrs_server_clock(void) { return now_s(); }

const char* msrs_server_last_error(void) { return g_server_err.c_str(); }

msrs_status msrs_server_create(msrs_server* out, const msrs_handle* models, int32_t n_models, const msrs_server_config* cfg) {
    if (!out) return sfail(MSRS_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!models || n_models < 1 || n_models > 64) return sfail(MSRS_ERR_ARG, "models must hold 1..64 handles");
    msrs_server_config d{};
    if (cfg) d = *cfg;
    const int n_streams = d.n_streams ? d.n_streams : 4;
    const int max_batch = d.max_batch ? d.max_batch : 32;
    const int max_pending = d.max_pending ? d.max_pending : 4096;
    const int idle_spin_us = d.idle_spin_us ? d.idle_spin_us : 10000;
    const size_t slot_bytes = d.slot_bytes ? d.slot_bytes : ((size_t)1 << 30);
    const size_t staging_bytes = d.staging_bytes ? d.staging_bytes : ((size_t)64 << 20);
    if (n_streams < 1 || n_streams > kMaxStreams) return sfail(MSRS_ERR_ARG, "n_streams must be in [1, 8]");
    if (max_batch < 1 || max_batch > kMaxBatch) return sfail(MSRS_ERR_ARG, "max_batch must be in [1, 256]");
    if (max_pending < 1) return sfail(MSRS_ERR_ARG, "max_pending must be positive");
    if (idle_spin_us < 0) return sfail(MSRS_ERR_ARG, "idle_spin_us must not be negative");
    int dev0 = -1;
    for (int i = 0; i < n_models; ++i) {
        Ctx* c = models[i];
        if (!c) return sfail(MSRS_ERR_ARG, "a model handle is NULL");
        if (!c->coarse_ready) return sfail(MSRS_ERR_STATE, "msrs_assemble_coarse must come first on every model");
        if (dev0 >= 0 && c->device != dev0) return sfail(MSRS_ERR_ARG, "models must live on one device");
        dev0 = c->device;
        if ((size_t)serve::Arena::round(c->n_nodes * 8) > slot_bytes)
            return sfail(MSRS_ERR_OOM, "slot_bytes is below one solution of a model");
        if ((size_t)serve::Arena::round((int64_t)c->n_bdry * 8) > staging_bytes)
            return sfail(MSRS_ERR_OOM, "staging_bytes is below one request of a model");
    }
    auto* s = new (std::nothrow) msrs_server_s();
    if (!s) return sfail(MSRS_ERR_OOM, "host allocation failed");
    s->models.assign(models, models + n_models);
    s->device = dev0;
    s->n_streams = n_streams;
    s->max_batch = max_batch;
    s->max_pending = max_pending;
    s->idle_spin_s = idle_spin_us * 1e-6;
    s->sched = serve::Scheduler(n_models);
    msrs_status st = MSRS_OK;
    std::string msg;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r, const char* what) {
        if (r != hipSuccess && e == hipSuccess) {
            e = r;
            msg = std::string(what) + ": " + hipGetErrorString(r);
        }
        return r == hipSuccess;
    };
    int64_t np_max = 0, nB_max = 0;
    for (Ctx* c : s->models) {
        np_max = std::max<int64_t>(np_max, c->Np);
        nB_max = std::max<int64_t>(nB_max, c->g_len());
    }
    if (chk(hipSetDevice(dev0), "hipSetDevice") && chk(hipMalloc((void**)&s->dslots, slot_bytes), "hipMalloc slots")) {
        s->dallocs.push_back(s->dslots);
        s->slots.reset((int64_t)slot_bytes);
    }
    if (e == hipSuccess && chk(hipHostMalloc((void**)&s->hstage, staging_bytes, hipHostMallocMapped), "hipHostMalloc staging") &&
        chk(hipHostGetDevicePointer((void**)&s->hstage_dev, s->hstage, 0), "hipHostGetDevicePointer"))
        s->stage.reset((int64_t)staging_bytes);
    if (e == hipSuccess) chk(hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking), "hipStreamCreate");
    s->lanes.resize(n_streams);
    for (auto& L : s->lanes) {
        if (e != hipSuccess) break;
        chk(hipStreamCreateWithFlags(&L.st, hipStreamNonBlocking), "hipStreamCreate");
        chk(hipEventCreateWithFlags(&L.ev, hipEventDisableTiming), "hipEventCreate");
        if (chk(hipMalloc((void**)&L.cbuf, sizeof(double) * (size_t)np_max * kOutPerLaunch), "hipMalloc cbuf")) s->dallocs.push_back(L.cbuf);
        if (chk(hipMalloc((void**)&L.gbuf, sizeof(double) * (size_t)nB_max * kOutPerLaunch), "hipMalloc gbuf")) s->dallocs.push_back(L.gbuf);
        if (chk(hipMalloc((void**)&L.zbuf, sizeof(double) * (size_t)np_max * kOutPerLaunch), "hipMalloc zbuf")) s->dallocs.push_back(L.zbuf);
    }
    if (e != hipSuccess) {
        st = e == hipErrorOutOfMemory ? MSRS_ERR_OOM : MSRS_ERR_HIP;
        msrs_server_destroy(s);
        return sfail(st, msg);
    }
    for (Ctx* c : s->models) c->served += 1;
    s->worker = std::thread(worker_main, s);
    *out = s;
    return MSRS_OK;
}

}  // extern "C"

namespace {
// Queue one request; the caller holds s->mu.
msrs_status submit_locked(msrs_server s, int32_t model, const double* f_host, double t_arrival, int64_t* ticket,
                          msrs_request_info* discard_info = nullptr, int64_t* discard_count = nullptr) {
    if (!f_host) return sfail(MSRS_ERR_ARG, "f_host is NULL");
    if (model < 0 || model >= (int)s->models.size()) return sfail(MSRS_ERR_ARG, "model index out of range");
    if (s->fatal != MSRS_OK) return sfail(s->fatal, s->fatal_msg);
    if (s->stop) return sfail(MSRS_ERR_STATE, "server is shutting down");
    if ((int64_t)s->reqs.size() >= s->max_pending) return sfail(MSRS_ERR_BUSY, "max_pending requests are unfetched");
    const Ctx& c = *s->models[model];
    const int64_t sb = (int64_t)c.n_bdry * 8;
    const int64_t off = s->stage.alloc(sb);
    if (off < 0) return sfail(MSRS_ERR_BUSY, "host staging for boundary data is full");
    std::memcpy(s->hstage + off, f_host, (size_t)sb);
    const int64_t id = s->next_id++;
    Req& r = s->reqs[id];
    r.model = model;
    r.stage_off = off;
    r.stage_bytes = sb;
    r.slot_bytes = c.n_nodes * 8;
    r.t_arrival = t_arrival > 0 ? t_arrival : now_s();
    r.discard_info = discard_info;
    r.discard_count = discard_count;
    s->sched.push(id, model, r.slot_bytes);
    s->n_submitted += 1;
    *ticket = id;
    return MSRS_OK;
}
}  // namespace

extern "C" {

msrs_status msrs_server_submit(msrs_server s, int32_t model, const double* f_host, double t_arrival, int64_t* ticket) {
    if (!valid(s)) return sfail(MSRS_ERR_ARG, "server is NULL");
    if (!ticket) return sfail(MSRS_ERR_ARG, "ticket is NULL");
    msrs_status st;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        st = submit_locked(s, model, f_host, t_arrival, ticket);
    }
    if (st == MSRS_OK) s->cv_work.notify_one();
    return st;
}

msrs_status msrs_server_submit_many(msrs_server s, int32_t n, const int32_t* models, const double* const* f_host,
                                    const double* t_arrival, int64_t* tickets, int32_t* n_done) {
    if (!valid(s)) return sfail(MSRS_ERR_ARG, "server is NULL");
    if (n < 0 || (n > 0 && (!models || !f_host || !tickets)) || !n_done) return sfail(MSRS_ERR_ARG, "NULL argument");
    msrs_status st = MSRS_OK;
    int k = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (; k < n; ++k) {
            st = submit_locked(s, models[k], f_host[k], t_arrival ? t_arrival[k] : 0.0, &tickets[k]);
            if (st != MSRS_OK) break;
        }
    }
    *n_done = k;
    if (k > 0) s->cv_work.notify_one();
    return st;
}

msrs_status msrs_server_replay(msrs_server s, int32_t n, const int32_t* models, const double* const* f_host,
                               const double* t_arrival, msrs_request_info* infos) {
    if (!valid(s)) return sfail(MSRS_ERR_ARG, "server is NULL");
    if (n < 0 || (n > 0 && (!models || !f_host || !infos))) return sfail(MSRS_ERR_ARG, "NULL argument");
    for (int i = 0; i < n; ++i) {
        if (models[i] < 0 || models[i] >= (int)s->models.size()) return sfail(MSRS_ERR_ARG, "model index out of range");
        if (!f_host[i]) return sfail(MSRS_ERR_ARG, "f_host has a NULL entry");
    }
    int64_t finished = 0;   // guarded by s->mu
    msrs_status st = MSRS_OK;
    int k = 0;
    for (; k < n; ++k) {
        const double ta = t_arrival ? t_arrival[k] : 0.0;
        if (ta > 0)
            while (now_s() < ta) {
            }
        for (;;) {
            int64_t ticket;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                st = submit_locked(s, models[k], f_host[k], ta, &ticket, &infos[k], &finished);
            }
            if (st != MSRS_ERR_BUSY) break;
            std::this_thread::yield();   // back-pressure: wait for staging / pending room
        }
        if (st != MSRS_OK) break;
        s->cv_work.notify_one();
    }
    // every queued request of this call reports through its info record
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return finished >= k; });
    if (st != MSRS_OK) return st;
    for (int i = 0; i < n; ++i)
        if (infos[i].status != MSRS_OK) return sfail(infos[i].status, s->fatal_msg.empty() ? "request failed" : s->fatal_msg);
    return MSRS_OK;
}

msrs_status msrs_server_wait(msrs_server s, int64_t ticket, double timeout_s) {
    if (!valid(s)) return sfail(MSRS_ERR_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end() || it->second.discard_info) return sfail(MSRS_ERR_ARG, "unknown ticket");
    auto ready = [&] { return it->second.state >= kDone; };
    if (timeout_s < 0) s->cv_done.wait(lk, ready);
    else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) return sfail(MSRS_ERR_BUSY, "request not finished");
    if (it->second.state == kFailed) return sfail(it->second.status, s->fatal_msg.empty() ? "request failed" : s->fatal_msg);
    return MSRS_OK;
}

msrs_status msrs_server_fetch(msrs_server s, int64_t ticket, double* u_out, msrs_request_info* info) {
    if (!valid(s)) return sfail(MSRS_ERR_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end() || it->second.discard_info) return sfail(MSRS_ERR_ARG, "unknown ticket");
    if (it->second.fetching) return sfail(MSRS_ERR_ARG, "ticket is being fetched by another call");
    it->second.fetching = true;
    s->cv_done.wait(lk, [&] { return it->second.state >= kDone; });
    Req r = it->second;
    msrs_status st = r.state == kFailed ? r.status : MSRS_OK;
    if (info) fill_info(r, st, info);
    if (st == MSRS_OK && u_out) {
        // the slot stays held (and unlisted for reuse) while the copy runs
        lk.unlock();
        hipError_t e = hipMemcpyAsync(u_out, s->dslots + r.slot_off, (size_t)r.slot_bytes, hipMemcpyDefault, s->copy);
        if (e == hipSuccess) e = hipStreamSynchronize(s->copy);
        lk.lock();
        if (e != hipSuccess) st = sfail(MSRS_ERR_HIP, std::string("copy-out: ") + hipGetErrorString(e));
    }
    if (r.slot_off >= 0) s->slots.release(r.slot_off, r.slot_bytes);
    if (r.stage_off >= 0) s->stage.release(r.stage_off, r.stage_bytes);
    s->reqs.erase(ticket);
    lk.unlock();
    s->cv_work.notify_one();
    if (st != MSRS_OK && g_server_err.empty()) g_server_err = "request failed";
    return st;
}

msrs_status msrs_server_get_stats(msrs_server s, msrs_server_stats* out) {
    if (!valid(s) || !out) return sfail(MSRS_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    out->submitted = s->n_submitted;
    out->completed = s->n_completed;
    out->batches = s->n_batches;
    out->max_in_flight = s->max_in_flight;
    out->peak_slot_bytes = s->peak_slot;
    out->slot_capacity = s->slots.capacity();
    out->admission_waits = s->stalls;
    out->mean_batch = s->n_batches ? (double)s->batch_reqs / (double)s->n_batches : 0.0;
    return s->fatal;
}

void msrs_server_destroy(msrs_server s) {
    if (!s) return;
    if (s->worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
            for (auto& it : s->sched.drop_all()) {
                Req& r = s->reqs[it.id];
                r.state = kFailed;
                r.status = MSRS_ERR_STATE;
            }
        }
        s->cv_work.notify_all();
        s->worker.join();
        s->cv_done.notify_all();
        for (Ctx* c : s->models) c->served -= 1;
    }
    for (auto& L : s->lanes) {
        if (L.st) { (void)hipStreamSynchronize(L.st); (void)hipStreamDestroy(L.st); }
        if (L.ev) (void)hipEventDestroy(L.ev);
    }
    if (s->copy) (void)hipStreamDestroy(s->copy);
    for (void* p : s->dallocs) (void)hipFree(p);
    if (s->hstage) (void)hipHostFree(s->hstage);
    delete s;
}

}  // extern "C"
