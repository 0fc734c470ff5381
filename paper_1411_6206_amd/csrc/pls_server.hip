// Serving runtime: continuous batching of recursive (sliding-window) reconstructions.
//
// A request is one sequence: a first window of nt frames reconstructed by plain L+S, then
// n_append frames appended one at a time (prior_ls_append).  The server runs up to
// max_active sequences at once, each driven by its own host worker on its own streams, so
// their kernels share the GPU.  A request is admitted when the device bytes it needs fit
// in the budget beside everything resident; handles of finished sequences stay resident
// (state, sample store, graphs) and are reused by later requests of the same geometry,
// and idle ones are evicted (oldest first) when an admission needs their room.  Pending
// requests are admitted oldest first among those that fit, so a small request is not held
// behind a large one that is waiting for memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "prior_ls.h"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

bool same_dims(const prior_ls_dims& a, const prior_ls_dims& b) {
    return a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.nt == b.nt && a.nc == b.nc &&
           a.wavelet_levels == b.wavelet_levels && a.gram_mode == b.gram_mode;
}

bool on_device(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

// A resident handle with the stream its calls are ordered on.
struct Resident {
    prior_ls_handle* h = nullptr;
    hipStream_t stream = nullptr;
    prior_ls_dims dims{};
    uint64_t bytes = 0;
    Clock::time_point idle_since{};
};

struct Job {
    int64_t ticket = 0;
    prior_ls_request req{};
    uint64_t need = 0;            // device bytes: plan + compact k-space of the largest frame
    Clock::time_point submitted{};
    Clock::time_point admitted{};
    Resident res{};
    bool reused = false;
    bool done = false;
    prior_ls_result result{};
};

void set_message(prior_ls_result& r, const std::string& m) {
    std::snprintf(r.message, sizeof(r.message), "%s", m.c_str());
}

}  // namespace

struct prior_ls_server {
    prior_ls_server_config cfg{};
    int device = 0;
    uint64_t budget = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Job*> pending;                 // submission order
    std::map<int64_t, Job*> jobs;             // every job not yet waited for
    std::list<Resident> idle;                 // resident handles without a sequence
    uint64_t used = 0;                        // bytes of running + idle residents
    uint64_t peak = 0;
    int64_t next_ticket = 1;
    int64_t submitted = 0, completed = 0, failed = 0, reused = 0, evicted = 0;
    int active = 0, peak_active = 0;
    bool stopping = false;
    std::vector<std::thread> workers;

    // Picks the oldest pending job that fits (reusing an idle handle of its geometry, or
    // evicting idle handles to make room); returns nullptr when none fits.  The handles to
    // destroy are returned through `evict` and destroyed by the caller without the lock.
    Job* admit_locked(std::vector<Resident>& evict) {
        for (auto it = pending.begin(); it != pending.end(); ++it) {
            Job* j = *it;
            auto same = std::find_if(idle.begin(), idle.end(),
                                     [&](const Resident& r) { return same_dims(r.dims, j->req.dims); });
            if (same != idle.end()) {
                j->res = *same;
                j->reused = true;
                idle.erase(same);
                if (j->need > j->res.bytes) {       // the sample store may grow
                    const uint64_t extra = j->need - j->res.bytes;
                    if (!make_room_locked(extra, evict)) {
                        idle.push_front(j->res);
                        j->res = Resident{};
                        j->reused = false;
                        continue;
                    }
                    used += extra;
                    j->res.bytes = j->need;
                }
            } else {
                if (!make_room_locked(j->need, evict)) continue;
                used += j->need;
                j->res.bytes = j->need;
            }
            peak = std::max(peak, used);
            pending.erase(it);
            return j;
        }
        return nullptr;
    }

    // Evicts idle handles (oldest first) until `bytes` more fit in the budget.
    bool make_room_locked(uint64_t bytes, std::vector<Resident>& evict) {
        uint64_t idle_bytes = 0;
        for (const Resident& r : idle) idle_bytes += r.bytes;
        if (used - idle_bytes + bytes > budget) return false;
        while (used + bytes > budget && !idle.empty()) {
            auto oldest = std::min_element(idle.begin(), idle.end(), [](const Resident& a, const Resident& b) {
                return a.idle_since < b.idle_since;
            });
            used -= oldest->bytes;
            evict.push_back(*oldest);
            idle.erase(oldest);
            ++evicted;
        }
        return used + bytes <= budget;
    }

    static void destroy_resident(Resident& r) {
        if (r.h) prior_ls_destroy(r.h);
        if (r.stream) (void)hipStreamDestroy(r.stream);
        r = Resident{};
    }

    void run(Job* j) {
        prior_ls_request& q = j->req;
        prior_ls_result& res = j->result;
        const int nw = q.n_append + 1;
        int rc = PRIOR_LS_OK;
        if (!j->res.h) {
            prior_ls_dims d = q.dims;
            d.hbm_budget = 0;                  // admission is the server's
            if (hipStreamCreateWithFlags(&j->res.stream, hipStreamNonBlocking) != hipSuccess) {
                (void)hipGetLastError();
                rc = PRIOR_LS_EHIP;
                set_message(res, "cannot create a stream");
            } else {
                rc = prior_ls_create(&d, j->res.stream, &j->res.h);
                if (rc) set_message(res, prior_ls_last_error(nullptr));
            }
            j->res.dims = q.dims;
        }
        const prior_ls_outputs none{nullptr, nullptr, nullptr, nullptr};
        for (int w = 0; w < nw && rc == PRIOR_LS_OK; ++w) {
            const bool last = w == nw - 1;
            const prior_ls_outputs* out = last ? &q.out : &none;
            prior_ls_stats st{};
            st.struct_size = sizeof(prior_ls_stats);
            const auto t0 = Clock::now();
            if (w == 0) {
                prior_ls_inputs in{};
                in.kspace = q.kspace0;
                in.mask = q.mask0;
                in.sens = q.sens;
                prior_ls_params p = q.first;
                p.lambda_p = 0.0;                  // the first instance has no priors
                rc = prior_ls_solve(j->res.h, &in, &p, out, &st);
            } else {
                const size_t P = (size_t)q.dims.ny * q.dims.nz;
                const size_t fk = (size_t)q.dims.nc * P * q.dims.nx * 8;
                rc = prior_ls_append(j->res.h, (const char*)q.kspace_frames + (w - 1) * fk,
                                     q.mask_frames + (w - 1) * P, &q.next, out, &st);
            }
            const double ms = ms_between(t0, Clock::now());
            if (q.latency_ms) q.latency_ms[w] = ms;
            if (q.stats) q.stats[w] = st;
            if (rc) set_message(res, prior_ls_last_error(j->res.h));
        }
        res.status = rc;
    }

    void worker() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            std::vector<Resident> evict;
            Job* j = nullptr;
            cv_work.wait(lk, [&] {
                if (!pending.empty()) {
                    j = admit_locked(evict);
                    if (j) return true;
                }
                return stopping && pending.empty();
            });
            if (!j) return;
            ++active;
            peak_active = std::max(peak_active, active);
            j->admitted = Clock::now();
            lk.unlock();
            for (Resident& r : evict) destroy_resident(r);
            run(j);
            lk.lock();
            --active;
            const auto now = Clock::now();
            j->result.reused_plan = j->reused ? 1 : 0;
            j->result.queue_ms = ms_between(j->submitted, j->admitted);
            j->result.run_ms = ms_between(j->admitted, now);
            j->result.total_ms = ms_between(j->submitted, now);
            j->result.state_bytes = j->res.bytes;
            if (j->reused) ++reused;
            if (j->result.status == PRIOR_LS_OK && j->res.h) {
                j->res.idle_since = now;
                idle.push_back(j->res);
                ++completed;
            } else {
                used -= j->res.bytes;
                Resident r = j->res;
                lk.unlock();
                destroy_resident(r);
                lk.lock();
                ++failed;
            }
            j->res = Resident{};
            j->done = true;
            cv_done.notify_all();
            cv_work.notify_all();                 // memory or a slot freed up
        }
    }
};

extern "C" {

int prior_ls_server_create(const prior_ls_server_config* cfg, prior_ls_server** out) {
    if (!out) return PRIOR_LS_EINVAL;
    *out = nullptr;
    if (!cfg || cfg->struct_size != sizeof(prior_ls_server_config)) return PRIOR_LS_EINVAL;
    if (cfg->max_active < 1 || cfg->max_active > 64 || cfg->reserved != 0) return PRIOR_LS_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return PRIOR_LS_EHIP;
    }
    auto* s = new prior_ls_server();
    s->cfg = *cfg;
    if (hipGetDevice(&s->device) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return PRIOR_LS_EHIP;
    }
    s->budget = cfg->hbm_budget;
    if (s->budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            (void)hipGetLastError();
            delete s;
            return PRIOR_LS_EHIP;
        }
        s->budget = (uint64_t)(0.9 * (double)fr);
    }
    for (int i = 0; i < cfg->max_active; ++i) s->workers.emplace_back([s] { s->worker(); });
    *out = s;
    return PRIOR_LS_OK;
}

int prior_ls_server_submit(prior_ls_server* s, const prior_ls_request* req, int64_t* ticket) {
    if (!s || !req || !ticket) return PRIOR_LS_EINVAL;
    if (req->struct_size != sizeof(prior_ls_request)) return PRIOR_LS_EINVAL;
    const prior_ls_dims& d = req->dims;
    if (d.struct_size != sizeof(prior_ls_dims)) return PRIOR_LS_EINVAL;
    const uint64_t plan = prior_ls_plan_bytes(&d);
    if (plan == 0) return PRIOR_LS_ESHAPE;
    if (req->first.struct_size != sizeof(prior_ls_params) ||
        req->next.struct_size != sizeof(prior_ls_params))
        return PRIOR_LS_EINVAL;
    if (req->n_append < 0 || req->reserved != 0) return PRIOR_LS_EINVAL;
    if (!on_device(req->kspace0) || !on_device(req->mask0)) return PRIOR_LS_EINVAL;
    if (d.nc > 1 && !on_device(req->sens)) return PRIOR_LS_EINVAL;
    if (req->n_append > 0 && (!on_device(req->kspace_frames) || !on_device(req->mask_frames)))
        return PRIOR_LS_EINVAL;
    // bytes of the compact k-space: one slot per frame, sized by the most sampled frame
    const size_t P = (size_t)d.ny * d.nz;
    const size_t nf = (size_t)d.nt + req->n_append;
    std::vector<uint8_t> m(nf * P);
    if (hipMemcpy(m.data(), req->mask0, d.nt * P, hipMemcpyDeviceToHost) != hipSuccess ||
        (req->n_append > 0 &&
         hipMemcpy(m.data() + d.nt * P, req->mask_frames, req->n_append * P, hipMemcpyDeviceToHost) != hipSuccess)) {
        (void)hipGetLastError();
        return PRIOR_LS_EHIP;
    }
    size_t ns_max = 1;
    for (size_t f = 0; f < nf; ++f) {
        size_t c = 0;
        for (size_t k = 0; k < P; ++k) c += m[f * P + k] != 0;
        ns_max = std::max(ns_max, c);
    }
    const uint64_t need = plan + ((uint64_t)d.nt * d.nx * d.nc * ns_max + 64) * 8;
    if (need > s->budget) return PRIOR_LS_ENOMEM;
    auto* j = new Job();
    j->req = *req;
    j->need = need;
    j->submitted = Clock::now();
    j->result.struct_size = sizeof(prior_ls_result);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) {
            delete j;
            return PRIOR_LS_EINVAL;
        }
        j->ticket = s->next_ticket++;
        s->jobs[j->ticket] = j;
        s->pending.push_back(j);
        ++s->submitted;
    }
    s->cv_work.notify_all();
    *ticket = j->ticket;
    return PRIOR_LS_OK;
}

int prior_ls_server_wait(prior_ls_server* s, int64_t ticket, prior_ls_result* result) {
    if (!s || !result || result->struct_size != sizeof(prior_ls_result)) return PRIOR_LS_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return PRIOR_LS_EINVAL;
    Job* j = it->second;
    s->cv_done.wait(lk, [&] { return j->done; });
    *result = j->result;
    s->jobs.erase(it);
    delete j;
    return PRIOR_LS_OK;
}

int prior_ls_server_info(prior_ls_server* s, prior_ls_server_stats* info) {
    if (!s || !info || info->struct_size != sizeof(prior_ls_server_stats)) return PRIOR_LS_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    info->budget = s->budget;
    info->used = s->used;
    info->peak_used = s->peak;
    info->submitted = s->submitted;
    info->completed = s->completed;
    info->failed = s->failed;
    info->reused = s->reused;
    info->evicted = s->evicted;
    info->queued = (int32_t)s->pending.size();
    info->active = s->active;
    info->peak_active = s->peak_active;
    info->resident_idle = (int32_t)s->idle.size();
    return PRIOR_LS_OK;
}

void prior_ls_server_destroy(prior_ls_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_work.notify_all();
    for (auto& t : s->workers) t.join();
    for (Resident& r : s->idle) prior_ls_server::destroy_resident(r);
    for (auto& kv : s->jobs) delete kv.second;
    delete s;
}

}  // extern "C"
