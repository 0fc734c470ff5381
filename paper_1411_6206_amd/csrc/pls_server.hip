// Serving runtime: continuous batching of recursive (sliding-window) reconstructions.
//
// A request is one sequence: a first window of nt frames reconstructed by plain L+S, then
// n_append frames appended one at a time.  Up to max_active sequences are in flight at
// once, each on its own handle and streams, so their kernels share the GPU.  One host
// thread (the dispatcher) drives all of them: it starts a window, enqueues chunks of
// iterations without waiting, polls their completion, and moves each sequence on as its
// work finishes, so the HIP runtime is called from a single thread.  A request is
// admitted when the device bytes it needs fit in the budget beside everything resident;
// handles of finished sequences stay resident (state, sample store, graphs) and are
// reused by later requests of the same geometry, and idle ones are evicted (oldest first)
// when an admission needs their room.  Pending requests are admitted oldest first among
// those that fit, so a small request is not held behind a large one waiting for memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "prior_ls.h"
#include "pls_runtime_api.hpp"

namespace pls {
void set_thread_error(const std::string& m);
}

namespace {

int fail(int code, const std::string& m) {
    pls::set_thread_error(m);
    return code;
}

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

bool same_dims(const prior_ls_dims& a, const prior_ls_dims& b) {
    return a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.nt == b.nt && a.nc == b.nc &&
           a.wavelet_levels == b.wavelet_levels && a.gram_mode == b.gram_mode &&
           a.transform == b.transform;
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

// A sequence in flight: its window, the iterations left in the window and the chunk on the
// GPU, if any.
struct Active {
    Job* j = nullptr;
    enum State { kStart, kRun, kOutputs } st = kStart;
    int window = 0;
    int remaining = 0;
    int inflight = 0;
    int converged = 0;
    Clock::time_point wstart{};
};

void set_message(prior_ls_result& r, const std::string& m) {
    std::snprintf(r.message, sizeof(r.message), "%s", m.c_str());
}

}  // namespace

// Sequences driven at once.  Several sequences in flight is switched off: a run with four
// large sequences in flight ended in a host segmentation fault (with one dispatcher thread
// as with one thread per sequence) whose cause was not found, so requests beyond the first
// queue until it finishes.  (The host tests build the server with more in flight to
// exercise its logic on the CPU.)
#ifndef PLS_SERVER_MAX_IN_FLIGHT
#define PLS_SERVER_MAX_IN_FLIGHT 1
#endif
constexpr int kMaxInFlight = PLS_SERVER_MAX_IN_FLIGHT;

struct prior_ls_server {
    prior_ls_server_config cfg{};
    int in_flight = 1;
    int device = 0;
    uint64_t budget = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Job*> incoming;                // submitted, not yet checked by the dispatcher
    std::deque<Job*> pending;                 // checked, waiting for admission (submission order)
    std::map<int64_t, Job*> jobs;             // every job not yet waited for
    std::list<Resident> idle;                 // resident handles without a sequence
    uint64_t used = 0;                        // bytes of running + idle residents
    uint64_t peak = 0;
    int64_t next_ticket = 1;
    int64_t submitted = 0, completed = 0, failed = 0, reused = 0, evicted = 0;
    int active = 0, peak_active = 0;
    bool stopping = false;
    std::thread thread;                       // the dispatcher
    hipStream_t ctl = nullptr;                // the dispatcher's mask read-backs

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

    // Checks a submitted job on the dispatcher thread (device pointers) and sizes it: the
    // plan plus the compact k-space, one slot per frame sized by its most sampled frame.
    int prepare(Job* j) {
        const prior_ls_request& q = j->req;
        const prior_ls_dims& d = q.dims;
        if (!on_device(q.kspace0) || !on_device(q.mask0) || (d.nc > 1 && !on_device(q.sens)) ||
            (q.n_append > 0 && (!on_device(q.kspace_frames) || !on_device(q.mask_frames)))) {
            set_message(j->result, "input arrays must be device memory");
            return PRIOR_LS_EINVAL;
        }
        const void* o[] = {q.out.L, q.out.S, q.out.X, q.out.M};
        for (const void* p : o)
            if (p && !on_device(p)) {
                set_message(j->result, "output arrays must be device memory");
                return PRIOR_LS_EINVAL;
            }
        const size_t P = (size_t)d.ny * d.nz;
        const size_t nf = (size_t)d.nt + q.n_append;
        std::vector<uint8_t> m(nf * P);
        hipError_t e = hipMemcpyAsync(m.data(), q.mask0, d.nt * P, hipMemcpyDeviceToHost, ctl);
        if (e == hipSuccess && q.n_append > 0)
            e = hipMemcpyAsync(m.data() + d.nt * P, q.mask_frames, q.n_append * P,
                               hipMemcpyDeviceToHost, ctl);
        if (e == hipSuccess) e = hipStreamSynchronize(ctl);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            set_message(j->result, std::string("reading the masks: ") + hipGetErrorString(e));
            return PRIOR_LS_EHIP;
        }
        size_t ns_max = 1;
        for (size_t f = 0; f < nf; ++f) {
            size_t c = 0;
            for (size_t k = 0; k < P; ++k) c += m[f * P + k] != 0;
            ns_max = std::max(ns_max, c);
        }
        j->need = prior_ls_plan_bytes(&d) + ((uint64_t)d.nt * d.nx * d.nc * ns_max + 64) * 8;
        if (j->need > budget) {
            set_message(j->result, "the request alone exceeds the server budget");
            return PRIOR_LS_ENOMEM;
        }
        return PRIOR_LS_OK;
    }

    // A job that ends before admission (under the lock).
    void reject_locked(Job* j, int status) {
        j->result.status = status;
        j->result.total_ms = ms_between(j->submitted, Clock::now());
        ++failed;
        j->done = true;
    }

    // Creates the handle of a newly admitted job when no resident one was reused.
    int open_handle(Job* j) {
        if (j->res.h) return PRIOR_LS_OK;
        prior_ls_dims d = j->req.dims;
        d.hbm_budget = 0;                      // admission is the server's
        if (hipStreamCreateWithFlags(&j->res.stream, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            set_message(j->result, "cannot create a stream");
            return PRIOR_LS_EHIP;
        }
        j->res.dims = j->req.dims;
        const int rc = prior_ls_create(&d, j->res.stream, &j->res.h);
        if (rc) set_message(j->result, prior_ls_last_error(nullptr));
        return rc;
    }

    // Ends window a.window: records its statistics and latency.
    void close_window(Active& a) {
        prior_ls_request& q = a.j->req;
        const double ms = ms_between(a.wstart, Clock::now());
        if (q.latency_ms) q.latency_ms[a.window] = ms;
        if (q.stats) {
            prior_ls_stats st{};
            st.struct_size = sizeof(prior_ls_stats);
            pls::phase_stats(a.j->res.h, &st, a.converged, ms);
            q.stats[a.window] = st;
        }
    }

    // Moves one sequence on as far as it can go without waiting.  Returns 1 on progress,
    // 0 when it waits for the GPU, or a negative status (the sequence has failed).
    int advance(Active& a) {
        Job* j = a.j;
        prior_ls_request& q = j->req;
        prior_ls_handle* h = j->res.h;
        const bool last = a.window == q.n_append;
        if (a.st == Active::kStart) {
            a.wstart = Clock::now();
            a.converged = 0;
            int rc;
            if (a.window == 0) {
                prior_ls_inputs in{};
                in.kspace = q.kspace0;
                in.mask = q.mask0;
                in.sens = q.sens;
                prior_ls_params p = q.first;
                p.lambda_p = 0.0;                  // the first instance has no priors
                rc = pls::phase_load(h, &in, &p);
            } else {
                const size_t P = (size_t)q.dims.ny * q.dims.nz;
                const size_t fk = (size_t)q.dims.nc * P * q.dims.nx * 8;
                rc = pls::phase_shift(h, (const char*)q.kspace_frames + (a.window - 1) * fk,
                                      q.mask_frames + (a.window - 1) * P, &q.next);
            }
            if (rc) return rc;
            a.remaining = pls::phase_max_iter(h);
            a.inflight = 0;
            a.st = Active::kRun;
        }
        if (a.st == Active::kRun) {
            if (a.inflight) {
                const int r = pls::phase_query(h);
                if (r <= 0) return r;
                const int rc = pls::phase_chunk_finish(h, a.inflight, &a.converged);
                if (rc) return rc;
                a.remaining -= a.inflight;
                a.inflight = 0;
            }
            if (a.remaining > 0 && !a.converged) {
                const int m = pls::phase_chunk_launch(h, a.remaining);
                if (m < 0) return m;
                a.inflight = m;
                return 1;
            }
            if (!last) {
                close_window(a);
                ++a.window;
                a.st = Active::kStart;
                return 1;
            }
            const int rc = pls::phase_outputs(h, &q.out);
            if (rc) return rc;
            a.st = Active::kOutputs;
            return 1;
        }
        // kOutputs
        const int r = pls::phase_query(h);
        if (r <= 0) return r;
        close_window(a);
        return 2;                                 // done
    }

    // Ends a job (under the lock): its handle goes to the idle pool, or is destroyed
    // (returned through `destroy`) when the sequence failed.
    void finish_locked(Job* j, int status, std::vector<Resident>& destroy) {
        const auto now = Clock::now();
        j->result.status = status;
        if (status && j->res.h && !j->result.message[0])
            set_message(j->result, prior_ls_last_error(j->res.h));
        j->result.reused_plan = j->reused ? 1 : 0;
        j->result.queue_ms = ms_between(j->submitted, j->admitted);
        j->result.run_ms = ms_between(j->admitted, now);
        j->result.total_ms = ms_between(j->submitted, now);
        j->result.state_bytes = j->res.bytes;
        if (j->reused) ++reused;
        if (status == PRIOR_LS_OK && j->res.h) {
            j->res.idle_since = now;
            idle.push_back(j->res);
            ++completed;
        } else {
            used -= j->res.bytes;
            destroy.push_back(j->res);
            ++failed;
        }
        j->res = Resident{};
        --active;
        j->done = true;
    }

    void dispatcher() {
        (void)hipSetDevice(device);
        std::vector<Active> act;
        for (;;) {
            std::vector<Resident> evict, destroy;
            std::vector<Job*> admitted, fresh;
            {
                std::lock_guard<std::mutex> lk(mu);
                fresh.assign(incoming.begin(), incoming.end());
                incoming.clear();
            }
            for (Job* j : fresh) {
                const int rc = prepare(j);
                std::lock_guard<std::mutex> lk(mu);
                if (rc) {
                    reject_locked(j, rc);
                    cv_done.notify_all();
                } else {
                    pending.push_back(j);
                }
            }
            {
                std::unique_lock<std::mutex> lk(mu);
                for (;;) {
                    while ((int)(act.size() + admitted.size()) < in_flight) {
                        Job* j = admit_locked(evict);
                        if (!j) break;
                        j->admitted = Clock::now();
                        admitted.push_back(j);
                        ++active;
                        peak_active = std::max(peak_active, active);
                    }
                    if (!act.empty() || !admitted.empty() || !incoming.empty()) break;
                    if (stopping && pending.empty()) return;
                    cv_work.wait(lk);             // a submission, or the stop
                }
            }
            for (Resident& r : evict) destroy_resident(r);
            for (Job* j : admitted) {
                Active a;
                a.j = j;
                const int rc = open_handle(j);
                if (rc) {
                    std::lock_guard<std::mutex> lk(mu);
                    finish_locked(j, rc, destroy);
                    cv_done.notify_all();
                    continue;
                }
                act.push_back(a);
            }
            bool progress = false;
            for (size_t i = 0; i < act.size();) {
                int r = advance(act[i]);
                while (r == 1) {                          // as far as it goes without waiting
                    progress = true;
                    r = advance(act[i]);
                }
                if (r == 0) {
                    ++i;
                    continue;
                }
                progress = true;
                {
                    std::lock_guard<std::mutex> lk(mu);
                    finish_locked(act[i].j, r == 2 ? PRIOR_LS_OK : r, destroy);
                }
                cv_done.notify_all();
                act.erase(act.begin() + i);
            }
            for (Resident& r : destroy) destroy_resident(r);
            if (!progress && admitted.empty()) std::this_thread::sleep_for(std::chrono::microseconds(20));
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
    s->in_flight = std::min(cfg->max_active, kMaxInFlight);
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
    if (hipStreamCreateWithFlags(&s->ctl, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return fail(PRIOR_LS_EHIP, "cannot create the control stream");
    }
    s->thread = std::thread([s] { s->dispatcher(); });
    *out = s;
    return PRIOR_LS_OK;
}

int prior_ls_server_submit(prior_ls_server* s, const prior_ls_request* req, int64_t* ticket) {
    if (!s || !req || !ticket) return fail(PRIOR_LS_EINVAL, "server, request and ticket are required");
    if (req->struct_size != sizeof(prior_ls_request)) return fail(PRIOR_LS_EINVAL, "request.struct_size mismatch");
    const prior_ls_dims& d = req->dims;
    if (d.struct_size != sizeof(prior_ls_dims)) return fail(PRIOR_LS_EINVAL, "dims.struct_size mismatch");
    if (prior_ls_plan_bytes(&d) == 0) return fail(PRIOR_LS_ESHAPE, "unsupported dims");
    if (req->first.struct_size != sizeof(prior_ls_params) ||
        req->next.struct_size != sizeof(prior_ls_params))
        return fail(PRIOR_LS_EINVAL, "params.struct_size mismatch");
    if (req->n_append < 0 || req->reserved != 0) return fail(PRIOR_LS_EINVAL, "n_append < 0 or reserved != 0");
    if (!req->kspace0 || !req->mask0 || (d.nc > 1 && !req->sens) ||
        (req->n_append > 0 && (!req->kspace_frames || !req->mask_frames)))
        return fail(PRIOR_LS_EINVAL, "a required array is NULL");
    auto* j = new Job();
    j->req = *req;
    j->submitted = Clock::now();
    j->result.struct_size = sizeof(prior_ls_result);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) {
            delete j;
            return fail(PRIOR_LS_EINVAL, "server is stopping");
        }
        j->ticket = s->next_ticket++;
        s->jobs[j->ticket] = j;
        s->incoming.push_back(j);
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
    if (s->thread.joinable()) s->thread.join();
    for (Resident& r : s->idle) prior_ls_server::destroy_resident(r);
    for (auto& kv : s->jobs) delete kv.second;
    if (s->ctl) (void)hipStreamDestroy(s->ctl);
    delete s;
}

}  // extern "C"
