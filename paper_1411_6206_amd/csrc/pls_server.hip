// Serving runtime: continuous batching of recursive (sliding-window) reconstructions.
//
// A request is one sequence: a first window of nt frames reconstructed by plain L+S, then
// n_append frames appended one at a time.  Up to max_active sequences of one batch class
// (the same phase-encode plane, transform, Gram mode and tile class; their nx, nt and nc may
// differ) are in flight together as a group: one host thread (the dispatcher) starts every
// member's next window (load or shift, on the member's own handle), then advances all of
// them with one batch (prior_ls_batch: one launch per kernel of an iteration for every
// member), each member running its own window's iteration count and stopping rule.  Members
// join a running group at window boundaries while the oldest pending request is of the
// group's class; a request of another class waits until the group drains, then starts the
// next group, which also gathers every request of its class already waiting.  A request
// is admitted when the device bytes it needs fit in the budget beside everything resident;
// handles of finished sequences stay resident (state, sample store, graphs) and are reused
// by later requests of the same geometry, and idle ones are evicted (oldest first) when an
// admission needs their room.  A new group starts with the oldest pending request that
// fits, so a small request is not held behind a large one waiting for memory.  Every
// sequence computes exactly what it computes alone.
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

// A sequence of the running group: its window and that window's start.
struct Member {
    Job* j = nullptr;
    int window = 0;
    Clock::time_point wstart{};
};

void set_message(prior_ls_result& r, const std::string& m) {
    std::snprintf(r.message, sizeof(r.message), "%s", m.c_str());
}

}  // namespace

// Members of a group at most (max_active is clamped to it).  Sequences only ever share the
// GPU as members of one batch: independently driven sequences on streams of their own were
// switched off after a run with four large ones in flight ended in a host segmentation
// fault whose cause was not found.
#ifndef PLS_SERVER_MAX_IN_FLIGHT
#define PLS_SERVER_MAX_IN_FLIGHT 64
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
    prior_ls_batch* batch = nullptr;          // over the running group's handles
    std::vector<prior_ls_handle*> batch_of;   // the handles `batch` was built over

    // Picks the oldest pending job that fits (reusing an idle handle of its geometry, or
    // evicting idle handles to make room); returns nullptr when none fits.  The handles to
    // destroy are returned through `evict` and destroyed by the caller without the lock.
    Job* admit_locked(std::vector<Resident>& evict) {
        for (auto it = pending.begin(); it != pending.end(); ++it) {
            if (!reserve_locked(*it, evict)) continue;
            Job* j = *it;
            pending.erase(it);
            return j;
        }
        return nullptr;
    }

    // A pending job that can share a batch with geometry `d` (pls::batch_compatible: the same
    // plane, transform, Gram mode and tile class; nx, nt and nc may differ) and fits: with
    // `oldest_only` only the oldest pending job qualifies (a running group does not overtake
    // older requests of other classes), else the oldest of that class (a group being formed
    // gathers what waits for it).
    Job* admit_same_locked(const prior_ls_dims& d, bool oldest_only, std::vector<Resident>& evict) {
        for (auto it = pending.begin(); it != pending.end(); ++it) {
            if (pls::batch_compatible((*it)->req.dims, d)) {
                if (!reserve_locked(*it, evict)) return nullptr;
                Job* j = *it;
                pending.erase(it);
                return j;
            }
            if (oldest_only) return nullptr;
        }
        return nullptr;
    }

    // Reserves job j's device bytes: an idle handle of its geometry (grown if its sample
    // store needs more) or new room, evicting idle handles as needed.  False if it does not
    // fit (nothing reserved).
    bool reserve_locked(Job* j, std::vector<Resident>& evict) {
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
                    return false;
                }
                used += extra;
                j->res.bytes = j->need;
            }
        } else {
            if (!make_room_locked(j->need, evict)) return false;
            used += j->need;
            j->res.bytes = j->need;
        }
        peak = std::max(peak, used);
        return true;
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

    // Ends member m's window: records its statistics and latency.
    void close_window(Member& m, int converged, double ms) {
        prior_ls_request& q = m.j->req;
        if (q.latency_ms) q.latency_ms[m.window] = ms;
        if (q.stats) {
            prior_ls_stats st{};
            st.struct_size = sizeof(prior_ls_stats);
            pls::phase_stats(m.j->res.h, &st, converged, ms);
            q.stats[m.window] = st;
        }
    }

    // Starts member m's window: the first window loads the problem, a later one slides the
    // window by the next frame.
    int start_window(Member& m) {
        prior_ls_request& q = m.j->req;
        prior_ls_handle* h = m.j->res.h;
        m.wstart = Clock::now();
        if (m.window == 0) {
            prior_ls_inputs in{};
            in.kspace = q.kspace0;
            in.mask = q.mask0;
            in.sens = q.sens;
            prior_ls_params p = q.first;
            p.lambda_p = 0.0;                      // the first instance has no priors
            return pls::phase_load(h, &in, &p);
        }
        const size_t P = (size_t)q.dims.ny * q.dims.nz;
        const size_t fk = (size_t)q.dims.nc * P * q.dims.nx * 8;
        return pls::phase_shift(h, (const char*)q.kspace_frames + (m.window - 1) * fk,
                                q.mask_frames + (m.window - 1) * P, &q.next);
    }

    // Writes member m's outputs and waits for them.
    int write_outputs(Member& m) {
        prior_ls_handle* h = m.j->res.h;
        int rc = pls::phase_outputs(h, &m.j->req.out);
        while (rc == PRIOR_LS_OK) {
            const int r = pls::phase_query(h);
            if (r == 1) break;
            if (r < 0) return r;
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
        return rc;
    }

    // One window of every member of the group: start them, advance them together as one
    // batch, record each window, write the outputs of finished sequences.  Members that
    // finish or fail leave the group (their jobs are finished through `done`: status per job).
    void run_window(std::vector<Member>& group, std::vector<std::pair<Job*, int>>& done) {
        std::vector<Member> live;
        for (Member& m : group) {
            const int rc = start_window(m);
            if (rc) done.push_back({m.j, rc});
            else live.push_back(m);
        }
        group.swap(live);
        if (group.empty()) return;
        std::vector<prior_ls_handle*> hs;
        for (Member& m : group) hs.push_back(m.j->res.h);
        if (hs != batch_of) {
            prior_ls_batch_destroy(batch);
            batch = nullptr;
            batch_of.clear();
            const int rc = prior_ls_batch_create(hs.data(), (int32_t)hs.size(), &batch);
            if (rc) {
                for (Member& m : group) {
                    set_message(m.j->result, prior_ls_last_error(nullptr));
                    done.push_back({m.j, rc});
                }
                group.clear();
                return;
            }
            batch_of = hs;
        }
        std::vector<int> target, status;
        std::vector<char> conv;
        std::vector<Clock::time_point> end;
        for (Member& m : group) target.push_back(pls::phase_max_iter(m.j->res.h));
        const int rc = pls::batch_run(batch, target, conv, status, end);
        live.clear();
        for (size_t i = 0; i < group.size(); ++i) {
            Member& m = group[i];
            const int st = rc ? rc : status[i];
            if (st) {
                if (rc) set_message(m.j->result, prior_ls_batch_last_error(batch));
                done.push_back({m.j, st});
                continue;
            }
            close_window(m, conv[i], ms_between(m.wstart, end[i]));
            if (m.window == m.j->req.n_append) {
                done.push_back({m.j, write_outputs(m)});
                continue;
            }
            ++m.window;
            live.push_back(m);
        }
        group.swap(live);
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
        std::vector<Member> group;
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
                    // a new group takes the oldest pending request that fits and every
                    // waiting request of its geometry; a running one takes more requests of
                    // its geometry while the oldest pending request is one of them
                    while ((int)(group.size() + admitted.size()) < in_flight) {
                        Job* j;
                        if (!group.empty()) j = admit_same_locked(group[0].j->req.dims, true, evict);
                        else if (!admitted.empty()) j = admit_same_locked(admitted[0]->req.dims, false, evict);
                        else j = admit_locked(evict);
                        if (!j) break;
                        j->admitted = Clock::now();
                        admitted.push_back(j);
                        ++active;
                        peak_active = std::max(peak_active, active);
                    }
                    if (!group.empty() || !admitted.empty() || !incoming.empty()) break;
                    if (stopping && pending.empty()) {
                        prior_ls_batch_destroy(batch);
                        batch = nullptr;
                        batch_of.clear();
                        return;
                    }
                    cv_work.wait(lk);             // a submission, or the stop
                }
            }
            for (Resident& r : evict) destroy_resident(r);
            std::vector<std::pair<Job*, int>> done;
            for (Job* j : admitted) {
                const int rc = open_handle(j);
                if (rc) done.push_back({j, rc});
                else group.push_back(Member{j, 0, {}});
            }
            if (!group.empty()) run_window(group, done);
            if (!done.empty()) {
                // a finished member's handle may go back to the idle pool (or be destroyed):
                // the batch over it goes first
                prior_ls_batch_destroy(batch);
                batch = nullptr;
                batch_of.clear();
                {
                    std::lock_guard<std::mutex> lk(mu);
                    for (auto& jd : done) finish_locked(jd.first, jd.second, destroy);
                }
                cv_done.notify_all();
            }
            for (Resident& r : destroy) destroy_resident(r);
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
