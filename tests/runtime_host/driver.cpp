// The library's runtime and serving dispatcher, host code as built for the GPU, driven on
// the CPU against stand-ins of HIP and of the kernels: sequences of five geometries (one
// with fully sampled appended frames, so its sample store grows), up to four of one
// geometry in flight as a batched group, a budget that forces queueing and evictions,
// submitted from a second thread; then the synchronous entry points on several handles
// from several threads at once, and batches.
#include <atomic>
#include <cstdio>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

#include <hip/hip_runtime.h>
#include "prior_ls.h"

struct Geo {
    int nx, ny, nz, nt, nc, dense_frames;
};
static const Geo kSmall[] = {{16, 16, 4, 5, 2, 0}, {24, 32, 8, 7, 3, 0}, {32, 32, 1, 6, 1, 0},
                             {16, 16, 4, 6, 2, 1}, {48, 32, 8, 8, 2, 0}};
// "full": the serving workload's volume classes at their real sizes, the 192x192x32 x 30
// frames x 8 coils class among them (four of it in flight), plus one with fully sampled
// appended frames so its sample store grows
static const Geo kFull[] = {{192, 192, 32, 30, 8, 0}, {128, 128, 16, 24, 4, 0},
                            {64, 64, 8, 16, 1, 0}, {192, 192, 32, 16, 4, 1},
                            {192, 192, 32, 30, 8, 0}};
static const Geo* kGeo = kSmall;

struct Seq {
    Geo g;
    int n_append;
    void *k0, *kf, *sens;
    uint8_t *m0, *mf;
    void* X;
    std::vector<double> lat;
    std::vector<prior_ls_stats> st;
    prior_ls_request rq{};
};

static void* dev_alloc(size_t n) {
    void* p = nullptr;
    hipMalloc(&p, n);
    // the full-size k-space arrays stay untouched (the stand-in kernels only read them)
    if (n < ((size_t)64 << 20)) std::memset(p, 0, n);
    return p;
}

static void make_seq(Seq& q, std::mt19937& rng) {
    const size_t P = (size_t)q.g.ny * q.g.nz, img = P * q.g.nx;
    q.k0 = dev_alloc((size_t)q.g.nc * q.g.nt * img * 8);
    q.kf = dev_alloc((size_t)(q.n_append ? q.n_append : 1) * q.g.nc * img * 8);
    q.sens = q.g.nc > 1 ? dev_alloc((size_t)q.g.nc * img * 8) : nullptr;
    q.m0 = (uint8_t*)dev_alloc((size_t)q.g.nt * P);
    q.mf = (uint8_t*)dev_alloc((size_t)(q.n_append ? q.n_append : 1) * P);
    for (size_t i = 0; i < (size_t)q.g.nt * P; ++i) q.m0[i] = rng() % 3 == 0;
    for (size_t i = 0; i < (size_t)q.n_append * P; ++i) q.mf[i] = q.g.dense_frames ? 1 : rng() % 4 == 0;
    q.X = dev_alloc((size_t)q.g.nt * img * 8);
    q.lat.assign(q.n_append + 1, 0.0);
    q.st.assign(q.n_append + 1, prior_ls_stats{});
    prior_ls_request& r = q.rq;
    r.struct_size = sizeof(r);
    r.dims = prior_ls_dims{sizeof(prior_ls_dims), q.g.nx, q.g.ny, q.g.nz, q.g.nt, q.g.nc, 2, 0, 0, 0};
    r.first = prior_ls_params{sizeof(prior_ls_params), 0.01, 0.01, 0.0, 0.0, 1, 8, 4, 1};
    r.next = prior_ls_params{sizeof(prior_ls_params), 0.01, 0.01, 0.2, 0.0, 1, 6, 3, 1};
    r.n_append = q.n_append;
    r.kspace0 = q.k0;
    r.mask0 = q.m0;
    r.kspace_frames = q.kf;
    r.mask_frames = q.mf;
    r.sens = q.sens;
    r.out = prior_ls_outputs{nullptr, nullptr, q.X, nullptr};
    r.stats = q.st.data();
    r.latency_ms = q.lat.data();
}

// "tune": the GPU autotuner test's sequence (32x48x8 x 12 frames x 3 coils, J = 2, chunks of
// 4): tune, step 12 and destroy; a fresh handle with the choice set by hand solves 12; a
// third with the choice set solves 0 iterations, steps 12 and is destroyed
static int tune_sequence(int rounds) {
    const int nx = 32, ny = 48, nz = 8, nt = 12, nc = 3;
    const size_t P = (size_t)ny * nz, img = P * nx;
    std::mt19937 rng(5);
    void* k = dev_alloc((size_t)nc * nt * img * 8);
    void* sens = dev_alloc((size_t)nc * img * 8);
    uint8_t* m = (uint8_t*)dev_alloc((size_t)nt * P);
    uint8_t* w = (uint8_t*)dev_alloc((size_t)nt * img);
    void* X[4];
    for (auto& x : X) x = dev_alloc((size_t)nt * img * 8);
    for (size_t i = 0; i < (size_t)nt * P; ++i) m[i] = rng() % 3 == 0;
    prior_ls_dims d{sizeof(prior_ls_dims), nx, ny, nz, nt, nc, 2, 0, 0, 0};
    prior_ls_params prm{sizeof(prior_ls_params), 0.01, 0.01, 0.0, 0.0, 1, 12, 4, 1};
    prior_ls_inputs in{k, m, sens, w, nullptr, nullptr, nullptr};
    prior_ls_outputs out{X[0], X[1], X[2], X[3]};
    int bad = 0;
    for (int r = 0; r < rounds; ++r) {
        prior_ls_tuning best{};
        best.struct_size = sizeof(best);
        prior_ls_stats st{};
        st.struct_size = sizeof(st);
        prior_ls_handle* h = nullptr;
        if (prior_ls_create(&d, nullptr, &h) || prior_ls_tune(h, &in, &prm, &best)) ++bad;
        if (prior_ls_step(h, 12, &out, &st) || st.iters != 12) ++bad;
        prior_ls_destroy(h);
        best.ms_per_iteration = 0.0;
        h = nullptr;
        if (prior_ls_create(&d, nullptr, &h) || prior_ls_set_tuning(h, &best)) ++bad;
        if (prior_ls_solve(h, &in, &prm, &out, &st) || st.iters != 12) ++bad;
        prior_ls_destroy(h);
        h = nullptr;
        prior_ls_params p0 = prm;
        p0.max_iter = 0;
        if (prior_ls_create(&d, nullptr, &h) || prior_ls_set_tuning(h, &best)) ++bad;
        if (prior_ls_solve(h, &in, &p0, nullptr, &st) || prior_ls_step(h, 12, &out, &st)) ++bad;
        prior_ls_destroy(h);
        std::printf("tune round %d: fork %d gram %d bp %d sparse grid %d\n", r, best.sparse_fork,
                    best.gram_blocks, best.bp_grid, best.sparse_grid);
    }
    for (void* p : {k, sens, (void*)m, (void*)w, X[0], X[1], X[2], X[3]}) hipFree(p);
    std::printf("tune done: bad %d\n", bad);
    return bad != 0;
}

int main(int argc, char** argv) {
    if (argc > 1 && std::strcmp(argv[1], "tune") == 0) return tune_sequence(5);
    const bool full = argc > 1 && std::strcmp(argv[1], "full") == 0;
    if (full) kGeo = kFull;
    std::mt19937 rng(11);
    const int N = full ? 12 : 40;
    std::vector<Seq> seqs(N);
    for (int i = 0; i < N; ++i) {
        // in "full" mode the first four requests are the 192x192x32 x 30 x 8 class
        seqs[i].g = (full && i < 4) ? kGeo[0] : kGeo[rng() % 5];
        seqs[i].n_append = full ? 1 + rng() % 3 : rng() % 4;
        make_seq(seqs[i], rng);
    }
    prior_ls_dims big{sizeof(prior_ls_dims), 48, 32, 8, 8, 2, 2, 0, 0, 0};
    if (full) big = prior_ls_dims{sizeof(prior_ls_dims), 192, 192, 32, 30, 8, 2, 0, 0, 0};
    prior_ls_server_config cfg{sizeof(cfg),
                               (uint64_t)(prior_ls_plan_bytes(&big) * (full ? 4.6 : 2.5)), 4, 0};
    prior_ls_server* s = nullptr;
    if (prior_ls_server_create(&cfg, &s)) return 1;
    std::vector<int64_t> tk(N, -1);
    std::atomic<int> submitted{0};
    std::thread sub([&] {
        for (int i = 0; i < N; ++i) {
            if (prior_ls_server_submit(s, &seqs[i].rq, &tk[i])) std::abort();
            submitted.store(i + 1);
            std::this_thread::sleep_for(std::chrono::microseconds(200));
        }
    });
    int bad = 0;
    for (int i = 0; i < N; ++i) {
        while (submitted.load() <= i) std::this_thread::yield();
        prior_ls_result r{};
        r.struct_size = sizeof(r);
        if (prior_ls_server_wait(s, tk[i], &r)) return 1;
        if (r.status) {
            ++bad;
            std::printf("request %d: status %d %s\n", i, r.status, r.message);
        }
        for (int w = 0; w <= seqs[i].n_append; ++w) {
            const int want = w == 0 ? 8 : 6;
            if (seqs[i].st[w].iters != want) {
                ++bad;
                std::printf("request %d window %d: %d iterations\n", i, w, seqs[i].st[w].iters);
            }
        }
    }
    sub.join();
    prior_ls_server_stats info{};
    info.struct_size = sizeof(info);
    prior_ls_server_info(s, &info);
    std::printf("server: completed %lld failed %lld reused %lld evicted %lld peak_active %d\n",
                (long long)info.completed, (long long)info.failed, (long long)info.reused,
                (long long)info.evicted, info.peak_active);
    prior_ls_server_destroy(s);
    // the synchronous entry points, one handle per thread, four threads at once
    std::vector<std::thread> th;
    std::atomic<int> sync_bad{0};
    for (int k = 0; k < 4; ++k)
        th.emplace_back([&, k] {
            Seq& q = seqs[k];
            prior_ls_handle* h = nullptr;
            if (prior_ls_create(&q.rq.dims, nullptr, &h)) {
                ++sync_bad;
                return;
            }
            prior_ls_inputs in{q.k0, q.m0, q.sens, nullptr, nullptr, nullptr, nullptr};
            prior_ls_stats st{};
            st.struct_size = sizeof(st);
            if (prior_ls_solve(h, &in, &q.rq.first, &q.rq.out, &st)) ++sync_bad;
            for (int j = 0; j < q.n_append; ++j) {
                const size_t P = (size_t)q.g.ny * q.g.nz;
                if (prior_ls_append(h, (char*)q.kf + (size_t)j * q.g.nc * P * q.g.nx * 8, q.mf + j * P,
                                    &q.rq.next, &q.rq.out, &st))
                    ++sync_bad;
            }
            if (prior_ls_step(h, 3, &q.rq.out, &st)) ++sync_bad;
            prior_ls_destroy(h);
        });
    for (auto& t : th) t.join();
    // a batch of three problems of one geometry with their own iteration counts and check
    // intervals, then a batched step; a batch of mixed geometries is refused
    {
        Seq q[3];
        prior_ls_handle* hb[3] = {nullptr, nullptr, nullptr};
        for (int k = 0; k < 3; ++k) {
            q[k].g = kGeo[1];
            q[k].n_append = 0;
            make_seq(q[k], rng);
            if (prior_ls_create(&q[k].rq.dims, nullptr, &hb[k])) ++sync_bad;
        }
        prior_ls_batch* b = nullptr;
        if (prior_ls_batch_create(hb, 3, &b)) ++sync_bad;
        prior_ls_inputs in[3];
        prior_ls_params pr[3];
        prior_ls_outputs out[3];
        prior_ls_stats st[3];
        const int iters[3] = {8, 5, 3}, ce[3] = {4, 2, 3};
        for (int k = 0; k < 3; ++k) {
            in[k] = prior_ls_inputs{q[k].k0, q[k].m0, q[k].sens, nullptr, nullptr, nullptr, nullptr};
            pr[k] = q[k].rq.first;
            pr[k].max_iter = iters[k];
            pr[k].check_every = ce[k];
            out[k] = q[k].rq.out;
            st[k] = prior_ls_stats{};
            st[k].struct_size = sizeof(prior_ls_stats);
        }
        if (prior_ls_batch_solve(b, in, pr, out, st)) ++sync_bad;
        for (int k = 0; k < 3; ++k)
            if (st[k].iters != iters[k]) {
                ++sync_bad;
                std::printf("batch problem %d: %d iterations\n", k, st[k].iters);
            }
        // after 8, 5 and 3 iterations the current iterates sit at different indices: a
        // batched step takes each problem from its own
        if (prior_ls_batch_step(b, 2, out, st)) ++sync_bad;
        if (st[0].iters != 10 || st[1].iters != 7 || st[2].iters != 5) {
            ++sync_bad;
            std::printf("batched step: %d %d %d iterations\n", st[0].iters, st[1].iters, st[2].iters);
        }
        prior_ls_batch_destroy(b);
        prior_ls_handle* h3[2] = {hb[1], hb[2]};
        if (prior_ls_batch_create(h3, 2, &b)) ++sync_bad;
        prior_ls_stats st2[2];
        for (auto& x : st2) {
            x = prior_ls_stats{};
            x.struct_size = sizeof(prior_ls_stats);
        }
        if (prior_ls_batch_step(b, 4, nullptr, st2)) ++sync_bad;
        if (st2[0].iters != 11 || st2[1].iters != 9) {
            ++sync_bad;
            std::printf("batched step: %d %d iterations\n", st2[0].iters, st2[1].iters);
        }
        prior_ls_batch_destroy(b);
        prior_ls_handle* other = nullptr;
        if (prior_ls_create(&seqs[0].rq.dims, nullptr, &other)) ++sync_bad;
        prior_ls_handle* mixed[2] = {hb[0], other};
        if (seqs[0].g.nx != kGeo[1].nx && prior_ls_batch_create(mixed, 2, &b) != PRIOR_LS_EINVAL) ++sync_bad;
        prior_ls_destroy(other);
        for (auto* h : hb) prior_ls_destroy(h);
    }
    std::printf("done: bad %d sync_bad %d\n", bad, sync_bad.load());
    return bad || sync_bad.load() || info.evicted == 0;
}
