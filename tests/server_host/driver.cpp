// Drives the serving runtime on the CPU with stand-in library phases: 200 requests of six
// geometries submitted from a thread, groups of up to four of one geometry, a budget that
// forces evictions.
#include <cstdio>
#include <thread>
#include <vector>
#include <random>
#include <atomic>
#include <chrono>
#include "prior_ls.h"
int main() {
  prior_ls_server_config cfg{sizeof(cfg), 0, 4, 0};
  std::mt19937 rng(7);
  int dimsets[6][5] = {{16,16,4,5,2},{24,32,8,7,3},{32,32,1,6,1},{16,16,4,6,2},{24,32,8,5,3},{32,32,1,7,1}};
  // a budget that fits about two of the largest: forces queueing and evictions
  prior_ls_dims big{sizeof(prior_ls_dims), 24,32,8,7,3, 2,0,0,0};
  cfg.hbm_budget = (uint64_t)(prior_ls_plan_bytes(&big) * 1.6);
  prior_ls_server* s = nullptr;
  if (prior_ls_server_create(&cfg, &s)) { printf("create failed\n"); return 1; }
  const int N = 200;
  static char fakedev[1 << 20];
  std::vector<std::vector<uint8_t>> masks(N);
  std::vector<std::vector<double>> lat(N);
  std::vector<std::vector<prior_ls_stats>> st(N);
  std::vector<prior_ls_request> rq(N);
  std::vector<int64_t> tk(N, -1);
  std::atomic<int> submitted{0};
  std::thread sub([&] {
    for (int i = 0; i < N; ++i) {
      int* g = dimsets[rng() % 6];
      int na = 1 + rng() % 3;
      prior_ls_request& r = rq[i];
      r = prior_ls_request{};
      r.struct_size = sizeof(r);
      r.dims = prior_ls_dims{sizeof(prior_ls_dims), g[0], g[1], g[2], g[3], g[4], 2, 0, 0, 0};
      r.first = prior_ls_params{sizeof(prior_ls_params), 0.01, 0.01, 0, 0, 1, 8, 4, 1};
      r.next = r.first; r.next.max_iter = 6;
      r.n_append = na;
      size_t P = (size_t)g[1] * g[2];
      masks[i].assign((g[3] + na) * P, 0);
      for (size_t k = 0; k < masks[i].size(); k += 3) masks[i][k] = 1;
      r.kspace0 = fakedev; r.mask0 = masks[i].data();
      r.kspace_frames = fakedev; r.mask_frames = masks[i].data() + g[3] * P;
      r.sens = fakedev;
      lat[i].resize(na + 1); st[i].resize(na + 1);
      r.latency_ms = lat[i].data(); r.stats = st[i].data();
      int64_t t;
      int rc = prior_ls_server_submit(s, &r, &t);
      if (rc) { printf("submit %d rc %d %s\n", i, rc, prior_ls_last_error(nullptr)); std::abort(); }
      tk[i] = t;
      submitted.store(i + 1, std::memory_order_release);
      std::this_thread::sleep_for(std::chrono::microseconds(rng() % 300));
    }
  });
  int bad = 0;
  for (int i = 0; i < N; ++i) {
    while (submitted.load(std::memory_order_acquire) <= i) std::this_thread::yield();
    prior_ls_result res{}; res.struct_size = sizeof(res);
    if (prior_ls_server_wait(s, tk[i], &res)) { printf("wait failed\n"); return 1; }
    if (res.status) { ++bad; printf("req %d status %d %s\n", i, res.status, res.message); }
    for (int w = 0; w <= rq[i].n_append; ++w) {
      int want = w == 0 ? rq[i].first.max_iter : rq[i].next.max_iter;
      if (st[i][w].iters != want || !(lat[i][w] > 0)) { ++bad; printf("req %d window %d iters %d lat %g\n", i, w, st[i][w].iters, lat[i][w]); }
    }
  }
  sub.join();
  prior_ls_server_stats info{}; info.struct_size = sizeof(info);
  prior_ls_server_info(s, &info);
  printf("done: completed %lld failed %lld reused %lld evicted %lld peak_active %d peak %llu budget %llu bad %d\n",
         (long long)info.completed, (long long)info.failed, (long long)info.reused, (long long)info.evicted,
         info.peak_active, (unsigned long long)info.peak_used, (unsigned long long)info.budget, bad);
  prior_ls_server_destroy(s);
  return bad || info.peak_used > info.budget;
}
