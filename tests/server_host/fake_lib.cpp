// Fake library calls: a handle is heap memory that every call reads and writes, and a
// chunk "runs" until a deadline, so use after destroy, two callers on one handle or a
// premature read show up under the sanitizers or as failed checks.
#include <chrono>
#include <cstring>
#include <string>
#include <thread>
#include <vector>
#include "prior_ls.h"
#include "pls_runtime_api.hpp"
using Clk = std::chrono::steady_clock;
struct prior_ls_handle { prior_ls_dims d; void* stream; int busy; long work; prior_ls_params p;
                         Clk::time_point ready; int inflight; int iters; char pad[4096]; };
static thread_local std::string g_err;
namespace pls { void set_thread_error(const std::string& m) { g_err = m; } }
static void touch(prior_ls_handle* h) { for (int i = 0; i < 4096; i += 64) h->pad[i]++; }
extern "C" {
uint64_t prior_ls_plan_bytes(const prior_ls_dims* d) {
  if (!d || d->nx <= 0) return 0;
  return (uint64_t)d->nx * d->ny * d->nz * d->nt * 40 + (uint64_t)d->nc * d->nx * d->ny * d->nz * 8;
}
int prior_ls_create(const prior_ls_dims* d, void* s, prior_ls_handle** out) {
  auto* h = new prior_ls_handle(); h->d = *d; h->stream = s; std::memset(h->pad, 1, sizeof h->pad);
  *out = h; return 0;
}
void prior_ls_destroy(prior_ls_handle* h) { if (!h) return; if (h->inflight) std::abort(); std::memset(h->pad, 0, sizeof h->pad); delete h; }
const char* prior_ls_last_error(const prior_ls_handle* h) { return h ? "" : g_err.c_str(); }
}
// A batch records its handles; running it reads and writes every one of them, so a batch
// over a destroyed handle or over a handle with a chunk in flight fails the run.
struct prior_ls_batch { std::vector<prior_ls_handle*> hs; char pad[256]; };
extern "C" {
int prior_ls_batch_create(prior_ls_handle* const* hs, int32_t n, prior_ls_batch** out) {
  if (!hs || n < 1 || !out) return -1;
  auto* b = new prior_ls_batch(); b->hs.assign(hs, hs + n);
  for (auto* h : b->hs) touch(h);
  *out = b; return 0;
}
void prior_ls_batch_destroy(prior_ls_batch* b) { delete b; }
const char* prior_ls_batch_last_error(const prior_ls_batch*) { return ""; }
}
namespace pls {
int phase_load(prior_ls_handle* h, const prior_ls_inputs* in, const prior_ls_params* p) {
  if (!in->kspace || !in->mask) return -1; touch(h); h->p = *p; h->iters = 0; return 0; }
int phase_shift(prior_ls_handle* h, const void* kf, const uint8_t* mf, const prior_ls_params* p) {
  if (!kf || !mf) return -1; touch(h); h->p = *p; h->iters = 0; return 0; }
int phase_chunk_launch(prior_ls_handle* h, int remaining) {
  if (h->inflight) std::abort();
  int m = remaining < h->p.check_every ? remaining : h->p.check_every;
  h->inflight = m; h->ready = Clk::now() + std::chrono::microseconds(30 * m); touch(h); return m; }
int phase_query(prior_ls_handle* h) { touch(h); return Clk::now() >= h->ready ? 1 : 0; }
int phase_chunk_finish(prior_ls_handle* h, int m, int* conv) {
  if (Clk::now() < h->ready || h->inflight != m) std::abort();
  h->inflight = 0; h->iters += m; *conv = 0; return 0; }
int phase_outputs(prior_ls_handle* h, const prior_ls_outputs*) { h->ready = Clk::now() + std::chrono::microseconds(50); return 0; }
void phase_stats(prior_ls_handle* h, prior_ls_stats* st, int conv, double ms) { st->iters = h->iters; st->converged = conv; st->ms = ms; }
int phase_max_iter(const prior_ls_handle* h) { return h->p.max_iter; }
bool batch_compatible(const prior_ls_dims& a, const prior_ls_dims& b) {
  return a.ny == b.ny && a.nz == b.nz && a.gram_mode == b.gram_mode && a.transform == b.transform &&
         (a.nt <= 16 ? 0 : a.nt <= 32 ? 1 : 2) == (b.nt <= 16 ? 0 : b.nt <= 32 ? 1 : 2) &&
         a.wavelet_levels == b.wavelet_levels; }
int batch_run(prior_ls_batch* b, const std::vector<int>& target, std::vector<char>& conv,
              std::vector<int>& status, std::vector<Clk::time_point>& done_at) {
  const size_t n = b->hs.size();
  if (target.size() != n) std::abort();
  conv.assign(n, 0); status.assign(n, 0); done_at.assign(n, Clk::now());
  int most = 0;
  for (size_t i = 0; i < n; ++i) {
    prior_ls_handle* h = b->hs[i];
    if (h->inflight) std::abort();
    touch(h);
    most = target[i] > most ? target[i] : most;
  }
  for (int k = 0; k < most; ++k) {
    std::this_thread::sleep_for(std::chrono::microseconds(30));
    for (size_t i = 0; i < n; ++i)
      if (k < target[i]) {
        touch(b->hs[i]);
        ++b->hs[i]->iters;
        if (k + 1 == target[i]) done_at[i] = Clk::now();
      }
  }
  return 0;
}
}
