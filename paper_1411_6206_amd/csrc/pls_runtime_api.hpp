// Phases of a solve / append, for the serving dispatcher, which drives many handles from one
// host thread: it starts a window, enqueues chunks of iterations without waiting, polls their
// completion, and enqueues the outputs, so no call blocks on another sequence's GPU work.
// Every function returns a PRIOR_LS_* status unless stated otherwise; messages go to the
// handle (prior_ls_last_error).
#pragma once

#include <chrono>
#include <vector>

#include "prior_ls.h"

namespace pls {

// Loads a window (prior_ls_solve's load and step (0)); blocks for the sample counts.
int phase_load(prior_ls_handle* h, const prior_ls_inputs* in, const prior_ls_params* p);
// Slides the window by one frame (prior_ls_append's shift and warm step (0)).
int phase_shift(prior_ls_handle* h, const void* kspace_frame, const uint8_t* mask_frame,
                const prior_ls_params* p);
// Enqueues the next chunk of at most `remaining` iterations; returns its length (> 0) or a
// negative status.
int phase_chunk_launch(prior_ls_handle* h, int remaining);
// 1 when the last enqueued chunk (or output write) has completed, 0 if not yet, or a
// negative status.
int phase_query(prior_ls_handle* h);
// After completion: takes the chunk's statistics (m iterations); *converged per the tol rule.
int phase_chunk_finish(prior_ls_handle* h, int m, int* converged);
// Enqueues the output writes of the resident window.
int phase_outputs(prior_ls_handle* h, const prior_ls_outputs* out);
// Statistics of the window so far.
void phase_stats(prior_ls_handle* h, prior_ls_stats* st, int converged, double ms);
// Iterations of the window (params.max_iter of the last load / shift).
int phase_max_iter(const prior_ls_handle* h);

// Problems that can share one batch (prior_ls_batch_create accepts them together): the same
// phase-encode plane, transform and depth, Gram mode and Gram tile class (nt <= 16, 17..32 or
// 33..64; the temporal transform: one nt).  nx, nt and nc may differ.
bool batch_compatible(const prior_ls_dims& a, const prior_ls_dims& b);

// Runs the loaded windows of a batch's handles together: handle i does up to target[i]
// iterations under the parameters of its last load / shift (its own check interval and
// tolerance), after the work already queued on its stream.  Blocks until all are done.
// converged[i], status[i] (ENONFINITE) and done_at[i] (when its last chunk was seen
// complete) out; returns a status for the batch as a whole (EHIP: message in
// prior_ls_batch_last_error).
int batch_run(prior_ls_batch* b, const std::vector<int>& target, std::vector<char>& converged,
              std::vector<int>& status, std::vector<std::chrono::steady_clock::time_point>& done_at);

}  // namespace pls
