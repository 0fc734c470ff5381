// Host runtime and C ABI of the Priori L+S library: argument validation, device state,
// set-up (sample lists, kx inverse DFT, layout permutations, step (0)), the iteration
// schedule of Algorithm 1 (captured per chunk into a hipGraph and replayed), convergence
// checks and output.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "prior_ls.h"
#include "pls_kernels.hpp"
#include "pls_runtime_api.hpp"

using pls::DcArgs;

namespace {
thread_local std::string g_create_error;
}

// Message of a failed call that has no handle (create, server calls) on this thread.
namespace pls {
void set_thread_error(const std::string& m) { g_create_error = m; }
}

namespace {

constexpr int kStatRec = 128;         // doubles per iteration record ([16, 16 + nt): sigma)
constexpr int kMatDoubles = 64 * 64;   // an nt x nt matrix (V, W) at the largest nt
constexpr int kOpFloats = 128 * 128;   // the real-expanded back-projection operand
constexpr int kMaxChunk = 1024;
constexpr int kMaxGramBlocks = 2048;  // largest Gram split the tuner tries

struct HipError {
    hipError_t e;
    std::string where;
};

#define PLS_HIP(call)                                                        \
    do {                                                                     \
        hipError_t e_ = (call);                                              \
        if (e_ != hipSuccess) throw HipError{e_, #call};                     \
    } while (0)

bool is_pow2_div(int n, int J) { return n == 1 || (n % (1 << J)) == 0; }

int check_dims(const prior_ls_dims* d, std::string& msg) {
    if (!d) {
        msg = "dims is NULL";
        return PRIOR_LS_EINVAL;
    }
    if (d->struct_size != sizeof(prior_ls_dims)) {
        msg = "dims.struct_size mismatch";
        return PRIOR_LS_EINVAL;
    }
    if (d->transform != PRIOR_LS_T_HAAR && d->transform != PRIOR_LS_T_TFFT &&
        d->transform != PRIOR_LS_T_DB4) {
        msg = "unknown transform";
        return PRIOR_LS_EINVAL;
    }
    if (d->gram_mode < PRIOR_LS_GRAM_FP64 || d->gram_mode > PRIOR_LS_GRAM_BF16X3) {
        msg = "unknown gram_mode";
        return PRIOR_LS_EINVAL;
    }
    if (d->nx < 1 || d->ny < 1 || d->nz < 1 || d->nt < 1 || d->nc < 1) {
        msg = "dimensions must be >= 1";
        return PRIOR_LS_ESHAPE;
    }
    if (d->nt > PRIOR_LS_MAX_NT) {
        msg = "nt > 64 is not supported";
        return PRIOR_LS_ESHAPE;
    }
    if (d->nc > 64) {
        msg = "nc > 64 is not supported";
        return PRIOR_LS_ESHAPE;
    }
    if (!pls::dc_supported(d->ny, d->nz)) {
        msg = "unsupported (ny, nz) phase-encode plane";
        return PRIOR_LS_ESHAPE;
    }
    if (!pls::xifft_supported(d->nx)) {
        msg = "unsupported readout length nx";
        return PRIOR_LS_ESHAPE;
    }
    const int J = d->wavelet_levels;
    if (J < 0 || J > 3) {
        msg = "wavelet_levels must be in [0, 3]";
        return PRIOR_LS_ESHAPE;
    }
    if (d->transform == PRIOR_LS_T_TFFT) {                     // J is not used
        if (d->nt > 32) {
            msg = "the temporal transform takes at most 32 frames";
            return PRIOR_LS_ESHAPE;
        }
        return PRIOR_LS_OK;
    }
    if (d->transform == PRIOR_LS_T_DB4 && !pls::db4_supported(d->nx, d->ny, d->nz)) {
        msg = "unsupported shape for the Daubechies transform";
        return PRIOR_LS_ESHAPE;
    }
    if (!is_pow2_div(d->nx, J) || !is_pow2_div(d->ny, J) || !is_pow2_div(d->nz, J)) {
        msg = "every spatial axis of size > 1 must be divisible by 2^wavelet_levels";
        return PRIOR_LS_ESHAPE;
    }
    // the sparse kernel covers (2^J)^3 blocks with z across the lanes of one wave
    if (d->nz > 1 && (d->nz % (1 << J)) != 0) {
        msg = "nz must be divisible by 2^wavelet_levels";
        return PRIOR_LS_ESHAPE;
    }
    return PRIOR_LS_OK;
}

struct Sizes {
    size_t N, I, P;
    uint64_t base_bytes;
    int gblocks, gentries, dcb, spb;
};

// Workgroups (= partial sums) of one sparse update under a tuning.
int sparse_launch_blocks(const prior_ls_dims& d, const prior_ls_tuning& t) {
    if (d.transform == PRIOR_LS_T_TFFT) return pls::sparse_tfft_blocks(d.nx * d.ny * d.nz, d.nt);
    if (d.transform == PRIOR_LS_T_DB4) return pls::sparse_db4_blocks(d.nx, d.nt);
    return pls::sparse_haar_blocks(d.wavelet_levels, d.nx, d.ny, d.nz, d.nt, t.sparse_grid);
}

// Workgroups of the sparse update at most (any tuning): the size of its partial sums.
int sparse_blocks(const prior_ls_dims& d) {
    if (d.transform == PRIOR_LS_T_TFFT) return pls::sparse_tfft_blocks(d.nx * d.ny * d.nz, d.nt);
    if (d.transform == PRIOR_LS_T_DB4) return pls::sparse_db4_blocks(d.nx, d.nt);
    const int J = d.wavelet_levels;
    const int B = 1 << J;
    const int ZW = d.nz > 1 ? B : 1;
    const int YW = 64 / ZW;
    const int nyt = (d.ny + 4 * YW - 1) / (4 * YW);
    return nyt * (d.nz / ZW) * (d.nx / B) * d.nt;
}

Sizes sizes_of(const prior_ls_dims& d) {
    Sizes s;
    s.P = (size_t)d.ny * d.nz;
    s.N = s.P * d.nx;
    s.I = s.N * d.nt;
    s.gblocks = pls::gram_blocks((int)s.N, kMaxGramBlocks);   // the largest split tuning tries
    s.gentries = pls::gram_tiles(d.nt) * 256;
    s.dcb = pls::dc_blocks(d.ny, d.nz, d.nx, d.nt);
    s.spb = sparse_blocks(d);
    uint64_t b = 0;
    b += 5 * s.I * 8;                                   // C, L[2], S[2]
    b += (uint64_t)d.nc * s.N * 8;                      // sensitivities (ones when nc == 1)
    b += 2 * s.I;                                       // weights, support of T(S)
    b += (uint64_t)2 * d.nt * s.P + 64 * 8;             // masks (two copies), sigma of L
    b += (uint64_t)d.nt * s.P * (2 + 4) + 3 * (d.nt + 1) * 4;  // sidx, plist, ns, offsets
    b += (uint64_t)(d.nx + d.ny + d.nz) * 8;            // twiddles
    b += (uint64_t)s.gblocks * s.gentries * 8 + s.gentries * 8;
    b += kOpFloats * 4 + 2 * kMatDoubles * 16 + 64 * 8;   // W operand, V and W, sigma
    if (d.transform == PRIOR_LS_T_TFFT) b += 2 * 64 * 64 * 4;
    if (d.transform == PRIOR_LS_T_DB4) b += s.I * 8;      // coefficient scratch
    b += (uint64_t)s.dcb * 32 + (uint64_t)s.spb * 8 + (uint64_t)kMaxChunk * kStatRec * 8;
    s.base_bytes = b;
    return s;
}

}  // namespace

struct prior_ls_handle {
    prior_ls_dims d{};
    hipStream_t ustream = nullptr;   // the caller's stream
    hipStream_t stream = nullptr;    // the handle's own stream (capturable)
    hipStream_t side = nullptr;      // second stream: the sparse update runs beside the
                                     // Gram / eigensolve / back-projection chain
    hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_fork = nullptr, ev_join = nullptr;
    hipEvent_t ev_bp = nullptr, ev_chg = nullptr;   // statistics iterations: the change pass
                                                    // (side stream) after the back-projection
    hipEvent_t ev_chunk = nullptr;   // end of the last enqueued chunk / output write
    int device = 0;
    Sizes sz{};
    uint64_t owned = 0;
    std::vector<void*> allocs;
    // state
    float2* C = nullptr;
    float2* L[2] = {nullptr, nullptr};
    float2* S[2] = {nullptr, nullptr};
    float2* sens = nullptr;
    float2* ones = nullptr;          // the unit coil of a single-coil problem (nc == 1)
    float *Wtf = nullptr, *Wti = nullptr;   // temporal transform: forward / inverse operands
    float2* dz = nullptr;                   // Daubechies transform: coefficient scratch
    uint8_t* w = nullptr;
    bool has_w = false, has_sens = false;
    float2* dh = nullptr;
    size_t dh_cap = 0;
    // the compact k-space is a ring of nt frame slots of slot_cap entries each; logical
    // frame t lives in slot slot_of[t] (dh_off[t] = slot_of[t] * slot_cap), so a new
    // frame replaces the oldest one in place
    size_t slot_cap = 0;
    std::vector<int> slot_of;
    uint8_t* mask_d = nullptr;       // [nt][P] masks of the window, logical frame order
    uint8_t* mask_tmp = nullptr;
    uint8_t* supp = nullptr;         // support of T(S) of the last sparse update (0 / 255)
    double* sigL = nullptr;          // singular values of the last L, by rank
    int *dh_off = nullptr, *ns = nullptr, *plist = nullptr, *line_off = nullptr;
    int16_t* sidx = nullptr;
    float2 *twx = nullptr, *twy = nullptr, *twz = nullptr;
    double *gpart = nullptr, *gred = nullptr;
    double *V = nullptr, *Wd = nullptr;
    float* Wop = nullptr;
    double* sigma_prev = nullptr;
    double *dc_part = nullptr, *sp_part = nullptr, *ch_part = nullptr;
    double* stats_d = nullptr;
    double* stats_h = nullptr;
    // op scratch (lazy)
    float2 *T1 = nullptr, *T2 = nullptr;
    double *Vop = nullptr, *Wdop = nullptr;
    float* Wopop = nullptr;
    // iteration
    int cur = 0;
    int iters = 0;
    bool loaded = false;
    prior_ls_params params{};
    prior_ls_tuning tuning{sizeof(prior_ls_tuning), 0, 0, 0, 0, 0.0};
    std::map<std::pair<int, int>, hipGraphExec_t> graphs;
    std::vector<hipGraph_t> graph_objs;
    std::string err;
    double last[kStatRec] = {0};

    template <class T>
    T* alloc(size_t bytes) {
        if (d.hbm_budget && owned + bytes > d.hbm_budget) throw std::bad_alloc();
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, bytes ? bytes : 1);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw std::bad_alloc();
        }
        allocs.push_back(p);
        owned += bytes;
        return static_cast<T*>(p);
    }
    void release(void* p, size_t bytes) {
        if (!p) return;
        auto it = std::find(allocs.begin(), allocs.end(), p);
        if (it != allocs.end()) allocs.erase(it);
        (void)hipFree(p);
        owned -= bytes;
    }
    void clear_graphs() {
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
        for (auto g : graph_objs) (void)hipGraphDestroy(g);
        graphs.clear();
        graph_objs.clear();
    }
};

namespace {

int fail(prior_ls_handle* h, int code, const std::string& m) {
    if (h) h->err = m;
    return code;
}

void upload_twiddles(float2* dst, int n, hipStream_t s) {
    std::vector<float2> tw(n);
    for (int m = 0; m < n; ++m) {
        const double ang = -2.0 * M_PI * (double)m / (double)n;
        tw[m] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
    PLS_HIP(hipMemcpyAsync(dst, tw.data(), n * sizeof(float2), hipMemcpyHostToDevice, s));
    PLS_HIP(hipStreamSynchronize(s));
}

bool is_device_ptr(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

// Step (3) with the handle's sparsifying transform.
int launch_sparse_any(const prior_ls_handle* h, const pls::SparseArgs& sa, hipStream_t s) {
    if (h->d.transform == PRIOR_LS_T_TFFT) return pls::launch_sparse_tfft(sa, s);
    if (h->d.transform == PRIOR_LS_T_DB4) {
        pls::SparseArgs a = sa;
        a.levels = h->d.wavelet_levels;
        a.Z = h->dz;
        return pls::launch_sparse_db4(a, s);
    }
    return pls::launch_sparse(h->d.wavelet_levels, sa, s);
}

// MFMA operands of the unitary temporal DFT (64 x 64 FP32, real-expanded, as the
// back-projection's): forward F[f][t] = exp(-2 pi i f t / nt) / sqrt(nt) with rows (Re f,
// Im f) and columns (Re t, Im t); inverse F^H with rows (Re t, Im t) and its columns in the
// order in which the forward product leaves its rows in the accumulator registers.
void upload_tfft_operands(prior_ls_handle* h) {
    const int nt = h->d.nt;
    const int NTP = nt <= 16 ? 16 : 32, K2 = 2 * NTP;
    std::vector<float> wf(64 * 64, 0.f), wi(64 * 64, 0.f);
    const double sc = 1.0 / std::sqrt((double)nt);
    auto expand = [&](std::vector<double>& m, double sign) {
        // m[o][k], o = (component, output index), k = (component, input index)
        for (int a = 0; a < nt; ++a)
            for (int b = 0; b < nt; ++b) {
                const double ang = sign * 2.0 * M_PI * (double)((long)a * b % nt) / nt;
                const double re = std::cos(ang) * sc, im = std::sin(ang) * sc;
                m[a * K2 + b] = re;
                m[a * K2 + NTP + b] = -im;
                m[(NTP + a) * K2 + b] = im;
                m[(NTP + a) * K2 + NTP + b] = re;
            }
    };
    std::vector<double> F(K2 * K2, 0.0), G(K2 * K2, 0.0);
    expand(F, -1.0);
    expand(G, +1.0);
    for (int o = 0; o < K2; ++o)
        for (int k = 0; k < K2; ++k) {
            wf[o * K2 + k] = (float)F[o * K2 + k];
            // column k = 4 ks + g of the inverse's operand takes forward output row
            // 16 (ks / 4) + 4 g + ks % 4
            const int ks = k / 4, g = k % 4;
            const int row = 16 * (ks / 4) + 4 * g + ks % 4;
            wi[o * K2 + k] = (float)G[o * K2 + row];
        }
    PLS_HIP(hipMemcpyAsync(h->Wtf, wf.data(), wf.size() * sizeof(float), hipMemcpyHostToDevice, h->stream));
    PLS_HIP(hipMemcpyAsync(h->Wti, wi.data(), wi.size() * sizeof(float), hipMemcpyHostToDevice, h->stream));
    PLS_HIP(hipStreamSynchronize(h->stream));
}

// One iteration of Algorithm 1 on the resident state.  Steps (1)-(2) (Gram, eigensolve,
// back-projection) run on the main stream while step (3) (sparse update) runs on the side
// stream from the end of the Gram pass on; both only read C = M - S, S and L of the
// previous iterate, and step (4) (data consistency) joins them.  ev (optional): 2 timing events around each of the 7 kernels,
// recorded on the stream the kernel runs on.
void enqueue_iteration(prior_ls_handle* h, int slot, bool stats, hipEvent_t* ev = nullptr) {
    const prior_ls_dims& d = h->d;
    const Sizes& sz = h->sz;
    // The sparse update forks off after the Gram pass (it then fills the GPU beside the
    // one-block eigensolve instead of competing with the Gram for bandwidth), or, with
    // tuning.sparse_fork = 1, at the start of the iteration.  With sparse_fork = 2 it runs
    // on the main stream after the Gram pass, so every kernel runs alone.
    const bool serial = h->tuning.sparse_fork == 2;
    hipStream_t s = h->stream, s2 = serial ? h->stream : h->side;
    const int p = h->cur, q = 1 - p;
    double* rec = h->stats_d + (size_t)slot * kStatRec;
    auto mark = [&](int k, hipStream_t st) {
        if (ev) PLS_HIP(hipEventRecord(ev[k], st));
    };
    const bool fork_first = h->tuning.sparse_fork == 1;
    if (fork_first) {
        PLS_HIP(hipEventRecord(h->ev_fork, s));
        PLS_HIP(hipStreamWaitEvent(s2, h->ev_fork, 0));
    }
    // steps (1)-(2): Gram, eigensolve, W, L_k = C W   [main stream]
    mark(0, s);
    pls::GramArgs ga{h->C, h->gpart, (int)sz.N, d.nt, 0, h->tuning.gram_blocks};
    const int gb = pls::launch_gram(d.gram_mode, ga, s);
    mark(1, s);
    if (!fork_first && !serial) {
        PLS_HIP(hipEventRecord(h->ev_fork, s));
        PLS_HIP(hipStreamWaitEvent(s2, h->ev_fork, 0));
    }
    // step (3): S_k = T^-1 soft(T(M_{k-1} - L_{k-1}))   (M = C + S)   [side stream]
    pls::SparseArgs sa{};
    sa.C = h->C;
    sa.S = h->S[p];
    sa.Lp = h->L[p];
    sa.w = h->has_w ? h->w : nullptr;
    sa.Sout = h->S[q];
    sa.supp = h->supp;
    sa.part = h->sp_part;
    sa.nx = d.nx;
    sa.ny = d.ny;
    sa.nz = d.nz;
    sa.nt = d.nt;
    sa.lambda_S = (float)h->params.lambda_S;
    mark(6, s2);
    sa.Wf = h->Wtf;
    sa.Wi = h->Wti;
    sa.max_grid = h->tuning.sparse_grid;
    const int spb = launch_sparse_any(h, sa, s2);
    mark(7, s2);
    if (!serial) PLS_HIP(hipEventRecord(h->ev_join, s2));
    mark(2, s);
    pls::launch_gram_reduce(h->gpart, gb, sz.gentries, h->gred, s);
    mark(3, s);
    pls::EigArgs ea{};
    ea.gram = h->gred;
    ea.V = h->V;
    ea.warm = 1;
    ea.Wop = h->Wop;
    ea.Wd = h->Wd;
    ea.sigma_prev = h->sigma_prev;
    ea.stat = rec;
    ea.sigL = h->sigL;
    ea.nt = d.nt;
    ea.lambda_L = h->params.lambda_L;
    ea.lambda_p = h->params.lambda_p;
    ea.relative = h->params.lambda_L_relative;
    mark(4, s);
    pls::launch_eig(ea, s);
    mark(5, s);
    pls::BpArgs ba{h->C, h->L[q], h->Wop, (int)sz.N, d.nt, h->tuning.bp_grid};
    mark(8, s);
    pls::launch_bp(ba, s);
    mark(9, s);
    // the change of the iterate for the stopping test: on the side stream once the
    // back-projection and the sparse update are done, beside the data-consistency pass (it
    // reads only the iterates, which nothing overwrites before the statistics kernel)
    if (stats && !serial) {
        PLS_HIP(hipEventRecord(h->ev_bp, s));
        PLS_HIP(hipStreamWaitEvent(s2, h->ev_bp, 0));
    }
    mark(14, s2);
    if (stats)
        pls::launch_change(pls::ChangeArgs{h->L[q], h->S[q], h->L[p], h->S[p], h->ch_part,
                                           (long)sz.I}, s2);
    mark(15, s2);
    if (stats && !serial) PLS_HIP(hipEventRecord(h->ev_chg, s2));
    // step (4): data consistency -> C = M_k - S_k   (joins the sparse update)
    if (!serial) PLS_HIP(hipStreamWaitEvent(s, h->ev_join, 0));
    DcArgs da{};
    da.L = h->L[q];
    da.S = h->S[q];
    da.C = h->C;
    da.sens = h->has_sens ? h->sens : h->ones;
    da.dh = h->dh;
    da.dh_off = h->dh_off;
    da.ns = h->ns;
    da.sidx = h->sidx;
    da.twy = h->twy;
    da.twz = h->twz;
    da.part = h->dc_part;
    da.nx = d.nx;
    da.nt = d.nt;
    da.nc = d.nc;
    da.inv_p = 1.0f / (float)sz.P;
    mark(10, s);
    const int dcb = pls::launch_dc(d.ny, d.nz, da, s);
    mark(11, s);
    // statistics are reduced only where they are read: the last iteration of a chunk
    if (stats && !serial) PLS_HIP(hipStreamWaitEvent(s, h->ev_chg, 0));
    mark(12, s);
    if (stats) {
        pls::StatsArgs st{h->dc_part, dcb, h->ch_part, pls::change_blocks((long)sz.I), h->sp_part,
                          spb, rec, (double)sz.P, h->params.lambda_S};
        pls::launch_stats(st, s);
    }
    mark(13, s);
    h->cur = q;
}

void run_chunk(prior_ls_handle* h, int n) {
    const bool graph = h->params.use_graph != 0;
    if (!graph) {
        for (int j = 0; j < n; ++j) enqueue_iteration(h, j, j == n - 1);
        PLS_HIP(hipGetLastError());
        return;
    }
    const auto key = std::make_pair(n, h->cur);
    auto it = h->graphs.find(key);
    if (it == h->graphs.end()) {
        const int cur0 = h->cur;
        hipGraph_t g = nullptr;
        PLS_HIP(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
        for (int j = 0; j < n; ++j) enqueue_iteration(h, j, j == n - 1);
        hipError_t le = hipGetLastError();
        PLS_HIP(hipStreamEndCapture(h->stream, &g));
        PLS_HIP(le);
        hipGraphExec_t ex = nullptr;
        PLS_HIP(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
        h->graph_objs.push_back(g);
        it = h->graphs.emplace(key, ex).first;
        h->cur = cur0;
    }
    PLS_HIP(hipGraphLaunch(it->second, h->stream));
    if (n % 2) h->cur = 1 - h->cur;
}

// Iterations run in chunks of at most check_every (one hipGraph replay each); after a chunk
// its last statistics record is read back for the stopping rule.
int chunk_size(const prior_ls_handle* h, int remaining) {
    const int ce = std::max(1, std::min(h->params.check_every, kMaxChunk));
    return std::min(ce, remaining);
}

// Enqueues m iterations and the read-back of their last statistics record, then records
// ev_chunk on the handle's stream.
void chunk_launch(prior_ls_handle* h, int m) {
    run_chunk(h, m);
    PLS_HIP(hipMemcpyAsync(h->stats_h, h->stats_d + (size_t)(m - 1) * kStatRec,
                           kStatRec * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    PLS_HIP(hipEventRecord(h->ev_chunk, h->stream));
}

// Once ev_chunk has completed: takes the chunk's statistics; status (ENONFINITE possible).
int chunk_finish(prior_ls_handle* h, int m, bool& converged) {
    std::memcpy(h->last, h->stats_h, sizeof(h->last));
    h->iters += m;
    if (h->last[7] != 0.0) return fail(h, PRIOR_LS_ENONFINITE, "non-finite value in the iterate");
    const double rel = h->last[2] > 0 ? std::sqrt(h->last[1] / h->last[2]) : INFINITY;
    converged = h->params.tol > 0 && rel < h->params.tol;
    return PRIOR_LS_OK;
}

// Runs n iterations in chunks; returns status (ENONFINITE possible), fills h->last.
int iterate(prior_ls_handle* h, int n, bool& converged) {
    converged = false;
    int done = 0;
    while (done < n) {
        const int m = chunk_size(h, n - done);
        chunk_launch(h, m);
        PLS_HIP(hipEventSynchronize(h->ev_chunk));
        done += m;
        const int r = chunk_finish(h, m, converged);
        if (r) return r;
        if (converged) break;
    }
    return PRIOR_LS_OK;
}

void write_outputs(prior_ls_handle* h, const prior_ls_outputs* out) {
    if (!out) return;
    const prior_ls_dims& d = h->d;
    const int p = h->cur;
    hipStream_t s = h->stream;
    if (out->L) pls::launch_unpack(h->L[p], nullptr, (float2*)out->L, d.nt, d.nx, d.ny, d.nz, s);
    if (out->S) pls::launch_unpack(h->S[p], nullptr, (float2*)out->S, d.nt, d.nx, d.ny, d.nz, s);
    if (out->X) pls::launch_unpack(h->L[p], h->S[p], (float2*)out->X, d.nt, d.nx, d.ny, d.nz, s);
    if (out->M) pls::launch_unpack(h->C, h->S[p], (float2*)out->M, d.nt, d.nx, d.ny, d.nz, s);
    PLS_HIP(hipGetLastError());
}

void fill_stats(prior_ls_handle* h, prior_ls_stats* st, bool converged, double ms) {
    if (!st) return;
    const double* r = h->last;
    st->iters = h->iters;
    st->converged = converged ? 1 : 0;
    st->nonfinite = r[7] != 0.0;
    st->sigma_count = h->d.nt;
    st->eig_sweeps = (int32_t)r[6];
    st->reserved = 0;
    st->rel_change = r[2] > 0 ? std::sqrt(r[1] / r[2]) : INFINITY;
    st->resid_norm = std::sqrt(std::max(r[0], 0.0));
    st->nuclear_norm = r[4];
    st->l1_weighted = r[3];
    st->tau_L = r[5];
    st->objective = 0.5 * r[0] + r[5] * r[4] + h->params.lambda_S * r[3];
    for (int i = 0; i < PRIOR_LS_MAX_NT; ++i) st->sigma[i] = i < h->d.nt ? r[16 + i] : 0.0;
    st->ms = ms;
}

int check_params(prior_ls_handle* h, const prior_ls_params* p) {
    if (!p) return fail(h, PRIOR_LS_EINVAL, "params is NULL");
    if (p->struct_size != sizeof(prior_ls_params)) return fail(h, PRIOR_LS_EINVAL, "params.struct_size mismatch");
    if (!(p->lambda_L >= 0) || !(p->lambda_S >= 0)) return fail(h, PRIOR_LS_EINVAL, "lambda_L and lambda_S must be >= 0");
    if (!(p->lambda_p >= 0 && p->lambda_p <= 1)) return fail(h, PRIOR_LS_EINVAL, "lambda_p must be in [0, 1]");
    if (!(p->tol >= 0)) return fail(h, PRIOR_LS_EINVAL, "tol must be >= 0");
    if (p->max_iter < 0) return fail(h, PRIOR_LS_EINVAL, "max_iter must be >= 0");
    if (p->check_every < 1) return fail(h, PRIOR_LS_EINVAL, "check_every must be >= 1");
    return PRIOR_LS_OK;
}

void set_identity_V(prior_ls_handle* h, double* V) {
    const int n = h->d.nt;
    std::vector<double> I(2 * n * n, 0.0);
    for (int i = 0; i < n; ++i) I[2 * (i * n + i)] = 1.0;
    PLS_HIP(hipMemcpyAsync(V, I.data(), I.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
    PLS_HIP(hipStreamSynchronize(h->stream));
}

DcArgs dc_args(prior_ls_handle* h, const float2* L, const float2* S, float2* C) {
    DcArgs da{};
    da.L = L;
    da.S = S;
    da.C = C;
    da.sens = h->has_sens ? h->sens : h->ones;
    da.dh = h->dh;
    da.dh_off = h->dh_off;
    da.ns = h->ns;
    da.sidx = h->sidx;
    da.twy = h->twy;
    da.twz = h->twz;
    da.part = h->dc_part;
    da.nx = h->d.nx;
    da.nt = h->d.nt;
    da.nc = h->d.nc;
    da.inv_p = 1.0f / (float)h->sz.P;
    da.blocks = h->sz.dcb;
    return da;
}

int load_problem(prior_ls_handle* h, const prior_ls_inputs* in, const prior_ls_params* p) {
    const prior_ls_dims& d = h->d;
    const Sizes& sz = h->sz;
    hipStream_t s = h->stream;
    h->clear_graphs();
    h->params = *p;
    h->loaded = false;
    // sample lists
    pls::launch_mask_scan(in->mask, d.ny, d.nz, d.nt, h->sidx, h->plist, h->ns, s);
    PLS_HIP(hipGetLastError());
    std::vector<int> ns(d.nt), off(d.nt), loff(d.nt + 1);
    PLS_HIP(hipMemcpyAsync(ns.data(), h->ns, d.nt * sizeof(int), hipMemcpyDeviceToHost, s));
    PLS_HIP(hipStreamSynchronize(s));
    int lines = 0, ns_max = 1;
    for (int t = 0; t < d.nt; ++t) {
        loff[t] = lines;
        lines += d.nc * ns[t];
        ns_max = std::max(ns_max, ns[t]);
    }
    loff[d.nt] = lines;
    const size_t slot = (size_t)d.nx * d.nc * ns_max;
    const size_t total = slot * d.nt;
    if (total > (size_t)INT32_MAX) return fail(h, PRIOR_LS_ESHAPE, "sampled data exceed 2^31 entries");
    h->slot_cap = slot;
    h->slot_of.resize(d.nt);
    for (int t = 0; t < d.nt; ++t) {
        h->slot_of[t] = t;
        off[t] = (int)(slot * t);
    }
    PLS_HIP(hipMemcpyAsync(h->mask_d, in->mask, (size_t)d.nt * sz.P, hipMemcpyDeviceToDevice, s));
    if (total > h->dh_cap || !h->dh) {
        h->release(h->dh, (h->dh_cap + 64) * sizeof(float2));
        h->dh = nullptr;
        h->dh_cap = 0;
        try {
            // +64: a clamped gather of an empty frame at the end still reads inside
            h->dh = h->alloc<float2>((total + 64) * sizeof(float2));
        } catch (const std::bad_alloc&) {
            return fail(h, PRIOR_LS_ENOMEM, "cannot allocate the compact k-space (hbm_budget or device memory)");
        }
        h->dh_cap = total;
    }
    PLS_HIP(hipMemcpyAsync(h->dh_off, off.data(), d.nt * sizeof(int), hipMemcpyHostToDevice, s));
    PLS_HIP(hipMemcpyAsync(h->line_off, loff.data(), (d.nt + 1) * sizeof(int), hipMemcpyHostToDevice, s));
    pls::XiArgs xa{};
    xa.kspace = (const float2*)in->kspace;
    xa.plist = h->plist;
    xa.line_off = h->line_off;
    xa.ns = h->ns;
    xa.dh_off = h->dh_off;
    xa.dh = h->dh;
    xa.twx = h->twx;
    xa.nx = d.nx;
    xa.nt = d.nt;
    xa.nc = d.nc;
    xa.P = (int)sz.P;
    xa.total_lines = lines;
    xa.scale = (float)(1.0 / std::sqrt((double)d.nx * (double)sz.P));
    pls::launch_xifft(d.nx, xa, s);
    // coils, weights, sigma prior
    h->has_sens = in->sens != nullptr;
    if (h->has_sens) {
        if (!h->sens) h->sens = h->alloc<float2>((size_t)d.nc * sz.N * sizeof(float2));
        pls::launch_pack((const float2*)in->sens, nullptr, h->sens, d.nc, d.nx, d.ny, d.nz, s);
    }
    h->has_w = in->prior_w != nullptr;
    if (h->has_w)
        pls::launch_pack_weights(in->prior_w, h->w, d.nt, d.nx, d.ny, d.nz,
                                 d.transform == PRIOR_LS_T_HAAR ? d.wavelet_levels : 0, s);
    std::vector<double> sp(d.nt, 0.0);
    if (p->lambda_p > 0 && in->sigma_prev) {
        // host or device memory: read once per solve, sorted on the host
        if (is_device_ptr(in->sigma_prev)) {
            PLS_HIP(hipMemcpyAsync(sp.data(), in->sigma_prev, d.nt * sizeof(double),
                                   hipMemcpyDeviceToHost, s));
            PLS_HIP(hipStreamSynchronize(s));
        } else {
            for (int i = 0; i < d.nt; ++i) sp[i] = in->sigma_prev[i];
        }
        std::sort(sp.begin(), sp.end(), [](double a, double b) { return a > b; });
    }
    PLS_HIP(hipMemcpyAsync(h->sigma_prev, sp.data(), d.nt * sizeof(double), hipMemcpyHostToDevice, s));
    set_identity_V(h, h->V);
    PLS_HIP(hipMemsetAsync(h->supp, 0, sz.I, s));
    PLS_HIP(hipMemsetAsync(h->sigL, 0, 64 * sizeof(double), s));
    // step (0)
    h->cur = 0;
    if (in->L0) {
        pls::launch_pack((const float2*)in->L0, nullptr, h->L[0], d.nt, d.nx, d.ny, d.nz, s);
        pls::launch_pack((const float2*)in->S0, nullptr, h->S[0], d.nt, d.nx, d.ny, d.nz, s);
        DcArgs da = dc_args(h, h->L[0], h->S[0], h->C);
        pls::launch_dc(d.ny, d.nz, da, s);
    } else {
        DcArgs da = dc_args(h, nullptr, nullptr, h->C);
        pls::launch_dc(d.ny, d.nz, da, s);
        PLS_HIP(hipMemsetAsync(h->S[0], 0, sz.I * sizeof(float2), s));
        PLS_HIP(hipMemcpyAsync(h->L[0], h->C, sz.I * sizeof(float2), hipMemcpyDeviceToDevice, s));
    }
    PLS_HIP(hipGetLastError());
    PLS_HIP(hipStreamSynchronize(s));
    h->iters = 0;
    std::memset(h->last, 0, sizeof(h->last));
    h->loaded = true;
    return PRIOR_LS_OK;
}

void ensure_op_scratch(prior_ls_handle* h) {
    const Sizes& sz = h->sz;
    if (!h->T1) h->T1 = h->alloc<float2>(sz.I * sizeof(float2));
    if (!h->T2) h->T2 = h->alloc<float2>(sz.I * sizeof(float2));
    if (!h->Vop) h->Vop = h->alloc<double>(2 * kMatDoubles * sizeof(double));
    if (!h->Wdop) h->Wdop = h->alloc<double>(2 * kMatDoubles * sizeof(double));
    if (!h->Wopop) h->Wopop = h->alloc<float>(kOpFloats * sizeof(float));
}

// Work of a call runs on the handle's stream, after everything already queued on the
// caller's stream; the caller's stream then waits for the handle's work.
void enter(prior_ls_handle* h) {
    PLS_HIP(hipEventRecord(h->ev_in, h->ustream));
    PLS_HIP(hipStreamWaitEvent(h->stream, h->ev_in, 0));
}
void leave(prior_ls_handle* h) {
    PLS_HIP(hipEventRecord(h->ev_out, h->stream));
    PLS_HIP(hipStreamWaitEvent(h->ustream, h->ev_out, 0));
}

template <class F>
int guarded(prior_ls_handle* h, F&& f) {
    try {
        return f();
    } catch (const HipError& e) {
        return fail(h, PRIOR_LS_EHIP, e.where + ": " + hipGetErrorString(e.e));
    } catch (const std::bad_alloc&) {
        return fail(h, PRIOR_LS_ENOMEM, "device allocation failed or hbm_budget exceeded");
    }
}

// Grows every frame slot of the compact k-space to `cap` entries, keeping the data of the
// frames in them (the buffer moves, so captured graphs are dropped).
void grow_slots(prior_ls_handle* h, size_t cap) {
    const int nt = h->d.nt;
    float2* nd = h->alloc<float2>((cap * nt + 64) * sizeof(float2));
    for (int k = 0; k < nt; ++k)
        PLS_HIP(hipMemcpyAsync(nd + k * cap, h->dh + k * h->slot_cap, h->slot_cap * sizeof(float2),
                               hipMemcpyDeviceToDevice, h->stream));
    PLS_HIP(hipStreamSynchronize(h->stream));
    h->release(h->dh, (h->dh_cap + 64) * sizeof(float2));
    h->dh = nd;
    h->dh_cap = cap * nt;
    h->slot_cap = cap;
    h->clear_graphs();
}

// The parameters an iteration graph captures by value; a change drops the graphs.
bool same_captured_params(const prior_ls_params& a, const prior_ls_params& b) {
    return a.lambda_L == b.lambda_L && a.lambda_S == b.lambda_S && a.lambda_p == b.lambda_p &&
           a.lambda_L_relative == b.lambda_L_relative && a.use_graph == b.use_graph;
}

// The new window of an append (the sliding-window recursion): masks and sample lists
// shifted, the new frame's compact k-space in the dropped frame's slot, L and S shifted as
// the warm start, the previous window's support and singular values as priors, and the
// warm start's data-consistency step.  Blocks only for the new frame's sample count.
int shift_window(prior_ls_handle* h, const void* kspace_frame, const uint8_t* mask_frame,
                 const prior_ls_params* params) {
    const prior_ls_dims& d = h->d;
    const Sizes& sz = h->sz;
    const int nt = d.nt;
    const size_t P = sz.P, N = sz.N;
    hipStream_t s = h->stream;
    // masks of the new window: frames 1..nt-1, then the new one
    if (nt > 1)
        PLS_HIP(hipMemcpyAsync(h->mask_tmp, h->mask_d + P, (nt - 1) * P, hipMemcpyDeviceToDevice, s));
    PLS_HIP(hipMemcpyAsync(h->mask_tmp + (nt - 1) * P, mask_frame, P, hipMemcpyDeviceToDevice, s));
    std::swap(h->mask_d, h->mask_tmp);
    pls::launch_mask_scan(h->mask_d, d.ny, d.nz, nt, h->sidx, h->plist, h->ns, s);
    PLS_HIP(hipGetLastError());
    int ns_new = 0;
    PLS_HIP(hipMemcpyAsync(&ns_new, h->ns + (nt - 1), sizeof(int), hipMemcpyDeviceToHost, s));
    PLS_HIP(hipStreamSynchronize(s));
    // the new frame takes the slot of the dropped one
    const size_t need = (size_t)d.nx * d.nc * ns_new;
    if (need * nt > (size_t)INT32_MAX) return fail(h, PRIOR_LS_ESHAPE, "sampled data exceed 2^31 entries");
    if (need > h->slot_cap) {
        try {
            grow_slots(h, need);
        } catch (const std::bad_alloc&) {
            return fail(h, PRIOR_LS_ENOMEM, "cannot grow the compact k-space (hbm_budget or device memory)");
        }
    }
    std::rotate(h->slot_of.begin(), h->slot_of.begin() + 1, h->slot_of.end());
    std::vector<int> off(nt);
    for (int t = 0; t < nt; ++t) off[t] = (int)(h->slot_of[t] * h->slot_cap);
    const int loff[2] = {0, d.nc * ns_new};
    PLS_HIP(hipMemcpyAsync(h->dh_off, off.data(), nt * sizeof(int), hipMemcpyHostToDevice, s));
    PLS_HIP(hipMemcpyAsync(h->line_off, loff, 2 * sizeof(int), hipMemcpyHostToDevice, s));
    // kx inverse DFT of the new frame's sampled lines into its slot
    pls::XiArgs xa{};
    xa.kspace = (const float2*)kspace_frame;
    xa.plist = h->plist + (size_t)(nt - 1) * P;
    xa.line_off = h->line_off;
    xa.ns = h->ns + (nt - 1);
    xa.dh_off = h->dh_off + (nt - 1);
    xa.dh = h->dh;
    xa.twx = h->twx;
    xa.nx = d.nx;
    xa.nt = 1;
    xa.nc = d.nc;
    xa.P = (int)P;
    xa.total_lines = loff[1];
    xa.scale = (float)(1.0 / std::sqrt((double)d.nx * (double)P));
    pls::launch_xifft(d.nx, xa, s);
    // warm start: L and S shifted by one frame, the new frame from the previous newest
    const int p = h->cur, q = 1 - p;
    const size_t fb = N * sizeof(float2);
    for (float2** A : {h->L, h->S}) {
        if (nt > 1)
            PLS_HIP(hipMemcpyAsync(A[q], A[p] + N, (nt - 1) * fb, hipMemcpyDeviceToDevice, s));
        PLS_HIP(hipMemcpyAsync(A[q] + (nt - 1) * N, A[p] + (nt - 1) * N, fb, hipMemcpyDeviceToDevice, s));
    }
    h->cur = q;
    // a-priori knowledge: support of T(S) shifted the same way, singular values of L
    if (d.transform == PRIOR_LS_T_TFFT) {
        // a coefficient is a temporal frequency of the window: the support carries over
        PLS_HIP(hipMemcpyAsync(h->w, h->supp, (size_t)nt * N, hipMemcpyDeviceToDevice, s));
    } else {
        if (nt > 1) PLS_HIP(hipMemcpyAsync(h->w, h->supp + N, (nt - 1) * N, hipMemcpyDeviceToDevice, s));
        PLS_HIP(hipMemcpyAsync(h->w + (nt - 1) * N, h->supp + (nt - 1) * N, N, hipMemcpyDeviceToDevice, s));
    }
    PLS_HIP(hipMemcpyAsync(h->sigma_prev, h->sigL, nt * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (!h->has_w || !same_captured_params(h->params, *params)) h->clear_graphs();
    h->has_w = true;
    h->params = *params;
    set_identity_V(h, h->V);
    // step (0) of the new window: one data-consistency step from Y = L + S
    DcArgs da = dc_args(h, h->L[h->cur], h->S[h->cur], h->C);
    pls::launch_dc(d.ny, d.nz, da, s);
    PLS_HIP(hipGetLastError());
    h->iters = 0;
    std::memset(h->last, 0, sizeof(h->last));
    return PRIOR_LS_OK;
}

int check_inputs(prior_ls_handle* h, const prior_ls_inputs* in, const prior_ls_params* params) {
    if (!in) return fail(h, PRIOR_LS_EINVAL, "inputs is NULL");
    const int rc = check_params(h, params);
    if (rc) return rc;
    if (!in->kspace || !in->mask) return fail(h, PRIOR_LS_EINVAL, "kspace and mask are required");
    if (h->d.nc > 1 && !in->sens) return fail(h, PRIOR_LS_EINVAL, "sens is required when nc > 1");
    if ((in->L0 == nullptr) != (in->S0 == nullptr)) return fail(h, PRIOR_LS_EINVAL, "L0 and S0: both or neither");
    if (params->lambda_p > 0 && !in->sigma_prev) return fail(h, PRIOR_LS_EINVAL, "sigma_prev is required when lambda_p > 0");
    const void* dev[] = {in->kspace, in->mask, in->sens, in->prior_w, in->L0, in->S0};
    for (const void* p : dev)
        if (p && !is_device_ptr(p)) return fail(h, PRIOR_LS_EINVAL, "input array is not device memory");
    return PRIOR_LS_OK;
}

int check_tuning(prior_ls_handle* h, const prior_ls_tuning* t) {
    if (!t || t->struct_size != sizeof(prior_ls_tuning)) return fail(h, PRIOR_LS_EINVAL, "tuning.struct_size mismatch");
    if (t->gram_blocks != 0 && (t->gram_blocks < 64 || t->gram_blocks > kMaxGramBlocks))
        return fail(h, PRIOR_LS_EINVAL, "gram_blocks must be 0 or in [64, 2048]");
    if (t->bp_grid != 0 && (t->bp_grid < 64 || t->bp_grid > 65536))
        return fail(h, PRIOR_LS_EINVAL, "bp_grid must be 0 or in [64, 65536]");
    if (t->sparse_fork < 0 || t->sparse_fork > 2) return fail(h, PRIOR_LS_EINVAL, "sparse_fork must be 0, 1 or 2");
    if (t->sparse_grid != 0 && (t->sparse_grid < 64 || t->sparse_grid > 65536))
        return fail(h, PRIOR_LS_EINVAL, "sparse_grid must be 0 or in [64, 65536]");
    return PRIOR_LS_OK;
}

// Milliseconds per iteration of one chunk of the current choice: the chunk is captured and
// run once untimed, then replayed between two events.
double time_choice(prior_ls_handle* h, const prior_ls_inputs* in, const prior_ls_params* p,
                   hipEvent_t e0, hipEvent_t e1) {
    if (load_problem(h, in, p) != PRIOR_LS_OK) return -1.0;
    const int n = std::max(1, std::min(p->check_every, kMaxChunk));
    run_chunk(h, n);
    PLS_HIP(hipEventRecord(e0, h->stream));
    run_chunk(h, n);
    PLS_HIP(hipEventRecord(e1, h->stream));
    PLS_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    PLS_HIP(hipEventElapsedTime(&ms, e0, e1));
    return (double)ms / n;
}

}  // namespace

namespace pls {

int phase_load(prior_ls_handle* h, const prior_ls_inputs* in, const prior_ls_params* p) {
    h->err.clear();
    const int rc = check_params(h, p);
    if (rc) return rc;
    return guarded(h, [&]() -> int { return load_problem(h, in, p); });
}

int phase_shift(prior_ls_handle* h, const void* kspace_frame, const uint8_t* mask_frame,
                const prior_ls_params* p) {
    h->err.clear();
    if (!h->loaded) return fail(h, PRIOR_LS_EINVAL, "append before solve");
    const int rc = check_params(h, p);
    if (rc) return rc;
    return guarded(h, [&]() -> int { return shift_window(h, kspace_frame, mask_frame, p); });
}

int phase_chunk_launch(prior_ls_handle* h, int remaining) {
    return guarded(h, [&]() -> int {
        const int m = chunk_size(h, remaining);
        chunk_launch(h, m);
        return m;
    });
}

int phase_query(prior_ls_handle* h) {
    const hipError_t e = hipEventQuery(h->ev_chunk);
    if (e == hipSuccess) return 1;
    if (e == hipErrorNotReady) return 0;
    (void)hipGetLastError();
    return fail(h, PRIOR_LS_EHIP, std::string("hipEventQuery: ") + hipGetErrorString(e));
}

int phase_chunk_finish(prior_ls_handle* h, int m, int* converged) {
    bool c = false;
    const int r = chunk_finish(h, m, c);
    *converged = c ? 1 : 0;
    return r;
}

int phase_outputs(prior_ls_handle* h, const prior_ls_outputs* out) {
    return guarded(h, [&]() -> int {
        write_outputs(h, out);
        PLS_HIP(hipEventRecord(h->ev_chunk, h->stream));
        return PRIOR_LS_OK;
    });
}

void phase_stats(prior_ls_handle* h, prior_ls_stats* st, int converged, double ms) {
    fill_stats(h, st, converged != 0, ms);
}

int phase_max_iter(const prior_ls_handle* h) { return h->params.max_iter; }

}  // namespace pls

extern "C" {

const char* prior_ls_strerror(int status) {
    switch (status) {
        case PRIOR_LS_OK: return "success";
        case PRIOR_LS_EINVAL: return "invalid argument";
        case PRIOR_LS_ESHAPE: return "unsupported shape";
        case PRIOR_LS_ENOMEM: return "out of device memory or over the HBM budget";
        case PRIOR_LS_EHIP: return "HIP runtime error";
        case PRIOR_LS_ENONFINITE: return "non-finite value in the iterate";
    }
    return "unknown status";
}

const char* prior_ls_last_error(const prior_ls_handle* h) {
    return h ? h->err.c_str() : g_create_error.c_str();
}

uint64_t prior_ls_plan_bytes(const prior_ls_dims* dims) {
    std::string m;
    if (check_dims(dims, m) != PRIOR_LS_OK) return 0;
    return sizes_of(*dims).base_bytes;
}

int prior_ls_create(const prior_ls_dims* dims, void* stream, prior_ls_handle** out) {
    if (!out) {
        g_create_error = "out is NULL";
        return PRIOR_LS_EINVAL;
    }
    *out = nullptr;
    std::string msg;
    const int rc = check_dims(dims, msg);
    if (rc != PRIOR_LS_OK) {
        g_create_error = msg;
        return rc;
    }
    const Sizes sz = sizes_of(*dims);
    if (dims->hbm_budget && sz.base_bytes > dims->hbm_budget) {
        g_create_error = "plan exceeds hbm_budget";
        return PRIOR_LS_ENOMEM;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        g_create_error = "no HIP device";
        return PRIOR_LS_EHIP;
    }
    auto* h = new prior_ls_handle();
    h->d = *dims;
    h->ustream = (hipStream_t)stream;
    h->sz = sz;
    const int r = guarded(h, [&]() -> int {
        PLS_HIP(hipGetDevice(&h->device));
        PLS_HIP(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
        PLS_HIP(hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
        PLS_HIP(hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming));
        PLS_HIP(hipEventCreateWithFlags(&h->ev_out, hipEventDisableTiming));
        PLS_HIP(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
        PLS_HIP(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
        PLS_HIP(hipEventCreateWithFlags(&h->ev_bp, hipEventDisableTiming));
        PLS_HIP(hipEventCreateWithFlags(&h->ev_chg, hipEventDisableTiming));
        PLS_HIP(hipEventCreateWithFlags(&h->ev_chunk, hipEventDisableTiming));
        const prior_ls_dims& d = h->d;
        h->C = h->alloc<float2>(sz.I * sizeof(float2));
        for (int k = 0; k < 2; ++k) {
            h->L[k] = h->alloc<float2>(sz.I * sizeof(float2));
            h->S[k] = h->alloc<float2>(sz.I * sizeof(float2));
        }
        if (d.nc > 1) h->sens = h->alloc<float2>((size_t)d.nc * sz.N * sizeof(float2));
        if (d.nc == 1) {
            h->ones = h->alloc<float2>(sz.N * sizeof(float2));
            const std::vector<float2> one(sz.N, make_float2(1.f, 0.f));
            PLS_HIP(hipMemcpyAsync(h->ones, one.data(), sz.N * sizeof(float2), hipMemcpyHostToDevice, h->stream));
            PLS_HIP(hipStreamSynchronize(h->stream));
        }
        h->w = h->alloc<uint8_t>(sz.I);
        h->supp = h->alloc<uint8_t>(sz.I);
        h->mask_d = h->alloc<uint8_t>((size_t)d.nt * sz.P);
        h->mask_tmp = h->alloc<uint8_t>((size_t)d.nt * sz.P);
        h->sigL = h->alloc<double>(64 * sizeof(double));
        h->sidx = h->alloc<int16_t>((size_t)d.nt * sz.P * sizeof(int16_t));
        h->plist = h->alloc<int>((size_t)d.nt * sz.P * sizeof(int));
        h->ns = h->alloc<int>((d.nt + 1) * sizeof(int));
        h->dh_off = h->alloc<int>((d.nt + 1) * sizeof(int));
        h->line_off = h->alloc<int>((d.nt + 1) * sizeof(int));
        h->twx = h->alloc<float2>(d.nx * sizeof(float2));
        h->twy = h->alloc<float2>(d.ny * sizeof(float2));
        h->twz = h->alloc<float2>(d.nz * sizeof(float2));
        h->gpart = h->alloc<double>((size_t)sz.gblocks * sz.gentries * sizeof(double));
        h->gred = h->alloc<double>(sz.gentries * sizeof(double));
        h->V = h->alloc<double>(2 * kMatDoubles * sizeof(double));
        h->Wd = h->alloc<double>(2 * kMatDoubles * sizeof(double));
        h->Wop = h->alloc<float>(kOpFloats * sizeof(float));
        h->sigma_prev = h->alloc<double>(64 * sizeof(double));
        h->dc_part = h->alloc<double>((size_t)sz.dcb * sizeof(double));
        h->ch_part = h->alloc<double>((size_t)pls::change_blocks((long)sz.I) * 2 * sizeof(double));
        h->sp_part = h->alloc<double>((size_t)std::max(sz.spb, 1) * sizeof(double));
        h->stats_d = h->alloc<double>((size_t)kMaxChunk * kStatRec * sizeof(double));
        if (d.transform == PRIOR_LS_T_TFFT) {
            h->Wtf = h->alloc<float>(64 * 64 * sizeof(float));
            h->Wti = h->alloc<float>(64 * 64 * sizeof(float));
        }
        if (d.transform == PRIOR_LS_T_DB4) h->dz = h->alloc<float2>(sz.I * sizeof(float2));
        PLS_HIP(hipHostMalloc((void**)&h->stats_h, kStatRec * sizeof(double), hipHostMallocDefault));
        upload_twiddles(h->twx, d.nx, h->stream);
        upload_twiddles(h->twy, d.ny, h->stream);
        upload_twiddles(h->twz, d.nz, h->stream);
        if (d.transform == PRIOR_LS_T_TFFT) upload_tfft_operands(h);
        PLS_HIP(hipMemsetAsync(h->stats_d, 0, (size_t)kMaxChunk * kStatRec * sizeof(double), h->stream));
        PLS_HIP(hipStreamSynchronize(h->stream));
        return PRIOR_LS_OK;
    });
    if (r != PRIOR_LS_OK) {
        g_create_error = h->err;
        prior_ls_destroy(h);
        return r;
    }
    *out = h;
    return PRIOR_LS_OK;
}

void prior_ls_destroy(prior_ls_handle* h) {
    if (!h) return;
    // everything queued on either stream completes before any graph, array or buffer the
    // work may still use is released
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->side) (void)hipStreamSynchronize(h->side);
    h->clear_graphs();
    for (void* p : h->allocs) (void)hipFree(p);
    if (h->stats_h) (void)hipHostFree(h->stats_h);
    if (h->ev_in) (void)hipEventDestroy(h->ev_in);
    if (h->ev_out) (void)hipEventDestroy(h->ev_out);
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    if (h->ev_bp) (void)hipEventDestroy(h->ev_bp);
    if (h->ev_chg) (void)hipEventDestroy(h->ev_chg);
    if (h->ev_chunk) (void)hipEventDestroy(h->ev_chunk);
    if (h->side) (void)hipStreamDestroy(h->side);
    if (h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

int prior_ls_solve(prior_ls_handle* h, const prior_ls_inputs* in, const prior_ls_params* params,
                   const prior_ls_outputs* out, prior_ls_stats* stats) {
    if (!h) return PRIOR_LS_EINVAL;
    h->err.clear();
    const auto t0 = std::chrono::steady_clock::now();
    int rc = check_inputs(h, in, params);
    if (rc) return rc;
    if (stats && stats->struct_size != sizeof(prior_ls_stats))
        return fail(h, PRIOR_LS_EINVAL, "stats.struct_size mismatch");
    if (out) {
        const void* o[] = {out->L, out->S, out->X, out->M};
        for (const void* p : o)
            if (p && !is_device_ptr(p)) return fail(h, PRIOR_LS_EINVAL, "output array is not device memory");
    }
    return guarded(h, [&]() -> int {
        enter(h);
        int r = load_problem(h, in, params);
        if (r) return r;
        bool conv = false;
        r = iterate(h, params->max_iter, conv);
        write_outputs(h, out);
        leave(h);
        PLS_HIP(hipStreamSynchronize(h->stream));
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        fill_stats(h, stats, conv, ms);
        return r;
    });
}

int prior_ls_set_tuning(prior_ls_handle* h, const prior_ls_tuning* t) {
    if (!h) return PRIOR_LS_EINVAL;
    h->err.clear();
    const int rc = check_tuning(h, t);
    if (rc) return rc;
    h->tuning = *t;
    h->clear_graphs();
    return PRIOR_LS_OK;
}

int prior_ls_get_tuning(const prior_ls_handle* h, prior_ls_tuning* t) {
    if (!h || !t || t->struct_size != sizeof(prior_ls_tuning)) return PRIOR_LS_EINVAL;
    *t = h->tuning;
    return PRIOR_LS_OK;
}

int prior_ls_tune(prior_ls_handle* h, const prior_ls_inputs* in, const prior_ls_params* params,
                  prior_ls_tuning* best) {
    if (!h) return PRIOR_LS_EINVAL;
    h->err.clear();
    int rc = check_inputs(h, in, params);
    if (rc) return rc;
    if (best && best->struct_size != sizeof(prior_ls_tuning))
        return fail(h, PRIOR_LS_EINVAL, "tuning.struct_size mismatch");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    rc = guarded(h, [&]() -> int {
        PLS_HIP(hipEventCreate(&e0));
        PLS_HIP(hipEventCreate(&e1));
        enter(h);
        prior_ls_params p = *params;
        p.use_graph = 1;
        prior_ls_tuning cur = h->tuning;
        h->tuning = cur;
        double best_ms = time_choice(h, in, &p, e0, e1);
        if (best_ms < 0) return fail(h, PRIOR_LS_EINVAL, "cannot load the problem");
        // one knob at a time, each from the best choice so far
        // the serial schedule (2) can win for small problems, where the second stream's
        // fork and join cost more than the overlap saves
        const int forks[] = {0, 1, 2};
        const int grams[] = {256, 512, 1024, 2048};
        const int grids[] = {1024, 2048, 4096, 8192};
        // fewer sparse-update workgroups leave more bandwidth to the chain it runs beside
        const int sgrids[] = {256, 512, 1024, 2048};
        auto trial = [&](prior_ls_tuning t) {
            h->tuning = t;
            h->clear_graphs();
            const double ms = time_choice(h, in, &p, e0, e1);
            if (ms >= 0 && ms < best_ms) {
                best_ms = ms;
                cur = t;
            }
        };
        for (int v : forks) {
            prior_ls_tuning t = cur;
            t.sparse_fork = v;
            if (v != cur.sparse_fork) trial(t);
        }
        for (int v : grams) {
            prior_ls_tuning t = cur;
            t.gram_blocks = v;
            if (v != cur.gram_blocks) trial(t);
        }
        for (int v : grids) {
            prior_ls_tuning t = cur;
            t.bp_grid = v;
            if (v != cur.bp_grid) trial(t);
        }
        if (h->d.transform == PRIOR_LS_T_HAAR)
            for (int v : sgrids) {
                prior_ls_tuning t = cur;
                t.sparse_grid = v;
                if (v != cur.sparse_grid) trial(t);
            }
        cur.ms_per_iteration = best_ms;
        h->tuning = cur;
        h->clear_graphs();
        h->params = *params;
        const int r = load_problem(h, in, params);
        leave(h);
        PLS_HIP(hipStreamSynchronize(h->stream));
        if (best) *best = cur;
        return r;
    });
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return rc;
}

int prior_ls_step(prior_ls_handle* h, int32_t n_iter, const prior_ls_outputs* out, prior_ls_stats* stats) {
    if (!h) return PRIOR_LS_EINVAL;
    h->err.clear();
    const auto t0 = std::chrono::steady_clock::now();
    if (!h->loaded) return fail(h, PRIOR_LS_EINVAL, "step before solve");
    if (n_iter < 0) return fail(h, PRIOR_LS_EINVAL, "n_iter must be >= 0");
    if (stats && stats->struct_size != sizeof(prior_ls_stats))
        return fail(h, PRIOR_LS_EINVAL, "stats.struct_size mismatch");
    if (out) {
        const void* o[] = {out->L, out->S, out->X, out->M};
        for (const void* p : o)
            if (p && !is_device_ptr(p)) return fail(h, PRIOR_LS_EINVAL, "output array is not device memory");
    }
    return guarded(h, [&]() -> int {
        enter(h);
        bool conv = false;
        const int r = iterate(h, n_iter, conv);
        write_outputs(h, out);
        leave(h);
        PLS_HIP(hipStreamSynchronize(h->stream));
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        fill_stats(h, stats, conv, ms);
        return r;
    });
}

int prior_ls_append(prior_ls_handle* h, const void* kspace_frame, const uint8_t* mask_frame,
                    const prior_ls_params* params, const prior_ls_outputs* out,
                    prior_ls_stats* stats) {
    if (!h) return PRIOR_LS_EINVAL;
    h->err.clear();
    const auto t0 = std::chrono::steady_clock::now();
    if (!h->loaded) return fail(h, PRIOR_LS_EINVAL, "append before solve");
    int rc = check_params(h, params);
    if (rc) return rc;
    if (stats && stats->struct_size != sizeof(prior_ls_stats))
        return fail(h, PRIOR_LS_EINVAL, "stats.struct_size mismatch");
    if (!kspace_frame || !mask_frame) return fail(h, PRIOR_LS_EINVAL, "kspace_frame and mask_frame are required");
    if (!is_device_ptr(kspace_frame) || !is_device_ptr(mask_frame))
        return fail(h, PRIOR_LS_EINVAL, "input array is not device memory");
    if (out) {
        const void* o[] = {out->L, out->S, out->X, out->M};
        for (const void* p : o)
            if (p && !is_device_ptr(p)) return fail(h, PRIOR_LS_EINVAL, "output array is not device memory");
    }
    return guarded(h, [&]() -> int {
        enter(h);
        int r = shift_window(h, kspace_frame, mask_frame, params);
        if (r) return r;
        bool conv = false;
        r = iterate(h, params->max_iter, conv);
        write_outputs(h, out);
        leave(h);
        PLS_HIP(hipStreamSynchronize(h->stream));
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        fill_stats(h, stats, conv, ms);
        return r;
    });
}

int prior_ls_step_timed(prior_ls_handle* h, int32_t n_iter, double* kernel_ms,
                        int32_t* kernel_launches, prior_ls_stats* stats) {
    if (!h) return PRIOR_LS_EINVAL;
    h->err.clear();
    const auto t0 = std::chrono::steady_clock::now();
    if (!h->loaded) return fail(h, PRIOR_LS_EINVAL, "step before solve");
    if (n_iter < 1 || n_iter > kMaxChunk) return fail(h, PRIOR_LS_EINVAL, "n_iter must be in [1, 1024]");
    if (!kernel_ms) return fail(h, PRIOR_LS_EINVAL, "kernel_ms is NULL");
    if (stats && stats->struct_size != sizeof(prior_ls_stats))
        return fail(h, PRIOR_LS_EINVAL, "stats.struct_size mismatch");
    constexpr int kEv = 16;
    std::vector<hipEvent_t> ev((size_t)n_iter * kEv, nullptr);
    const int r = guarded(h, [&]() -> int {
        for (auto& e : ev) PLS_HIP(hipEventCreate(&e));
        enter(h);
        for (int j = 0; j < n_iter; ++j) enqueue_iteration(h, j, j == n_iter - 1, &ev[(size_t)j * kEv]);
        PLS_HIP(hipGetLastError());
        PLS_HIP(hipMemcpyAsync(h->stats_h, h->stats_d + (size_t)(n_iter - 1) * kStatRec,
                               kStatRec * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        leave(h);
        PLS_HIP(hipStreamSynchronize(h->stream));
        std::memcpy(h->last, h->stats_h, sizeof(h->last));
        h->iters += n_iter;
        // event pair of each kernel in the ABI order gram, reduce, eig, sparse, bp, dc, stats,
        // change
        const int pair[PRIOR_LS_NKERNELS] = {0, 2, 4, 6, 8, 10, 12, 14};
        for (int k = 0; k < PRIOR_LS_NKERNELS; ++k) {
            double tot = 0.0;
            for (int j = 0; j < n_iter; ++j) {
                float ms = 0.f;
                PLS_HIP(hipEventElapsedTime(&ms, ev[(size_t)j * kEv + pair[k]],
                                            ev[(size_t)j * kEv + pair[k] + 1]));
                tot += ms;
            }
            kernel_ms[k] = tot;
            if (kernel_launches) kernel_launches[k] = k >= 6 ? 1 : n_iter;   // statistics: last iteration
        }
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        fill_stats(h, stats, false, ms);
        return h->last[7] != 0.0 ? fail(h, PRIOR_LS_ENONFINITE, "non-finite value in the iterate") : PRIOR_LS_OK;
    });
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    return r;
}

int prior_ls_op_dc(prior_ls_handle* h, const void* Y, void* M, double* resid_norm) {
    if (!h) return PRIOR_LS_EINVAL;
    h->err.clear();
    if (!h->loaded) return fail(h, PRIOR_LS_EINVAL, "no problem loaded (call solve first)");
    if (!is_device_ptr(Y) || !is_device_ptr(M)) return fail(h, PRIOR_LS_EINVAL, "Y and M must be device memory");
    return guarded(h, [&]() -> int {
        const prior_ls_dims& d = h->d;
        ensure_op_scratch(h);
        enter(h);
        hipStream_t s = h->stream;
        pls::launch_pack((const float2*)Y, nullptr, h->T1, d.nt, d.nx, d.ny, d.nz, s);
        DcArgs da = dc_args(h, h->T1, nullptr, h->T2);
        const int dcb = pls::launch_dc(d.ny, d.nz, da, s);
        double* rec = h->stats_d + (size_t)(kMaxChunk - 1) * kStatRec;
        pls::StatsArgs st{h->dc_part, dcb, nullptr, 0, h->sp_part, 0, rec, (double)h->sz.P, 0.0};
        pls::launch_stats(st, s);
        pls::launch_unpack(h->T2, nullptr, (float2*)M, d.nt, d.nx, d.ny, d.nz, s);
        PLS_HIP(hipGetLastError());
        double r0 = 0;
        PLS_HIP(hipMemcpyAsync(&r0, rec, sizeof(double), hipMemcpyDeviceToHost, s));
        leave(h);
        PLS_HIP(hipStreamSynchronize(s));
        if (resid_norm) *resid_norm = std::sqrt(std::max(r0, 0.0));
        return PRIOR_LS_OK;
    });
}

int prior_ls_op_svt(prior_ls_handle* h, const void* C, void* L, double* sigma) {
    if (!h) return PRIOR_LS_EINVAL;
    h->err.clear();
    if (!h->loaded) return fail(h, PRIOR_LS_EINVAL, "no problem loaded (call solve first)");
    if (!is_device_ptr(C) || !is_device_ptr(L)) return fail(h, PRIOR_LS_EINVAL, "C and L must be device memory");
    return guarded(h, [&]() -> int {
        const prior_ls_dims& d = h->d;
        ensure_op_scratch(h);
        enter(h);
        hipStream_t s = h->stream;
        pls::launch_pack((const float2*)C, nullptr, h->T1, d.nt, d.nx, d.ny, d.nz, s);
        pls::GramArgs ga{h->T1, h->gpart, (int)h->sz.N, d.nt, 0, h->tuning.gram_blocks};
        const int gb = pls::launch_gram(d.gram_mode, ga, s);
        pls::launch_gram_reduce(h->gpart, gb, h->sz.gentries, h->gred, s);
        set_identity_V(h, h->Vop);
        double* rec = h->stats_d + (size_t)(kMaxChunk - 1) * kStatRec;
        pls::EigArgs ea{};
        ea.gram = h->gred;
        ea.V = h->Vop;
        ea.warm = 1;
        ea.Wop = h->Wopop;
        ea.Wd = h->Wdop;
        ea.sigma_prev = h->sigma_prev;
        ea.stat = rec;
        ea.nt = d.nt;
        ea.lambda_L = h->params.lambda_L;
        ea.lambda_p = h->params.lambda_p;
        ea.relative = h->params.lambda_L_relative;
        pls::launch_eig(ea, s);
        pls::BpArgs ba{h->T1, h->T2, h->Wopop, (int)h->sz.N, d.nt, h->tuning.bp_grid};
        pls::launch_bp(ba, s);
        pls::launch_unpack(h->T2, nullptr, (float2*)L, d.nt, d.nx, d.ny, d.nz, s);
        PLS_HIP(hipGetLastError());
        double rr[kStatRec];
        PLS_HIP(hipMemcpyAsync(rr, rec, sizeof(rr), hipMemcpyDeviceToHost, s));
        leave(h);
        PLS_HIP(hipStreamSynchronize(s));
        if (sigma)
            for (int i = 0; i < d.nt; ++i) sigma[i] = rr[16 + i];
        return PRIOR_LS_OK;
    });
}

int prior_ls_op_sparse(prior_ls_handle* h, const void* Xm, const void* Lp, void* S) {
    if (!h) return PRIOR_LS_EINVAL;
    h->err.clear();
    if (!h->loaded) return fail(h, PRIOR_LS_EINVAL, "no problem loaded (call solve first)");
    if (!is_device_ptr(Xm) || !is_device_ptr(Lp) || !is_device_ptr(S))
        return fail(h, PRIOR_LS_EINVAL, "Xm, Lp and S must be device memory");
    return guarded(h, [&]() -> int {
        const prior_ls_dims& d = h->d;
        ensure_op_scratch(h);
        enter(h);
        hipStream_t s = h->stream;
        pls::launch_pack((const float2*)Xm, nullptr, h->T1, d.nt, d.nx, d.ny, d.nz, s);
        pls::launch_pack((const float2*)Lp, nullptr, h->T2, d.nt, d.nx, d.ny, d.nz, s);
        pls::SparseArgs sa{};
        sa.C = h->T1;
        sa.S = nullptr;
        sa.Lp = h->T2;
        sa.w = h->has_w ? h->w : nullptr;
        sa.Sout = h->T1;
        sa.part = h->sp_part;
        sa.nx = d.nx;
        sa.ny = d.ny;
        sa.nz = d.nz;
        sa.nt = d.nt;
        sa.lambda_S = (float)h->params.lambda_S;
        sa.Wf = h->Wtf;
        sa.Wi = h->Wti;
        launch_sparse_any(h, sa, s);
        pls::launch_unpack(h->T1, nullptr, (float2*)S, d.nt, d.nx, d.ny, d.nz, s);
        PLS_HIP(hipGetLastError());
        leave(h);
        PLS_HIP(hipStreamSynchronize(s));
        return PRIOR_LS_OK;
    });
}

}  // extern "C"

// ================================================================ batches
// A batch advances several loaded handles together: every kernel of an iteration is launched
// once for all of them (grid z = problem), each problem's blocks reading its argument block
// from device memory.  The problems share the phase-encode plane (ny, nz), the sparsifying
// transform and its depth, the Gram mode and the Gram tile class (nt <= 16, 17..32 or 33..64), which
// fix the kernel instances; nx, nt and nc may differ.  Each launch takes the largest of the
// problems' grids; a problem's blocks beyond its own grid return at once and its blocks
// stride over its work by its own grid, so it computes exactly what it computes alone.
// Problems stop on their own terms (their iteration count, or convergence checked at their
// own chunk boundaries, as when run alone); the blocks of a stopped problem return at once.

struct prior_ls_batch {
    std::vector<prior_ls_handle*> hs;
    int device = 0;
    prior_ls_dims d{};
    Sizes sz{};
    prior_ls_tuning tuning{};
    hipStream_t stream = nullptr, side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_done = nullptr, ev_h = nullptr;
    hipEvent_t ev_bp = nullptr, ev_chg = nullptr;
    char* dev = nullptr;       // argument arrays [kernel][phase][problem] and activity flags
    char* host = nullptr;      // pinned staging of the same layout
    size_t bytes = 0;
    size_t off[9] = {0};       // gram, reduce, eig, bp, sparse, dc, stats, change, active
    int grid[9] = {0};         // launch grid per kernel (as off; [8]: the Daubechies x-line
                               // passes): the largest problem's
    std::vector<int> staged_cur;   // every problem's iterate index when the arguments were staged
    std::map<std::pair<int, int>, hipGraphExec_t> graphs;
    std::vector<hipGraph_t> graph_objs;
    std::string err;
    void clear_graphs() {
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
        for (auto g : graph_objs) (void)hipGraphDestroy(g);
        graphs.clear();
        graph_objs.clear();
    }
};

namespace {

constexpr int kMaxBatch = 4096;

int bfail(prior_ls_batch* b, int code, const std::string& m) {
    if (b) b->err = m;
    return code;
}


// Argument block array of kernel k for phase `phase` (iteration j of a chunk uses phase
// j % 2).
template <class T>
T* barr(prior_ls_batch* b, char* base, int k, int phase) {
    return reinterpret_cast<T*>(base + b->off[k]) + (size_t)phase * b->hs.size();
}

// Argument blocks of every problem for both phases: phase 0 reads problem i's current
// iterate (index cur), phase 1 the other one, so problems whose iterate indices differ
// share a launch.  Written to the pinned staging area and copied to the device; every
// problem's cur is recorded in b->staged_cur.
void batch_upload_args(prior_ls_batch* b) {
    const int n = (int)b->hs.size();
    b->staged_cur.resize(n);
    for (int k = 0; k < 9; ++k) b->grid[k] = 1;
    for (int ph = 0; ph < 2; ++ph) {
        for (int i = 0; i < n; ++i) {
            prior_ls_handle* h = b->hs[i];
            const prior_ls_dims& d = h->d;
            const Sizes& sz = h->sz;
            const int p = h->cur ^ ph, q = 1 - p;
            b->staged_cur[i] = h->cur;
            const int gb = pls::gram_blocks((int)sz.N, b->tuning.gram_blocks);
            barr<pls::GramArgs>(b, b->host, 0, ph)[i] =
                pls::GramArgs{h->C, h->gpart, (int)sz.N, d.nt,
                              pls::gram_vpb((int)sz.N, b->tuning.gram_blocks), b->tuning.gram_blocks};
            barr<pls::ReduceArgs>(b, b->host, 1, ph)[i] =
                pls::ReduceArgs{h->gpart, h->gred, gb, sz.gentries};
            pls::EigArgs ea{};
            ea.gram = h->gred;
            ea.V = h->V;
            ea.warm = 1;
            ea.Wop = h->Wop;
            ea.Wd = h->Wd;
            ea.sigma_prev = h->sigma_prev;
            ea.stat = h->stats_d;            // + slot * kStatRec at launch
            ea.sigL = h->sigL;
            ea.nt = d.nt;
            ea.lambda_L = h->params.lambda_L;
            ea.lambda_p = h->params.lambda_p;
            ea.relative = h->params.lambda_L_relative;
            barr<pls::EigArgs>(b, b->host, 2, ph)[i] = ea;
            barr<pls::BpArgs>(b, b->host, 3, ph)[i] =
                pls::BpArgs{h->C, h->L[q], h->Wop, (int)sz.N, d.nt, b->tuning.bp_grid};
            pls::SparseArgs sa{};
            sa.C = h->C;
            sa.S = h->S[p];
            sa.Lp = h->L[p];
            sa.w = h->has_w ? h->w : nullptr;
            sa.Sout = h->S[q];
            sa.supp = h->supp;
            sa.part = h->sp_part;
            sa.nx = d.nx;
            sa.ny = d.ny;
            sa.nz = d.nz;
            sa.nt = d.nt;
            sa.lambda_S = (float)h->params.lambda_S;
            sa.Wf = h->Wtf;
            sa.Wi = h->Wti;
            sa.max_grid = b->tuning.sparse_grid;
            sa.blocks = sparse_launch_blocks(d, b->tuning);
            sa.levels = d.wavelet_levels;
            sa.Z = h->dz;
            barr<pls::SparseArgs>(b, b->host, 4, ph)[i] = sa;
            barr<DcArgs>(b, b->host, 5, ph)[i] = dc_args(h, h->L[q], h->S[q], h->C);
            const int chb = pls::change_blocks((long)sz.I);
            barr<pls::StatsArgs>(b, b->host, 6, ph)[i] =
                pls::StatsArgs{h->dc_part, sz.dcb, h->ch_part, chb, h->sp_part, sa.blocks,
                               h->stats_d, (double)sz.P, h->params.lambda_S};
            barr<pls::ChangeArgs>(b, b->host, 7, ph)[i] =
                pls::ChangeArgs{h->L[q], h->S[q], h->L[p], h->S[p], h->ch_part, (long)sz.I, chb};
            // launch grids: the largest problem's (per kernel, as the offsets)
            const int own[9] = {gb, 0, 1, pls::bp_blocks((int)sz.N, b->tuning.bp_grid), sa.blocks,
                                sz.dcb, 1, chb,
                                d.transform == PRIOR_LS_T_DB4
                                    ? pls::sparse_db4_line_blocks(d.ny, d.nz, d.nt) : 0};
            for (int k = 0; k < 9; ++k) b->grid[k] = std::max(b->grid[k], own[k]);
        }
    }
    PLS_HIP(hipMemcpyAsync(b->dev, b->host, b->off[8], hipMemcpyHostToDevice, b->stream));
    PLS_HIP(hipStreamSynchronize(b->stream));
}

// One iteration of every active problem (the schedule of enqueue_iteration, batched),
// reading the argument blocks of phase p.
void enqueue_batch_iteration(prior_ls_batch* b, int slot, bool stats, int p) {
    const prior_ls_dims& d = b->d;
    const int n = (int)b->hs.size();
    const bool serial = b->tuning.sparse_fork == 2;
    hipStream_t s = b->stream, s2 = serial ? b->stream : b->side;
    const int* act = reinterpret_cast<const int*>(b->dev + b->off[8]);
    const long rec = (long)slot * kStatRec;
    const bool fork_first = b->tuning.sparse_fork == 1;
    if (fork_first) {
        PLS_HIP(hipEventRecord(b->ev_fork, s));
        PLS_HIP(hipStreamWaitEvent(s2, b->ev_fork, 0));
    }
    const pls::Batched<pls::GramArgs> bg{n, barr<pls::GramArgs>(b, b->dev, 0, p), act, 0, b->grid[0]};
    pls::launch_gram_batched(d.gram_mode, barr<pls::GramArgs>(b, b->host, 0, p)[0], &bg, s);
    if (!fork_first && !serial) {
        PLS_HIP(hipEventRecord(b->ev_fork, s));
        PLS_HIP(hipStreamWaitEvent(s2, b->ev_fork, 0));
    }
    const pls::Batched<pls::SparseArgs> bs{n, barr<pls::SparseArgs>(b, b->dev, 4, p), act, 0,
                                           b->grid[4], b->grid[8]};
    const pls::SparseArgs& sa0 = barr<pls::SparseArgs>(b, b->host, 4, p)[0];
    if (d.transform == PRIOR_LS_T_TFFT) pls::launch_sparse_tfft_batched(sa0, &bs, s2);
    else if (d.transform == PRIOR_LS_T_DB4) pls::launch_sparse_db4_batched(sa0, &bs, s2);
    else pls::launch_sparse_batched(d.wavelet_levels, sa0, &bs, s2);
    if (!serial) PLS_HIP(hipEventRecord(b->ev_join, s2));
    const pls::Batched<pls::ReduceArgs> br{n, barr<pls::ReduceArgs>(b, b->dev, 1, p), act, 0, 0};
    pls::launch_gram_reduce_batched(barr<pls::ReduceArgs>(b, b->host, 1, p)[0], &br, s);
    const pls::Batched<pls::EigArgs> be{n, barr<pls::EigArgs>(b, b->dev, 2, p), act, rec, 0};
    pls::launch_eig_batched(barr<pls::EigArgs>(b, b->host, 2, p)[0], &be, s);
    const pls::Batched<pls::BpArgs> bb{n, barr<pls::BpArgs>(b, b->dev, 3, p), act, 0, b->grid[3]};
    pls::launch_bp_batched(barr<pls::BpArgs>(b, b->host, 3, p)[0], &bb, s);
    // the change of the iterate beside the data-consistency pass (as enqueue_iteration)
    if (stats) {
        if (!serial) {
            PLS_HIP(hipEventRecord(b->ev_bp, s));
            PLS_HIP(hipStreamWaitEvent(s2, b->ev_bp, 0));
        }
        const pls::Batched<pls::ChangeArgs> bc{n, barr<pls::ChangeArgs>(b, b->dev, 7, p), act, 0, b->grid[7]};
        pls::launch_change_batched(barr<pls::ChangeArgs>(b, b->host, 7, p)[0], &bc, s2);
        if (!serial) PLS_HIP(hipEventRecord(b->ev_chg, s2));
    }
    if (!serial) PLS_HIP(hipStreamWaitEvent(s, b->ev_join, 0));
    const pls::Batched<DcArgs> bd{n, barr<DcArgs>(b, b->dev, 5, p), act, 0, b->grid[5]};
    pls::launch_dc_batched(d.ny, d.nz, barr<DcArgs>(b, b->host, 5, p)[0], &bd, s);
    if (stats) {
        if (!serial) PLS_HIP(hipStreamWaitEvent(s, b->ev_chg, 0));
        const pls::Batched<pls::StatsArgs> bt{n, barr<pls::StatsArgs>(b, b->dev, 6, p), act, rec, 0};
        pls::launch_stats_batched(barr<pls::StatsArgs>(b, b->host, 6, p)[0], &bt, s);
    }
}

// m iterations (phases 0, 1, 0, ...), captured into a graph per m when use_graph.
void run_batch_chunk(prior_ls_batch* b, int m, bool graph) {
    if (!graph) {
        for (int j = 0; j < m; ++j) enqueue_batch_iteration(b, j, j == m - 1, j & 1);
        PLS_HIP(hipGetLastError());
        return;
    }
    const auto key = std::make_pair(m, 0);
    auto it = b->graphs.find(key);
    if (it == b->graphs.end()) {
        hipGraph_t g = nullptr;
        PLS_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        for (int j = 0; j < m; ++j) enqueue_batch_iteration(b, j, j == m - 1, j & 1);
        hipError_t le = hipGetLastError();
        PLS_HIP(hipStreamEndCapture(b->stream, &g));
        PLS_HIP(le);
        hipGraphExec_t ex = nullptr;
        PLS_HIP(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
        b->graph_objs.push_back(g);
        it = b->graphs.emplace(key, ex).first;
    }
    PLS_HIP(hipGraphLaunch(it->second, b->stream));
}

// Advances problem i by up to target[i] iterations, stopping it early on convergence (tested
// where it would be alone: after every check_every iterations of its own and after its last)
// or on a non-finite iterate.  The handles' streams must have reached the batch (their work
// before this call is ordered by the caller).  conv[i], status[i] out; done_at (optional)
// receives the host time at which problem i's last chunk was seen complete.
void batch_iterate(prior_ls_batch* b, const std::vector<int>& target, std::vector<char>& conv,
                   std::vector<int>& status,
                   std::vector<std::chrono::steady_clock::time_point>* done_at = nullptr) {
    const int n = (int)b->hs.size();
    std::vector<int> done(n, 0);
    int* act = reinterpret_cast<int*>(b->host + b->off[8]);
    int* act_d = reinterpret_cast<int*>(b->dev + b->off[8]);
    conv.assign(n, 0);
    status.assign(n, PRIOR_LS_OK);
    for (int i = 0; i < n; ++i) act[i] = target[i] > 0 ? 1 : 0;
    if (done_at) done_at->assign(n, std::chrono::steady_clock::now());
    const bool graph = b->hs[0]->params.use_graph != 0;
    for (;;) {
        int m = kMaxChunk;
        bool any = false, restage = b->staged_cur.size() != (size_t)n;
        for (int i = 0; i < n; ++i) {
            if (!act[i]) continue;
            const prior_ls_handle* h = b->hs[i];
            const int ce = std::max(1, std::min(h->params.check_every, kMaxChunk));
            m = std::min(m, std::min(ce - done[i] % ce, target[i] - done[i]));
            any = true;
            if (!restage && b->staged_cur[i] != h->cur) restage = true;
        }
        if (!any) break;
        // phase 0 must read every active problem's current iterate
        if (restage) batch_upload_args(b);
        PLS_HIP(hipMemcpyAsync(act_d, act, n * sizeof(int), hipMemcpyHostToDevice, b->stream));
        run_batch_chunk(b, m, graph);
        for (int i = 0; i < n; ++i) {
            if (!act[i]) continue;
            prior_ls_handle* h = b->hs[i];
            PLS_HIP(hipMemcpyAsync(h->stats_h, h->stats_d + (size_t)(m - 1) * kStatRec,
                                   kStatRec * sizeof(double), hipMemcpyDeviceToHost, b->stream));
        }
        PLS_HIP(hipEventRecord(b->ev_done, b->stream));
        PLS_HIP(hipEventSynchronize(b->ev_done));
        for (int i = 0; i < n; ++i) {
            if (!act[i]) continue;
            prior_ls_handle* h = b->hs[i];
            const int ce = std::max(1, std::min(h->params.check_every, kMaxChunk));
            done[i] += m;
            h->iters += m;
            if (m % 2) h->cur = 1 - h->cur;
            if (done_at) (*done_at)[i] = std::chrono::steady_clock::now();
            std::memcpy(h->last, h->stats_h, sizeof(h->last));
            if (h->last[7] != 0.0) {
                status[i] = fail(h, PRIOR_LS_ENONFINITE, "non-finite value in the iterate");
                act[i] = 0;
                continue;
            }
            if (done[i] % ce == 0 || done[i] == target[i]) {
                const double rel = h->last[2] > 0 ? std::sqrt(h->last[1] / h->last[2]) : INFINITY;
                if (h->params.tol > 0 && rel < h->params.tol) {
                    conv[i] = 1;
                    act[i] = 0;
                }
            }
            if (done[i] >= target[i]) act[i] = 0;
        }
    }
}

// The batch stream waits for the work queued so far on every handle's stream.
void batch_join_handles(prior_ls_batch* b) {
    for (prior_ls_handle* h : b->hs) {
        PLS_HIP(hipEventRecord(b->ev_h, h->stream));
        PLS_HIP(hipStreamWaitEvent(b->stream, b->ev_h, 0));
    }
}

// Outputs and statistics of every problem on its own stream after the batch's work.
void batch_finish(prior_ls_batch* b, const prior_ls_outputs* out, prior_ls_stats* stats,
                  const std::vector<char>& conv, double ms) {
    PLS_HIP(hipEventRecord(b->ev_done, b->stream));
    for (size_t i = 0; i < b->hs.size(); ++i) {
        prior_ls_handle* h = b->hs[i];
        PLS_HIP(hipStreamWaitEvent(h->stream, b->ev_done, 0));
        write_outputs(h, out ? &out[i] : nullptr);
        leave(h);
    }
    for (size_t i = 0; i < b->hs.size(); ++i) {
        prior_ls_handle* h = b->hs[i];
        PLS_HIP(hipStreamSynchronize(h->stream));
        fill_stats(h, stats ? &stats[i] : nullptr, conv[i] != 0, ms);
    }
}

template <class F>
int bguarded(prior_ls_batch* b, F&& f) {
    try {
        return f();
    } catch (const HipError& e) {
        return bfail(b, PRIOR_LS_EHIP, e.where + ": " + hipGetErrorString(e.e));
    } catch (const std::bad_alloc&) {
        return bfail(b, PRIOR_LS_ENOMEM, "host or device allocation failed");
    }
}

int batch_check_io(prior_ls_batch* b, const prior_ls_outputs* out, prior_ls_stats* stats) {
    for (size_t i = 0; i < b->hs.size(); ++i) {
        if (stats && stats[i].struct_size != sizeof(prior_ls_stats))
            return bfail(b, PRIOR_LS_EINVAL, "stats[" + std::to_string(i) + "].struct_size mismatch");
        if (out) {
            const void* o[] = {out[i].L, out[i].S, out[i].X, out[i].M};
            for (const void* q : o)
                if (q && !is_device_ptr(q))
                    return bfail(b, PRIOR_LS_EINVAL, "outputs[" + std::to_string(i) + "] is not device memory");
        }
    }
    return PRIOR_LS_OK;
}

int first_status(const std::vector<int>& st) {
    for (int s : st)
        if (s) return s;
    return PRIOR_LS_OK;
}

}  // namespace

namespace pls {

// Problems that can share a batch's launches: the same kernel instances (plane shape,
// transform and depth, Gram mode and tile class; the temporal transform's instance depends on
// nt itself).  nx, nt and nc may differ.
bool batch_compatible(const prior_ls_dims& a, const prior_ls_dims& b) {
    if (a.ny != b.ny || a.nz != b.nz || a.gram_mode != b.gram_mode || a.transform != b.transform)
        return false;
    auto tile_class = [](int nt) { return nt <= 16 ? 0 : (nt <= 32 ? 1 : 2); };
    if (tile_class(a.nt) != tile_class(b.nt)) return false;
    if (a.transform == PRIOR_LS_T_TFFT) return a.nt == b.nt;
    return a.wavelet_levels == b.wavelet_levels;
}

int batch_run(prior_ls_batch* b, const std::vector<int>& target, std::vector<char>& converged,
              std::vector<int>& status, std::vector<std::chrono::steady_clock::time_point>& done_at) {
    if (!b || target.size() != b->hs.size()) return bfail(b, PRIOR_LS_EINVAL, "one target per problem");
    b->err.clear();
    return bguarded(b, [&]() -> int {
        PLS_HIP(hipSetDevice(b->device));
        batch_upload_args(b);        // loads and shifts may have moved arrays or changed lambdas
        batch_join_handles(b);
        batch_iterate(b, target, converged, status, &done_at);
        return PRIOR_LS_OK;
    });
}

}  // namespace pls

extern "C" {

int prior_ls_batch_create(prior_ls_handle* const* handles, int32_t count, prior_ls_batch** out) {
    if (!out) return PRIOR_LS_EINVAL;
    *out = nullptr;
    if (!handles || count < 1 || count > kMaxBatch) {
        pls::set_thread_error("handles is NULL or count outside [1, 4096]");
        return PRIOR_LS_EINVAL;
    }
    for (int i = 0; i < count; ++i) {
        if (!handles[i]) {
            pls::set_thread_error("handles[" + std::to_string(i) + "] is NULL");
            return PRIOR_LS_EINVAL;
        }
        for (int j = 0; j < i; ++j)
            if (handles[j] == handles[i]) {
                pls::set_thread_error("a handle appears twice in the batch");
                return PRIOR_LS_EINVAL;
            }
        if (!pls::batch_compatible(handles[i]->d, handles[0]->d) || handles[i]->device != handles[0]->device) {
            pls::set_thread_error("the handles of a batch need one phase-encode plane (ny, nz), "
                                  "transform and depth, Gram mode, Gram tile class (nt <= 16, "
                                  "17..32 or 33..64; the temporal transform: one nt) and device");
            return PRIOR_LS_EINVAL;
        }
    }
    auto* b = new (std::nothrow) prior_ls_batch();
    if (!b) return PRIOR_LS_ENOMEM;
    b->hs.assign(handles, handles + count);
    b->d = handles[0]->d;
    b->sz = handles[0]->sz;
    b->device = handles[0]->device;
    b->tuning = handles[0]->tuning;
    const int rc = bguarded(b, [&]() -> int {
        PLS_HIP(hipSetDevice(b->device));
        PLS_HIP(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
        PLS_HIP(hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking));
        PLS_HIP(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
        PLS_HIP(hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming));
        PLS_HIP(hipEventCreateWithFlags(&b->ev_done, hipEventDisableTiming));
        PLS_HIP(hipEventCreateWithFlags(&b->ev_h, hipEventDisableTiming));
        PLS_HIP(hipEventCreateWithFlags(&b->ev_bp, hipEventDisableTiming));
        PLS_HIP(hipEventCreateWithFlags(&b->ev_chg, hipEventDisableTiming));
        const size_t sizes[8] = {sizeof(pls::GramArgs), sizeof(pls::ReduceArgs), sizeof(pls::EigArgs),
                                 sizeof(pls::BpArgs), sizeof(pls::SparseArgs), sizeof(DcArgs),
                                 sizeof(pls::StatsArgs), sizeof(pls::ChangeArgs)};
        size_t o = 0;
        for (int k = 0; k < 8; ++k) {
            b->off[k] = o;
            o += (2 * (size_t)count * sizes[k] + 255) / 256 * 256;
        }
        b->off[8] = o;
        b->bytes = o + ((size_t)count * sizeof(int) + 255) / 256 * 256;
        void* dp = nullptr;
        PLS_HIP(hipMalloc(&dp, b->bytes));
        b->dev = static_cast<char*>(dp);
        void* hp = nullptr;
        PLS_HIP(hipHostMalloc(&hp, b->bytes, hipHostMallocDefault));
        b->host = static_cast<char*>(hp);
        std::memset(b->host, 0, b->bytes);
        return PRIOR_LS_OK;
    });
    if (rc) {
        pls::set_thread_error(b->err);
        prior_ls_batch_destroy(b);
        return rc;
    }
    *out = b;
    return PRIOR_LS_OK;
}

void prior_ls_batch_destroy(prior_ls_batch* b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->side) (void)hipStreamSynchronize(b->side);
    b->clear_graphs();
    if (b->dev) (void)hipFree(b->dev);
    if (b->host) (void)hipHostFree(b->host);
    hipEvent_t evs[] = {b->ev_fork, b->ev_join, b->ev_done, b->ev_h, b->ev_bp, b->ev_chg};
    for (hipEvent_t e : evs)
        if (e) (void)hipEventDestroy(e);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    if (b->side) (void)hipStreamDestroy(b->side);
    delete b;
}

const char* prior_ls_batch_last_error(const prior_ls_batch* b) {
    return b ? b->err.c_str() : "";
}

int prior_ls_batch_solve(prior_ls_batch* b, const prior_ls_inputs* in, const prior_ls_params* params,
                         const prior_ls_outputs* out, prior_ls_stats* stats) {
    if (!b) return PRIOR_LS_EINVAL;
    b->err.clear();
    if (!in || !params) return bfail(b, PRIOR_LS_EINVAL, "inputs and params are required");
    const auto t0 = std::chrono::steady_clock::now();
    const int n = (int)b->hs.size();
    for (int i = 0; i < n; ++i) {
        prior_ls_handle* h = b->hs[i];
        h->err.clear();
        const int rc = check_inputs(h, &in[i], &params[i]);
        if (rc) return bfail(b, rc, "problem " + std::to_string(i) + ": " + h->err);
    }
    int rc = batch_check_io(b, out, stats);
    if (rc) return rc;
    return bguarded(b, [&]() -> int {
        std::vector<int> target(n);
        for (int i = 0; i < n; ++i) {
            prior_ls_handle* h = b->hs[i];
            enter(h);
            const int r = load_problem(h, &in[i], &params[i]);
            if (r) return bfail(b, r, "problem " + std::to_string(i) + ": " + h->err);
            target[i] = params[i].max_iter;
        }
        PLS_HIP(hipSetDevice(b->device));
        batch_upload_args(b);
        batch_join_handles(b);
        std::vector<char> conv;
        std::vector<int> st;
        batch_iterate(b, target, conv, st);
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        batch_finish(b, out, stats, conv, ms);
        const int r = first_status(st);
        if (r) b->err = "a problem of the batch reached a non-finite iterate";
        return r;
    });
}

int prior_ls_batch_step(prior_ls_batch* b, int32_t n_iter, const prior_ls_outputs* out,
                        prior_ls_stats* stats) {
    if (!b) return PRIOR_LS_EINVAL;
    b->err.clear();
    if (n_iter < 0) return bfail(b, PRIOR_LS_EINVAL, "n_iter must be >= 0");
    const auto t0 = std::chrono::steady_clock::now();
    const int n = (int)b->hs.size();
    for (int i = 0; i < n; ++i) {
        const prior_ls_handle* h = b->hs[i];
        if (!h->loaded) return bfail(b, PRIOR_LS_EINVAL, "problem " + std::to_string(i) + " is not loaded");
    }
    int rc = batch_check_io(b, out, stats);
    if (rc) return rc;
    return bguarded(b, [&]() -> int {
        for (prior_ls_handle* h : b->hs) enter(h);
        PLS_HIP(hipSetDevice(b->device));
        batch_upload_args(b);
        batch_join_handles(b);
        std::vector<char> conv;
        std::vector<int> st;
        batch_iterate(b, std::vector<int>(n, n_iter), conv, st);
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        batch_finish(b, out, stats, conv, ms);
        const int r = first_status(st);
        if (r) b->err = "a problem of the batch reached a non-finite iterate";
        return r;
    });
}

}  // extern "C"
