// Stand-ins of the library's kernel launchers for the CPU build of its host code: each
// enqueues, on the launch stream, work that reads and writes the arrays the kernel would,
// at the extents its arguments imply (so a wrong size or a buffer freed too early is caught
// by the sanitizers), and takes some time (so streams and sequences overlap).  The sample
// lists and the compact k-space use the kernels' own index arithmetic.
#include <chrono>
#include <cstring>
#include <thread>

#include "pls_kernels.hpp"

namespace pls {
namespace {
void work_us(int us) { std::this_thread::sleep_for(std::chrono::microseconds(us)); }
template <class T>
void touch(T* p, size_t n) {
    if (!p || !n) return;
    volatile char a = *(volatile char*)p;
    volatile char b = *((volatile char*)(p + n) - 1);
    (void)a;
    (void)b;
    std::memset((void*)p, 0, sizeof(T));
    std::memset((void*)(p + n - 1), 0, sizeof(T));
}
template <class T>
void look(const T* p, size_t n) {
    if (!p || !n) return;
    volatile char a = *(const volatile char*)p;
    volatile char b = *((const volatile char*)(p + n) - 1);
    (void)a;
    (void)b;
}
}  // namespace

bool dc_supported(int ny, int nz) { return ny >= 16 && ny <= 256 && nz >= 1 && nz <= 32; }
bool xifft_supported(int nx) { return nx >= 16 && nx <= 256; }
int dc_blocks(int ny, int nz, int nx, int nt) { return nx * nt; }
int gram_tiles(int nt) { return nt <= 16 ? 3 : 10; }
int gram_vpb(int N, int target) {
    const int t = target > 0 ? target : 512;
    const int vpb = (N + t - 1) / t;
    return (vpb + 127) / 128 * 128;
}
int gram_blocks(int N, int target) {
    const int vpb = gram_vpb(N, target);
    return (N + vpb - 1) / vpb;
}

int launch_dc(int ny, int nz, const DcArgs& a, hipStream_t s) {
    DcArgs c = a;
    fh_stream(s)->push([c, ny, nz] {
        const size_t P = (size_t)ny * nz, I = P * c.nx * c.nt;
        look(c.L, c.L ? I : 0);
        look(c.S, c.S ? I : 0);
        look(c.sens, c.sens ? (size_t)c.nc * c.nx * P : 0);
        for (int t = 0; t < c.nt; ++t) {
            look(c.sidx + t * P, P);
            const size_t n = (size_t)c.nx * c.nc * c.ns[t];
            look(c.dh + c.dh_off[t], n ? n : 1);
        }
        touch(c.C, I);
        touch(c.part, (size_t)c.nx * c.nt);
        work_us(60);
    });
    return c.nx * c.nt;
}

bool launch_xifft(int nx, const XiArgs& a, hipStream_t s) {
    XiArgs c = a;
    fh_stream(s)->push([c, nx] {
        for (int line = 0; line < c.total_lines; ++line) {
            int t = 0;
            while (line >= c.line_off[t + 1]) ++t;
            const int rem = line - c.line_off[t];
            const int coil = rem / c.ns[t], smp = rem % c.ns[t];
            const int pos = c.plist[(size_t)t * c.P + smp];
            for (int x = 0; x < nx; ++x) {
                const float2 v = c.kspace[((size_t)(coil * c.nt + t) * c.P + pos) * nx + x];
                c.dh[c.dh_off[t] + ((size_t)x * c.nc + coil) * c.ns[t] + smp] = v;
            }
        }
        work_us(30);
    });
    return true;
}

void launch_mask_scan(const uint8_t* mask, int ny, int nz, int nt, int16_t* sidx, int* plist,
                      int* ns, hipStream_t s) {
    fh_stream(s)->push([=] {
        const int P = ny * nz;
        for (int t = 0; t < nt; ++t) {
            int k = 0;
            for (int i = 0; i < P; ++i) {
                if (mask[(size_t)t * P + i]) {
                    sidx[(size_t)t * P + i] = (int16_t)k;
                    plist[(size_t)t * P + k] = i;
                    ++k;
                } else {
                    sidx[(size_t)t * P + i] = -1;
                }
            }
            ns[t] = k;
        }
    });
}

void launch_pack(const float2* in, const float2* in2, float2* out, int F, int nx, int ny, int nz,
                 hipStream_t s) {
    fh_stream(s)->push([=] {
        const size_t n = (size_t)F * nx * ny * nz;
        look(in, n);
        look(in2, in2 ? n : 0);
        touch(out, n);
        work_us(10);
    });
}
void launch_unpack(const float2* a, const float2* b, float2* out, int F, int nx, int ny, int nz,
                   hipStream_t s) {
    launch_pack(a, b, out, F, nx, ny, nz, s);
}
void launch_pack_weights(const uint8_t* in, uint8_t* out, int nt, int nx, int ny, int nz, int J,
                         hipStream_t s) {
    fh_stream(s)->push([=] {
        const size_t n = (size_t)nt * nx * ny * nz;
        look(in, n);
        touch(out, n);
    });
}
void launch_add(const float2* a, const float2* b, float2* out, size_t n, hipStream_t s) {
    fh_stream(s)->push([=] {
        look(a, n);
        look(b, n);
        touch(out, n);
    });
}
int launch_gram(int mode, const GramArgs& a, hipStream_t s) {
    GramArgs c = a;
    const int gb = gram_blocks(c.N, c.target_blocks);
    fh_stream(s)->push([c, gb] {
        look(c.C, (size_t)c.N * c.nt);
        touch(c.part, (size_t)gb * gram_tiles(c.nt) * 256);
        work_us(20);
    });
    return gb;
}
void launch_gram_reduce(const double* part, int blocks, int entries, double* out, hipStream_t s) {
    fh_stream(s)->push([=] {
        look(part, (size_t)blocks * entries);
        touch(out, (size_t)entries);
    });
}
void launch_eig(const EigArgs& a, hipStream_t s) {
    EigArgs c = a;
    fh_stream(s)->push([c] {
        touch(c.V, (size_t)2 * c.nt * c.nt);
        touch(c.Wd, (size_t)2 * c.nt * c.nt);
        look(c.sigma_prev, (size_t)c.nt);
        if (c.sigL) touch(c.sigL, (size_t)c.nt);
        c.stat[4] = c.stat[5] = c.stat[6] = 1.0;
        work_us(30);
    });
}
int bp_blocks(int N, int max_grid) {
    const int tiles = (N + 63) / 64, cap = max_grid > 0 ? max_grid : 2048;
    return tiles < cap ? tiles : cap;
}
void launch_bp(const BpArgs& a, hipStream_t s) {
    BpArgs c = a;
    fh_stream(s)->push([c] {
        look(c.C, (size_t)c.N * c.nt);
        touch(c.L, (size_t)c.N * c.nt);
        work_us(20);
    });
}
int sparse_haar_blocks(int levels, int nx, int ny, int nz, int nt, int max_grid) {
    const int B = 1 << levels, ZW = nz > 1 ? B : 1, YW = 64 / ZW;
    const int items = ((ny + 4 * YW - 1) / (4 * YW)) * (nz / ZW) * (nx / B) * nt;
    return (max_grid > 0 && max_grid < items) ? max_grid : items;
}
int launch_sparse(int levels, const SparseArgs& a, hipStream_t s) {
    SparseArgs c = a;
    const int blocks = sparse_haar_blocks(levels, c.nx, c.ny, c.nz, c.nt, c.max_grid);
    fh_stream(s)->push([c, blocks] {
        const size_t I = (size_t)c.nx * c.ny * c.nz * c.nt;
        look(c.C, I);
        look(c.S, c.S ? I : 0);
        look(c.Lp, I);
        look(c.w, c.w ? I : 0);
        touch(c.Sout, I);
        if (c.supp) touch(c.supp, I);
        touch(c.part, (size_t)blocks);
        work_us(40);
    });
    return blocks;
}
int sparse_tfft_blocks(int N, int nt) {
    int m = nt;
    for (int r : {2, 3, 5, 7})
        while (m > 1 && m % r == 0) m /= r;
    const int per_block = (nt >= 1 && nt <= 32 && m == 1) ? 256 : 64;
    const int b = (N + per_block - 1) / per_block;
    return b < 2048 ? b : 2048;
}
int launch_sparse_tfft(const SparseArgs& a, hipStream_t s) {
    SparseArgs c = a;
    const int blocks = sparse_tfft_blocks(c.nx * c.ny * c.nz, c.nt);
    fh_stream(s)->push([c, blocks] {
        const size_t I = (size_t)c.nx * c.ny * c.nz * c.nt;
        look(c.C, I);
        look(c.S, c.S ? I : 0);
        look(c.Lp, I);
        look(c.w, c.w ? I : 0);
        look(c.Wf, 64 * 64);
        look(c.Wi, 64 * 64);
        touch(c.Sout, I);
        if (c.supp) touch(c.supp, I);
        touch(c.part, (size_t)blocks);
        work_us(40);
    });
    return blocks;
}

int sparse_db4_blocks(int nx, int nt) { return nx * nt; }
int sparse_db4_line_blocks(int ny, int nz, int nt) { return nt * ((ny * nz + 31) / 32); }
bool db4_supported(int nx, int ny, int nz) { return nx <= 256 && ny * nz <= 8192; }
int launch_sparse_db4(const SparseArgs& a, hipStream_t s) {
    SparseArgs c = a;
    const int blocks = sparse_db4_blocks(c.nx, c.nt);
    fh_stream(s)->push([c, blocks] {
        const size_t I = (size_t)c.nx * c.ny * c.nz * c.nt;
        look(c.C, I);
        look(c.S, c.S ? I : 0);
        look(c.Lp, I);
        look(c.w, c.w ? I : 0);
        touch(c.Z, I);
        touch(c.Sout, I);
        if (c.supp) touch(c.supp, I);
        touch(c.part, (size_t)blocks);
        work_us(40);
    });
    return blocks;
}

int change_blocks(long n) {
    const long b = ((n + 1) / 2 + 2047) / 2048;
    return (int)(b < 1 ? 1 : (b > 2048 ? 2048 : b));
}

void launch_change(const ChangeArgs& a, hipStream_t s) {
    ChangeArgs c = a;
    fh_stream(s)->push([c] {
        look(c.L, (size_t)c.n);
        look(c.S, (size_t)c.n);
        look(c.Lold, (size_t)c.n);
        look(c.Sold, (size_t)c.n);
        touch(c.part, (size_t)change_blocks(c.n) * 2);
        work_us(20);
    });
}

void launch_stats(const StatsArgs& a, hipStream_t s) {
    StatsArgs c = a;
    fh_stream(s)->push([c] {
        look(c.dc_part, (size_t)c.dc_blocks);
        look(c.ch_part, (size_t)c.ch_blocks * 2);
        look(c.sp_part, (size_t)c.sp_blocks);
        c.stat[0] = 1.0;
        c.stat[1] = 1.0;
        c.stat[2] = 4.0;
        c.stat[3] = 1.0;
        c.stat[7] = 0.0;
    });
}

// Batched launchers: every problem's argument block (already on the "device") goes
// through the single-problem stand-in; the activity flags are not consulted (touching a
// stopped problem's arrays is harmless).
int launch_gram_batched(int mode, const GramArgs& a0, const Batched<GramArgs>* bt, hipStream_t s) {
    if (!bt) return launch_gram(mode, a0, s);
    int r = 0;
    for (int b = 0; b < bt->count; ++b) r = launch_gram(mode, bt->args[b], s);
    return r;
}
void launch_gram_reduce_batched(const ReduceArgs& a0, const Batched<ReduceArgs>* bt, hipStream_t s) {
    if (!bt) return launch_gram_reduce(a0.part, a0.blocks, a0.entries, a0.out, s);
    for (int b = 0; b < bt->count; ++b) {
        const ReduceArgs& r = bt->args[b];
        launch_gram_reduce(r.part, r.blocks, r.entries, r.out, s);
    }
}
void launch_eig_batched(const EigArgs& a0, const Batched<EigArgs>* bt, hipStream_t s) {
    if (!bt) return launch_eig(a0, s);
    for (int b = 0; b < bt->count; ++b) {
        EigArgs e = bt->args[b];
        e.stat += bt->rec_off;
        launch_eig(e, s);
    }
}
void launch_bp_batched(const BpArgs& a0, const Batched<BpArgs>* bt, hipStream_t s) {
    if (!bt) return launch_bp(a0, s);
    for (int b = 0; b < bt->count; ++b) launch_bp(bt->args[b], s);
}
int launch_sparse_batched(int levels, const SparseArgs& a0, const Batched<SparseArgs>* bt,
                          hipStream_t s) {
    if (!bt) return launch_sparse(levels, a0, s);
    int r = 0;
    for (int b = 0; b < bt->count; ++b) r = launch_sparse(levels, bt->args[b], s);
    return r;
}
int launch_sparse_db4_batched(const SparseArgs& a0, const Batched<SparseArgs>* bt, hipStream_t s) {
    if (!bt) return launch_sparse_db4(a0, s);
    int r = 0;
    for (int b = 0; b < bt->count; ++b) r = launch_sparse_db4(bt->args[b], s);
    return r;
}
int launch_sparse_tfft_batched(const SparseArgs& a0, const Batched<SparseArgs>* bt, hipStream_t s) {
    if (!bt) return launch_sparse_tfft(a0, s);
    int r = 0;
    for (int b = 0; b < bt->count; ++b) r = launch_sparse_tfft(bt->args[b], s);
    return r;
}
void launch_stats_batched(const StatsArgs& a0, const Batched<StatsArgs>* bt, hipStream_t s) {
    if (!bt) return launch_stats(a0, s);
    for (int b = 0; b < bt->count; ++b) {
        StatsArgs c = bt->args[b];
        c.stat += bt->rec_off;
        launch_stats(c, s);
    }
}
void launch_change_batched(const ChangeArgs& a0, const Batched<ChangeArgs>* bt, hipStream_t s) {
    if (!bt) return launch_change(a0, s);
    for (int b = 0; b < bt->count; ++b) launch_change(bt->args[b], s);
}
int launch_dc_batched(int ny, int nz, const DcArgs& a0, const Batched<DcArgs>* bt, hipStream_t s) {
    if (!bt) return launch_dc(ny, nz, a0, s);
    int r = 0;
    for (int b = 0; b < bt->count; ++b) r = launch_dc(ny, nz, bt->args[b], s);
    return r;
}

}  // namespace pls
