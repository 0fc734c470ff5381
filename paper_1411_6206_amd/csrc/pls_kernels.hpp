// Kernel argument blocks and host-side launchers of the Priori L+S library.
//
// Internal layouts (device, owned by the handle):
//   image state C, L, S      complex64 [nt][nx][nz][ny]   (each (t, x) plane contiguous)
//   coil sensitivities       complex64 [nc][nx][nz][ny]
//   prior weights            uint8     [nt][nx][nz][ny]   block-local (in-place) Haar order
//   compact hybrid data dh   complex64, frame t at dh_off[t], index (x * nc + c) * ns[t] + s:
//                            the unitary kx-IDFT of sample s of frame t, scaled by 1/sqrt(ny nz)
//   sample map sidx          int16 [nt][nz][ny]: sample index of (kz, ky) or -1
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace pls {

struct DcArgs {
    const float2* L;       // new iterate (Y = L + S); L NULL means Y = 0
    const float2* S;       // NULL means S = 0
    float2* C;             // out: C = M - S = L - E^H(E Y - d); also holds Y between coils,
                           // so it must not alias L or S
    const float2* sens;    // [nc][nx][nz][ny]; a single unit coil is an array of ones
    const float2* dh;
    const int* dh_off;
    const int* ns;
    const int16_t* sidx;
    const float2* twy;     // exp(-2 pi i m / ny)
    const float2* twz;     // exp(-2 pi i m / nz)
    double* part;          // per block: sum |r|^2 of its residual entries (scaled by 1/(ny nz))
    int nx, nt, nc;
    float inv_p;           // 1 / (ny nz)
    int blocks;            // this problem's workgroups, (nx / planes per block) nt: the grid
                           // when launched alone; blocks beyond it (a batch launched with a
                           // larger problem's grid) return at once
};

struct XiArgs {
    const float2* kspace;  // user layout [nc][nt][nz][ny][nx]
    const int* plist;      // [nt][ny nz] sample positions z * ny + y in sample order
    const int* line_off;   // [nt + 1] prefix of nc * ns
    const int* ns;
    const int* dh_off;
    float2* dh;
    const float2* twx;     // exp(-2 pi i m / nx)
    int nx, nt, nc, P, total_lines;
    float scale;           // 1 / sqrt(nx * ny * nz)
};

bool dc_supported(int ny, int nz);
bool xifft_supported(int nx);
// Launch the data-consistency pass over all (t, x) planes.  Returns the number of blocks
// (rows of DcArgs::part written), 0 if the shape is unsupported.
int launch_dc(int ny, int nz, const DcArgs& a, hipStream_t s);
int dc_blocks(int ny, int nz, int nx, int nt);
bool launch_xifft(int nx, const XiArgs& a, hipStream_t s);

// ---------------------------------------------------------------- setup kernels
void launch_mask_scan(const uint8_t* mask, int ny, int nz, int nt, int16_t* sidx, int* plist,
                      int* ns, hipStream_t s);
// user [F][nz][ny][nx] -> internal [F][nx][nz][ny]; in2 (optional) is added
void launch_pack(const float2* in, const float2* in2, float2* out, int F, int nx, int ny,
                 int nz, hipStream_t s);
// internal [F][nx][nz][ny] -> user [F][nz][ny][nx]; out = a + b (b optional)
void launch_unpack(const float2* a, const float2* b, float2* out, int F, int nx, int ny,
                   int nz, hipStream_t s);
// canonical Haar layout [nt][nz][ny][nx] -> internal block-local [nt][nx][nz][ny]
void launch_pack_weights(const uint8_t* in, uint8_t* out, int nt, int nx, int ny, int nz,
                         int levels, hipStream_t s);
void launch_add(const float2* a, const float2* b, float2* out, size_t n, hipStream_t s);

// ---------------------------------------------------------------- Gram / eig / LS
struct GramArgs {
    const float2* C;       // [nt][N]
    double* part;          // [blocks][NTILE * 256]
    int N, nt, vox_per_block;
    int target_blocks;     // split of the voxels into about this many blocks (0 = default)
};
// returns number of blocks
int launch_gram(int mode, const GramArgs& a, hipStream_t s);
int gram_blocks(int N, int target = 0);
int gram_vpb(int N, int target);   // voxels per Gram block
int gram_tiles(int nt);
void launch_gram_reduce(const double* part, int blocks, int entries, double* out, hipStream_t s);

struct EigArgs {
    const double* gram;    // reduced tiles
    double* V;             // [nt][nt] complex (re, im interleaved) eigenvectors, in/out (warm start)
    int warm;              // use V as the starting basis
    float* Wop;            // MFMA A-operand of the back-projection: [64][64] (or [32][32])
    double* Wd;            // W = V diag(phi) V^H, complex [nt][nt] (FP64 copy)
    const double* sigma_prev;  // [nt] descending, zero padded
    double* stat;          // per-iteration record (see pls_stats layout in the runtime)
    double* sigL;          // [nt] singular values of the new L by rank (descending), or NULL
    int nt;
    double lambda_L, lambda_p;
    int relative;
};
void launch_eig(const EigArgs& a, hipStream_t s);

struct BpArgs {
    const float2* C;
    float2* L;
    const float* Wop;
    int N, nt;
    int max_grid;          // workgroups at most (0 = default)
};
void launch_bp(const BpArgs& a, hipStream_t s);
int bp_blocks(int N, int max_grid);   // back-projection workgroups of one problem

struct SparseArgs {
    const float2* C;       // M - S (so M - L_prev = C + S - L_prev)
    const float2* S;       // previous S (may be NULL: zero)
    const float2* Lp;      // previous L
    const uint8_t* w;      // internal block-local weights or NULL
    float2* Sout;
    uint8_t* supp;         // 255 where a coefficient survives the shrinkage, else 0 (same
                           // layout as w), or NULL
    double* part;          // per block: weighted l1 of the shrunk coefficients
    int nx, ny, nz, nt;
    float lambda_S;
    const float* Wf;       // temporal transform only: MFMA operands of the forward DFT and
    const float* Wi;       // of the inverse (its columns in the forward's output order)
    int max_grid;          // Haar transform: workgroups at most, each looping over tiles
                           // (0 = one per tile)
    int blocks;            // this problem's workgroups (= partial sums); set by the launcher
                           // for one problem, by the batch for each of its problems
    int levels;            // Daubechies transform: J
    float2* Z;             // Daubechies transform: scratch image array (coefficients)
};
// returns number of blocks
int launch_sparse(int levels, const SparseArgs& a, hipStream_t s);
// workgroups (= partial sums) of the Haar sparse update for a max_grid cap
int sparse_haar_blocks(int levels, int nx, int ny, int nz, int nt, int max_grid);
int launch_sparse_tfft(const SparseArgs& a, hipStream_t s);
int sparse_tfft_blocks(int N, int nt);   // workgroups (= partial sums) of the temporal update
// Daubechies-4 update (three passes: x lines, (y, z) planes, x lines; a.Z the scratch array,
// a.levels J): returns the partial sums written (nt * nx, one per plane).
int launch_sparse_db4(const SparseArgs& a, hipStream_t s);
int sparse_db4_blocks(int nx, int nt);
int sparse_db4_line_blocks(int ny, int nz, int nt);   // workgroups of each x-line pass
bool db4_supported(int nx, int ny, int nz);

// Change of the iterate for the stopping test: per block, sum |Y - Yold|^2 and sum |Yold|^2
// over its elements (Y = L + S, Yold = Lold + Sold, each formed in FP32, summed in FP64).
struct ChangeArgs {
    const float2* L;
    const float2* S;
    const float2* Lold;
    const float2* Sold;
    double* part;          // [blocks][2]
    long n;                // complex elements of each array
    int blocks;            // this problem's workgroups, change_blocks(n); set as for SparseArgs
};
int change_blocks(long n);
void launch_change(const ChangeArgs& a, hipStream_t s);

struct StatsArgs {
    const double* dc_part;
    int dc_blocks;
    const double* ch_part; // [ch_blocks][2] change partials; ch_blocks 0: stat[1] = stat[2] = 0
    int ch_blocks;
    const double* sp_part;
    int sp_blocks;
    double* stat;          // per-iteration record
    double p_scale;        // ny * nz (residual scaling)
    double lambda_S;
};
void launch_stats(const StatsArgs& a, hipStream_t s);

// ---------------------------------------------------------------- batched launches
// A kernel reads its argument block through a source.  ArgOne carries the block by value
// (one problem per launch).  ArgBatch serves several problems of one geometry in one
// launch: the blocks with blockIdx.z == b work on problem b, read args[b] from device
// memory, return at once while active[b] is 0, and add rec_off to the statistics-record
// pointer (eigensolver and statistics kernels: the iteration's slot in the chunk).
template <class A>
__device__ __forceinline__ void offset_record(A&, long) {}
__device__ __forceinline__ void offset_record(EigArgs& a, long off) { a.stat += off; }
__device__ __forceinline__ void offset_record(StatsArgs& a, long off) { a.stat += off; }

template <class A>
struct ArgOne {
    A a;
    __device__ __forceinline__ bool skip() const { return false; }
    __device__ __forceinline__ A get() const { return a; }
};

template <class A>
struct ArgBatch {
    const A* args;         // [count] (device)
    const int* active;     // [count] (device), or NULL: all active
    long rec_off;
    __device__ __forceinline__ bool skip() const { return active && active[blockIdx.z] == 0; }
    __device__ __forceinline__ A get() const {
        A a = args[blockIdx.z];
        offset_record(a, rec_off);
        return a;
    }
};

// A batched launch: `count` problems (grid z), their device argument blocks, the per-problem
// activity flags (device, or NULL), the record offset, and the launch grid along x (the
// largest of the problems' own grids: problems of a batch may differ in nx, nt and nc; 0 =
// the grid of problem 0's host argument block).  Every kernel returns at once in the
// workgroups beyond its problem's own grid, and strides over its problem's work by that own
// grid, so a problem computes in a batch exactly what it computes alone.
template <class A>
struct Batched {
    int count;
    const A* args;
    const int* active;
    long rec_off;
    int grid;
    int grid2 = 0;         // a second pass's grid where a launcher runs two (0: its own)
    ArgBatch<A> src() const { return ArgBatch<A>{args, active, rec_off}; }
};

// Launches kernel template KERN (its last template parameter is the argument source) with
// the remaining template arguments given after the fixed ones: for one problem (BT NULL)
// with argument block A by value, else for the batch *BT with the grid's z extent set to
// the problem count.
#define PLS_LAUNCH(GRID, BLOCK, STREAM, A, BT, KERN, ...)                                   \
    PLS_LAUNCH_SHMEM(GRID, BLOCK, 0, STREAM, A, BT, KERN, __VA_ARGS__)

// The same with SHMEM bytes of dynamic LDS.
#define PLS_LAUNCH_SHMEM(GRID, BLOCK, SHMEM, STREAM, A, BT, KERN, ...)                      \
    do {                                                                                    \
        using PlsA_ = std::decay_t<decltype(A)>;                                            \
        if (BT) {                                                                           \
            dim3 g_ = (GRID);                                                               \
            g_.z = (unsigned)(BT)->count;                                                   \
            hipLaunchKernelGGL((KERN<__VA_ARGS__, ::pls::ArgBatch<PlsA_>>), g_, (BLOCK),     \
                               (SHMEM), (STREAM), (BT)->src());                              \
        } else {                                                                            \
            hipLaunchKernelGGL((KERN<__VA_ARGS__, ::pls::ArgOne<PlsA_>>), (GRID), (BLOCK),  \
                               (SHMEM), (STREAM), ::pls::ArgOne<PlsA_>{(A)});                \
        }                                                                                   \
    } while (0)

struct ReduceArgs {
    const double* part;    // [blocks][entries]
    double* out;           // [entries]
    int blocks, entries;
};

int launch_gram_batched(int mode, const GramArgs& a0, const Batched<GramArgs>* bt, hipStream_t s);
void launch_gram_reduce_batched(const ReduceArgs& a0, const Batched<ReduceArgs>* bt, hipStream_t s);
void launch_eig_batched(const EigArgs& a0, const Batched<EigArgs>* bt, hipStream_t s);
void launch_bp_batched(const BpArgs& a0, const Batched<BpArgs>* bt, hipStream_t s);
int launch_sparse_batched(int levels, const SparseArgs& a0, const Batched<SparseArgs>* bt,
                          hipStream_t s);
int launch_sparse_tfft_batched(const SparseArgs& a0, const Batched<SparseArgs>* bt, hipStream_t s);
int launch_sparse_db4_batched(const SparseArgs& a0, const Batched<SparseArgs>* bt, hipStream_t s);
void launch_stats_batched(const StatsArgs& a0, const Batched<StatsArgs>* bt, hipStream_t s);
void launch_change_batched(const ChangeArgs& a0, const Batched<ChangeArgs>* bt, hipStream_t s);
int launch_dc_batched(int ny, int nz, const DcArgs& a0, const Batched<DcArgs>* bt, hipStream_t s);

}  // namespace pls
