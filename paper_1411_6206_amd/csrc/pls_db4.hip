// Step (3) of Algorithm 1 with T the orthonormal four-tap Daubechies wavelet, periodic, in
// the standard (tensor-product) decomposition: the full J-level 1D transform along each
// spatial axis of size > 1.  One level along an axis of length n maps u to
//   a_k = sum_m h_m u[(2k + m) mod n],  d_k = sum_m g_m u[(2k + m) mod n],  g_m = (-1)^m h_{3-m},
// stored as [a | d] (canonical Mallat order); its inverse is the adjoint,
//   u[2k] = h0 a_k + h2 a_{k-1} + g0 d_k + g2 d_{k-1},
//   u[2k+1] = h1 a_k + h3 a_{k-1} + g1 d_k + g3 d_{k-1}   (k - 1 mod n / 2).
// The axes commute, so the update runs as three passes over the frames:
//   1. x lines: Z = T_x (X - L_prev) into a scratch array;
//   2. (y, z) planes: T_y, T_z, the weighted soft threshold (support and weighted l1 partial
//      sums as in the Haar update), T_z^{-1}, T_y^{-1}, in place;
//   3. x lines: S = T_x^{-1} Z.
// Each pass stages its lines or plane in LDS; a level reads its inputs into registers, waits
// at a block barrier, and writes its outputs in place.
#include "pls_common.hpp"
#include "pls_kernels.hpp"

namespace pls {

// Daubechies' four-tap scaling filter, (1 + sqrt 3, 3 + sqrt 3, 3 - sqrt 3, 1 - sqrt 3) / (4 sqrt 2)
constexpr float kH0 = 0.482962913144534143f, kH1 = 0.836516303737807906f;
constexpr float kH2 = 0.224143868042013381f, kH3 = -0.129409522551260381f;
// wavelet filter g_m = (-1)^m h_{3-m}
constexpr float kG0 = kH3, kG1 = -kH2, kG2 = kH1, kG3 = -kH0;

constexpr int kDbThreads = 256;
constexpr int kDbLinePts = 16;       // x-line passes: positions p of the plane per block
constexpr int kDbMaxNx = 256;
constexpr int kDbMaxPlane = 256 * 32;
constexpr int kDbLineItems = kDbMaxNx / 2 * kDbLinePts / kDbThreads;   // (n / 2) x 16 / 256
constexpr int kDbPlaneThreads = 512;                                   // plane pass
static_assert(kDbMaxPlane / 2 <= 8 * kDbPlaneThreads, "plane items per thread exceed 8");

__device__ __forceinline__ float2 fma2(float s, float2 u, float2 acc) {
    return make_float2(fmaf(s, u.x, acc.x), fmaf(s, u.y, acc.y));
}

// Item e = tid + NTH q of a level with `lines` lines of length n is (line l, output k),
// k < n / 2, with k or l the fast index (k_fast).  The pair is advanced incrementally from
// one q to the next (no division per item).
template <int NTH>
struct DbItems {
    int f, s, df, ds, F;
    __device__ __forceinline__ DbItems(int tid, int fast_range) : F(fast_range) {
        f = tid % F;
        s = tid / F;
        df = NTH % F;
        ds = NTH / F;
    }
    __device__ __forceinline__ void next() {
        f += df;
        s += ds;
        if (f >= F) {
            f -= F;
            s += 1;
        }
    }
};

// One analysis level on LDS lines: `lines` lines, element i of line l at l * ls + i * es,
// length n (even).  Items (l, k), k < n / 2, are dealt to the NTH threads; at most MAXIT each.
template <int NTH, int MAXIT>
__device__ __forceinline__ void db4_level_fwd(float2* u, int lines, int n, int ls, int es,
                                              int tid, bool k_fast) {
    const int h = n >> 1, items = lines * h;
    float2 ra[MAXIT], rd[MAXIT];
    {
        DbItems<NTH> it(tid, k_fast ? h : lines);
#pragma unroll
        for (int q = 0; q < MAXIT; ++q, it.next()) {
            if (tid + q * NTH < items) {
                const int k = k_fast ? it.f : it.s, l = k_fast ? it.s : it.f;
                const float2* b = u + l * ls;
                const int i0 = 2 * k;
                const int i2 = i0 + 2 < n ? i0 + 2 : i0 + 2 - n;
                const int i3 = i0 + 3 < n ? i0 + 3 : i0 + 3 - n;
                const float2 u0 = b[i0 * es], u1 = b[(i0 + 1) * es], u2 = b[i2 * es], u3 = b[i3 * es];
                float2 av = make_float2(0.f, 0.f), dv = make_float2(0.f, 0.f);
                av = fma2(kH0, u0, av); av = fma2(kH1, u1, av); av = fma2(kH2, u2, av); av = fma2(kH3, u3, av);
                dv = fma2(kG0, u0, dv); dv = fma2(kG1, u1, dv); dv = fma2(kG2, u2, dv); dv = fma2(kG3, u3, dv);
                ra[q] = av;
                rd[q] = dv;
            }
        }
    }
    __syncthreads();
    {
        DbItems<NTH> it(tid, k_fast ? h : lines);
#pragma unroll
        for (int q = 0; q < MAXIT; ++q, it.next()) {
            if (tid + q * NTH < items) {
                const int k = k_fast ? it.f : it.s, l = k_fast ? it.s : it.f;
                u[l * ls + k * es] = ra[q];
                u[l * ls + (h + k) * es] = rd[q];
            }
        }
    }
    __syncthreads();
}

// The adjoint level: [a | d] -> u on the same lines.
template <int NTH, int MAXIT>
__device__ __forceinline__ void db4_level_inv(float2* u, int lines, int n, int ls, int es,
                                              int tid, bool k_fast) {
    const int h = n >> 1, items = lines * h;
    float2 re[MAXIT], ro[MAXIT];
    {
        DbItems<NTH> it(tid, k_fast ? h : lines);
#pragma unroll
        for (int q = 0; q < MAXIT; ++q, it.next()) {
            if (tid + q * NTH < items) {
                const int k = k_fast ? it.f : it.s, l = k_fast ? it.s : it.f;
                const float2* b = u + l * ls;
                const int km = k == 0 ? h - 1 : k - 1;
                const float2 a0 = b[k * es], a1 = b[km * es];
                const float2 d0 = b[(h + k) * es], d1 = b[(h + km) * es];
                float2 ev = make_float2(0.f, 0.f), od = make_float2(0.f, 0.f);
                ev = fma2(kH0, a0, ev); ev = fma2(kH2, a1, ev); ev = fma2(kG0, d0, ev); ev = fma2(kG2, d1, ev);
                od = fma2(kH1, a0, od); od = fma2(kH3, a1, od); od = fma2(kG1, d0, od); od = fma2(kG3, d1, od);
                re[q] = ev;
                ro[q] = od;
            }
        }
    }
    __syncthreads();
    {
        DbItems<NTH> it(tid, k_fast ? h : lines);
#pragma unroll
        for (int q = 0; q < MAXIT; ++q, it.next()) {
            if (tid + q * NTH < items) {
                const int k = k_fast ? it.f : it.s, l = k_fast ? it.s : it.f;
                u[l * ls + (2 * k) * es] = re[q];
                u[l * ls + (2 * k + 1) * es] = ro[q];
            }
        }
    }
    __syncthreads();
}

__device__ __forceinline__ int db4_line_blocks(const SparseArgs& a) {
    return a.nt * ((a.ny * a.nz + kDbLinePts - 1) / kDbLinePts);
}

// Passes 1 and 3: block = frame t and 16 consecutive plane positions p (16 x-lines, 128
// bytes per x row: one cache line), all nx in LDS as [x][p].  INV = false: U = C + S - L_prev,
// J forward levels, Z out; INV = true: Z in, J inverse levels, S out.
template <bool INV, class SRC>
__global__ void __launch_bounds__(kDbThreads) pls_db4_x_kernel(SRC src) {
    if (src.skip()) return;
    const SparseArgs a = src.get();
    if ((int)blockIdx.x >= db4_line_blocks(a)) return;   // beyond this problem's grid (batches)
    __shared__ float2 u[kDbMaxNx * kDbLinePts];
    const int tid = threadIdx.x;
    const int P = a.ny * a.nz;
    const int pb = (P + kDbLinePts - 1) / kDbLinePts;
    const int t = blockIdx.x / pb;
    const int p0 = (blockIdx.x % pb) * kDbLinePts;
    const int nx = a.nx;
    const bool has_s = a.S != nullptr;
    const float2* Sp = has_s ? a.S : a.C;
#pragma unroll 4
    for (int e = tid; e < nx * kDbLinePts; e += kDbThreads) {
        const int x = e / kDbLinePts, pl = e % kDbLinePts;
        const int p = p0 + pl;
        const bool ok = p < P;
        const size_t gi = ((size_t)t * nx + x) * P + (ok ? p : P - 1);
        float2 v;
        if constexpr (INV) {
            v = a.Z[gi];
        } else {
            const float2 c = a.C[gi], sv = Sp[gi], l = a.Lp[gi];
            v = csub(has_s ? cadd(c, sv) : c, l);
        }
        u[e] = ok ? v : make_float2(0.f, 0.f);
    }
    __syncthreads();
    const int J = nx > 1 ? a.levels : 0;
    if constexpr (!INV) {
        for (int j = 0; j < J; ++j)
            db4_level_fwd<kDbThreads, kDbLineItems>(u, kDbLinePts, nx >> j, 1, kDbLinePts, tid, false);
    } else {
        for (int j = J - 1; j >= 0; --j)
            db4_level_inv<kDbThreads, kDbLineItems>(u, kDbLinePts, nx >> j, 1, kDbLinePts, tid, false);
    }
#pragma unroll 4
    for (int e = tid; e < nx * kDbLinePts; e += kDbThreads) {
        const int x = e / kDbLinePts, pl = e % kDbLinePts;
        const int p = p0 + pl;
        if (p < P) {
            const size_t gi = ((size_t)t * nx + x) * P + p;
            if constexpr (INV) a.Sout[gi] = u[e];
            else a.Z[gi] = u[e];
        }
    }
}

// Pass 2: block = plane (t, x), [z][y] in LDS (P points of dynamic LDS).  T_y (rows), T_z
// (columns), the weighted soft threshold of every coefficient, then the inverses; one
// weighted-l1 partial per block.  NTH threads with at most MAXIT items each per level
// (NTH MAXIT >= P / 2).
template <int NTH, int MAXIT, class SRC>
__global__ void __launch_bounds__(NTH) pls_db4_plane_kernel(SRC src) {
    if (src.skip()) return;
    const SparseArgs a = src.get();
    if ((int)blockIdx.x >= a.nt * a.nx) return;   // beyond this problem's grid (batches)
    extern __shared__ float2 u[];
    __shared__ double red[NTH / kWave];
    const int tid = threadIdx.x;
    const int ny = a.ny, nz = a.nz, P = ny * nz;
    const size_t base = (size_t)blockIdx.x * P;   // plane (t, x) = blockIdx.x
#pragma unroll 4
    for (int e = tid; e < P; e += NTH) u[e] = a.Z[base + e];
    __syncthreads();
    const int Jy = ny > 1 ? a.levels : 0, Jz = nz > 1 ? a.levels : 0;
    for (int j = 0; j < Jy; ++j) db4_level_fwd<NTH, MAXIT>(u, nz, ny >> j, ny, 1, tid, true);
    for (int j = 0; j < Jz; ++j) db4_level_fwd<NTH, MAXIT>(u, ny, nz >> j, 1, ny, tid, false);
    const bool has_w = a.w != nullptr;
    float l1 = 0.f;
    for (int e = tid; e < P; e += NTH) {
        // soft threshold of the complex magnitude: u (1 - tau / |u|) where |u| > tau
        const float omw = has_w ? weight_complement(a.w[base + e]) : 1.0f;
        const float tau = a.lambda_S * omw;
        const float2 v = u[e];
        const float m2 = fmaf(v.x, v.x, v.y * v.y);
        const bool keep = m2 > tau * tau;
        const float rm = __builtin_amdgcn_rsqf(keep ? m2 : 1.0f);
        const float sc = fmaf(-tau, rm, 1.0f);
        u[e] = keep ? make_float2(v.x * sc, v.y * sc) : make_float2(0.f, 0.f);
        l1 = fmaf(omw, keep ? fmaf(m2, rm, -tau) : 0.f, l1);
        if (a.supp) a.supp[base + e] = keep ? 255 : 0;
    }
    __syncthreads();
    for (int j = Jz - 1; j >= 0; --j) db4_level_inv<NTH, MAXIT>(u, ny, nz >> j, 1, ny, tid, false);
    for (int j = Jy - 1; j >= 0; --j) db4_level_inv<NTH, MAXIT>(u, nz, ny >> j, ny, 1, tid, true);
#pragma unroll 4
    for (int e = tid; e < P; e += NTH) a.Z[base + e] = u[e];
    const double s = block_sum<NTH>((double)l1, red);
    if (tid == 0) a.part[blockIdx.x] = s;
}

int sparse_db4_blocks(int nx, int nt) { return nx * nt; }

int sparse_db4_line_blocks(int ny, int nz, int nt) {
    return nt * ((ny * nz + kDbLinePts - 1) / kDbLinePts);
}

bool db4_supported(int nx, int ny, int nz) {
    return nx <= kDbMaxNx && ny * nz <= kDbMaxPlane;
}

int launch_sparse_db4_batched(const SparseArgs& a0, const Batched<SparseArgs>* bt, hipStream_t s) {
    SparseArgs a = a0;
    a.blocks = sparse_db4_blocks(a.nx, a.nt);
    const int own_lines = sparse_db4_line_blocks(a.ny, a.nz, a.nt);
    // a batch's grid is its largest problem's, per pass: bt->grid holds the plane pass's,
    // bt->grid2 the line passes' (every problem of a batch has this plane)
    const int grid_planes = (bt && bt->grid > 0) ? bt->grid : a.blocks;
    const int grid_lines = (bt && bt->grid2 > 0) ? bt->grid2 : own_lines;
    const int P = a.ny * a.nz;
    const size_t lds = (size_t)P * sizeof(float2);
    constexpr int NT = kDbPlaneThreads;
    PLS_LAUNCH(dim3(grid_lines), dim3(kDbThreads), s, a, bt, pls_db4_x_kernel, false);
    // items per thread and level at most P / 2 / NT, rounded up to a compiled bound
    const int need = (P / 2 + NT - 1) / NT;
    if (need <= 2)
        PLS_LAUNCH_SHMEM(dim3(grid_planes), dim3(NT), lds, s, a, bt, pls_db4_plane_kernel, NT, 2);
    else if (need <= 4)
        PLS_LAUNCH_SHMEM(dim3(grid_planes), dim3(NT), lds, s, a, bt, pls_db4_plane_kernel, NT, 4);
    else if (need <= 6)
        PLS_LAUNCH_SHMEM(dim3(grid_planes), dim3(NT), lds, s, a, bt, pls_db4_plane_kernel, NT, 6);
    else
        PLS_LAUNCH_SHMEM(dim3(grid_planes), dim3(NT), lds, s, a, bt, pls_db4_plane_kernel, NT, 8);
    PLS_LAUNCH(dim3(grid_lines), dim3(kDbThreads), s, a, bt, pls_db4_x_kernel, true);
    return a.blocks;
}

int launch_sparse_db4(const SparseArgs& a, hipStream_t s) {
    return launch_sparse_db4_batched(a, nullptr, s);
}

}  // namespace pls
