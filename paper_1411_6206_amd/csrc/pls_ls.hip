// Low-rank and sparse updates of Algorithm 1 and the per-iteration statistics.
//
//  * back-projection, steps (1)-(2): L = C W on FP32 MFMA (v_mfma_f32_16x16x4f32) with the
//    frame-space operator W from the eigensolver, real-expanded: [Re L | Im L]^T =
//    Wr^T [Re C | Im C]^T, 16 voxels per MFMA column block;
//  * sparse update, step (3): S = T^{-1} soft(T(X - L_prev), lambda_S (1 - w)) with T the
//    J-level orthonormal Haar (nonstandard pyramid) computed in place on (2^J)^3 blocks:
//    x in registers, y and z across the lanes of a wave;
//  * fixed-order FP64 reduction of the per-block partial sums into one record per iteration.
#include <algorithm>

#include "pls_common.hpp"
#include "pls_fft.hpp"
#include "pls_kernels.hpp"

namespace pls {

typedef float f4 __attribute__((ext_vector_type(4)));

// A copy of x the compiler cannot see through, so loads addressed with it are not hoisted
// out of a loop (which would pin their registers for the loop's duration).
__device__ __forceinline__ int unhoisted(int x) {
    int y;
    asm volatile("v_mov_b32 %0, %1" : "=v"(y) : "v"(x));
    return y;
}

// Copies a real-expanded K2 x K2 MFMA A operand (row o, column k at o * K2 + k) into LDS in
// fragment order: element (mb, ks) of lane l (row 16 mb + l % 16, column 4 ks + l / 16) at
// fragment (mb * KS / 4 + ks / 4) * 64 + l, component ks % 4, so a lane fetches the operands
// of four consecutive k steps with one 16-byte read.  The caller adds the barrier.
template <int K2>
__device__ __forceinline__ void load_fragments(const float* W, f4* frag) {
    constexpr int MB = K2 / 16, KQ = K2 / 16, NF = MB * KQ * 64;
    for (int e = threadIdx.x; e < NF; e += blockDim.x) {
        const int l = e & 63, q = (e >> 6) % KQ, mb = e / (64 * KQ);
        const int base = (16 * mb + (l & 15)) * K2 + 16 * q + (l >> 4);
        f4 v;
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = W[base + 4 * j];
        frag[e] = v;
    }
}


// ---------------------------------------------------------------- back-projection
// The operand lives in LDS in fragment order rather than in 64 VGPRs, for occupancy.
template <int NB, class SRC>
__global__ void __launch_bounds__(256) pls_bp_kernel(SRC src) {
    if (src.skip()) return;
    const BpArgs a = src.get();
    constexpr int NTP = 16 * NB, K2 = 2 * NTP, MB = K2 / 16, KS = K2 / 4, KH = NTP / 4;
    constexpr int KQ = KS / 4;
    __shared__ f4 frag[MB * KQ * 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i16 = lane & 15, g = lane >> 4;
    load_fragments<K2>(a.Wop, frag);
    __syncthreads();
    const int N = a.N;
    const int stride = gridDim.x * 4 * 16;
    // frames are clamped into range and voxels into the volume, so every load is valid and
    // issued without a branch; out-of-range values are zeroed by selects
    auto load_tile = [&](int v0, float2 (&cb)[KH]) __attribute__((always_inline)) {
        const int v = v0 + i16;
        const int vc = v < N ? v : N - 1;
#pragma unroll
        for (int kk = 0; kk < KH; ++kk) {
            const int f = 4 * kk + g;
            const int fc = f < a.nt ? f : a.nt - 1;
            const float2 x = a.C[fc * N + vc];
            cb[kk] = (f < a.nt && v < N) ? x : make_float2(0.f, 0.f);
        }
    };
    int v0 = (blockIdx.x * 4 + wave) * 16;
    if (v0 >= N) return;
    float2 cb[KH];
    load_tile(v0, cb);
    for (; v0 < N; v0 += stride) {
        // fetch the next tile before this one's products (software pipelining)
        float2 nb[KH];
        const int vn = v0 + stride;
        load_tile(vn < N ? vn : v0, nb);
        const int fl = unhoisted(lane);
        f4 acc[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) acc[mb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
            f4 af[MB];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) af[mb] = frag[(mb * KQ + q) * 64 + fl];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int ks = 4 * q + j;
                const float b = ks < KH ? cb[ks].x : cb[ks - KH].y;
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
                    acc[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[mb][j], b, acc[mb], 0, 0, 0);
            }
        }
        const int v = v0 + i16;
        if (v < N) {
#pragma unroll
            for (int mb = 0; mb < MB / 2; ++mb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int f = 16 * mb + 4 * g + r;
                    if (f < a.nt) a.L[f * N + v] = make_float2(acc[mb][r], acc[mb + MB / 2][r]);
                }
        }
#pragma unroll
        for (int kk = 0; kk < KH; ++kk) cb[kk] = nb[kk];
    }
}

int bp_blocks(int N, int max_grid) {
    const int tiles = (N + 63) / 64;
    const int cap = max_grid > 0 ? max_grid : 2048;
    return tiles < cap ? tiles : cap;
}

// Each output voxel is formed by one lane whatever the grid, so a batch launched with a
// larger problem's grid computes every problem exactly as alone.
void launch_bp_batched(const BpArgs& a, const Batched<BpArgs>* bt, hipStream_t s) {
    const int grid = (bt && bt->grid > 0) ? bt->grid : bp_blocks(a.N, a.max_grid);
    if (a.nt <= 16)
        PLS_LAUNCH(dim3(grid), dim3(256), s, a, bt, pls_bp_kernel, 1);
    else if (a.nt <= 32)
        PLS_LAUNCH(dim3(grid), dim3(256), s, a, bt, pls_bp_kernel, 2);
    else
        PLS_LAUNCH(dim3(grid), dim3(256), s, a, bt, pls_bp_kernel, 4);
}

void launch_bp(const BpArgs& a, hipStream_t s) { launch_bp_batched(a, nullptr, s); }

// ---------------------------------------------------------------- sparse update
__device__ __forceinline__ float2 shfl_xor2(float2 v, int m) {
    return make_float2(__shfl_xor(v.x, m, kWave), __shfl_xor(v.y, m, kWave));
}

// (own, partner) -> a or d of the orthonormal 2-point Haar; self-inverse
__device__ __forceinline__ float2 haar_pair(float2 u, float2 p, bool second) {
    constexpr float s = 0.70710678118654752440f;
    return second ? make_float2((p.x - u.x) * s, (p.y - u.y) * s)
                  : make_float2((u.x + p.x) * s, (u.y + p.y) * s);
}

template <int J, bool ZA>
__device__ __forceinline__ void haar_level(float2 (&v)[1 << J], int l, int yl, int zl, int lane) {
    constexpr int B = 1 << J;
    constexpr int ZW = ZA ? B : 1;
    constexpr int YW = 64 / ZW;
    const int st = 1 << l;
    const bool lane_in = ((yl & (st - 1)) == 0) && ((zl & (st - 1)) == 0);
    // x: registers k and k + st, k a multiple of 2 st
#pragma unroll
    for (int k = 0; k < B; ++k) {
        if ((k & (2 * st - 1)) == 0 && k + st < B && lane_in) {
            const float2 u0 = v[k], u1 = v[k + st];
            v[k] = haar_pair(u0, u1, false);
            v[k + st] = haar_pair(u1, u0, true);
        }
    }
    // y: lanes differing in bit l
#pragma unroll
    for (int k = 0; k < B; ++k) {
        if ((k & (st - 1)) == 0) {
            const float2 p = shfl_xor2(v[k], st);
            if (lane_in) v[k] = haar_pair(v[k], p, (yl >> l) & 1);
        }
    }
    if constexpr (ZA) {
#pragma unroll
        for (int k = 0; k < B; ++k) {
            if ((k & (st - 1)) == 0) {
                const float2 p = shfl_xor2(v[k], st * YW);
                if (lane_in) v[k] = haar_pair(v[k], p, (zl >> l) & 1);
            }
        }
    }
    (void)lane;
}

template <int J, bool ZA, class SRC>
__global__ void __launch_bounds__(256) pls_sparse_kernel(SRC src) {
    if (src.skip()) return;
    const SparseArgs a = src.get();
    if ((int)blockIdx.x >= a.blocks) return;   // beyond this problem's grid (batches)
    constexpr int B = 1 << J;
    constexpr int ZW = ZA ? B : 1;
    constexpr int YW = 64 / ZW;
    constexpr int XW = B;
    __shared__ double red[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int yl = lane % YW, zl = lane / YW;
    const int nyt = (a.ny + 4 * YW - 1) / (4 * YW);
    const int nzt = a.nz / ZW;
    const int tiles = nyt * nzt * (a.nx / B);
    const bool has_s = a.S != nullptr, has_w = a.w != nullptr;
    const float2* Sp = has_s ? a.S : a.C;
    const uint8_t* wp = has_w ? a.w : reinterpret_cast<const uint8_t*>(a.C);
    float l1 = 0.f;
    // work item = (frame t, tile); a workgroup takes items blockIdx.x, + blocks, ...
    for (int item = blockIdx.x; item < tiles * a.nt; item += a.blocks) {
        int tile = item % tiles;
        const int t = item / tiles;
        const int yt = tile % nyt;
        tile /= nyt;
        const int zt = tile % nzt;
        const int xt = tile / nzt;
        const int y = yt * 4 * YW + wave * YW + yl;
        const int z = zt * ZW + zl;
        const bool valid = y < a.ny;
        // Every lane loads from a valid address (y clamped into the volume, absent arrays
        // replaced by C) and discards with selects, so the loads of all XW rows and all
        // arrays are in flight together.
        const int yc = valid ? y : a.ny - 1;
        float2 v[XW], sv[XW], lv[XW];
        int gi[XW];
        uint8_t wq[XW];
#pragma unroll
        for (int k = 0; k < XW; ++k) {
            gi[k] = ((t * a.nx + xt * XW + k) * a.nz + z) * a.ny + yc;
            v[k] = a.C[gi[k]];
            sv[k] = Sp[gi[k]];
            lv[k] = a.Lp[gi[k]];
            wq[k] = wp[gi[k]];
        }
#pragma unroll
        for (int k = 0; k < XW; ++k) {
            const float2 u = has_s ? cadd(v[k], sv[k]) : v[k];
            v[k] = valid ? csub(u, lv[k]) : make_float2(0.f, 0.f);
        }
        for (int l = 0; l < J; ++l) haar_level<J, ZA>(v, l, yl, zl, lane);
#pragma unroll
        for (int k = 0; k < XW; ++k) {
            // soft threshold of the complex magnitude: u (1 - tau / |u|) where |u| > tau
            const float omw = has_w ? weight_complement(wq[k]) : 1.0f;
            const float tau = a.lambda_S * omw;
            const float2 u = v[k];
            const float m2 = fmaf(u.x, u.x, u.y * u.y);
            const bool keep = valid && m2 > tau * tau;
            const float rm = __builtin_amdgcn_rsqf(keep ? m2 : 1.0f);
            const float sc = fmaf(-tau, rm, 1.0f);
            v[k] = keep ? make_float2(u.x * sc, u.y * sc) : make_float2(0.f, 0.f);
            l1 = fmaf(omw, keep ? fmaf(m2, rm, -tau) : 0.f, l1);
            if (a.supp && valid) a.supp[gi[k]] = keep ? 255 : 0;
        }
        for (int l = J - 1; l >= 0; --l) haar_level<J, ZA>(v, l, yl, zl, lane);
        if (valid) {
#pragma unroll
            for (int k = 0; k < XW; ++k) a.Sout[gi[k]] = v[k];
        }
    }
    const double s = block_sum<256>((double)l1, red);
    if (threadIdx.x == 0) a.part[blockIdx.x] = s;
}

int sparse_haar_blocks(int levels, int nx, int ny, int nz, int nt, int max_grid) {
    const int B = 1 << levels;
    const int ZW = nz > 1 ? B : 1;
    const int YW = 64 / ZW;
    const int nyt = (ny + 4 * YW - 1) / (4 * YW);
    const int items = nyt * (nz / ZW) * (nx / B) * nt;
    return (max_grid > 0 && max_grid < items) ? max_grid : items;
}

template <int J, bool ZA>
static int sparse_launch_t(const SparseArgs& a0, const Batched<SparseArgs>* bt, hipStream_t s) {
    SparseArgs a = a0;
    a.blocks = sparse_haar_blocks(J, a.nx, a.ny, a.nz, a.nt, a.max_grid);
    const int grid = (bt && bt->grid > 0) ? bt->grid : a.blocks;
    PLS_LAUNCH(dim3(grid), dim3(256), s, a, bt, pls_sparse_kernel, J, ZA);
    return a.blocks;
}

int launch_sparse_batched(int levels, const SparseArgs& a, const Batched<SparseArgs>* bt,
                          hipStream_t s) {
    const bool za = a.nz > 1;
    switch (levels) {
        case 0: return za ? sparse_launch_t<0, true>(a, bt, s) : sparse_launch_t<0, false>(a, bt, s);
        case 1: return za ? sparse_launch_t<1, true>(a, bt, s) : sparse_launch_t<1, false>(a, bt, s);
        case 2: return za ? sparse_launch_t<2, true>(a, bt, s) : sparse_launch_t<2, false>(a, bt, s);
        case 3: return za ? sparse_launch_t<3, true>(a, bt, s) : sparse_launch_t<3, false>(a, bt, s);
    }
    return 0;
}

int launch_sparse(int levels, const SparseArgs& a, hipStream_t s) {
    return launch_sparse_batched(levels, a, nullptr, s);
}

// ---------------------------------------------------------------- sparse update, temporal T
// Step (3) with T the unitary DFT along the frames of each voxel: per tile of 16 voxels a
// wave forms U = X - L_prev (all frames), Z = F U on FP32 MFMA (real-expanded, like the
// back-projection), soft-thresholds Z in the accumulator registers, and forms S = F^H Z_s
// with a second MFMA product.  The accumulator of the first product holds row
// 16 mb + 4 g + r in register (mb, r) of lane group g, which is the B operand that the
// second product's instruction 4 mb + r takes from lane group g once the inverse operator's
// columns are listed in that order (done on the host): no data moves between the two.
// frame counts whose DFT factors into radices 2, 3, 4, 5 and 7 (an in-register FFT)
static bool tfft_smooth(int nt) {
    int m = nt;
    for (int r : {2, 3, 5, 7})
        while (m > 1 && m % r == 0) m /= r;
    return nt >= 1 && nt <= 32 && m == 1;
}

int sparse_tfft_blocks(int N, int nt) {
    const int per_block = tfft_smooth(nt) ? 256 : 64;   // voxels per workgroup and step
    const int b = (N + per_block - 1) / per_block;
    return b < 2048 ? b : 2048;
}

// The operands of both products live in LDS in fragment order, not in registers: 128
// fewer VGPRs, so four waves per SIMD instead of two hide the memory latency.
template <int NB, class SRC>
__global__ void __launch_bounds__(256, 4) pls_tfft_sparse_kernel(SRC src) {
    if (src.skip()) return;
    const SparseArgs a = src.get();
    if ((int)blockIdx.x >= a.blocks) return;   // beyond this problem's grid (batches)
    constexpr int NTP = 16 * NB, K2 = 2 * NTP, MB = K2 / 16, KS = K2 / 4, KH = NTP / 4;
    constexpr int KQ = KS / 4;                 // groups of four k steps
    constexpr int NF = MB * KQ * 64;           // 16-byte fragments per operand
    __shared__ double red[4];
    // element (mb, ks) of lane l of an operand at fragment (mb * KQ + ks / 4) * 64 + l,
    // component ks % 4
    __shared__ f4 fragF[NF], fragI[NF];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i16 = lane & 15, g = lane >> 4;
    load_fragments<K2>(a.Wf, fragF);
    load_fragments<K2>(a.Wi, fragI);
    __syncthreads();
    const int N = a.nx * a.ny * a.nz;
    const int nt = a.nt;
    const int stride = a.blocks * 4 * 16;
    const bool has_s = a.S != nullptr, has_w = a.w != nullptr;
    const float2* Sp = has_s ? a.S : a.C;
    const uint8_t* wp = has_w ? a.w : reinterpret_cast<const uint8_t*>(a.C);
    // frames clamped into range and voxels into the volume: every load is valid
    auto load_tile = [&](int v0, float2 (&cb)[KH]) __attribute__((always_inline)) {
        const int v = v0 + i16;
        const int vc = v < N ? v : N - 1;
        float2 c[KH], sv[KH], l[KH];
#pragma unroll
        for (int kk = 0; kk < KH; ++kk) {
            const int f = 4 * kk + g;
            const int idx = (f < nt ? f : nt - 1) * N + vc;
            c[kk] = a.C[idx];
            sv[kk] = Sp[idx];
            l[kk] = a.Lp[idx];
        }
#pragma unroll
        for (int kk = 0; kk < KH; ++kk) {
            const float2 u = has_s ? cadd(c[kk], sv[kk]) : c[kk];
            cb[kk] = (4 * kk + g < nt && v < N) ? csub(u, l[kk]) : make_float2(0.f, 0.f);
        }
    };
    float l1 = 0.f;
    int v0 = (blockIdx.x * 4 + wave) * 16;
    float2 cb[KH];
    if (v0 < N) load_tile(v0, cb);
    for (; v0 < N; v0 += stride) {
        float2 nb[KH];
        const int vn = v0 + stride;
        load_tile(vn < N ? vn : v0, nb);
        const int v = v0 + i16;
        const int vc = v < N ? v : N - 1;
        const int fl = unhoisted(lane);
        // Z = F U
        f4 z[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) z[mb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < KQ; ++q) {
            f4 af[MB];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) af[mb] = fragF[(mb * KQ + q) * 64 + fl];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int ks = 4 * q + j;
                const float b = ks < KH ? cb[ks].x : cb[ks - KH].y;
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
                    z[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[mb][j], b, z[mb], 0, 0, 0);
            }
        }
        // soft threshold of frequency f = 16 mb + 4 g + r (real part in z[mb], imaginary
        // part in z[mb + MB/2])
        uint8_t wq[MB / 2][4];
#pragma unroll
        for (int mb = 0; mb < MB / 2; ++mb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int f = 16 * mb + 4 * g + r;
                wq[mb][r] = wp[(f < nt ? f : nt - 1) * N + vc];
            }
#pragma unroll
        for (int mb = 0; mb < MB / 2; ++mb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int f = 16 * mb + 4 * g + r;
                const bool valid = f < nt && v < N;
                const float omw = has_w ? weight_complement(wq[mb][r]) : 1.0f;
                const float tau = a.lambda_S * omw;
                const float zr = z[mb][r], zi = z[mb + MB / 2][r];
                const float m2 = fmaf(zr, zr, zi * zi);
                const bool keep = valid && m2 > tau * tau;
                const float rm = __builtin_amdgcn_rsqf(keep ? m2 : 1.0f);
                const float sc = keep ? fmaf(-tau, rm, 1.0f) : 0.0f;
                z[mb][r] = zr * sc;
                z[mb + MB / 2][r] = zi * sc;
                l1 = fmaf(omw, keep ? fmaf(m2, rm, -tau) : 0.f, l1);
                if (a.supp && valid) a.supp[f * N + v] = keep ? 255 : 0;
            }
        // S = F^H Z_s: instruction 4 mb + r takes register (mb, r) as its B operand
        f4 o[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) o[mb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            // k steps 4 mb .. 4 mb + 3 of the inverse: fragment group mb
            f4 ai[MB];
#pragma unroll
            for (int mo = 0; mo < MB; ++mo) ai[mo] = fragI[(mo * KQ + mb) * 64 + fl];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float b = z[mb][r];
#pragma unroll
                for (int mo = 0; mo < MB; ++mo)
                    o[mo] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[mo][r], b, o[mo], 0, 0, 0);
            }
        }
        if (v < N) {
#pragma unroll
            for (int mb = 0; mb < MB / 2; ++mb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int f = 16 * mb + 4 * g + r;
                    if (f < nt) a.Sout[f * N + v] = make_float2(o[mb][r], o[mb + MB / 2][r]);
                }
        }
#pragma unroll
        for (int kk = 0; kk < KH; ++kk) cb[kk] = nb[kk];
    }
    const double s = block_sum<256>((double)l1, red);
    if (threadIdx.x == 0) a.part[blockIdx.x] = s;
}

// The same step for frame counts with radices 2, 3, 4, 5 and 7 only: one thread per voxel
// holds all its frames, U = X - L_prev, and takes the unitary DFT along them as an
// in-register FFT (natural order in and out), shrinks, and transforms back.  Every load
// and store of a wave covers 64 consecutive voxels of one frame.  The FFT needs a tenth of
// the dense product's arithmetic, so the pass is bound by memory, not by the MFMA chain.
template <int NT, class SRC>
__global__ void __launch_bounds__(256) pls_tfft_fft_kernel(SRC src) {
    if (src.skip()) return;
    const SparseArgs a = src.get();
    if ((int)blockIdx.x >= a.blocks) return;   // beyond this problem's grid (batches)
    __shared__ double red[4];
    const int N = a.nx * a.ny * a.nz;
    const bool has_s = a.S != nullptr, has_w = a.w != nullptr;
    const float2* Sp = has_s ? a.S : a.C;
    const uint8_t* wp = has_w ? a.w : reinterpret_cast<const uint8_t*>(a.C);
    const float scale = 1.0f / sqrtf((float)NT);
    float l1 = 0.f;
    for (int v = blockIdx.x * 256 + threadIdx.x; v < N; v += a.blocks * 256) {
        float2 x[NT];
#pragma unroll
        for (int f = 0; f < NT; ++f) {
            const size_t i = (size_t)f * N + v;
            const float2 c = a.C[i], sv = Sp[i], l = a.Lp[i];
            x[f] = csub(has_s ? cadd(c, sv) : c, l);
        }
        dft<NT, false>(x);
        uint8_t wq[NT];
#pragma unroll
        for (int k = 0; k < NT; ++k) wq[k] = wp[(size_t)k * N + v];
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            const float omw = has_w ? weight_complement(wq[k]) : 1.0f;
            const float tau = a.lambda_S * omw;
            const float zr = x[k].x * scale, zi = x[k].y * scale;
            const float m2 = fmaf(zr, zr, zi * zi);
            const bool keep = m2 > tau * tau;
            const float rm = __builtin_amdgcn_rsqf(keep ? m2 : 1.0f);
            // shrunk coefficient, with the inverse transform's 1/sqrt(NT) folded in
            const float sc = keep ? fmaf(-tau, rm, 1.0f) * scale : 0.0f;
            x[k] = make_float2(zr * sc, zi * sc);
            l1 = fmaf(omw, keep ? fmaf(m2, rm, -tau) : 0.f, l1);
            if (a.supp) a.supp[(size_t)k * N + v] = keep ? 255 : 0;
        }
        dft<NT, true>(x);
#pragma unroll
        for (int f = 0; f < NT; ++f) a.Sout[(size_t)f * N + v] = x[f];
    }
    const double sum = block_sum<256>((double)l1, red);
    if (threadIdx.x == 0) a.part[blockIdx.x] = sum;
}

template <int NT>
static int tfft_fft_launch(const SparseArgs& a0, const Batched<SparseArgs>* bt, hipStream_t s) {
    SparseArgs a = a0;
    a.blocks = sparse_tfft_blocks(a.nx * a.ny * a.nz, NT);
    const int grid = (bt && bt->grid > 0) ? bt->grid : a.blocks;
    PLS_LAUNCH(dim3(grid), dim3(256), s, a, bt, pls_tfft_fft_kernel, NT);
    return a.blocks;
}

int launch_sparse_tfft_batched(const SparseArgs& a, const Batched<SparseArgs>* bt, hipStream_t s) {
    switch (a.nt) {
        case 1: return tfft_fft_launch<1>(a, bt, s);
        case 2: return tfft_fft_launch<2>(a, bt, s);
        case 3: return tfft_fft_launch<3>(a, bt, s);
        case 4: return tfft_fft_launch<4>(a, bt, s);
        case 5: return tfft_fft_launch<5>(a, bt, s);
        case 6: return tfft_fft_launch<6>(a, bt, s);
        case 7: return tfft_fft_launch<7>(a, bt, s);
        case 8: return tfft_fft_launch<8>(a, bt, s);
        case 9: return tfft_fft_launch<9>(a, bt, s);
        case 10: return tfft_fft_launch<10>(a, bt, s);
        case 12: return tfft_fft_launch<12>(a, bt, s);
        case 14: return tfft_fft_launch<14>(a, bt, s);
        case 15: return tfft_fft_launch<15>(a, bt, s);
        case 16: return tfft_fft_launch<16>(a, bt, s);
        case 18: return tfft_fft_launch<18>(a, bt, s);
        case 20: return tfft_fft_launch<20>(a, bt, s);
        case 21: return tfft_fft_launch<21>(a, bt, s);
        case 24: return tfft_fft_launch<24>(a, bt, s);
        case 25: return tfft_fft_launch<25>(a, bt, s);
        case 27: return tfft_fft_launch<27>(a, bt, s);
        case 28: return tfft_fft_launch<28>(a, bt, s);
        case 30: return tfft_fft_launch<30>(a, bt, s);
        case 32: return tfft_fft_launch<32>(a, bt, s);
    }
    // other frame counts (a prime factor above 7): the dense product on MFMA
    SparseArgs a1 = a;
    a1.blocks = sparse_tfft_blocks(a.nx * a.ny * a.nz, a.nt);
    const int grid = (bt && bt->grid > 0) ? bt->grid : a1.blocks;
    if (a.nt <= 16)
        PLS_LAUNCH(dim3(grid), dim3(256), s, a1, bt, pls_tfft_sparse_kernel, 1);
    else
        PLS_LAUNCH(dim3(grid), dim3(256), s, a1, bt, pls_tfft_sparse_kernel, 2);
    return a1.blocks;
}

int launch_sparse_tfft(const SparseArgs& a, hipStream_t s) {
    return launch_sparse_tfft_batched(a, nullptr, s);
}

// ---------------------------------------------------------------- statistics
// stat record (doubles): [0] ||r||^2, [1] ||Y - Yold||^2, [2] ||Yold||^2, [3] weighted l1,
// [4] nuclear norm, [5] tau_L, [6] Jacobi sweeps, [7] non-finite flag, [16, 16 + nt) sigma
template <int NTH, class SRC>
__global__ void __launch_bounds__(NTH) pls_stats_kernel(SRC src) {
    static_assert(NTH == 256, "one block of 256 threads");
    if (src.skip()) return;
    const StatsArgs a = src.get();
    __shared__ double red[4];
    // each thread sums its partials b = tid + 256 m in four interleaved accumulators (m mod
    // 4, so four loads are in flight) added in a fixed order
    double p0[4] = {0.0, 0.0, 0.0, 0.0}, p1[4] = {0.0, 0.0, 0.0, 0.0};
    double p2[4] = {0.0, 0.0, 0.0, 0.0}, p3[4] = {0.0, 0.0, 0.0, 0.0};
    int b = threadIdx.x;
    for (; b + 3 * 256 < a.dc_blocks; b += 4 * 256) {
#pragma unroll
        for (int k = 0; k < 4; ++k) p0[k] += a.dc_part[b + 256 * k];
    }
    for (int k = 0; b < a.dc_blocks; b += 256, ++k) p0[k] += a.dc_part[b];
    b = threadIdx.x;
    for (; b + 3 * 256 < a.ch_blocks; b += 4 * 256) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double* q = a.ch_part + 2 * (b + 256 * k);
            p1[k] += q[0];
            p2[k] += q[1];
        }
    }
    for (int k = 0; b < a.ch_blocks; b += 256, ++k) {
        const double* q = a.ch_part + 2 * b;
        p1[k] += q[0];
        p2[k] += q[1];
    }
    b = threadIdx.x;
    for (; b + 3 * 256 < a.sp_blocks; b += 4 * 256) {
#pragma unroll
        for (int k = 0; k < 4; ++k) p3[k] += a.sp_part[b + 256 * k];
    }
    for (int k = 0; b < a.sp_blocks; b += 256, ++k) p3[k] += a.sp_part[b];
    double s0 = (p0[0] + p0[1]) + (p0[2] + p0[3]), s1 = (p1[0] + p1[1]) + (p1[2] + p1[3]);
    double s2 = (p2[0] + p2[1]) + (p2[2] + p2[3]), s3 = (p3[0] + p3[1]) + (p3[2] + p3[3]);
    s0 = block_sum<256>(s0, red);
    s1 = block_sum<256>(s1, red);
    s2 = block_sum<256>(s2, red);
    s3 = block_sum<256>(s3, red);
    if (threadIdx.x == 0) {
        a.stat[0] = s0 * a.p_scale;
        a.stat[1] = s1;
        a.stat[2] = s2;
        a.stat[3] = s3;
        const bool bad = !isfinite(s0) || !isfinite(s1) || !isfinite(s2) || !isfinite(s3) ||
                         !isfinite(a.stat[4]);
        a.stat[7] = bad ? 1.0 : 0.0;
    }
}

void launch_stats_batched(const StatsArgs& a, const Batched<StatsArgs>* bt, hipStream_t s) {
    PLS_LAUNCH(dim3(1), dim3(256), s, a, bt, pls_stats_kernel, 256);
}

// ---------------------------------------------------------------- change of the iterate
// ||Y - Yold||^2 and ||Yold||^2 for the stopping test (step (4)'s relative change), a
// streaming pass over the four image arrays.  Each thread takes pairs of elements (16-byte
// loads) in a grid-stride loop; the grid depends on n only, so the sums are deterministic.
constexpr int kChangeThreads = 256;
constexpr int kChangeMaxBlocks = 2048;

int change_blocks(long n) {
    const long pairs = (n + 1) / 2;
    const long per_block = (long)kChangeThreads * 8;   // at least 8 pairs per thread
    const long b = (pairs + per_block - 1) / per_block;
    return (int)std::min<long>(std::max<long>(b, 1), kChangeMaxBlocks);
}

// 32 registers: its waves then fit beside two waves of the data-consistency kernel it runs
// next to (240 registers each of the SIMD's 512)
template <int NTH, class SRC>
__global__ void __launch_bounds__(NTH) __attribute__((amdgpu_num_vgpr(32)))
pls_change_kernel(SRC src) {
    if (src.skip()) return;
    const ChangeArgs a = src.get();
    if ((int)blockIdx.x >= a.blocks) return;   // beyond this problem's grid (batches)
    __shared__ double red[NTH / kWave];
    double d2 = 0.0, y2 = 0.0;
    auto add = [&](float2 l, float2 sv, float2 lo, float2 so) __attribute__((always_inline)) {
        const float2 y = cadd(l, sv), yo = cadd(lo, so);
        const double dx = (double)y.x - yo.x, dy = (double)y.y - yo.y;
        d2 = fma(dx, dx, fma(dy, dy, d2));
        y2 = fma((double)yo.x, (double)yo.x, fma((double)yo.y, (double)yo.y, y2));
    };
    const long npair = a.n / 2;
    const float4* L4 = reinterpret_cast<const float4*>(a.L);
    const float4* S4 = reinterpret_cast<const float4*>(a.S);
    const float4* Lo4 = reinterpret_cast<const float4*>(a.Lold);
    const float4* So4 = reinterpret_cast<const float4*>(a.Sold);
    const long stride = (long)a.blocks * NTH;
    for (long i = (long)blockIdx.x * NTH + threadIdx.x; i < npair; i += stride) {
        const float4 l = L4[i], sv = S4[i], lo = Lo4[i], so = So4[i];
        add(make_float2(l.x, l.y), make_float2(sv.x, sv.y), make_float2(lo.x, lo.y),
            make_float2(so.x, so.y));
        add(make_float2(l.z, l.w), make_float2(sv.z, sv.w), make_float2(lo.z, lo.w),
            make_float2(so.z, so.w));
    }
    if ((a.n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        const long e = a.n - 1;
        add(a.L[e], a.S[e], a.Lold[e], a.Sold[e]);
    }
    d2 = block_sum<NTH>(d2, red);
    y2 = block_sum<NTH>(y2, red);
    if (threadIdx.x == 0) {
        a.part[2 * blockIdx.x] = d2;
        a.part[2 * blockIdx.x + 1] = y2;
    }
}

void launch_change_batched(const ChangeArgs& a0, const Batched<ChangeArgs>* bt, hipStream_t s) {
    ChangeArgs a = a0;
    a.blocks = change_blocks(a.n);
    const int grid = (bt && bt->grid > 0) ? bt->grid : a.blocks;
    PLS_LAUNCH(dim3(grid), dim3(kChangeThreads), s, a, bt, pls_change_kernel, kChangeThreads);
}

void launch_change(const ChangeArgs& a, hipStream_t s) { launch_change_batched(a, nullptr, s); }

void launch_stats(const StatsArgs& a, hipStream_t s) { launch_stats_batched(a, nullptr, s); }

}  // namespace pls
