// Step (1) of Algorithm 1, first half: the Gram matrix G = C^H C of the Casorati matrix
// C = X - S (voxels x frames), its Hermitian eigendecomposition G = V diag(sigma^2) V^H,
// and the frame-space operator W = V diag(sigma_tilde / sigma) V^H that turns the
// singular-value soft threshold (step 1) and the singular-value prior (step 2) into one
// product L = C W.
//
// The Gram is accumulated on the real-expanded matrix R = [Re C | Im C] (N x 2*16*NB) with
// MFMA: G_R = R^T R holds Re G = A^T A + B^T B and Im G = A^T B - B^T A (A = Re C,
// B = Im C).  Only the tiles on and above the diagonal are formed.
#include "pls_common.hpp"
#include "pls_kernels.hpp"
#include "prior_ls.h"

namespace pls {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kGramBlocks = 512;

template <int NB>
constexpr int npair() { return (2 * NB) * (2 * NB + 1) / 2; }

int gram_tiles(int nt) { return nt <= 16 ? npair<1>() : (nt <= 32 ? npair<2>() : npair<4>()); }

// Voxels per block for a target block count (0 = the default), a multiple of 128.
int gram_vpb(int N, int target) {
    const int t = target > 0 ? target : kGramBlocks;
    int vpb = (N + t - 1) / t;
    return (vpb + 127) / 128 * 128;
}

int gram_blocks(int N, int target) {
    const int vpb = gram_vpb(N, target);
    return (N + vpb - 1) / vpb;
}

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// Fixed-order sum of the 4 waves' FP32 16x16 accumulators, (w0 + w2) + (w1 + w3) in FP64,
// stored as FP64 partial tiles; v_mfma_f32_16x16xK output: register r of a lane holds row
// 4 (lane / 16) + r, column lane % 16.
template <int NP, bool UNUSED>
__device__ __forceinline__ void gram_block_store(const f4 (&acc)[NP], double (*red)[NP * 256],
                                                 double* part, int lane, int wave) {
    const int slot = lane;
    double d[NP][4];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int r = 0; r < 4; ++r) d[p][r] = (double)acc[p][r];
    if (wave >= 2) {
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int r = 0; r < 4; ++r) red[wave - 2][p * 256 + r * 64 + slot] = d[p][r];
    }
    __syncthreads();
    if (wave < 2) {
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int r = 0; r < 4; ++r) d[p][r] += red[wave][p * 256 + r * 64 + slot];
    }
    __syncthreads();
    if (wave == 1) {
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int r = 0; r < 4; ++r) red[0][p * 256 + r * 64 + slot] = d[p][r];
    }
    __syncthreads();
    if (wave == 0) {
        double* out = part + (size_t)blockIdx.x * NP * 256;
        const int g = lane >> 4, i16 = lane & 15;
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                out[p * 256 + (4 * g + r) * 16 + i16] = d[p][r] + red[0][p * 256 + r * 64 + slot];
    }
}

// ---------------------------------------------------------------- FP64 MFMA Gram
// Lane (i, g) = (lane % 16, lane / 16).  A wave takes chunks of 16 voxels; lane group g
// covers voxels 4g..4g+3 of the chunk, one per K step of v_mfma_f64_16x16x4.  The lane
// loads frames i and 16 + i of those voxels (32 contiguous bytes per frame).
template <int NB, class SRC>
__global__ void __launch_bounds__(256) pls_gram_f64_kernel(SRC src) {
    if (src.skip()) return;
    GramArgs a = src.get();
    constexpr int NT4 = 2 * NB;
    constexpr int NP = npair<NB>();
    __shared__ double red[2][NP * 256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i16 = lane & 15, g = lane >> 4;
    const size_t vb = (size_t)blockIdx.x * a.vox_per_block;
    if (vb >= (size_t)a.N) return;             // beyond this problem's grid (batches)
    const size_t ve = min((size_t)a.N, vb + a.vox_per_block);
    d4 acc[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) acc[p] = d4{0.0, 0.0, 0.0, 0.0};

    for (size_t cb = vb + wave * 16; cb < ve; cb += 64) {
        const size_t v = cb + 4 * g;
        float2 x[NB][4];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int f = nb * 16 + i16;
            if (f < a.nt && v < ve) {
                const float4* src = reinterpret_cast<const float4*>(a.C + (size_t)f * a.N + v);
                const float4 u0 = src[0], u1 = src[1];
                x[nb][0] = make_float2(u0.x, u0.y);
                x[nb][1] = make_float2(u0.z, u0.w);
                x[nb][2] = make_float2(u1.x, u1.y);
                x[nb][3] = make_float2(u1.z, u1.w);
            } else {
#pragma unroll
                for (int s = 0; s < 4; ++s) x[nb][s] = make_float2(0.f, 0.f);
            }
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            double op[NT4];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                op[nb] = (double)x[nb][s].x;
                op[NB + nb] = (double)x[nb][s].y;
            }
            int p = 0;
#pragma unroll
            for (int I = 0; I < NT4; ++I)
#pragma unroll
                for (int J = I; J < NT4; ++J, ++p)
                    acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(op[I], op[J], acc[p], 0, 0, 0);
        }
    }
    // fixed-order reduction over the 4 waves: (w0 + w2) + (w1 + w3)
    const int slot = lane;  // acc[p][r] -> red[.][p * 256 + r * 64 + lane]
    if (wave >= 2) {
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int r = 0; r < 4; ++r) red[wave - 2][p * 256 + r * 64 + slot] = acc[p][r];
    }
    __syncthreads();
    if (wave < 2) {
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[p][r] += red[wave][p * 256 + r * 64 + slot];
    }
    __syncthreads();
    if (wave == 1) {
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int r = 0; r < 4; ++r) red[0][p * 256 + r * 64 + slot] = acc[p][r];
    }
    __syncthreads();
    if (wave == 0) {
        double* out = a.part + (size_t)blockIdx.x * NP * 256;
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                // v_mfma_f64_16x16x4 output: register r of a lane holds row lane/16 + 4 r,
                // column lane % 16 (the f32 variant uses row 4 (lane/16) + r instead)
                const int row = g + 4 * r, col = i16;
                out[p * 256 + row * 16 + col] = acc[p][r] + red[0][p * 256 + r * 64 + slot];
            }
    }
}

// ---------------------------------------------------------------- FP32 MFMA Gram
// Same lane mapping as the FP64 kernel with v_mfma_f32_16x16x4f32; FP32 accumulation within
// a wave (a few hundred voxels per entry), FP64 across waves and blocks.
template <int NB, class SRC>
__global__ void __launch_bounds__(256) pls_gram_f32_kernel(SRC src) {
    if (src.skip()) return;
    GramArgs a = src.get();
    constexpr int NT4 = 2 * NB;
    constexpr int NP = npair<NB>();
    __shared__ double red[2][NP * 256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i16 = lane & 15, g = lane >> 4;
    const size_t vb = (size_t)blockIdx.x * a.vox_per_block;
    if (vb >= (size_t)a.N) return;             // beyond this problem's grid (batches)
    const size_t ve = min((size_t)a.N, vb + a.vox_per_block);
    f4 acc[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) acc[p] = f4{0.f, 0.f, 0.f, 0.f};
    for (size_t cb = vb + wave * 16; cb < ve; cb += 64) {
        const size_t v = cb + 4 * g;
        float2 x[NB][4];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int f = nb * 16 + i16;
            if (f < a.nt && v < ve) {
                const float4* src = reinterpret_cast<const float4*>(a.C + (size_t)f * a.N + v);
                const float4 u0 = src[0], u1 = src[1];
                x[nb][0] = make_float2(u0.x, u0.y);
                x[nb][1] = make_float2(u0.z, u0.w);
                x[nb][2] = make_float2(u1.x, u1.y);
                x[nb][3] = make_float2(u1.z, u1.w);
            } else {
#pragma unroll
                for (int s = 0; s < 4; ++s) x[nb][s] = make_float2(0.f, 0.f);
            }
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            float op[NT4];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                op[nb] = x[nb][s].x;
                op[NB + nb] = x[nb][s].y;
            }
            int p = 0;
#pragma unroll
            for (int I = 0; I < NT4; ++I)
#pragma unroll
                for (int J = I; J < NT4; ++J, ++p)
                    acc[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(op[I], op[J], acc[p], 0, 0, 0);
        }
    }
    gram_block_store<NP, false>(acc, red, a.part, lane, wave);
}

// ---------------------------------------------------------------- split-BF16 Gram
// x = hi + lo with hi = bf16(x), lo = bf16(x - hi); R^T R ~ hi^T hi + hi^T lo + lo^T hi on
// v_mfma_f32_16x16x32_bf16 (the lo^T lo term, ~2^-16 relative, is dropped).  Lane (i, g)
// holds 8 consecutive voxels 8g..8g+7 of a 32-voxel chunk for frames i and 16 + i; A and B
// use the same (lane, element) -> voxel mapping, which is all a Gram needs.
template <int NB, class SRC>
__global__ void __launch_bounds__(256) pls_gram_bf16x3_kernel(SRC src) {
    if (src.skip()) return;
    GramArgs a = src.get();
    constexpr int NT4 = 2 * NB;
    constexpr int NP = npair<NB>();
    __shared__ double red[2][NP * 256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i16 = lane & 15, g = lane >> 4;
    const size_t vb = (size_t)blockIdx.x * a.vox_per_block;
    if (vb >= (size_t)a.N) return;             // beyond this problem's grid (batches)
    const size_t ve = min((size_t)a.N, vb + a.vox_per_block);
    f4 acc[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) acc[p] = f4{0.f, 0.f, 0.f, 0.f};
    for (size_t cb = vb + wave * 32; cb < ve; cb += 128) {
        const size_t v = cb + 8 * g;
        bf8 hi[NT4], lo[NT4];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int f = nb * 16 + i16;
            float re[8], im[8];
            if (f < a.nt && v < ve) {
                const float4* src = reinterpret_cast<const float4*>(a.C + (size_t)f * a.N + v);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float4 u = src[k];
                    re[2 * k] = u.x;
                    im[2 * k] = u.y;
                    re[2 * k + 1] = u.z;
                    im[2 * k + 1] = u.w;
                }
            } else {
#pragma unroll
                for (int k = 0; k < 8; ++k) re[k] = im[k] = 0.f;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const __bf16 hr = (__bf16)re[k], hm = (__bf16)im[k];
                hi[nb][k] = hr;
                lo[nb][k] = (__bf16)(re[k] - (float)hr);
                hi[NB + nb][k] = hm;
                lo[NB + nb][k] = (__bf16)(im[k] - (float)hm);
            }
        }
        int p = 0;
#pragma unroll
        for (int I = 0; I < NT4; ++I)
#pragma unroll
            for (int J = I; J < NT4; ++J, ++p) {
                acc[p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hi[I], hi[J], acc[p], 0, 0, 0);
                acc[p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hi[I], lo[J], acc[p], 0, 0, 0);
                acc[p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lo[I], hi[J], acc[p], 0, 0, 0);
            }
    }
    gram_block_store<NP, false>(acc, red, a.part, lane, wave);
}

// ---------------------------------------------------------------- windows of 33..64 frames
// 64 frames make 8 real-expanded column blocks and 36 tiles on and above the diagonal, too
// many accumulators for one wave.  Here the 4 waves of a block split the tiles instead of
// the voxels: wave w forms tiles 9 w .. 9 w + 8 (in the order of the other kernels) over every
// voxel of the block, and writes them without a cross-wave reduction.  MODE: 0 FP64 MFMA,
// 1 FP32 MFMA, 2 split BF16 (the lane mappings and operand splits of the kernels above).
constexpr int kWideTiles = 36, kWideTilesPerWave = 9;

struct WidePairs {
    int I[kWideTiles], J[kWideTiles];
};
constexpr WidePairs wide_pairs() {
    WidePairs t{{}, {}};
    int p = 0;
    for (int i = 0; i < 8; ++i)
        for (int j = i; j < 8; ++j, ++p) {
            t.I[p] = i;
            t.J[p] = j;
        }
    return t;
}
constexpr WidePairs kWidePairs = wide_pairs();

template <int MODE, int W>
__device__ __forceinline__ void gram_wide_wave(const GramArgs& a, size_t vb, size_t ve, int lane) {
    constexpr int NB = 4, NT4 = 8, PW = kWideTilesPerWave;
    const int i16 = lane & 15, g = lane >> 4;
    using Acc = typename std::conditional<MODE == 0, d4, f4>::type;
    Acc acc[PW];
#pragma unroll
    for (int q = 0; q < PW; ++q) acc[q] = Acc{0, 0, 0, 0};
    if constexpr (MODE != 2) {
        using T = typename std::conditional<MODE == 0, double, float>::type;
        for (size_t cb = vb; cb < ve; cb += 16) {
            const size_t v = cb + 4 * g;
            float2 x[NB][4];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int f = nb * 16 + i16;
                if (f < a.nt && v < ve) {
                    const float4* src = reinterpret_cast<const float4*>(a.C + (size_t)f * a.N + v);
                    const float4 u0 = src[0], u1 = src[1];
                    x[nb][0] = make_float2(u0.x, u0.y);
                    x[nb][1] = make_float2(u0.z, u0.w);
                    x[nb][2] = make_float2(u1.x, u1.y);
                    x[nb][3] = make_float2(u1.z, u1.w);
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k) x[nb][k] = make_float2(0.f, 0.f);
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                T op[NT4];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    op[nb] = (T)x[nb][k].x;
                    op[NB + nb] = (T)x[nb][k].y;
                }
                sfor<PW>([&](auto qI) __attribute__((always_inline)) {
                    constexpr int q = decltype(qI)::value;
                    constexpr int I = kWidePairs.I[W * PW + q], J = kWidePairs.J[W * PW + q];
                    if constexpr (MODE == 0)
                        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(op[I], op[J], acc[q], 0, 0, 0);
                    else
                        acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(op[I], op[J], acc[q], 0, 0, 0);
                });
            }
        }
    } else {
        for (size_t cb = vb; cb < ve; cb += 32) {
            const size_t v = cb + 8 * g;
            bf8 hi[NT4], lo[NT4];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int f = nb * 16 + i16;
                float re[8], im[8];
                if (f < a.nt && v < ve) {
                    const float4* src = reinterpret_cast<const float4*>(a.C + (size_t)f * a.N + v);
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const float4 u = src[k];
                        re[2 * k] = u.x;
                        im[2 * k] = u.y;
                        re[2 * k + 1] = u.z;
                        im[2 * k + 1] = u.w;
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < 8; ++k) re[k] = im[k] = 0.f;
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const __bf16 hr = (__bf16)re[k], hm = (__bf16)im[k];
                    hi[nb][k] = hr;
                    lo[nb][k] = (__bf16)(re[k] - (float)hr);
                    hi[NB + nb][k] = hm;
                    lo[NB + nb][k] = (__bf16)(im[k] - (float)hm);
                }
            }
            sfor<PW>([&](auto qI) __attribute__((always_inline)) {
                constexpr int q = decltype(qI)::value;
                constexpr int I = kWidePairs.I[W * PW + q], J = kWidePairs.J[W * PW + q];
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hi[I], hi[J], acc[q], 0, 0, 0);
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hi[I], lo[J], acc[q], 0, 0, 0);
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lo[I], hi[J], acc[q], 0, 0, 0);
            });
        }
    }
    double* out = a.part + (size_t)blockIdx.x * kWideTiles * 256;
#pragma unroll
    for (int q = 0; q < PW; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            // FP64 MFMA output: register r holds row g + 4 r; FP32 / BF16: row 4 g + r
            const int row = MODE == 0 ? g + 4 * r : 4 * g + r;
            out[(W * PW + q) * 256 + row * 16 + i16] = (double)acc[q][r];
        }
}

template <int MODE, class SRC>
__global__ void __launch_bounds__(256) pls_gram_wide_kernel(SRC src) {
    if (src.skip()) return;
    GramArgs a = src.get();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const size_t vb = (size_t)blockIdx.x * a.vox_per_block;
    if (vb >= (size_t)a.N) return;             // beyond this problem's grid (batches)
    const size_t ve = min((size_t)a.N, vb + a.vox_per_block);
    switch (wave) {
        case 0: gram_wide_wave<MODE, 0>(a, vb, ve, lane); break;
        case 1: gram_wide_wave<MODE, 1>(a, vb, ve, lane); break;
        case 2: gram_wide_wave<MODE, 2>(a, vb, ve, lane); break;
        default: gram_wide_wave<MODE, 3>(a, vb, ve, lane); break;
    }
}

// Batched: every argument block must already hold vox_per_block = gram_vpb(N, target_blocks)
// (the kernel reads it from there); a0 is problem 0's block, for the launch shape.
int launch_gram_batched(int mode, const GramArgs& a0, const Batched<GramArgs>* bt, hipStream_t s) {
    GramArgs a = a0;
    const int vpb = gram_vpb(a.N, a.target_blocks);
    a.vox_per_block = vpb;
    const int own = (a.N + vpb - 1) / vpb;
    const int grid = (bt && bt->grid > 0) ? bt->grid : own;
    const bool one = a.nt <= 16;
    if (a.nt > 32) {
        if (mode == PRIOR_LS_GRAM_FP32) PLS_LAUNCH(dim3(grid), dim3(256), s, a, bt, pls_gram_wide_kernel, 1);
        else if (mode == PRIOR_LS_GRAM_BF16X3) PLS_LAUNCH(dim3(grid), dim3(256), s, a, bt, pls_gram_wide_kernel, 2);
        else PLS_LAUNCH(dim3(grid), dim3(256), s, a, bt, pls_gram_wide_kernel, 0);
    } else if (mode == PRIOR_LS_GRAM_FP32) {
        if (one) PLS_LAUNCH(dim3(grid), dim3(256), s, a, bt, pls_gram_f32_kernel, 1);
        else PLS_LAUNCH(dim3(grid), dim3(256), s, a, bt, pls_gram_f32_kernel, 2);
    } else if (mode == PRIOR_LS_GRAM_BF16X3) {
        if (one) PLS_LAUNCH(dim3(grid), dim3(256), s, a, bt, pls_gram_bf16x3_kernel, 1);
        else PLS_LAUNCH(dim3(grid), dim3(256), s, a, bt, pls_gram_bf16x3_kernel, 2);
    } else {
        if (one) PLS_LAUNCH(dim3(grid), dim3(256), s, a, bt, pls_gram_f64_kernel, 1);
        else PLS_LAUNCH(dim3(grid), dim3(256), s, a, bt, pls_gram_f64_kernel, 2);
    }
    return own;
}

int launch_gram(int mode, const GramArgs& a, hipStream_t s) {
    return launch_gram_batched(mode, a, nullptr, s);
}

// out[e] = sum over the per-block partials in a fixed order: a block covers 16 entries
// (one 128-byte row segment per partial) with 16 row groups; group g sums the partials
// b = g + 16 m into eight accumulators (m mod 8, so eight loads are in flight), adds them in
// index order, and the 16 group sums are added in group order.
template <int NTH, class SRC>
__global__ void __launch_bounds__(NTH) pls_gram_reduce_kernel(SRC src) {
    static_assert(NTH == 256, "16 row groups of 16 entries");
    if (src.skip()) return;
    const ReduceArgs ra = src.get();
    const double* part = ra.part;
    double* out = ra.out;
    const int blocks = ra.blocks, entries = ra.entries;
    __shared__ double red[16][16];
    // on the critical path while the sparse update shares the CUs: issue before its waves
    __builtin_amdgcn_s_setprio(3);
    const int le = threadIdx.x & 15, g = threadIdx.x >> 4;
    const int e = blockIdx.x * 16 + le;
    const int ec = e < entries ? e : entries - 1;
    double s[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) s[k] = 0.0;
    int b = g;
    for (; b + 7 * 16 < blocks; b += 8 * 16) {
#pragma unroll
        for (int k = 0; k < 8; ++k) s[k] += part[(size_t)(b + 16 * k) * entries + ec];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (b + 16 * k < blocks) s[k] += part[(size_t)(b + 16 * k) * entries + ec];
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) t += s[k];
    red[g][le] = t;
    __syncthreads();
    if (g == 0 && e < entries) {
        double u = 0.0;
#pragma unroll
        for (int k = 0; k < 16; ++k) u += red[k][le];
        out[e] = u;
    }
}

void launch_gram_reduce_batched(const ReduceArgs& a, const Batched<ReduceArgs>* bt, hipStream_t s) {
    PLS_LAUNCH(dim3((a.entries + 15) / 16), dim3(256), s, a, bt, pls_gram_reduce_kernel, 256);
}

void launch_gram_reduce(const double* part, int blocks, int entries, double* out, hipStream_t s) {
    launch_gram_reduce_batched(ReduceArgs{part, out, blocks, entries}, nullptr, s);
}

// ---------------------------------------------------------------- Hermitian eigensolver
// Cyclic complex Jacobi in FP64 with round-robin pair ordering (all n/2 disjoint
// rotations of a round applied at once), warm-started from the previous iteration's
// eigenvectors: A = V^H G V is then nearly diagonal and one or two sweeps suffice.
constexpr int kEigThreads = 512;    // one block of eight waves: it shares its CU with the sparse update
constexpr int kMaxSweeps = 30;

__device__ __forceinline__ double gram_real(const double* red, int NB, int c1, int c2) {
    int I = c1 / 16, J = c2 / 16, i = c1 % 16, j = c2 % 16;
    if (I > J) {
        int t = I; I = J; J = t;
        t = i; i = j; j = t;
    }
    const int NT4 = 2 * NB;
    const int p = I * NT4 - I * (I - 1) / 2 + (J - I);
    return red[p * 256 + i * 16 + j];
}

// Pair k of round r in the round-robin ordering of n (even) indices; r, k < n - 1.
__device__ __forceinline__ void rr_pair(int n, int r, int k, int& p, int& q) {
    const int m = n - 1;
    int pp = r + k;                 // < 2m
    pp = pp >= m ? pp - m : pp;
    int qq = r - k + m;             // in (0, 2m)
    qq = qq >= m ? qq - m : qq;
    p = k == 0 ? m : pp;
    q = k == 0 ? r : qq;
}

// FP64 reciprocal and reciprocal square root: hardware approximations refined by two
// Newton steps (each doubles the correct bits) instead of the IEEE division / sqrt
// sequences.  Used for the Jacobi rotation parameters only.
__device__ __forceinline__ double rcp64(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = y * fma(-x, y, 2.0);
    y = y * fma(-x, y, 2.0);
    return y;
}
__device__ __forceinline__ double rsq64(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-0.5 * x * y, y, 1.5);
    y = y * fma(-0.5 * x * y, y, 1.5);
    return y;
}

// Jacobi rotation that zeroes the (p, q) entry of a Hermitian matrix with diagonal entries
// app, aqq and off-diagonal entry (cr + i ci): J = [[cs, sn e], [-sn conj(e), cs]],
// e = c / |c|, with the tangent t of the real symmetric rotation on |c|.  cs is formed as
// 1 / sqrt(1 + t^2) and sn = t cs, so J is unitary to FP64 rounding whatever the accuracy
// of t.
__device__ __forceinline__ void jacobi_rot(double app, double aqq, double cr, double ci,
                                           double& cs, double& sn, double& er, double& ei) {
    const double ac2 = cr * cr + ci * ci;
    cs = 1.0;
    sn = 0.0;
    er = 1.0;
    ei = 0.0;
    if (ac2 > 1e-300) {
        const double inv_ac = rsq64(ac2);
        const double th = (aqq - app) * 0.5 * inv_ac;
        double t;
        if (fabs(th) > 1e150) {
            t = 0.5 * rcp64(th);
        } else {
            const double h = fma(th, th, 1.0);
            t = (th >= 0 ? 1.0 : -1.0) * rcp64(fabs(th) + h * rsq64(h));
        }
        cs = rsq64(fma(t, t, 1.0));
        sn = t * cs;
        er = cr * inv_ac;
        ei = ci * inv_ac;
    }
}

// The sums of a and b over the block, each in the fixed order of block_sum, with one pair
// of barriers for both.  red holds 2 (NT / 64) doubles.
template <int NT>
__device__ __forceinline__ void block_sum2(double& a, double& b, double* red) {
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) {
        red[w] = a;
        red[NT / kWave + w] = b;
    }
    __syncthreads();
    double sa = 0.0, sb = 0.0;
#pragma unroll
    for (int i = 0; i < NT / kWave; ++i) {
        sa += red[i];
        sb += red[NT / kWave + i];
    }
    a = sa;
    b = sb;
}

// One block of NT threads, for windows of at most NMAX frames.  With NMAX <= 32 the rotated
// matrix is double-buffered (a round reads one copy and writes the other) and every wave
// derives the round's rotations for itself, so a round needs a single block barrier.  With
// NMAX = 64 one copy of A and the eigenvectors fill most of the LDS: a round updates A in
// place (each item owns one 2x2 block of it) after a second barrier that lets every wave
// read the round's diagonal blocks first; the set-up products are staged in registers.
template <int NT, int NMAX, class SRC>
__global__ void __launch_bounds__(NT) pls_eig_kernel(SRC src) {
    if (src.skip()) return;
    const EigArgs a = src.get();
    constexpr int NW = NT / 64;
    constexpr bool DB = NMAX <= 32;
    constexpr int NBUF = DB ? 2 : 1;
    constexpr int NSTG = DB ? 1 : (NMAX * NMAX + NT - 1) / NT;   // staged set-up entries
    // Ab[0] / Ab[1]: the two copies of A (real, imaginary); Ab[1] holds T in the set-up
    __shared__ double Ab[NBUF][2][NMAX][NMAX + 1];
    __shared__ double Vr[NMAX][NMAX + 1], Vi[NMAX][NMAX + 1];
    __shared__ double rc[NW][NMAX / 2], rs[NW][NMAX / 2], rer[NW][NMAX / 2], rei[NW][NMAX / 2];
    __shared__ double red[2 * NW];
    __shared__ double sig[NMAX], phi[NMAX], phi_r[NMAX], sig_r[NMAX];
    __shared__ int rank_of[NMAX];
    double (*Ar)[NMAX + 1] = Ab[0][0];
    double (*Ai)[NMAX + 1] = Ab[0][1];
    // one block on the critical path while the sparse update fills the other CUs (and
    // possibly this one): its waves issue first
    __builtin_amdgcn_s_setprio(3);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int n = a.nt;
    const int ne = n + (n & 1);
    const int NB = n <= 16 ? 1 : (n <= 32 ? 2 : 4);
    const int NTP = 16 * NB;

    // G (complex Hermitian, n x n; padded index decoupled): into T (NMAX = 32) or A
    double (*Gr)[NMAX + 1] = DB ? Ab[NBUF - 1][0] : Ab[0][0];
    double (*Gi)[NMAX + 1] = DB ? Ab[NBUF - 1][1] : Ab[0][1];
    for (int idx = tid; idx < ne * ne; idx += NT) {
        const int i = idx / ne, j = idx % ne;
        double gr = 0.0, gi = 0.0;
        if (i < n && j < n) {
            gr = gram_real(a.gram, NB, i, j) + gram_real(a.gram, NB, NTP + i, NTP + j);
            gi = gram_real(a.gram, NB, i, NTP + j) - gram_real(a.gram, NB, j, NTP + i);
        }
        Gr[i][j] = gr;
        Gi[i][j] = gi;
        double vr = (i == j) ? 1.0 : 0.0, vi = 0.0;
        if (a.warm && i < n && j < n) {
            vr = a.V[2 * (i * n + j)];
            vi = a.V[2 * (i * n + j) + 1];
        }
        Vr[i][j] = vr;
        Vi[i][j] = vi;
    }
    __syncthreads();
    if constexpr (DB) {
        double (*Tr)[NMAX + 1] = Ab[1][0];
        double (*Ti)[NMAX + 1] = Ab[1][1];
        // A = V^H (G V): first G V into Ar, then V^H (.) into Tr.  A thread forms a 2 x 2
        // block of entries (ne is even), so that each operand it reads from LDS serves two
        // entries; every entry is summed over k in order, as one entry per thread would.
        const int hb = ne / 2;
        for (int b = tid; b < hb * hb; b += NT) {
            const int i0 = 2 * (b / hb), j0 = 2 * (b % hb);
            double sr[2][2] = {}, si[2][2] = {};
            for (int k = 0; k < ne; ++k) {
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const double tr = Tr[i0 + a][k], ti = Ti[i0 + a][k];
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        sr[a][c] += tr * Vr[k][j0 + c] - ti * Vi[k][j0 + c];
                        si[a][c] += tr * Vi[k][j0 + c] + ti * Vr[k][j0 + c];
                    }
                }
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    Ar[i0 + a][j0 + c] = sr[a][c];
                    Ai[i0 + a][j0 + c] = si[a][c];
                }
        }
        __syncthreads();
        for (int b = tid; b < hb * hb; b += NT) {
            const int i0 = 2 * (b / hb), j0 = 2 * (b % hb);
            double sr[2][2] = {}, si[2][2] = {};
            for (int k = 0; k < ne; ++k) {
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const double vr = Vr[k][i0 + a], vi = Vi[k][i0 + a];
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        // conj(V[k][i]) * (GV)[k][j]
                        sr[a][c] += vr * Ar[k][j0 + c] + vi * Ai[k][j0 + c];
                        si[a][c] += vr * Ai[k][j0 + c] - vi * Ar[k][j0 + c];
                    }
                }
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    Tr[i0 + a][j0 + c] = sr[a][c];
                    Ti[i0 + a][j0 + c] = si[a][c];
                }
        }
        __syncthreads();
        for (int idx = tid; idx < ne * ne; idx += NT) {
            const int i = idx / ne, j = idx % ne;
            // symmetrise: A = (T + T^H) / 2
            Ar[i][j] = 0.5 * (Tr[i][j] + Tr[j][i]);
            Ai[i][j] = (i == j) ? 0.0 : 0.5 * (Ti[i][j] - Ti[j][i]);
        }
        __syncthreads();
    } else {
        // the same products with A as the only matrix buffer: each thread forms its entries
        // in registers, and writes them after a barrier
        double sr[NSTG], si[NSTG];
#pragma unroll
        for (int q = 0; q < NSTG; ++q) {
            const int idx = tid + q * NT;
            sr[q] = si[q] = 0.0;
            if (idx < ne * ne) {
                const int i = idx / ne, j = idx % ne;
                for (int k = 0; k < ne; ++k) {   // (G V)[i][j]
                    sr[q] += Ar[i][k] * Vr[k][j] - Ai[i][k] * Vi[k][j];
                    si[q] += Ar[i][k] * Vi[k][j] + Ai[i][k] * Vr[k][j];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NSTG; ++q) {
            const int idx = tid + q * NT;
            if (idx < ne * ne) {
                Ar[idx / ne][idx % ne] = sr[q];
                Ai[idx / ne][idx % ne] = si[q];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NSTG; ++q) {
            const int idx = tid + q * NT;
            sr[q] = si[q] = 0.0;
            if (idx < ne * ne) {
                const int i = idx / ne, j = idx % ne;
                for (int k = 0; k < ne; ++k) {   // conj(V[k][i]) * (GV)[k][j]
                    sr[q] += Vr[k][i] * Ar[k][j] + Vi[k][i] * Ai[k][j];
                    si[q] += Vr[k][i] * Ai[k][j] - Vi[k][i] * Ar[k][j];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NSTG; ++q) {
            const int idx = tid + q * NT;
            if (idx < ne * ne) {
                Ar[idx / ne][idx % ne] = sr[q];
                Ai[idx / ne][idx % ne] = si[q];
            }
        }
        __syncthreads();
        // symmetrise: A = (A + A^H) / 2, read before written
#pragma unroll
        for (int q = 0; q < NSTG; ++q) {
            const int idx = tid + q * NT;
            sr[q] = si[q] = 0.0;
            if (idx < ne * ne) {
                const int i = idx / ne, j = idx % ne;
                sr[q] = 0.5 * (Ar[i][j] + Ar[j][i]);
                si[q] = (i == j) ? 0.0 : 0.5 * (Ai[i][j] - Ai[j][i]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NSTG; ++q) {
            const int idx = tid + q * NT;
            if (idx < ne * ne) {
                Ar[idx / ne][idx % ne] = sr[q];
                Ai[idx / ne][idx % ne] = si[q];
            }
        }
        __syncthreads();
    }

    const int half = ne / 2;
    int sweeps = 0, cur = 0;
    for (; sweeps < kMaxSweeps && ne > 1; ++sweeps) {
        double (*Cr)[NMAX + 1] = Ab[cur][0];
        double (*Ci)[NMAX + 1] = Ab[cur][1];
        double off = 0.0, dg = 0.0;
        for (int idx = tid; idx < ne * ne; idx += NT) {
            const int i = idx / ne, j = idx % ne;
            if (i == j) dg += Cr[i][i] * Cr[i][i];
            else off += Cr[i][j] * Cr[i][j] + Ci[i][j] * Ci[i][j];
        }
        block_sum2<NT>(off, dg, red);
        // relative off-diagonal norm below 1e-8: eigenvector errors of that order (times
        // the inverse gap) are far below the FP32 resolution of W
        if (!(off > 1e-16 * dg)) break;   // also stops on NaN
        for (int r = 0; r < ne - 1; ++r) {
            double (*Sr)[NMAX + 1] = Ab[cur][0];
            double (*Si)[NMAX + 1] = Ab[cur][1];
            double (*Dr)[NMAX + 1] = Ab[DB ? cur ^ 1 : cur][0];
            double (*Di)[NMAX + 1] = Ab[DB ? cur ^ 1 : cur][1];
            // this wave's copy of the round's rotations (every wave computes the same ones).
            // Their inputs are read first (every lane reads a valid pair), then, with
            // NMAX <= 32, this thread's item entries, which arrive while the rotations'
            // dependent arithmetic runs (the LDS returns a wave's reads in issue order)
            int rp, rq;
            rr_pair(ne, r, lane < half ? lane : 0, rp, rq);
            const double rapp = Sr[rp][rp], raqq = Sr[rq][rq], rcr = Sr[rp][rq], rci = Si[rp][rq];
            const bool has_a = DB && tid < half * half, has_v = DB && tid < ne * half;
            int ip = 0, iq = 0, iu = 0, iw = 0, ial = 0, ibe = 0, vi = 0, vu = 0, vw = 0, vbe = 0;
            double e00r = 0, e00i = 0, e01r = 0, e01i = 0, e10r = 0, e10i = 0, e11r = 0, e11i = 0;
            double w0r = 0, w0i = 0, w1r = 0, w1i = 0;
            if constexpr (DB) {
                // S is read-only this round and a V entry belongs to one item: the entries
                // do not depend on the rotations.  Absent items read item 0.
                const int ia = has_a ? tid : 0;
                ial = ia / half;
                ibe = ia % half;
                rr_pair(ne, r, ial, ip, iq);
                rr_pair(ne, r, ibe, iu, iw);
                e00r = Sr[ip][iu]; e00i = Si[ip][iu]; e01r = Sr[ip][iw]; e01i = Si[ip][iw];
                e10r = Sr[iq][iu]; e10i = Si[iq][iu]; e11r = Sr[iq][iw]; e11i = Si[iq][iw];
                const int iv = has_v ? tid : 0;
                vi = iv / half;
                vbe = iv % half;
                rr_pair(ne, r, vbe, vu, vw);
                w0r = Vr[vi][vu]; w0i = Vi[vi][vu]; w1r = Vr[vi][vw]; w1i = Vi[vi][vw];
            }
            if (lane < half) {
                double cs, sn, er, ei;
                jacobi_rot(rapp, raqq, rcr, rci, cs, sn, er, ei);
                rc[wv][lane] = cs;
                rs[wv][lane] = sn;
                rer[wv][lane] = er;
                rei[wv][lane] = ei;
            }
            // the LDS executes a wave's accesses in issue order: keep the compiler from
            // moving the reads below above the writes
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // one copy of A: every wave has read the diagonal blocks it needs before any
            // item overwrites them
            if constexpr (!DB) __syncthreads();
            // D = J^H S J on every 2x2 block; J = [[cs, sn e], [-sn conj(e), cs]].  An A item
            // (al, be) < (half, half) rotates one 2x2 block of S into D; a V item (i, be)
            // rotates two entries of row i of V in place.  Each item's reads come first and
            // its writes last, so the caller can interleave two items.
            struct AItem {
                int p, q, u, w;
                bool diag;
                double c1, s1, e1r, e1i, c2, s2, e2r, e2i;
                double b00r, b00i, b01r, b01i, b10r, b10i, b11r, b11i;
            };
            struct VItem {
                int i, u, w;
                double c2, s2, e2r, e2i, v0r, v0i, v1r, v1i;
            };
            auto a_load = [&](int idx) __attribute__((always_inline)) {
                AItem x;
                const int al = idx / half, be = idx % half;
                rr_pair(ne, r, al, x.p, x.q);
                rr_pair(ne, r, be, x.u, x.w);
                x.diag = al == be;
                x.c1 = rc[wv][al]; x.s1 = rs[wv][al]; x.e1r = rer[wv][al]; x.e1i = rei[wv][al];
                x.c2 = rc[wv][be]; x.s2 = rs[wv][be]; x.e2r = rer[wv][be]; x.e2i = rei[wv][be];
                x.b00r = Sr[x.p][x.u]; x.b00i = Si[x.p][x.u]; x.b01r = Sr[x.p][x.w]; x.b01i = Si[x.p][x.w];
                x.b10r = Sr[x.q][x.u]; x.b10i = Si[x.q][x.u]; x.b11r = Sr[x.q][x.w]; x.b11i = Si[x.q][x.w];
                return x;
            };
            auto a_finish = [&](const AItem& x) __attribute__((always_inline)) {
                const double c1 = x.c1, s1 = x.s1, e1r = x.e1r, e1i = x.e1i;
                const double c2 = x.c2, s2 = x.s2, e2r = x.e2r, e2i = x.e2i;
                // X = J1^H B, J1^H = [[c1, -s1 e1], [s1 conj(e1), c1]]
                const double x00r = c1 * x.b00r - s1 * (e1r * x.b10r - e1i * x.b10i);
                const double x00i = c1 * x.b00i - s1 * (e1r * x.b10i + e1i * x.b10r);
                const double x01r = c1 * x.b01r - s1 * (e1r * x.b11r - e1i * x.b11i);
                const double x01i = c1 * x.b01i - s1 * (e1r * x.b11i + e1i * x.b11r);
                const double x10r = s1 * (e1r * x.b00r + e1i * x.b00i) + c1 * x.b10r;
                const double x10i = s1 * (e1r * x.b00i - e1i * x.b00r) + c1 * x.b10i;
                const double x11r = s1 * (e1r * x.b01r + e1i * x.b01i) + c1 * x.b11r;
                const double x11i = s1 * (e1r * x.b01i - e1i * x.b01r) + c1 * x.b11i;
                // Y = X J2: Y[:,0] = X[:,0] c2 - X[:,1] s2 conj(e2); Y[:,1] = X[:,0] s2 e2 + X[:,1] c2
                double y00r = c2 * x00r - s2 * (x01r * e2r + x01i * e2i);
                double y00i = c2 * x00i - s2 * (x01i * e2r - x01r * e2i);
                double y10r = c2 * x10r - s2 * (x11r * e2r + x11i * e2i);
                double y10i = c2 * x10i - s2 * (x11i * e2r - x11r * e2i);
                double y01r = s2 * (x00r * e2r - x00i * e2i) + c2 * x01r;
                double y01i = s2 * (x00r * e2i + x00i * e2r) + c2 * x01i;
                double y11r = s2 * (x10r * e2r - x10i * e2i) + c2 * x11r;
                double y11i = s2 * (x10r * e2i + x10i * e2r) + c2 * x11i;
                if (x.diag) {
                    y01r = y01i = y10r = y10i = 0.0;
                    y00i = y11i = 0.0;
                }
                Dr[x.p][x.u] = y00r; Di[x.p][x.u] = y00i;
                Dr[x.p][x.w] = y01r; Di[x.p][x.w] = y01i;
                Dr[x.q][x.u] = y10r; Di[x.q][x.u] = y10i;
                Dr[x.q][x.w] = y11r; Di[x.q][x.w] = y11i;
            };
            auto v_load = [&](int idx) __attribute__((always_inline)) {
                VItem x;
                x.i = idx / half;
                const int be = idx % half;
                rr_pair(ne, r, be, x.u, x.w);
                x.c2 = rc[wv][be]; x.s2 = rs[wv][be]; x.e2r = rer[wv][be]; x.e2i = rei[wv][be];
                x.v0r = Vr[x.i][x.u]; x.v0i = Vi[x.i][x.u]; x.v1r = Vr[x.i][x.w]; x.v1i = Vi[x.i][x.w];
                return x;
            };
            // V <- V J
            auto v_finish = [&](const VItem& x) __attribute__((always_inline)) {
                Vr[x.i][x.u] = x.c2 * x.v0r - x.s2 * (x.v1r * x.e2r + x.v1i * x.e2i);
                Vi[x.i][x.u] = x.c2 * x.v0i - x.s2 * (x.v1i * x.e2r - x.v1r * x.e2i);
                Vr[x.i][x.w] = x.s2 * (x.v0r * x.e2r - x.v0i * x.e2i) + x.c2 * x.v1r;
                Vi[x.i][x.w] = x.s2 * (x.v0r * x.e2i + x.v0i * x.e2r) + x.c2 * x.v1i;
            };
            if constexpr (DB) {
                // every thread takes at most one A item (half^2 <= 256) and one V item
                // (ne half <= 512), their entries loaded above; only the rotations are read
                // here
                // the launcher takes NT >= ne half, so no item is left over
                AItem xa;
                xa.p = ip; xa.q = iq; xa.u = iu; xa.w = iw;
                xa.diag = ial == ibe;
                xa.c1 = rc[wv][ial]; xa.s1 = rs[wv][ial]; xa.e1r = rer[wv][ial]; xa.e1i = rei[wv][ial];
                xa.c2 = rc[wv][ibe]; xa.s2 = rs[wv][ibe]; xa.e2r = rer[wv][ibe]; xa.e2i = rei[wv][ibe];
                xa.b00r = e00r; xa.b00i = e00i; xa.b01r = e01r; xa.b01i = e01i;
                xa.b10r = e10r; xa.b10i = e10i; xa.b11r = e11r; xa.b11i = e11i;
                VItem xv;
                xv.i = vi; xv.u = vu; xv.w = vw;
                xv.c2 = rc[wv][vbe]; xv.s2 = rs[wv][vbe]; xv.e2r = rer[wv][vbe]; xv.e2i = rei[wv][vbe];
                xv.v0r = w0r; xv.v0i = w0i; xv.v1r = w1r; xv.v1i = w1i;
                if (has_a) a_finish(xa);
                if (has_v) v_finish(xv);
            } else {
                for (int it = tid; it < half * half + ne * half; it += NT) {
                    if (it < half * half) a_finish(a_load(it));
                    else v_finish(v_load(it - half * half));
                }
            }
            // every entry of D was written (the pairs partition the indices); the next round
            // reads D and overwrites S, whose last readers are behind this barrier
            __syncthreads();
            if constexpr (DB) cur ^= 1;
        }
    }
    double (*Acur)[NMAX + 1] = Ab[cur][0];

    // spectrum, descending ranks (ties broken by index), thresholds
    if (tid < n) sig[tid] = sqrt(fmax(Acur[tid][tid], 0.0));
    __syncthreads();
    if (tid < n) {
        int rk = 0;
        const double si = sig[tid];
        for (int j = 0; j < n; ++j) rk += (sig[j] > si) || (sig[j] == si && j < tid);
        rank_of[tid] = rk;
    }
    __syncthreads();
    double s1 = 0.0;
    for (int j = 0; j < n; ++j) s1 = fmax(s1, sig[j]);
    const double tau = a.relative ? a.lambda_L * s1 : a.lambda_L;
    double nuc_part = 0.0;
    if (tid < n) {
        const double sg = sig[tid];
        const double hat = fmax(sg - tau, 0.0);
        const double prev = a.sigma_prev ? a.sigma_prev[rank_of[tid]] : 0.0;
        double tgt = hat - a.lambda_p * (hat - prev);
        if (sg <= 1e-3 * s1) tgt = 0.0;
        const double ph = sg > 0.0 ? tgt / sg : 0.0;
        phi[tid] = ph;
        nuc_part = tgt;
        // this frame's factors of the nuclear norm, at its rank
        phi_r[rank_of[tid]] = ph;
        sig_r[rank_of[tid]] = sg;
        a.stat[16 + rank_of[tid]] = sg;
        if (a.sigL) a.sigL[rank_of[tid]] = tgt;
    }
    __syncthreads();
    // nuclear norm summed in rank order for determinism (the terms are independent loads)
    if (tid == 0) {
        double nuc = 0.0;
        for (int k = 0; k < n; ++k) nuc += phi_r[k] * sig_r[k];
        a.stat[4] = nuc;
        a.stat[5] = tau;
        a.stat[6] = (double)sweeps;
    }
    (void)nuc_part;
    // W = V diag(phi) V^H and its real-expanded MFMA operand.  A thread forms a 2 x 2 block
    // of entries (NTP is even), each summed over k in order.
    const int K2 = 2 * NTP;
    const int hw = NTP / 2;
    for (int b = tid; b < hw * hw; b += NT) {
        const int t0 = 2 * (b / hw), j0 = 2 * (b % hw);
        double wr[2][2] = {}, wi[2][2] = {};
        for (int k = 0; k < n; ++k) {
            const double pk = phi[k];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                // V[t][k] phi_k conj(V[j][k]); rows at or beyond n hold zeros of W
                const double pr = Vr[t0 + e][k] * pk, pi = Vi[t0 + e][k] * pk;
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    wr[e][c] += pr * Vr[j0 + c][k] + pi * Vi[j0 + c][k];
                    wi[e][c] += pi * Vr[j0 + c][k] - pr * Vi[j0 + c][k];
                }
            }
        }
#pragma unroll
        for (int e = 0; e < 2; ++e)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int t = t0 + e, j = j0 + c;
                const bool in = t < n && j < n;
                const double vr = in ? wr[e][c] : 0.0, vi = in ? wi[e][c] : 0.0;
                if (in) {
                    a.Wd[2 * (t * n + j)] = vr;
                    a.Wd[2 * (t * n + j) + 1] = vi;
                }
                // Wr[k][o]: k = input (Re frames 0..NTP-1, Im frames NTP..), o = output
                // likewise.  A operand = Wr^T: Aop[o][k]
                const float fr = (float)vr, fi = (float)vi;
                a.Wop[(j)*K2 + t] = fr;               // Wr[t][j]         =  Re W
                a.Wop[(j)*K2 + NTP + t] = -fi;        // Wr[NTP+t][j]     = -Im W
                a.Wop[(NTP + j) * K2 + t] = fi;       // Wr[t][NTP+j]     =  Im W
                a.Wop[(NTP + j) * K2 + NTP + t] = fr; // Wr[NTP+t][NTP+j] =  Re W
            }
    }
    for (int idx = tid; idx < n * n; idx += NT) {
        const int i = idx / n, j = idx % n;
        a.V[2 * idx] = Vr[i][j];
        a.V[2 * idx + 1] = Vi[i][j];
    }
}

// With NMAX <= 32 a thread takes at most one A item and one V item per round, so the block
// needs ne half <= NT threads (ne = nt rounded up to even).  Fewer waves make the round's
// block barrier cheaper: windows of up to 16 frames take two waves (4-18% faster than eight
// at nt = 3..16), one problem of 17..24 frames five (about 5% faster at nt = 24); results
// are the same bit for bit.  A batch holds one tile class, so problem 0's nt bounds every
// member's only up to 16 frames: batches of 17..32 frames keep eight waves.
void launch_eig_batched(const EigArgs& a, const Batched<EigArgs>* bt, hipStream_t s) {
    const int ne = a.nt + (a.nt & 1);
    if (a.nt <= 16) PLS_LAUNCH(dim3(1), dim3(128), s, a, bt, pls_eig_kernel, 128, 16);
    else if (a.nt <= 32 && !bt && ne * (ne / 2) <= 320)
        PLS_LAUNCH(dim3(1), dim3(320), s, a, bt, pls_eig_kernel, 320, 32);
    else if (a.nt <= 32) PLS_LAUNCH(dim3(1), dim3(kEigThreads), s, a, bt, pls_eig_kernel, kEigThreads, 32);
    else PLS_LAUNCH(dim3(1), dim3(kEigThreads), s, a, bt, pls_eig_kernel, kEigThreads, 64);
}

void launch_eig(const EigArgs& a, hipStream_t s) {
    launch_eig_batched(a, nullptr, s);
}

}  // namespace pls
