// Data consistency, step (4) of Algorithm 1, and the set-up kx inverse DFT.
//
// For a Cartesian mask that is constant along kx, F^H m F = F_yz^H m F_yz per x plane,
// so with the data taken once through the unitary kx-IDFT (dh, see pls_xifft) the
// normal operator needs only 2D (y, z) FFTs.  One block owns PB (t, x) planes and, for
// every coil c, forms C_c Y, transforms it, replaces the sampled entries by the residual
// F(C_c Y) - dh and zeroes the rest, transforms back and accumulates conj(C_c) times the
// result.  It writes C = L - sum_c conj(C_c) F^H(m F(C_c Y) - dh) = M - S.
#pragma once

#include "pls_fft.hpp"
#include "pls_kernels.hpp"

namespace pls {

template <int NY, int NZ>
struct DcCfg {
    static constexpr int P = NY * NZ;
    static constexpr bool kHas3 = (NY % 3 == 0);
    static constexpr bool kHas7 = (NZ % 7 == 0);      // nz = 14: radix 14 = 2 x 7 along z
    // planes of 6144+ points with a factor 3 take 24 points per thread: two passes per axis
    // (e.g. 192 = 8 x 24, 32 = 4 x 8) instead of three, at 256 registers and 2 waves/SIMD
    static constexpr bool kWide = kHas3 && !kHas7 && P >= 24 * 256;
    static constexpr int Q0 = kHas7 ? 28 : (kWide ? 24 : (kHas3 ? 12 : 16));
    static constexpr int Q = (P / Q0 > 512) ? P / 512 : Q0;
    // blocks of 256 threads (128 for planes under 1024 points): smaller planes share a
    // block, which measured 7-34% faster than one 128-thread block per plane
    static constexpr int TT = (P >= 1024) ? 256 : 128;
    static constexpr int PB = (P / Q >= TT) ? 1 : (TT * Q) / P;
    static constexpr int T = PB * P / Q;
    // Y = L + S is parked in the output array between coils (not kept in registers), and
    // the frame's sample indices of the thread's points stay in registers (two per
    // register) instead of being looked up in LDS for every coil
    // LDS rows carry one unused point per 16 (Geom YSW = 16): the first pass of each y
    // transform (stage length 1) writes butterfly j's points to y = j R + r, a stride of R
    // points, and with unpadded rows of a power-of-two length a stride of 8 or 16 points put
    // the lanes of a write on the same few banks.  Measured on one data-consistency pass
    // (same outputs bit for bit): 128x16 planes -7% (1 coil) and -14% (4 coils), 64x8 -4% /
    // -10%, 192x32 x 8 coils -3%.  Not for nz = 14 (its 28-point tile then spills
    // registers, +10%) nor the 12-point 192-wide planes (no conflicts to remove).  Rows are
    // PADY points longer still where that spreads the row-to-row lanes of a pass further.
    static constexpr int YSW = (kHas7 || (NY == 192 && Q == 12)) ? 0 : 16;
    static constexpr int PADY = YSW == 0 ? 0 : (Q == 24 ? 12 : (NY == 48 ? 4 : (NY == 96 ? 2 : 0)));
    // waves per SIMD the register allocation must allow: 2, except the 28-point tiles of
    // nz = 14 with rows of 16 or 32 (8 and 16 planes per block), which spill to scratch at
    // 2 and measured faster at 1 with the overflow in AGPRs (same outputs bit for bit): 16x14
    // -4%, 32x14 -24%; 64x14 and 128x14 measured 18-40% slower that way and keep 2
    static constexpr int MINW = (kHas7 && NY <= 32) ? 1 : 2;
    using G = Geom<NY, NZ, PB, Q, PADY, 32, MINW, YSW>;
};

// Register distribution of a first pass of radix R along axis AX: element (i, r) of a
// thread sits at plane-batch offset rel + r * STEP of plane pb (unpadded global layout).
template <class G, int AX, int R>
struct Dist {
    using M = PassMap<G, AX, R>;
    static constexpr int NB = M::NB;
    static constexpr int JN = M::JN;
    static constexpr int STEP = (AX == 0) ? JN : JN * G::NY;
    int pb[NB];     // plane of the batch
    int rel[NB];    // offset inside the plane of element (i, 0)
    __device__ __forceinline__ Dist(int tid) {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            int line, j;
            M::map(tid, i, line, j);
            if constexpr (AX == 0) {
                pb[i] = line / G::NZ;
                rel[i] = (line % G::NZ) * G::NY + j;
            } else {
                pb[i] = line / G::NY;
                rel[i] = j * G::NY + (line % G::NY);
            }
        }
    }
};

template <class G, class SRC>
__global__ void __launch_bounds__(G::T, G::MINW) pls_dc_kernel(SRC src) {
    if (src.skip()) return;
    const DcArgs a = src.get();
    if ((int)blockIdx.x >= a.blocks) return;   // beyond this problem's grid (batches)
    constexpr int Q = G::Q, P = G::P, NY = G::NY, NZ = G::NZ, PB = G::PB, T = G::T;
    constexpr int R0 = radix_in<G>();
    constexpr int RL = radix_out<G>();
    constexpr int AXL = G::NPZ > 0 ? 1 : 0;
    // staged compact data of one coil (all planes of the batch); one buffer suffices when
    // the transform has block barriers (see the coil loop), else two alternate
    constexpr int NST = (PB * P < 1024) ? PB * P : 1024;
    constexpr int NSTT = (NST + T - 1) / T;   // staged entries per thread
    constexpr int NBUF = (G::NPZ > 0) ? 1 : 2;
    using D0 = Dist<G, 0, R0>;
    using DL = Dist<G, AXL, RL>;
    __shared__ float2 lds[G::LDS_ELEMS];
    __shared__ float2 twt[G::TW_ELEMS];      // per-pass twiddle tables
    __shared__ float2 dhs[NBUF][NST];
    __shared__ double red[T / kWave];
    const int tid = threadIdx.x;
    tw_fill<G>(twt, a.twy, a.twz, tid);

    // Blocks are dealt round-robin to the 8 XCDs; renumber them so that each XCD works on a
    // contiguous range of (x, t) planes and the coil maps of an x plane stay in its L2.
    const int nb = a.blocks;
    const int lb = (nb % 8 == 0) ? (blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8 : blockIdx.x;
    const int t = lb % a.nt;
    const int x0 = (lb / a.nt) * PB;
    const int nvalid = a.nx - x0;              // planes of this batch that exist (>= 1)
    const int pbv = nvalid < PB ? nvalid : PB;
    const int plane0 = (t * a.nx + x0) * P;    // element offset of plane (t, x0)
    // Loads are issued unconditionally from always-valid addresses and blended with uniform
    // selects, so the compiler can issue a whole group before waiting: absent operands read
    // a valid stand-in array whose value is then discarded by a select (never multiplied,
    // so whatever the stand-in holds cannot leak in).
    const bool has_y = (a.L != nullptr);
    const bool has_s = has_y && (a.S != nullptr);
    const float2* Lp = has_y ? a.L : a.C;
    const float2* Sp = has_s ? a.S : Lp;
    const D0 d0(tid);
    const int nst = a.ns[t];
    const float2* dh_t = a.dh + a.dh_off[t];
    const int16_t* sid_t = a.sidx + t * P;
    // sample index (or -1) of each point of the thread in the distribution the forward
    // transform leaves, packed two per register; -1 also marks points of absent planes
    static_assert(Q % 2 == 0, "sample indices are packed in pairs");
    uint32_t sidp[Q / 2];
    {
        const DL dl(tid);
#pragma unroll
        for (int i = 0; i < DL::NB; ++i) {
            const bool ok = dl.pb[i] < nvalid;
#pragma unroll
            for (int r = 0; r < RL; ++r) {
                const int q = i * RL + r;
                const int sv = ok ? (int)sid_t[dl.rel[i] + r * DL::STEP] : -1;
                const uint32_t h = (uint32_t)sv & 0xffffu;
                if (q % 2 == 0) sidp[q / 2] = h;
                else sidp[q / 2] |= h << 16;
            }
        }
    }
    // the compact data of coil c for the batch: entry pb * nst + s, contiguous in memory when
    // PB == 1 (index (x * nc + c) * nst + s)
    const bool staged = pbv * nst <= NST;
    auto stage_load = [&](int c, float2 (&buf)[NSTT]) __attribute__((always_inline)) {
#pragma unroll
        for (int k = 0; k < NSTT; ++k) {
            const int e0 = tid + k * T;
            const bool in = staged && e0 < pbv * nst;
            const int e = in ? e0 : 0;                 // unused entries read a valid address
            const int pb = nst > 0 ? e / nst : 0;
            const int s = e - pb * nst;
            const float2 d = dh_t[((x0 + pb) * a.nc + c) * nst + s];
            buf[k] = in ? d : make_float2(0.f, 0.f);
        }
    };
    float2 dnext[NSTT];
    stage_load(0, dnext);

    float2 acc[Q], v[Q];
    // Y = L + S at element gi
    auto form_y = [&](int gi) __attribute__((always_inline)) {
        const float2 l = Lp[gi], sv = Sp[gi];
        float2 yv = has_s ? cadd(l, sv) : l;
        if (!has_y) yv = make_float2(0.f, 0.f);
        return yv;
    };
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[q] = make_float2(0.f, 0.f);

    double res2 = 0.0;
    __syncthreads();  // twiddle tables and sample map visible
    for (int c = 0; c < a.nc; ++c) {
        const int tidc = opaque(tid);
        const D0 e0(tidc);
        const DL el(tidc);
        const int buf = (NBUF == 2) ? (c & 1) : 0;
        // stage coil c's compact data (loaded one coil ahead) and fetch coil c + 1's.  With
        // one buffer, its last reads (the previous coil's residual) precede the block barrier
        // inside the previous coil's inverse transform, which every wave has passed here;
        // with two, the buffer being written was last read two coils ago, before this
        // coil's barriers
#pragma unroll
        for (int k = 0; k < NSTT; ++k) {
            const int e = tidc + k * T;
            if (e < NST) dhs[buf][e] = dnext[k];
        }
        if constexpr (G::NPZ == 0) __syncthreads();   // no block barrier inside the transform
        if (c + 1 < a.nc) stage_load(c + 1, dnext);
        const float2* sc = a.sens + (c * a.nx + x0) * P;
#pragma unroll
        for (int i = 0; i < D0::NB; ++i) {
            const int pbc = min(e0.pb[i], nvalid - 1);
            const int o = pbc * P + e0.rel[i];
            const bool own = e0.pb[i] < nvalid;
#pragma unroll
            for (int r = 0; r < R0; ++r) {
                const int q = i * R0 + r;
                // Y = L + S is formed at the first coil and parked in the output array (each
                // thread rereads only the entries it wrote), so the later coils read one
                // array instead of two.  A single coil needs no parking; the wide
                // configurations (multi-coil volumes) park unconditionally
                float2 yv;
                const int gi = plane0 + o + r * D0::STEP;
                if (c == 0) {
                    yv = form_y(gi);
                    if (own && (Q >= 24 || a.nc > 1)) a.C[gi] = yv;
                } else {
                    yv = a.C[gi];
                }
                const float2 sv = sc[o + r * D0::STEP];
                v[q] = cmul(sv, yv);
            }
        }
        // rows of this wave were last read by this wave (previous inverse); the column
        // phases of the previous coil ended at the barrier inside fft2_inv, which also
        // orders the staging writes above before the reads below
        fft2_fwd<G>(v, lds, twt, tidc);
        // residual on the sampled entries; the compact data come from LDS when staged, else
        // from global memory (two copies of the loop under a block-uniform branch, so each
        // uses plain LDS or global loads rather than generic ones)
        auto residual = [&](auto stagedI) __attribute__((always_inline)) {
            constexpr bool kStaged = decltype(stagedI)::value;
            float r2 = 0.f;
#pragma unroll
            for (int i = 0; i < DL::NB; ++i) {
                const int pbc = min(el.pb[i], nvalid - 1);
                const float2* dh_p = dh_t + ((x0 + pbc) * a.nc + c) * nst;
#pragma unroll
                for (int r = 0; r < RL; ++r) {
                    const int q = i * RL + r;
                    const int s = (int)(int16_t)(sidp[q / 2] >> (16 * (q % 2)));
                    const int sc0 = s < 0 ? 0 : s;
                    float2 d;
                    if constexpr (kStaged) d = dhs[buf][pbc * nst + sc0];
                    else d = dh_p[sc0];
                    const bool smp = s >= 0;
                    const float2 rv = make_float2(smp ? fmaf(v[q].x, a.inv_p, -d.x) : 0.f,
                                                  smp ? fmaf(v[q].y, a.inv_p, -d.y) : 0.f);
                    r2 = fmaf(rv.x, rv.x, fmaf(rv.y, rv.y, r2));
                    v[q] = rv;
                }
            }
            res2 += (double)r2;
        };
        if (staged) residual(std::true_type{});
        else residual(std::false_type{});
        // the coil map of the accumulation is loaded before the last inverse pass, so the
        // loads are in flight during its LDS reads and arithmetic
        fft2_inv<G, 1>(v, lds, twt, tidc);
        float2 sacc[Q];
#pragma unroll
        for (int i = 0; i < D0::NB; ++i) {
            const int pbc = min(e0.pb[i], nvalid - 1);
            const int o = pbc * P + e0.rel[i];
#pragma unroll
            for (int r = 0; r < R0; ++r) sacc[i * R0 + r] = sc[o + r * D0::STEP];
        }
        fft2_inv<G, 2>(v, lds, twt, tidc);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            // acc += v conj(s), four FMAs
            acc[q].x = fmaf(v[q].x, sacc[q].x, fmaf(v[q].y, sacc[q].y, acc[q].x));
            acc[q].y = fmaf(v[q].y, sacc[q].x, fmaf(-v[q].x, sacc[q].y, acc[q].y));
        }
    }
#pragma unroll
    for (int i = 0; i < D0::NB; ++i) {
        if (d0.pb[i] < nvalid) {
            const int o = plane0 + d0.pb[i] * P + d0.rel[i];
#pragma unroll
            for (int r = 0; r < R0; ++r) {
                const int q = i * R0 + r;
                const int gi = o + r * D0::STEP;
                float2 l = Lp[gi];
                if (!has_y) l = make_float2(0.f, 0.f);
                a.C[gi] = csub(l, acc[q]);
            }
        }
    }
    const double s0 = block_sum<G::T>(res2, red);
    if (tid == 0) a.part[lb] = s0;
}

// Unitary inverse DFT along kx of every sampled (c, t, kz, ky) line, scaled by 1/sqrt(P),
// scattered into the compact hybrid layout.  A block takes PB consecutive lines (6144
// points); a line's frame, coil and sample index are looked up once (binary search of the
// line offsets) into LDS.  Lines are read whole (contiguous in kx); the results go through
// an LDS transpose so that consecutive lanes write consecutive samples s of one x (the
// lines of one (t, c) are consecutive in s).
template <int NX>
struct XiCfg {
    static constexpr int Q = DcCfg<NX, 1>::Q;
    static constexpr int PB = 6144 / NX;
    using G = Geom<NX, 1, PB, Q, 0, 32, 1>;
    static constexpr int LDT = NX + 1;   // transpose row pitch (odd: no bank-aligned columns)
};

template <int NX>
__global__ void __launch_bounds__(XiCfg<NX>::G::T) pls_xifft_kernel(XiArgs a) {
    using X = XiCfg<NX>;
    using G = typename X::G;
    constexpr int Q = G::Q, PB = G::PB, T = G::T, LDT = X::LDT;
    constexpr int R0 = radix_in<G>();
    constexpr int RL = radix_out<G>();
    constexpr int NLDS = (G::LDS_ELEMS > PB * LDT) ? G::LDS_ELEMS : PB * LDT;
    __shared__ float2 lds[NLDS];
    __shared__ float2 twt[G::TW_ELEMS];
    __shared__ long long lsrc[PB];   // per line: kspace offset of kx = 0, or -1 (no line)
    __shared__ int ldst[PB];         // per line: dh offset of x = 0
    __shared__ int lstr[PB];         // per line: dh stride between x (nc * ns[t])
    const int tid = threadIdx.x;
    tw_fill<G>(twt, a.twx, a.twx, tid);
    for (int pb = tid; pb < PB; pb += T) {
        const int line = blockIdx.x * PB + pb;
        long long src = -1;
        int dst = 0, str = 0;
        if (line < a.total_lines) {
            // frame: the last t with line_off[t] <= line (it has lines, so ns[t] > 0)
            int lo = 0, hi = a.nt - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (a.line_off[mid] <= line) lo = mid;
                else hi = mid - 1;
            }
            const int t = lo;
            const int rem = line - a.line_off[t];
            const int ns = a.ns[t];
            const int c = rem / ns;
            const int sidx = rem - c * ns;
            const int pos = a.plist[(size_t)t * a.P + sidx];
            src = ((long long)(c * a.nt + t) * a.P + pos) * NX;
            dst = a.dh_off[t] + c * ns + sidx;
            str = a.nc * ns;
        }
        lsrc[pb] = src;
        ldst[pb] = dst;
        lstr[pb] = str;
    }
    __syncthreads();
    float2 v[Q];
#pragma unroll
    for (int i = 0; i < Q / R0; ++i)
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            int pb, z, x;
            pos_in<G>(tid, i, r, pb, z, x);
            const long long src = lsrc[pb];
            const float2 val = a.kspace[src < 0 ? 0 : src + x];
            v[i * R0 + r] = src < 0 ? make_float2(0.f, 0.f) : val;
        }
    // inverse transform along the line (every pass is wave-local: NZ = 1)
    {
        constexpr int NP = G::NPY;
        sfor<NP>([&](auto pI) __attribute__((always_inline)) {
            constexpr int p = decltype(pI)::value;
            constexpr int R = G::PY.r[p];
            constexpr int LS = plan_prod(G::PY, p);
            fft_pass<G, 0, R, LS, true, p == 0, p == NP - 1, tw_find(G::TW, R, LS)>(v, lds, twt,
                                                                                   tid);
        });
    }
    // transpose through LDS: the last pass left this wave's reads done (wave-local), but
    // other waves may still read their lines, so wait for all before overwriting
    __syncthreads();
#pragma unroll
    for (int i = 0; i < Q / RL; ++i)
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            int pb, z, x;
            pass_pos<G, 0, RL>(tid, i, r, pb, z, x);
            lds[pb * LDT + x] = cscale(v[i * RL + r], a.scale);
        }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const int e = tid + k * T;          // PB * NX = Q * T entries
        const int pb = e % PB, x = e / PB;
        if (lsrc[pb] >= 0) a.dh[ldst[pb] + (size_t)x * lstr[pb]] = lds[pb * LDT + x];
    }
}

template <int NY, int NZ>
inline int dc_grid(int nx, int nt) {
    using C = DcCfg<NY, NZ>;
    return ((nx + C::PB - 1) / C::PB) * nt;
}

// bt NULL: one problem with argument block a; else the batch *bt (a: problem 0's block; the
// launch grid is bt->grid when set).  Returns this problem's (a's) block count.
template <int NY, int NZ>
inline int dc_launch_t(const DcArgs& a0, const Batched<DcArgs>* bt, hipStream_t s) {
    using G = typename DcCfg<NY, NZ>::G;
    DcArgs a = a0;
    a.blocks = dc_grid<NY, NZ>(a.nx, a.nt);
    const int grid = (bt && bt->grid > 0) ? bt->grid : a.blocks;
    PLS_LAUNCH(dim3(grid), dim3(G::T), s, a, bt, pls_dc_kernel, G);
    return a.blocks;
}

template <int NX>
inline void xifft_launch_t(const XiArgs& a, hipStream_t s) {
    using G = typename XiCfg<NX>::G;
    const int grid = (a.total_lines + G::PB - 1) / G::PB;
    if (grid > 0) hipLaunchKernelGGL((pls_xifft_kernel<NX>), dim3(grid), dim3(G::T), 0, s, a);
}

// Per-nz translation units (pls_dc_nz*.hip) instantiate the kernels; these return -1 when
// the shape is not theirs.
int dc_launch_nz1(int ny, const DcArgs& a, const Batched<DcArgs>* bt, hipStream_t s);
int dc_launch_nz4(int ny, const DcArgs& a, const Batched<DcArgs>* bt, hipStream_t s);
int dc_launch_nz8(int ny, const DcArgs& a, const Batched<DcArgs>* bt, hipStream_t s);
int dc_launch_nz14(int ny, const DcArgs& a, const Batched<DcArgs>* bt, hipStream_t s);
int dc_launch_nz16(int ny, const DcArgs& a, const Batched<DcArgs>* bt, hipStream_t s);
int dc_launch_nz32(int ny, const DcArgs& a, const Batched<DcArgs>* bt, hipStream_t s);
bool xifft_launch_any(int nx, const XiArgs& a, hipStream_t s);

}  // namespace pls

