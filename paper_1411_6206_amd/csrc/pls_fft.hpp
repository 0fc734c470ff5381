// LDS-staged mixed-radix Stockham FFT over (y, z) planes, wave64 / gfx950.
//
// A block owns PB planes of NY x NZ complex points (y fastest).  Every thread keeps
// Q points in registers.  A 1D FFT along one axis is a sequence of radix-R passes; in
// pass p (stage length Ls = product of the earlier radices on that axis) butterfly j
// of a line reads the points j + r*N/R, multiplies point r by exp(-+2 pi i k r/(Ls R))
// with k = j mod Ls, takes an R-point DFT in registers and writes point r to
// (j / Ls) Ls R + (j mod Ls) + r Ls (Stockham autosort: natural order in and out).
// Between passes the plane goes through LDS; the first pass of a transform reads the
// thread's registers and the last one leaves its result in registers.  Because the
// last pass of a transform writes exactly the positions that a first pass of the same
// radix reads, a forward transform whose last radix is the inverse transform's first
// radix hands its registers straight to the inverse (no LDS round trip), and the
// inverse's last pass returns the data in the distribution the forward pass read.
#pragma once

#include "pls_common.hpp"

namespace pls {

// ---------------------------------------------------------------- in-register DFTs
// The largest prime-power factor of R when it is a proper factor (then R / it is coprime to
// it), else 1.
constexpr int pfa_n1(int R) {
    int best = 1;
    int r = R;
    for (int p = 2; p <= r; ++p) {
        if (r % p != 0) continue;
        int q = 1;
        while (r % p == 0) {
            r /= p;
            q *= p;
        }
        if (q > best) best = q;
    }
    return best < R ? best : 1;
}
// x with a x = 1 mod m (m > 1, gcd(a, m) = 1)
constexpr int modinv_c(int a, int m) {
    for (int x = 1; x < m; ++x)
        if ((a * x) % m == 1) return x;
    return 1;
}

template <int R, bool INV>
__device__ __forceinline__ void dft(float2* x) {
    if constexpr (R == 1) {
    } else if constexpr (R == 2) {
        const float2 a = x[0], b = x[1];
        x[0] = cadd(a, b);
        x[1] = csub(a, b);
    } else if constexpr (R == 3) {
        constexpr float kS3 = 0.866025403784438646763723170752936183f;  // sqrt(3)/2
        const float2 t1 = cadd(x[1], x[2]);
        const float2 t2 = csub(x[1], x[2]);
        const float2 m1 = make_float2(fmaf(-0.5f, t1.x, x[0].x), fmaf(-0.5f, t1.y, x[0].y));
        // forward: -i * sqrt(3)/2 * t2, inverse: +i * sqrt(3)/2 * t2
        const float2 m2 = INV ? make_float2(-kS3 * t2.y, kS3 * t2.x)
                              : make_float2(kS3 * t2.y, -kS3 * t2.x);
        x[0] = cadd(x[0], t1);
        x[1] = cadd(m1, m2);
        x[2] = csub(m1, m2);
    } else if constexpr (R == 4) {
        const float2 a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
        const float2 c = cadd(x[1], x[3]), d = csub(x[1], x[3]);
        const float2 e = INV ? cmul_pi(d) : cmul_mi(d);
        x[0] = cadd(a, c);
        x[2] = csub(a, c);
        x[1] = cadd(b, e);
        x[3] = csub(b, e);
    } else if constexpr (R == 5 || R == 7) {
        // odd prime: the inputs j and R - j share their cosine terms and have opposite sine
        // terms, X[k] = x0 + sum_j cos(2 pi jk/R) (x_j + x_{R-j}) -+ i sin(2 pi jk/R)
        // (x_j - x_{R-j}), and X[R - k] takes the other sign
        constexpr int H = (R - 1) / 2;
        float2 t[H + 1], u[H + 1];
        float2 sum = x[0];
        sfor<H>([&](auto jI) __attribute__((always_inline)) {
            constexpr int j = decltype(jI)::value + 1;
            t[j] = cadd(x[j], x[R - j]);
            u[j] = csub(x[j], x[R - j]);
            sum = cadd(sum, t[j]);
        });
        float2 out[R];
        out[0] = sum;
        sfor<H>([&](auto kI) __attribute__((always_inline)) {
            constexpr int k = decltype(kI)::value + 1;
            float2 a = x[0], b = make_float2(0.f, 0.f);
            sfor<H>([&](auto jI) __attribute__((always_inline)) {
                constexpr int j = decltype(jI)::value + 1;
                constexpr double ang = 2.0 * kPi * ((j * k) % R) / R;
                constexpr float c = (float)cx_cos(ang), sn = (float)cx_sin(ang);
                a = make_float2(fmaf(c, t[j].x, a.x), fmaf(c, t[j].y, a.y));
                b = make_float2(fmaf(sn, u[j].x, b.x), fmaf(sn, u[j].y, b.y));
            });
            // forward: X[k] = a - i b, X[R - k] = a + i b; the inverse swaps them
            const float2 mib = make_float2(a.x + b.y, a.y - b.x);
            const float2 pib = make_float2(a.x - b.y, a.y + b.x);
            out[k] = INV ? pib : mib;
            out[R - k] = INV ? mib : pib;
        });
        sfor<R>([&](auto iI) __attribute__((always_inline)) { x[decltype(iI)::value] = out[decltype(iI)::value]; });
    } else if constexpr (pfa_n1(R) > 1) {
        // R = N1 N2 with N1, N2 coprime (Good-Thomas): with n = (N2 n1 + N1 n2) mod R and
        // k = (N2 E1 k1 + N1 E2 k2) mod R, E1 = N2^-1 mod N1, E2 = N1^-1 mod N2, the kernel
        // w_R^{nk} splits into w_N1^{n1 k1} w_N2^{n2 k2}: N1 DFTs of length N2, then N2 of
        // length N1, with no twiddle factors between them (the index maps are register
        // renamings)
        constexpr int N1 = pfa_n1(R), N2 = R / N1;
        constexpr int E1 = modinv_c(N2 % N1, N1), E2 = modinv_c(N1 % N2, N2);
        float2 t[R];
        sfor<N1>([&](auto aI) __attribute__((always_inline)) {
            constexpr int n1 = decltype(aI)::value;
            float2 y[N2];
            sfor<N2>([&](auto bI) __attribute__((always_inline)) {
                constexpr int n2 = decltype(bI)::value;
                y[n2] = x[(N2 * n1 + N1 * n2) % R];
            });
            dft<N2, INV>(y);
            sfor<N2>([&](auto kI) __attribute__((always_inline)) { t[n1 * N2 + decltype(kI)::value] = y[decltype(kI)::value]; });
        });
        sfor<N2>([&](auto kI) __attribute__((always_inline)) {
            constexpr int k2 = decltype(kI)::value;
            float2 z[N1];
            sfor<N1>([&](auto aI) __attribute__((always_inline)) { z[decltype(aI)::value] = t[decltype(aI)::value * N2 + k2]; });
            dft<N1, INV>(z);
            sfor<N1>([&](auto cI) __attribute__((always_inline)) {
                constexpr int k1 = decltype(cI)::value;
                x[(N2 * E1 * k1 + N1 * E2 * k2) % R] = z[k1];
            });
        });
    } else {
        // R = A B:  X[c + A d] = sum_b w_B^{bd} w_R^{bc} sum_a x[B a + b] w_A^{ac}
        constexpr int A = (R % 4 == 0) ? 4 : ((R % 2 == 0) ? 2 : ((R % 3 == 0) ? 3 : ((R % 5 == 0) ? 5 : 7)));
        constexpr int B = R / A;
        float2 t[R];
        sfor<B>([&](auto bI) __attribute__((always_inline)) {
            constexpr int b = decltype(bI)::value;
            float2 y[A];
            sfor<A>([&](auto aI) __attribute__((always_inline)) { y[decltype(aI)::value] = x[B * decltype(aI)::value + b]; });
            dft<A, INV>(y);
            sfor<A>([&](auto cI) __attribute__((always_inline)) {
                constexpr int c = decltype(cI)::value;
                t[c * B + b] = ctw<b * c, R, INV>(y[c]);
            });
        });
        sfor<A>([&](auto cI) __attribute__((always_inline)) {
            constexpr int c = decltype(cI)::value;
            float2 z[B];
            sfor<B>([&](auto bI) __attribute__((always_inline)) { z[decltype(bI)::value] = t[c * B + decltype(bI)::value]; });
            dft<B, INV>(z);
            sfor<B>([&](auto dI) __attribute__((always_inline)) { x[c + A * decltype(dI)::value] = z[decltype(dI)::value]; });
        });
    }
}

// ---------------------------------------------------------------- radix planning
struct RadixPlan {
    int n;
    int r[8];
};

constexpr int cgcd(int a, int b) { return b == 0 ? a : cgcd(b, a % b); }

// Factor N into radices that each divide Q (so every thread holds whole butterflies),
// each <= RMAX, sorted ascending.  n = -1 when impossible.
constexpr RadixPlan plan_axis(int N, int Q, int RMAX = 32) {
    RadixPlan p{0, {0, 0, 0, 0, 0, 0, 0, 0}};
    int rem = N;
    while (rem > 1) {
        int g = cgcd(rem, Q);
        if (g > RMAX) {
            int d = RMAX;
            while (d > 1 && g % d != 0) --d;
            g = d;
        }
        if (g <= 1 || p.n >= 8) {
            p.n = -1;
            return p;
        }
        p.r[p.n++] = g;
        rem /= g;
    }
    for (int i = 0; i < p.n; ++i)
        for (int j = i + 1; j < p.n; ++j)
            if (p.r[j] < p.r[i]) {
                int t = p.r[i];
                p.r[i] = p.r[j];
                p.r[j] = t;
            }
    return p;
}

constexpr int plan_prod(const RadixPlan& p, int upto) {
    int s = 1;
    for (int i = 0; i < upto; ++i) s *= p.r[i];
    return s;
}

// Stage length of the inverse pass of radix p.r[idx]: the inverse runs the radices in
// reverse order, so its stage length is the product of the radices after idx.
constexpr int plan_prod_after(const RadixPlan& p, int idx) {
    int s = 1;
    for (int u = p.n - 1; u > idx; --u) s *= p.r[u];
    return s;
}

// Per-pass twiddle tables.  A pass of radix R and stage length LS multiplies point r of
// butterfly k (k < LS) by exp(-+2 pi i k r / (LS R)); the table of that (R, LS) holds these
// factors (forward sign) at off + (r - 1) LS + k, so lanes that take consecutive butterflies
// read consecutive entries instead of a stride-r gather from the axis table.  One table
// serves every forward or inverse pass, on either axis, with the same (R, LS).
struct TwPlan {
    int n;
    int R[32], LS[32], off[32];
    int total;
};

constexpr TwPlan tw_add(TwPlan t, int R, int LS) {
    if (LS <= 1) return t;
    for (int i = 0; i < t.n; ++i)
        if (t.R[i] == R && t.LS[i] == LS) return t;
    t.R[t.n] = R;
    t.LS[t.n] = LS;
    t.off[t.n] = t.total;
    t.total += (R - 1) * LS;
    ++t.n;
    return t;
}

constexpr TwPlan tw_axis(TwPlan t, const RadixPlan& p) {
    for (int q = 1; q < p.n; ++q) t = tw_add(t, p.r[q], plan_prod(p, q));
    for (int idx = 0; idx + 1 < p.n; ++idx) t = tw_add(t, p.r[idx], plan_prod_after(p, idx));
    return t;
}

constexpr int tw_find(const TwPlan& t, int R, int LS) {
    for (int i = 0; i < t.n; ++i)
        if (t.R[i] == R && t.LS[i] == LS) return t.off[i];
    return -1;
}

// ---------------------------------------------------------------- plane geometry
template <int NY_, int NZ_, int PB_, int Q_, int PADY_, int RMAX_ = 32, int MINW_ = 1,
          int YSW_ = 0>
struct Geom {
    static constexpr int NY = NY_, NZ = NZ_, PB = PB_, Q = Q_;
    static constexpr int MINW = MINW_;   // launch bound: minimum waves per SIMD
    static constexpr int P = NY * NZ;
    static constexpr int T = PB * P / Q;
    // LDS layout: plane pb, row z, column y at pb * PS + z * LDY + ycol(y).  With YSW = 0
    // ycol(y) = y; with YSW = 16 one unused point follows every 16 points of a row,
    // ycol(y) = y + y / 16, so that the stride-R writes of a radix-R pass of stage length 1
    // (butterfly j writes y = j R + r) spread over the banks.  Every access of a pass is a
    // per-butterfly base plus a compile-time offset (ds_read/ds_write immediate); the padded
    // rows need a second base where a butterfly's points straddle a padding point (YCarry).
    // Rows are PADY points longer still.
    static constexpr int YSW = YSW_;
    static_assert(YSW == 0 || YSW == 16, "row padding: none or one point per 16");
    static constexpr int LDY = NY + (YSW > 0 ? NY / YSW : 0) + PADY_;
    __device__ static __forceinline__ int ycol(int y) { return YSW > 0 ? y + (y >> 4) : y; }
    static constexpr int PS = LDY * NZ;
    static constexpr int LDS_ELEMS = PS * PB;
    static constexpr RadixPlan PY = plan_axis(NY, Q, RMAX_);
    static constexpr RadixPlan PZ = plan_axis(NZ, Q, RMAX_);
    static constexpr int NPY = PY.n;
    static constexpr int NPZ = PZ.n;
    static constexpr TwPlan TW = tw_axis(tw_axis(TwPlan{0, {}, {}, {}, 0}, PY), PZ);
    static constexpr int TW_ELEMS = TW.total > 0 ? TW.total : 1;
    static_assert(PB * P % Q == 0, "Q must divide the block's points");
    static_assert(T % 64 == 0 && T <= 1024, "threads must be whole waves");
    static_assert(NPY >= 1 && NPZ >= 0, "axis not factorable with this Q");
};

// Wave-local LDS ordering.  The LDS executes the instructions of one wave in issue order,
// so a read issued after a write of the same wave sees it, and a write issued after a read
// cannot overtake it; only the compiler must be kept from moving LDS accesses across.
#define PLS_WAVE_SYNC() asm volatile("" ::: "memory")

// A copy of x the compiler cannot see through: address arithmetic derived from it is
// recomputed where it is used instead of being hoisted out of a loop (and pinning
// registers for its whole duration).
__device__ __forceinline__ int opaque(int x) {
    int y;
    asm volatile("v_mov_b32 %0, %1" : "=v"(y) : "v"(x));
    return y;
}

// Line ownership of a pass of radix R along axis AX (0 = y, 1 = z).  The lines of the axis
// (PB * NZ rows for y, PB * NY columns for z) are split evenly over the waves of the
// block, so every exchange between two passes of the same axis stays inside one wave;
// only the change of axis needs a block barrier.  Butterfly i of a thread is butterfly
// k = lane + 64 i of its wave: along y consecutive lanes take consecutive butterflies of
// a row, along z consecutive lanes take consecutive columns.
template <class G, int AX, int R>
struct PassMap {
    static constexpr int N = (AX == 0) ? G::NY : G::NZ;
    static constexpr int JN = N / R;
    static constexpr int NB = G::Q / R;
    static constexpr int LINES = (AX == 0) ? G::PB * G::NZ : G::PB * G::NY;
    static constexpr int W = G::T / 64;
    static constexpr int LPW = LINES / W;
    static constexpr int STRIDE = (AX == 0) ? 1 : G::LDY;
    static_assert(LINES % W == 0 && LPW * JN == 64 * NB, "lines do not split over waves");
    __device__ static __forceinline__ void map(int tid, int i, int& line, int& j) {
        const int k = (tid & 63) + 64 * i;
        const int w = tid >> 6;
        if constexpr (AX == 0) {
            line = w * LPW + k / JN;
            j = k % JN;
        } else {
            line = w * LPW + k % LPW;
            j = k / LPW;
        }
    }
    // LDS offset of point 0 of a line
    __device__ static __forceinline__ int lbase(int line) {
        if constexpr (AX == 0) return (line / G::NZ) * G::PS + (line % G::NZ) * G::LDY;
        else return (line / G::NY) * G::PS + G::ycol(line % G::NY);
    }
    // (plane, z, y) of element (i, r) in the distribution a first pass of this radix reads
    __device__ static __forceinline__ void pos(int tid, int i, int r, int& pb, int& z, int& y) {
        int line, j;
        map(tid, i, line, j);
        if constexpr (AX == 0) {
            pb = line / G::NZ;
            z = line % G::NZ;
            y = j + r * JN;
        } else {
            pb = line / G::NY;
            y = line % G::NY;
            z = j + r * JN;
        }
    }
};

// Position (plane, z, y) of element (i, r) of a thread's registers in the distribution
// that a first pass of radix R along axis AX reads.
template <class G, int AX, int R>
__device__ __forceinline__ void pass_pos(int tid, int i, int r, int& pb, int& z, int& y) {
    PassMap<G, AX, R>::pos(tid, i, r, pb, z, y);
}

// Padded rows (YSW = 16): a y pass touches y = y0 + c, with y0 the butterfly's
// lane-dependent part and c = r * step a compile-time constant.  Its column is
// ycol(y0) + c + c / 16 + carry, carry = ((y0 % 16) + (c % 16)) / 16.  The values y0 % 16
// can take in the pass are known at compile time; per r the carry is then never, always,
// or set exactly for the lanes with y0 % 16 >= thr[k] for one of a few thresholds.
struct YCarry {
    int cls[32];   // per r: -1 carry never, -2 always, k >= 0 threshold class k
    int thr[16];
    int nthr;
};

// y0 of butterfly k (lane + 64 i) of a y pass of radix R, stage length LS: the first point
// read (WRITE false) or written (WRITE true).
constexpr int ypass_y0(int k, int JN, int R, int LS, bool WRITE) {
    const int j = k % JN;
    return WRITE ? (j / LS) * LS * R + j % LS : j;
}

constexpr YCarry ycarry(int NBK, int JN, int R, int LS, bool WRITE) {
    YCarry c{{}, {}, 0};
    bool can[16] = {};
    for (int k = 0; k < NBK; ++k) can[ypass_y0(k, JN, R, LS, WRITE) & 15] = true;
    for (int r = 0; r < R; ++r) {
        const int d = (WRITE ? r * LS : r * JN) & 15;
        // smallest possible y0 % 16 that carries, and whether every possible value does
        int lo = 16;
        bool all = true;
        for (int u = 0; u < 16; ++u) {
            if (!can[u]) continue;
            if (u + d >= 16) lo = lo < u ? lo : u;
            else all = false;
        }
        if (lo == 16) {
            c.cls[r] = -1;
        } else if (all) {
            c.cls[r] = -2;
        } else {
            int k = 0;
            while (k < c.nthr && c.thr[k] != lo) ++k;
            if (k == c.nthr) c.thr[c.nthr++] = lo;
            c.cls[r] = k;
        }
    }
    return c;
}

// LDS offsets of the points r of butterfly (base = row base, y0) of a padded y pass, into
// off[]: one runtime base per threshold class, the rest compile-time immediates.
template <int R, int STEP, YCarry const& C>
__device__ __forceinline__ void ypad_offsets(int base, int y0, int (&off)[R]) {
    const int b0 = base + y0 + (y0 >> 4);
    int bk[C.nthr > 0 ? C.nthr : 1];
    sfor<C.nthr>([&](auto kI) __attribute__((always_inline)) {
        constexpr int k = decltype(kI)::value;
        constexpr int t = C.thr[k];
        bk[k] = b0 + ((y0 & 15) >= t ? 1 : 0);
    });
    sfor<R>([&](auto rI) __attribute__((always_inline)) {
        constexpr int r = decltype(rI)::value;
        constexpr int c = r * STEP;
        constexpr int cl = C.cls[r];
        constexpr int imm = c + (c >> 4) + (cl == -2 ? 1 : 0);
        if constexpr (cl >= 0) off[r] = bk[cl] + imm;
        else off[r] = b0 + imm;
    });
}

template <int NBK, int JN, int R, int LS, bool WRITE>
struct YCarryOf {
    static constexpr YCarry value = ycarry(NBK, JN, R, LS, WRITE);
};

// One Stockham pass.  With TWOFF < 0, tw = exp(-2 pi i m / N), m in [0, N), for this axis'
// length N; otherwise tw is a block of per-pass tables (TwPlan) and this pass' factors sit at
// TWOFF + (r - 1) LS + k.  Reads follow a block barrier or a wave-local sync of the previous
// pass; writes are followed by a wave-local sync (callers add the block barrier at a change
// of axis).
template <class G, int AX, int R, int LS, bool INV, bool IN_REG, bool OUT_REG, int TWOFF = -1>
__device__ __forceinline__ void fft_pass(float2 (&v)[G::Q], float2* lds, const float2* tw,
                                         int tid) {
    using M = PassMap<G, AX, R>;
    constexpr int N = M::N, JN = M::JN, NB = M::NB, STRIDE = M::STRIDE;
    static_assert(G::Q % R == 0 && N % (R * LS) == 0, "bad pass");
    int base[NB], jj[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        int line;
        M::map(tid, i, line, jj[i]);
        base[i] = M::lbase(line);
    }
    constexpr bool PADDED = (AX == 0 && G::YSW > 0);
    if constexpr (!IN_REG) {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            if constexpr (PADDED) {
                int off[R];
                ypad_offsets<R, JN, YCarryOf<64 * NB, JN, R, LS, false>::value>(base[i], jj[i], off);
#pragma unroll
                for (int r = 0; r < R; ++r) v[i * R + r] = lds[off[r]];
            } else {
                const float2* src = lds + base[i] + jj[i] * STRIDE;
#pragma unroll
                for (int r = 0; r < R; ++r) v[i * R + r] = src[r * JN * STRIDE];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        if constexpr (LS > 1) {
            const int k = jj[i] % LS;
            constexpr int step = N / (LS * R);
#pragma unroll
            for (int r = 1; r < R; ++r) {
                float2 w = (TWOFF >= 0) ? tw[TWOFF + (r - 1) * LS + k] : tw[k * r * step];
                if (INV) w.y = -w.y;
                v[i * R + r] = cmul(v[i * R + r], w);
            }
        }
        dft<R, INV>(&v[i * R]);
    }
    if constexpr (!OUT_REG) {
        PLS_WAVE_SYNC();   // this wave's reads of the lines it is about to overwrite are done
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int j = jj[i];
            if constexpr (PADDED) {
                int off[R];
                ypad_offsets<R, LS, YCarryOf<64 * NB, JN, R, LS, true>::value>(
                    base[i], (j / LS) * LS * R + (j % LS), off);
#pragma unroll
                for (int r = 0; r < R; ++r) lds[off[r]] = v[i * R + r];
            } else {
                float2* dst = lds + base[i] + ((j / LS) * LS * R + (j % LS)) * STRIDE;
#pragma unroll
                for (int r = 0; r < R; ++r) dst[r * LS * STRIDE] = v[i * R + r];
            }
        }
        PLS_WAVE_SYNC();
    }
}

// Fills the per-pass twiddle tables (G::TW_ELEMS entries of LDS) from the axis tables
// twy = exp(-2 pi i m / NY) and twz = exp(-2 pi i m / NZ).  The caller adds the barrier.
template <class G>
__device__ __forceinline__ void tw_fill(float2* twt, const float2* twy, const float2* twz,
                                        int tid) {
    sfor<G::TW.n>([&](auto iI) __attribute__((always_inline)) {
        constexpr int i = decltype(iI)::value;
        constexpr int R = G::TW.R[i], LS = G::TW.LS[i], off = G::TW.off[i];
        constexpr int M = R * LS;
        static_assert(G::NY % M == 0 || G::NZ % M == 0, "stage length outside both axes");
        for (int e = tid; e < (R - 1) * LS; e += G::T) {
            const int m = (e % LS) * (e / LS + 1);            // k r < M
            twt[off + e] = (G::NY % M == 0) ? twy[m * (G::NY / M)] : twz[m * (G::NZ / M)];
        }
    });
}

// Forward 2D transform: y passes (ascending radices) then z passes (ascending).
// Input: registers in the distribution of the first y pass; output: registers in the
// distribution of a first pass of radix (last z radix) along z (or y when NZ == 1).
// twt holds the per-pass tables tw_fill wrote.  The caller guarantees that no other wave
// still reads this block's rows (LDS).
template <class G>
__device__ __forceinline__ void fft2_fwd(float2 (&v)[G::Q], float2* lds, const float2* twt,
                                         int tid) {
    constexpr int NPY = G::NPY, NPZ = G::NPZ, NP = NPY + NPZ;
    sfor<NP>([&](auto pI) __attribute__((always_inline)) {
        constexpr int p = decltype(pI)::value;
        constexpr bool IN_REG = (p == 0);
        constexpr bool OUT_REG = (p == NP - 1);
        if constexpr (p < NPY) {
            constexpr int R = G::PY.r[p];
            constexpr int LS = plan_prod(G::PY, p);
            fft_pass<G, 0, R, LS, false, IN_REG, OUT_REG, tw_find(G::TW, R, LS)>(v, lds, twt, tid);
        } else {
            constexpr int q = p - NPY;
            constexpr int R = G::PZ.r[q];
            constexpr int LS = plan_prod(G::PZ, q);
            if constexpr (q == 0) __syncthreads();   // rows -> columns
            fft_pass<G, 1, R, LS, false, IN_REG, OUT_REG, tw_find(G::TW, R, LS)>(v, lds, twt, tid);
        }
    });
}

// Inverse 2D transform (unnormalised): z passes in descending radix order, then y passes
// in descending order.  Reads the registers fft2_fwd left and returns them in the
// distribution fft2_fwd read.  PART selects the passes: 0 all, 1 all but the last (which
// leaves its result in LDS), 2 the last only (reads LDS, returns the registers), so that a
// caller can issue global loads between the two.
template <class G, int PART = 0>
__device__ __forceinline__ void fft2_inv(float2 (&v)[G::Q], float2* lds, const float2* twt,
                                         int tid) {
    constexpr int NPY = G::NPY, NPZ = G::NPZ, NP = NPY + NPZ;
    sfor<NP>([&](auto pI) __attribute__((always_inline)) {
        constexpr int p = decltype(pI)::value;
        if constexpr ((PART == 1 && p == NP - 1) || (PART == 2 && p != NP - 1)) return;
        constexpr bool IN_REG = (p == 0);
        constexpr bool OUT_REG = (p == NP - 1);
        if constexpr (p < NPZ) {
            constexpr int idx = NPZ - 1 - p;          // radices reversed
            constexpr int R = G::PZ.r[idx];
            constexpr int LS = plan_prod_after(G::PZ, idx);
            fft_pass<G, 1, R, LS, true, IN_REG, OUT_REG, tw_find(G::TW, R, LS)>(v, lds, twt, tid);
        } else {
            constexpr int q = p - NPZ;
            constexpr int idx = NPY - 1 - q;
            constexpr int R = G::PY.r[idx];
            constexpr int LS = plan_prod_after(G::PY, idx);
            if constexpr (q == 0 && NPZ > 0) __syncthreads();   // columns -> rows
            fft_pass<G, 0, R, LS, true, IN_REG, OUT_REG, tw_find(G::TW, R, LS)>(v, lds, twt, tid);
        }
    });
}

// Input distribution of fft2_fwd (= output distribution of fft2_inv).
template <class G>
__device__ __forceinline__ void pos_in(int tid, int i, int r, int& pb, int& z, int& y) {
    constexpr int R0 = G::PY.r[0];
    pass_pos<G, 0, R0>(tid, i, r, pb, z, y);
}
// Output distribution of fft2_fwd (= input distribution of fft2_inv).
template <class G>
__device__ __forceinline__ void pos_out(int tid, int i, int r, int& pb, int& z, int& y) {
    if constexpr (G::NPZ > 0) {
        constexpr int RL = G::PZ.r[G::NPZ - 1];
        pass_pos<G, 1, RL>(tid, i, r, pb, z, y);
    } else {
        constexpr int RL = G::PY.r[G::NPY - 1];
        pass_pos<G, 0, RL>(tid, i, r, pb, z, y);
    }
}

// Radix of the element-grouping used by pos_in / pos_out.
template <class G>
constexpr int radix_in() { return G::PY.r[0]; }
template <class G>
constexpr int radix_out() { return G::NPZ > 0 ? G::PZ.r[G::NPZ - 1] : G::PY.r[G::NPY - 1]; }

}  // namespace pls
