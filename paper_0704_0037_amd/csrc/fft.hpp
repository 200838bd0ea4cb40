// Stockham FFT building blocks for lines held in LDS (gfx950, wave64).
//
// A length-L transform is split into passes of radix 2, 3, 4, 5, 6, 8 or 16.  Pass p with radix R
// and stride Ns (product of the radices before it) does L/R butterflies; butterfly j reads the
// elements j + r*L/R (r < R), multiplies element r by W^(r*k) with W = exp(-+2 pi i/(Ns*R)) and
// k = j mod Ns, does an R-point DFT and writes output r to (j - k)*R + k + r*Ns (self-sorting,
// no bit reversal).  The first pass (Ns = 1) needs no twiddles and reads straight from global
// memory, so zero padding is a predicated-off load; the last pass writes straight to global
// memory, so the pruned output of an inverse transform is a predicated-off store.
//
// DIR = -1 is the forward transform exp(-2 pi i jk/L), DIR = +1 the unnormalized inverse.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace dda {

constexpr int kMaxPass = 12;
#ifndef DDA_MAX_THREADS
#define DDA_MAX_THREADS 512   // block-size bound of the x / y pass kernels
#endif
// block-size bound of the x / y pass kernels per precision: single-precision lines need twice the
// lines per block for the same 128-byte runs on their transposed side, and fit the registers
#ifndef DDA_MAX_THREADS_F64
#define DDA_MAX_THREADS_F64 DDA_MAX_THREADS
#endif
template <typename R> constexpr int max_threads() { return sizeof(R) == 8 ? DDA_MAX_THREADS_F64 : 2 * DDA_MAX_THREADS; }
// padded lengths with kernels specialized at compile time (5-smooth sizes the workloads use most)
#define DDA_SPECIALIZED_LENGTHS(X) \
    X(32) X(48) X(60) X(64) X(72) X(80) X(96) X(120) X(128) X(160) X(192) X(200) X(256) X(320) X(384) X(512)

#ifndef DDA_ZMUL_THREADS
#define DDA_ZMUL_THREADS (3 * 64)  // block-size bound of the fused z-pass kernel
#endif
#ifndef DDA_TW_DERIVED
#define DDA_TW_DERIVED 1  // radix-8 twiddles w^3, w^5, w^6, w^7 formed from w, w^2, w^4 (0: all from the table)
#endif
#ifndef DDA_B2_COLMAJOR
#define DDA_B2_COLMAJOR 1  // y-pass output [Lx][c][Ly][nz] (0: [Ly][Lx][c][nz])
#endif
#ifndef DDA_ZMUL_OWN
#define DDA_ZMUL_OWN 1  // the fp64 z pass multiplies each thread's own component from registers
#endif
#ifndef DDA_ZMUL_WAVES_PER_EU
#define DDA_ZMUL_WAVES_PER_EU 3  // register budget of the z pass: three 3-wave blocks per CU at fp64
#endif
#ifndef DDA_LDS_CAP
#define DDA_LDS_CAP (96 * 1024)  // LDS bytes a matvec block may take
#endif

struct FftPlan {
    int L;                   // transform length
    int npass;               // number of passes (1 for L = 1, which uses radix 1); 0 = length not supported
    int tpl;                 // threads per line = L / largest radix (butterflies of the widest pass)
    int tpl1;                // threads per line for one butterfly per thread in every pass = L / smallest radix
    int tw_off;              // offset of the table exp(-2 pi i m / L), m < L, in the twiddle buffer
    int radix[kMaxPass];
    int ns[kMaxPass];        // product of the radices of the preceding passes
};

// Radix schedule for length L (5-smooth): 8s first, the leftover power of two as 16 (maxr 16), as
// a 6 together with one factor 3 (only where a radix-3 pass would need more than 64 threads per
// line), as 4*4, 4 or 2, then 5s and 3s; reversed for the inverse of a pass pair whose middle
// stays in registers.  Larger radices mean fewer passes over LDS.  A line gets tpl = L / (largest radix)
// threads, one per butterfly of its widest pass; a pass of smaller radix has more butterflies
// than threads, and each thread takes ceil(L / (R tpl)) of them, so no lane idles through the
// radix-8 passes that do most of the arithmetic.  tpl1 = L / (smallest radix) threads give one
// butterfly per thread in every pass (the fused z pass runs that way).  Used on the host to plan
// and on the device to specialize kernels for a length known at compile time.
// order: 0 the schedule above, 1 reversed, 2 ascending by radix (largest last), 3 descending
__host__ __device__ constexpr FftPlan make_plan(int L, int maxr, int order) {
    FftPlan p{};
    int r[kMaxPass] = {};
    int n = 0;
    if (L == 1) {
        r[n++] = 1;
    } else {
        int rem = L, p2 = 0, n3 = 0, n5 = 0;
        while (rem > 1 && rem % 2 == 0) rem /= 2, ++p2;
        while (rem > 1 && rem % 5 == 0) rem /= 5, ++n5;
        while (rem > 1 && rem % 3 == 0) rem /= 3, ++n3;
        if (rem != 1 || L < 1) return p;  // npass = 0: unsupported
        const int n8 = p2 / 3, left = p2 % 3;
        if (n8 + 2 + n3 + n5 > kMaxPass) return p;
        for (int i = 0; i < n8; ++i) r[n++] = 8;
        int m3 = n3;
        if (left == 1) {
            if (n8 > 0 && maxr >= 16) r[n - 1] = 16;
            else if (m3 > 0 && maxr >= 6 && L / 3 > 64) { r[n++] = 6; --m3; }  // 384 = 8 8 6: 64 threads, not 128
            else if (n8 > 0) { r[n - 1] = 4; r[n++] = 4; }
            else r[n++] = 2;
        } else if (left == 2) {
            r[n++] = 4;
        }
        for (int i = 0; i < n5; ++i) r[n++] = 5;
        for (int i = 0; i < m3; ++i) r[n++] = 3;
    }
    if (order == 1)
        for (int i = 0; i < n / 2; ++i) {
            const int t = r[i];
            r[i] = r[n - 1 - i];
            r[n - 1 - i] = t;
        }
    if (order >= 2)
        for (int i = 1; i < n; ++i)  // insertion sort
            for (int k = i; k > 0 && (order == 2 ? r[k - 1] > r[k] : r[k - 1] < r[k]); --k) {
                const int t = r[k];
                r[k] = r[k - 1];
                r[k - 1] = t;
            }
    int ns = 1, rmin = 1 << 30, rmax = 0;
    for (int i = 0; i < n; ++i) {
        p.radix[i] = r[i];
        p.ns[i] = ns;
        ns *= r[i];
        rmin = rmin < r[i] ? rmin : r[i];
        rmax = rmax > r[i] ? rmax : r[i];
    }
    p.L = L;
    p.npass = n;
    p.tpl = L / rmax;
    p.tpl1 = L / rmin;
    return p;
}

// threads per line of the fused z pass: one butterfly per thread in every pass when that fits
// in 64 (tpl1), else L / (largest radix) with several butterflies per thread in the passes of
// smaller radix (384 = 8 4 4 3: 48 threads, not 128)
// z-pass mode of a length.  One butterfly per thread in every pass (tpl1 threads per line, one
// column per round) where that fits in 64 threads and a line fills a good part of a wave;
// otherwise ("multi") L / (largest radix) threads per line, the forward plan with its largest
// radix last, several butterflies per thread in the other passes, each component in a wave of
// its own, and 64 / lanes columns per round (lanes = tpl rounded up to a power of two, at least
// 16): a short line alone would leave most of a wave idle through a round's whole chain of
// passes.  Measured per 2-vector z pass against one column per round: 48 -41 %, 64 -57 %, 96
// -23 %, 120 -19 %, 192 -7 %, 256 -11 %; but 160 (20 of 32 lanes busy) +16 % and 72 (9 of 16)
// +0 %, which keep one column per round.
__host__ __device__ constexpr int zmul_pow2_lanes(int tpl) {
    int w = 16;
    while (w < tpl) w *= 2;
    return w;
}
__host__ __device__ constexpr bool zmul_multi(const FftPlan &p) {
    return p.tpl1 > 64 ||
           (p.npass > 1 && p.tpl <= 32 && (4 * p.tpl >= 3 * zmul_pow2_lanes(p.tpl) || p.tpl <= 8));
}
__host__ __device__ constexpr int zmul_tpl(const FftPlan &p) { return zmul_multi(p) ? p.tpl : p.tpl1; }
// lanes per line (a power of two) and lines (columns) per wave in the multi mode
__host__ __device__ constexpr int zmul_lanes(const FftPlan &p) { return zmul_multi(p) ? zmul_pow2_lanes(p.tpl) : p.tpl1; }
__host__ __device__ constexpr int zmul_slots(const FftPlan &p) { return zmul_multi(p) ? 64 / zmul_lanes(p) : 1; }
// threads per component in the block: a whole wave in the multi mode
__host__ __device__ constexpr int zmul_ct(const FftPlan &p) { return zmul_multi(p) ? 64 : p.tpl1; }

__host__ __device__ constexpr int pow2_at_least(int n) {
    int w = 1;
    while (w < n) w *= 2;
    return w;
}

// bound on the butterflies a thread takes in a pass of radix R when a line has L / (largest
// radix) threads and no radix exceeds maxr
__host__ __device__ constexpr int bfly_per_thread(int R, int maxr) { return (maxr + R - 1) / R; }

// The plan a kernel uses: the compile-time plan for LC > 0 (all indices fold to constants), else
// the runtime plan passed as an argument.  tw_off always comes from the runtime plan.
template <int LC, int MAXR, int REV>
__device__ __forceinline__ FftPlan plan_of(const FftPlan &rt) {
    if constexpr (LC > 0) {
        constexpr FftPlan P = make_plan(LC, MAXR, REV);  // evaluated by the compiler
        static_assert(P.npass > 0, "unsupported specialized length");
        FftPlan p = P;
        p.tw_off = rt.tw_off;
        return p;
    } else {
        return rt;
    }
}

// LDS element index with one element of skew every 8, so radix-8 butterflies writing with a
// stride of 8 elements do not all land in the same banks.
__device__ __forceinline__ int pidx(int i) { return i + (i >> 3); }
__host__ __device__ constexpr int lds_line_stride(int L) { return L + (L >> 3) + 1; }

// ----------------------------------------------------------------------- small DFTs
template <int DIR, typename C> __device__ __forceinline__ void dft2(C *a) {
    C t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
}

template <int DIR, typename C> __device__ __forceinline__ void dft3(C *a) {
    using R = decltype(C::x);
    const R s3 = (R)0.86602540378443864676;  // sin(2 pi / 3)
    C s = cadd(a[1], a[2]);
    C d = csub(a[1], a[2]);
    C t = mk<C>(a[0].x - (R)0.5 * s.x, a[0].y - (R)0.5 * s.y);
    C u = mul_i<DIR>(cscale(d, s3));  // -i s3 (a1 - a2) forward
    a[0] = cadd(a[0], s);
    a[1] = cadd(t, u);
    a[2] = csub(t, u);
}

template <int DIR, typename C> __device__ __forceinline__ void dft4(C *a) {
    C t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
    C t2 = cadd(a[1], a[3]), t3 = mul_i<DIR>(csub(a[1], a[3]));
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, t3);
    a[3] = csub(t1, t3);
}

template <int DIR, typename C> __device__ __forceinline__ void dft5(C *a) {
    using R = decltype(C::x);
    const R c1 = (R)0.30901699437494742410;   // cos(2 pi/5)
    const R c2 = (R)-0.80901699437494742410;  // cos(4 pi/5)
    const R s1 = (R)0.95105651629515357212;   // sin(2 pi/5)
    const R s2 = (R)0.58778525229247312917;   // sin(4 pi/5)
    C b1 = cadd(a[1], a[4]), b2 = cadd(a[2], a[3]);
    C d1 = csub(a[1], a[4]), d2 = csub(a[2], a[3]);
    C t1 = mk<C>(a[0].x + c1 * b1.x + c2 * b2.x, a[0].y + c1 * b1.y + c2 * b2.y);
    C t2 = mk<C>(a[0].x + c2 * b1.x + c1 * b2.x, a[0].y + c2 * b1.y + c1 * b2.y);
    C u1 = mul_i<DIR>(mk<C>(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y));
    C u2 = mul_i<DIR>(mk<C>(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y));
    a[0] = cadd(a[0], cadd(b1, b2));
    a[1] = cadd(t1, u1);
    a[4] = csub(t1, u1);
    a[2] = cadd(t2, u2);
    a[3] = csub(t2, u2);
}

// 6 = 3 x 2: two-point DFTs of (a_i, a_(i+3)), the second output times w6^i, then three-point DFTs;
// output k2 + 2 k1 is the three-point DFT k1 of branch k2 (w6^((i + 3m)(k2 + 2k1)) =
// w6^(i k2) w3^(i k1) (-1)^(m k2))
template <int DIR, typename C> __device__ __forceinline__ void dft6(C *a) {
    using R = decltype(C::x);
    const R h = (R)0.5, s3 = (R)0.86602540378443864676;  // cos, sin of pi / 3
    C t0[3], t1[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        t0[i] = cadd(a[i], a[i + 3]);
        t1[i] = csub(a[i], a[i + 3]);
    }
    // w6 = exp(DIR 2 pi i / 6) = h + DIR i s3; w6^2 = -h + DIR i s3
    const R sd = DIR < 0 ? -s3 : s3;
    t1[1] = mk<C>(t1[1].x * h - t1[1].y * sd, t1[1].x * sd + t1[1].y * h);
    t1[2] = mk<C>(-t1[2].x * h - t1[2].y * sd, t1[2].x * sd - t1[2].y * h);
    dft3<DIR>(t0);
    dft3<DIR>(t1);
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
        a[2 * k1] = t0[k1];
        a[2 * k1 + 1] = t1[k1];
    }
}

// multiply by exp(DIR * 2 pi i m / 16) for the few m the radix-16 split needs
template <int DIR, typename C> __device__ __forceinline__ C rot16(C v, int m) {
    using R = decltype(C::x);
    const R c1 = (R)0.92387953251128675613, s1 = (R)0.38268343236508977173;
    const R h = (R)0.70710678118654752440;
    R c, s;  // cos, sin of pi m / 8
    switch (m) {
        case 1: c = c1; s = s1; break;
        case 2: c = h; s = h; break;
        case 3: c = s1; s = c1; break;
        case 4: c = 0; s = 1; break;
        case 6: c = -h; s = h; break;
        default: c = -c1; s = -s1; break;  // m = 9
    }
    // forward: (c - i s), inverse: (c + i s)
    const R ss = DIR < 0 ? -s : s;
    return mk<C>(v.x * c - v.y * ss, v.x * ss + v.y * c);
}

template <int DIR, typename C> __device__ __forceinline__ void dft8(C *a) {
    using R = decltype(C::x);
    const R h = (R)0.70710678118654752440;
    C e[4] = {a[0], a[2], a[4], a[6]};
    C o[4] = {a[1], a[3], a[5], a[7]};
    dft4<DIR>(e);
    dft4<DIR>(o);
    C o1 = o[1], o3 = o[3];
    if (DIR < 0) {
        o[1] = mk<C>((o1.x + o1.y) * h, (o1.y - o1.x) * h);
        o[3] = mk<C>((o3.y - o3.x) * h, -(o3.x + o3.y) * h);
    } else {
        o[1] = mk<C>((o1.x - o1.y) * h, (o1.x + o1.y) * h);
        o[3] = mk<C>(-(o3.x + o3.y) * h, (o3.x - o3.y) * h);
    }
    o[2] = mul_i<DIR>(o[2]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        a[k] = cadd(e[k], o[k]);
        a[k + 4] = csub(e[k], o[k]);
    }
}

template <int DIR, typename C> __device__ __forceinline__ void dft16(C *a) {
    // n = 4 n1 + n2: DFT-4 over n1 (stride 4), twiddle W16^(n2 k1), DFT-4 over n2
    C b[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        C t[4] = {a[n2], a[4 + n2], a[8 + n2], a[12 + n2]};
        dft4<DIR>(t);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) b[n2][k1] = (n2 * k1 == 0) ? t[k1] : rot16<DIR>(t[k1], n2 * k1);
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        C t[4] = {b[0][k1], b[1][k1], b[2][k1], b[3][k1]};
        dft4<DIR>(t);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) a[k1 + 4 * k2] = t[k2];
    }
}

template <int DIR, int RADIX, typename C> __device__ __forceinline__ void dftR(C *a) {
    if constexpr (RADIX == 1) (void)a;
    else if constexpr (RADIX == 2) dft2<DIR>(a);
    else if constexpr (RADIX == 3) dft3<DIR>(a);
    else if constexpr (RADIX == 4) dft4<DIR>(a);
    else if constexpr (RADIX == 5) dft5<DIR>(a);
    else if constexpr (RADIX == 6) dft6<DIR>(a);
    else if constexpr (RADIX == 8) dft8<DIR>(a);
    else if constexpr (RADIX == 16) dft16<DIR>(a);
}

// ------------------------------------------------------------- butterfly load / store
// a[r] *= w^(r k) (conjugated for the inverse), w = exp(-2 pi i step / L), from the table tw.
// With DDA_TW_DERIVED, radix 8 loads w, w^2, w^4 and forms the other four by products (fewer
// cached loads per butterfly, ~2 ulps more rounding).
// Twiddle source of a transform whose passes are all radix 8: the first L/8 entries of the
// length-L table staged in LDS (lds), the full table in global memory (glob).  A radix-8 pass
// reads w = lds[k step] (k step < L/8 there) and forms w^2, w^4 by squaring; other radices read
// the global table.
template <typename C> struct TwStaged {
    const C *lds;
    const C *glob;
};

template <int DIR, int RADIX, typename C>
__device__ __forceinline__ void twiddle(C *a, int k, int step, TwStaged<C> tw) {
    if constexpr (RADIX == 8) {
        const C w1 = tw.lds[k * step], w2 = cmul(w1, w1), w4 = cmul(w2, w2);
        const C w3 = cmul(w1, w2), w5 = cmul(w1, w4), w6 = cmul(w2, w4), w7 = cmul(w3, w4);
        const C w[8] = {w1, w1, w2, w3, w4, w5, w6, w7};
#pragma unroll
        for (int r = 1; r < 8; ++r) a[r] = cmul(a[r], DIR < 0 ? w[r] : cconj(w[r]));
    } else {
#pragma unroll
        for (int r = 1; r < RADIX; ++r) {
            C w = tw.glob[r * k * step];
            a[r] = cmul(a[r], DIR < 0 ? w : cconj(w));
        }
    }
}

template <int DIR, int RADIX, typename C>
__device__ __forceinline__ void twiddle(C *a, int k, int step, const C *__restrict__ tw) {
    if constexpr (DDA_TW_DERIVED && RADIX == 8) {
        const C w1 = tw[k * step], w2 = tw[2 * k * step], w4 = tw[4 * k * step];
        const C w3 = cmul(w1, w2), w5 = cmul(w1, w4), w6 = cmul(w2, w4), w7 = cmul(w3, w4);
        const C w[8] = {w1, w1, w2, w3, w4, w5, w6, w7};
#pragma unroll
        for (int r = 1; r < 8; ++r) a[r] = cmul(a[r], DIR < 0 ? w[r] : cconj(w[r]));
    } else {
#pragma unroll
        for (int r = 1; r < RADIX; ++r) {
            C w = tw[r * k * step];
            a[r] = cmul(a[r], DIR < 0 ? w : cconj(w));
        }
    }
}

// Load the R inputs of butterfly j through ld(index), twiddle, transform (into a[0..R-1]).
// UPPER_ZERO: the first pass of a zero-padded line (L >= 2n - 1, so every index >= L/2 is
// padding): inputs j + r L/R with r >= ceil(R/2) are zero without being loaded.
template <int DIR, int RADIX, typename C, class LD, bool UPPER_ZERO = false>
__device__ __forceinline__ void bfly_load(C *a, int j, int L, int Ns, const C *__restrict__ tw, LD ld) {
    const int q = L / RADIX;
#pragma unroll
    for (int r = 0; r < RADIX; ++r) a[r] = (UPPER_ZERO && 2 * r >= RADIX) ? czero<C>() : ld(j + r * q);
    if (Ns > 1) twiddle<DIR, RADIX>(a, j % Ns, q / Ns, tw);  // step = L / (Ns * RADIX)
    dftR<DIR, RADIX>(a);
}

template <int DIR, int RADIX, typename C, class LD, bool UPPER_ZERO = false>
__device__ __forceinline__ void bfly_load(C *a, int j, int L, int Ns, TwStaged<C> tw, LD ld) {
    const int q = L / RADIX;
#pragma unroll
    for (int r = 0; r < RADIX; ++r) a[r] = (UPPER_ZERO && 2 * r >= RADIX) ? czero<C>() : ld(j + r * q);
    if (Ns > 1) twiddle<DIR, RADIX>(a, j % Ns, q / Ns, tw);
    dftR<DIR, RADIX>(a);
}

// Twiddle and transform values already in registers (for a pass whose inputs a thread holds).
template <int DIR, int RADIX, typename C>
__device__ __forceinline__ void bfly_regs(C *a, int j, int L, int Ns, const C *__restrict__ tw) {
    if (Ns > 1) twiddle<DIR, RADIX>(a, j % Ns, L / RADIX / Ns, tw);
    dftR<DIR, RADIX>(a);
}

template <int RADIX, typename C, class ST>
__device__ __forceinline__ void bfly_store(const C *a, int j, int Ns, ST st) {
    const int k = j % Ns;
    const int base = (j - k) * RADIX + k;
#pragma unroll
    for (int r = 0; r < RADIX; ++r) st(base + r * Ns, a[r]);
}

// Runtime-radix dispatch.  MAXR bounds the radices a kernel supports (register array size).
template <int DIR, int MAXR, bool UPPER_ZERO = false, typename C, class LD>
__device__ __forceinline__ void load_rt(C *a, int R, int j, int L, int Ns, const C *__restrict__ tw, LD ld) {
    switch (R) {
        case 1: a[0] = ld(j); break;
        case 2: bfly_load<DIR, 2, C, LD, UPPER_ZERO>(a, j, L, Ns, tw, ld); break;
        case 3: bfly_load<DIR, 3, C, LD, UPPER_ZERO>(a, j, L, Ns, tw, ld); break;
        case 4: bfly_load<DIR, 4, C, LD, UPPER_ZERO>(a, j, L, Ns, tw, ld); break;
        case 5: bfly_load<DIR, 5, C, LD, UPPER_ZERO>(a, j, L, Ns, tw, ld); break;
        case 6: bfly_load<DIR, 6, C, LD, UPPER_ZERO>(a, j, L, Ns, tw, ld); break;
        case 8: if constexpr (MAXR >= 8) bfly_load<DIR, 8, C, LD, UPPER_ZERO>(a, j, L, Ns, tw, ld); break;
        default: if constexpr (MAXR >= 16) bfly_load<DIR, 16, C, LD, UPPER_ZERO>(a, j, L, Ns, tw, ld); break;
    }
}

template <int DIR, int MAXR, bool UPPER_ZERO = false, typename C, class LD>
__device__ __forceinline__ void load_rt(C *a, int R, int j, int L, int Ns, TwStaged<C> tw, LD ld) {
    switch (R) {
        case 1: a[0] = ld(j); break;
        case 2: bfly_load<DIR, 2, C, LD, UPPER_ZERO>(a, j, L, Ns, tw, ld); break;
        case 3: bfly_load<DIR, 3, C, LD, UPPER_ZERO>(a, j, L, Ns, tw, ld); break;
        case 4: bfly_load<DIR, 4, C, LD, UPPER_ZERO>(a, j, L, Ns, tw, ld); break;
        case 5: bfly_load<DIR, 5, C, LD, UPPER_ZERO>(a, j, L, Ns, tw, ld); break;
        case 6: bfly_load<DIR, 6, C, LD, UPPER_ZERO>(a, j, L, Ns, tw, ld); break;
        case 8: if constexpr (MAXR >= 8) bfly_load<DIR, 8, C, LD, UPPER_ZERO>(a, j, L, Ns, tw, ld); break;
        default: if constexpr (MAXR >= 16) bfly_load<DIR, 16, C, LD, UPPER_ZERO>(a, j, L, Ns, tw, ld); break;
    }
}

template <int DIR, int MAXR, typename C>
__device__ __forceinline__ void regs_rt(C *a, int R, int j, int L, int Ns, const C *__restrict__ tw) {
    switch (R) {
        case 1: break;
        case 2: bfly_regs<DIR, 2>(a, j, L, Ns, tw); break;
        case 3: bfly_regs<DIR, 3>(a, j, L, Ns, tw); break;
        case 4: bfly_regs<DIR, 4>(a, j, L, Ns, tw); break;
        case 5: bfly_regs<DIR, 5>(a, j, L, Ns, tw); break;
        case 6: bfly_regs<DIR, 6>(a, j, L, Ns, tw); break;
        case 8: if constexpr (MAXR >= 8) bfly_regs<DIR, 8>(a, j, L, Ns, tw); break;
        default: if constexpr (MAXR >= 16) bfly_regs<DIR, 16>(a, j, L, Ns, tw); break;
    }
}

template <int MAXR, typename C, class ST>
__device__ __forceinline__ void store_rt(const C *a, int R, int j, int Ns, ST st) {
    switch (R) {
        case 1: st(j, a[0]); break;
        case 2: bfly_store<2>(a, j, Ns, st); break;
        case 3: bfly_store<3>(a, j, Ns, st); break;
        case 4: bfly_store<4>(a, j, Ns, st); break;
        case 5: bfly_store<5>(a, j, Ns, st); break;
        case 6: bfly_store<6>(a, j, Ns, st); break;
        case 8: if constexpr (MAXR >= 8) bfly_store<8>(a, j, Ns, st); break;
        default: if constexpr (MAXR >= 16) bfly_store<16>(a, j, Ns, st); break;
    }
}

template <int B, int E, class F> __device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Ordering point between the read and write phases of an in-place LDS pass.  When every line
// lives inside one wavefront (WAVE), only that wave's lanes exchange data; LDS instructions of a
// wave complete in order, so a compiler barrier suffices.  Otherwise the whole block syncs.
template <bool WAVE> __device__ __forceinline__ void lds_sync() {
    if constexpr (WAVE) {
        __asm__ volatile("" ::: "memory");
        __builtin_amdgcn_wave_barrier();
        __asm__ volatile("" ::: "memory");
    } else {
        __syncthreads();
    }
}

// lines of a compile-time plan fit in one wavefront when its threads-per-line divides 64
template <int LC, int MAXR> __host__ __device__ constexpr bool wave_lines() {
    if constexpr (LC > 0) return 64 % make_plan(LC, MAXR, false).tpl == 0;
    else return false;
}

// One in-place pass of radix R over an LDS line: thread j loads butterflies j, j + tpl, ... (< L/R)
// into registers, the block syncs, then it stores them.  NB bounds the butterflies per thread.
template <int DIR, int R, int NB, bool WAVE, typename C, class TW, class LD, class ST>
__device__ __forceinline__ void lds_pass(int j, int L, int tpl, int Ns, TW tw, LD ld, ST st) {
    C a[NB][R];
    const int nb = L / R;
#pragma unroll
    for (int b = 0; b < NB; ++b)
        if (j + b * tpl < nb) bfly_load<DIR, R>(a[b], j + b * tpl, L, Ns, tw, ld);
    lds_sync<WAVE>();
#pragma unroll
    for (int b = 0; b < NB; ++b)
        if (j + b * tpl < nb) bfly_store<R>(a[b], j + b * tpl, Ns, st);
    lds_sync<WAVE>();
}

// Passes [p0, p1) in place on the LDS line `ln` (stride-skewed).  Every thread of the block
// must call this (it may contain barriers).  LC > 0 selects the plan make_plan(LC, MAXR, REV)
// known at compile time: passes are then unrolled with constant radices and strides, and when a
// line fits in a wave the passes sync only that wave; LC = 0 runs the runtime plan `pl`.
// ONE: the caller runs tpl1 threads per line (one butterfly per thread in every pass) instead of
// tpl.
// P2: the caller gives each line a power-of-two group of lanes (threads past the line's butterfly
// count idle), so a line whose group divides 64 lies within one wave.
template <int DIR, int MAXR, int LC, int REV, bool ONE, bool P2, typename C, class TW>
__device__ __forceinline__ void lds_passes_tw(C *ln, const FftPlan &pl, int p0, int p1, int j, TW tw) {
    auto ld = [&](int i) { return ln[pidx(i)]; };
    auto st = [&](int i, C v) { ln[pidx(i)] = v; };
    if constexpr (LC > 0) {
        constexpr FftPlan P = make_plan(LC, MAXR, REV);
        constexpr int T = ONE ? P.tpl1 : P.tpl;
        constexpr bool W = 64 % (P2 ? pow2_at_least(T) : T) == 0;
        static_for<1, P.npass>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            constexpr int R = P.radix[p], Ns = P.ns[p];
            constexpr int NB = (LC / R + T - 1) / T;
            if (p >= p0 && p < p1) lds_pass<DIR, R, NB, W, C>(j, LC, T, Ns, tw, ld, st);
        });
    } else {
        for (int p = p0; p < p1; ++p) {
            const int R = pl.radix[p], Ns = pl.ns[p], L = pl.L, T = ONE ? pl.tpl1 : pl.tpl;
            constexpr int M = ONE ? 1 : MAXR;  // butterflies per thread bound
            switch (R) {
                case 2: lds_pass<DIR, 2, bfly_per_thread(2, M), false, C>(j, L, T, Ns, tw, ld, st); break;
                case 3: lds_pass<DIR, 3, bfly_per_thread(3, M), false, C>(j, L, T, Ns, tw, ld, st); break;
                case 4: lds_pass<DIR, 4, bfly_per_thread(4, M), false, C>(j, L, T, Ns, tw, ld, st); break;
                case 5: lds_pass<DIR, 5, bfly_per_thread(5, M), false, C>(j, L, T, Ns, tw, ld, st); break;
                case 6: lds_pass<DIR, 6, bfly_per_thread(6, M), false, C>(j, L, T, Ns, tw, ld, st); break;
                case 8: if constexpr (MAXR >= 8) lds_pass<DIR, 8, bfly_per_thread(8, M), false, C>(j, L, T, Ns, tw, ld, st); break;
                default: if constexpr (MAXR >= 16) lds_pass<DIR, 16, 1, false, C>(j, L, T, Ns, tw, ld, st); break;
            }
        }
    }
}

template <int DIR, int MAXR, int LC, int REV, bool ONE = false, bool P2 = false, typename C>
__device__ __forceinline__ void lds_passes(C *ln, const FftPlan &pl, int p0, int p1, int j,
                                           const C *__restrict__ tw) {
    lds_passes_tw<DIR, MAXR, LC, REV, ONE, P2>(ln, pl, p0, p1, j, tw);
}
template <int DIR, int MAXR, int LC, int REV, bool ONE = false, bool P2 = false, typename C>
__device__ __forceinline__ void lds_passes(C *ln, const FftPlan &pl, int p0, int p1, int j, TwStaged<C> tw) {
    lds_passes_tw<DIR, MAXR, LC, REV, ONE, P2>(ln, pl, p0, p1, j, tw);
}

// true when every pass of the compile-time plan of length L is radix 8 (its twiddle bases fit in
// L/8 table entries)
__host__ __device__ constexpr bool all_radix8(int L, int maxr) {
    if (L <= 0) return false;
    const FftPlan P = make_plan(L, maxr, false);
    for (int p = 0; p < P.npass; ++p)
        if (P.radix[p] != 8) return false;
    return P.npass > 0;
}

// compile-time pass count of the specialized plan (0 for the runtime plan)
template <int LC, int MAXR> __host__ __device__ constexpr int npass_of() {
    if constexpr (LC > 0) return make_plan(LC, MAXR, false).npass;
    else return 0;
}

}  // namespace dda
