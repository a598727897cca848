// Power-of-two complex FFT building blocks of the gfx950 string-method
// kernels.  The zero-padded transforms of the dipolar convolution (Sec. II.A,
// eq. (6): a discrete convolution evaluated with FFTs) are built from these.
//
// fft_lines() transforms a set of lines held in LDS with Stockham passes of
// radix 16, 8, 4 or 2 (the widest radix a kernel instantiates is a template
// choice).  A wavefront owns a group of lines of 1024 elements in
// total, so every pass has exactly 1024/R butterflies per group, i.e.
// 16/R butterflies (16 complex values) per lane, and the lane reads all of
// its inputs before any lane of the wavefront writes: the pass can run in
// place with wavefront-level ordering only.
//
// The pass bodies are __host__ __device__ so that the host test suite can
// run them with the 64 lanes of a wavefront emulated one after another
// (all reads, then all writes), which is exactly the lockstep semantics the
// device relies on.
#pragma once

#include <hip/hip_runtime.h>

namespace ssm {

// exp(-2 pi i k / 16), k = 0..15, to double precision
constexpr double kW16re[16] = {
    1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508977,
    0.0, -0.38268343236508977, -0.70710678118654752, -0.92387953251128674,
    -1.0, -0.92387953251128674, -0.70710678118654752, -0.38268343236508977,
    0.0, 0.38268343236508977, 0.70710678118654752, 0.92387953251128674};
constexpr double kW16im[16] = {
    0.0, -0.38268343236508977, -0.70710678118654752, -0.92387953251128674,
    -1.0, -0.92387953251128674, -0.70710678118654752, -0.38268343236508977,
    0.0, 0.38268343236508977, 0.70710678118654752, 0.92387953251128674,
    1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508977};

template <typename V>
__host__ __device__ __forceinline__ V mk(decltype(V::x) a, decltype(V::x) b) { V r; r.x = a; r.y = b; return r; }
template <typename V>
__host__ __device__ __forceinline__ V cadd(V a, V b) { return mk<V>(a.x + b.x, a.y + b.y); }
template <typename V>
__host__ __device__ __forceinline__ V csub(V a, V b) { return mk<V>(a.x - b.x, a.y - b.y); }
template <typename V>
__host__ __device__ __forceinline__ V cmul(V a, V b) { return mk<V>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
// a * conj(b)
template <typename V>
__host__ __device__ __forceinline__ V cmulc(V a, V b) { return mk<V>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y); }
template <bool INV, typename V>
__host__ __device__ __forceinline__ V twm(V a, V w) { return INV ? cmulc(a, w) : cmul(a, w); }

// a * exp(-2 pi i e/16) (conjugate twiddle for INV).  Called with e a
// compile-time constant after unrolling, so the trivial factors 1, -1, -i, i
// cost no multiplications (x * 0 cannot be folded away in IEEE arithmetic).
template <bool INV, typename V>
__host__ __device__ __forceinline__ V twc16(V a, int e)
{
    using S = decltype(V::x);
    e &= 15;
    if (e == 0) return a;
    if (e == 8) return mk<V>(-a.x, -a.y);
    if (e == 4) return INV ? mk<V>(-a.y, a.x) : mk<V>(a.y, -a.x);
    if (e == 12) return INV ? mk<V>(a.y, -a.x) : mk<V>(-a.y, a.x);
    return cmul(a, mk<V>((S)kW16re[e], (S)(INV ? -kW16im[e] : kW16im[e])));
}

// 1: butterflies with a non-trivial twiddle in the in-register DFTs use the
// fused form of twfma16 (fewer instructions; the difference output carries
// the rounding of the sum once more)
#ifndef SSM_FFT_FMA_BFLY
#define SSM_FFT_FMA_BFLY 1
#endif

// u + v * exp(-2 pi i e/16) (conjugate twiddle for INV) for e not a
// multiple of 4, as fused multiply-adds.  For e = 2, 6, 10, 14 the twiddle's
// parts have equal magnitude: one sum or difference of v's parts, then one
// fused multiply-add per output part.
template <bool INV, typename V>
__host__ __device__ __forceinline__ V twfma16(V u, V v, int e)
{
    using S = decltype(V::x);
    e &= 15;
    const S c = (S)kW16re[e], s = (S)(INV ? -kW16im[e] : kW16im[e]);
    if ((e & 3) == 2) {
        // s = +-c: u + c (v.x - (s/c) v.y, v.y + (s/c) v.x)
        const bool same = (s > 0) == (c > 0);
        const S ax = same ? v.x - v.y : v.x + v.y;
        const S ay = same ? v.y + v.x : v.y - v.x;
        return mk<V>(fma(c, ax, u.x), fma(c, ay, u.y));
    }
    return mk<V>(fma(c, v.x, fma(-s, v.y, u.x)), fma(c, v.y, fma(s, v.x, u.y)));
}

// In-register R-point DFT (R = 1, 2, 4, 8, 16), natural order in and out:
// bit-reversal permutation, then radix-2 decimation-in-time stages.
template <typename V, int R, bool INV>
__host__ __device__ __forceinline__ void dft_reg(V (&a)[R])
{
    if (R == 1) return;
    constexpr int LR = (R == 2) ? 1 : (R == 4) ? 2 : (R == 8) ? 3 : 4;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        int r = 0;
#pragma unroll
        for (int b = 0; b < LR; ++b) r |= ((i >> b) & 1) << (LR - 1 - b);
        if (r > i) { V t = a[i]; a[i] = a[r]; a[r] = t; }
    }
#pragma unroll
    for (int len = 2; len <= R; len <<= 1) {
        const int half = len >> 1;
#pragma unroll
        for (int i = 0; i < R; i += len) {
#pragma unroll
            for (int j = 0; j < half; ++j) {
                const int e = j * (16 / len);
                const V u = a[i + j];
                if (SSM_FFT_FMA_BFLY && (e & 3)) {
                    // u + w v straight into FMAs, u - w v as 2u - (u + w v):
                    // 6 instructions instead of a product and two sums (8)
                    const V t = twfma16<INV>(u, a[i + j + half], e);
                    a[i + j] = t;
                    a[i + j + half] = mk<V>(decltype(V::x)(2) * u.x - t.x, decltype(V::x)(2) * u.y - t.y);
                } else {
                    const V v = twc16<INV>(a[i + j + half], e);
                    a[i + j] = cadd(u, v);
                    a[i + j + half] = csub(u, v);
                }
            }
        }
    }
}

// LDS layout of the line buffers.  With SSM_LDS_PAD=1 one pad element
// follows every 16, which spreads the strided Stockham writes (stride R) over
// all banks at the cost of per-element address arithmetic (more registers);
// measured on gfx950 the registers cost more than the conflicts, so the
// default layout is dense.  lds_pad(i) is the physical index of element i.
#ifndef SSM_LDS_PAD
#define SSM_LDS_PAD 0
#endif
__host__ __device__ __forceinline__ int lds_pad(int i) { return SSM_LDS_PAD ? i + (i >> 4) : i; }
// physical size of a buffer of n elements
__host__ __device__ __forceinline__ int lds_padded_size(int n) { return SSM_LDS_PAD ? n + (n >> 4) + 1 : n; }

// One radix-R Stockham pass over a group of gl lines of length m = 2^lm
// (line stride ls) starting at element off0 of buf (padded layout).
// lns = log2 of the sub-transform length already done.  twl[e] =
// exp(-2 pi i e / (2 TST m)), e < 2 TST m (conjugated for the inverse), so
// the pass twiddle W_{Ns R}^{r k} is twl[TST ((r k) << (lm+1-lns-lr))]
// (TST = 3: the lines are the thirds of lines of length 3m, whose table
// serves them).
template <typename V, int R, bool INV, int TST = 1>
struct Pass {
    static constexpr int LR = (R == 2) ? 1 : (R == 4) ? 2 : (R == 8) ? 3 : 4;
    static constexpr int B = 16 / R;  // butterflies per lane

    __host__ __device__ static void read(const V* buf, int off0, int ls, int lm, int lns, int gl,
                                         const V* twl, int lane, V (&v)[B][R])
    {
        const int q = 1 << (lm - LR), lq = lm - LR;
        const int nbf = gl << lq;
        const int Ns = 1 << lns;
        const int tsh = lm + 1 - lns - LR;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int g = lane + 64 * b;
            if (g < nbf) {
                const int line = g >> lq, j = g & (q - 1), k = j & (Ns - 1);
                const int i0 = off0 + line * ls + j;
#pragma unroll
                for (int r = 0; r < R; ++r) v[b][r] = buf[lds_pad(i0 + r * q)];
                if (lns > 0) {
#pragma unroll
                    for (int r = 1; r < R; ++r) v[b][r] = twm<INV>(v[b][r], twl[TST * ((r * k) << tsh)]);
                }
                dft_reg<V, R, INV>(v[b]);
            }
        }
    }

    __host__ __device__ static void write(V* buf, int off0, int ls, int lm, int lns, int gl,
                                          int lane, const V (&v)[B][R])
    {
        const int q = 1 << (lm - LR), lq = lm - LR;
        const int nbf = gl << lq;
        const int Ns = 1 << lns;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int g = lane + 64 * b;
            if (g < nbf) {
                const int line = g >> lq, j = g & (q - 1), k = j & (Ns - 1);
                const int i0 = off0 + line * ls + ((j >> lns) << (lns + LR)) + k;
#pragma unroll
                for (int r = 0; r < R; ++r) buf[lds_pad(i0 + r * Ns)] = v[b][r];
            }
        }
    }
};

// Physical index of element i in a line buffer with one pad element after
// every 2^PADL (PADL = 0: dense).  Pads spread the strided Stockham
// accesses over the LDS banks.
template <int PADL>
__host__ __device__ __forceinline__ int padx(int i) { return PADL ? i + (i >> PADL) : i; }
// pad log2 used for lines of length 2^LM: at most the line length, so that
// every line starts at a multiple of the pad unit
__host__ __device__ constexpr int pad_for(int padl, int lm) { return padl == 0 ? 0 : (padl < lm ? padl : lm); }

// One radix-R pass as above with the line length 2^LM, the sub-transform
// length 2^LNS and the line stride 2^LM fixed at compile time: every index
// is a per-lane base plus constant offsets.  Groups hold 1024 elements, so
// butterfly b of a lane is g = lane + 64 b.  Lines are stored with pad
// log2 PADL (padx); the element offsets a pass adds to its per-lane base
// never cross a pad boundary differently from the offset itself, so
// padx(i0 + o) = padx(i0) + o + (o >> PADL).  Twiddle e of W_{2^(LM+1)} is
// twl[e << TWS] (TWS = 0: a table of exactly 2^(LM+1) entries).
// XOR swizzle of the low 4 index bits with the next 4 (a permutation within
// every aligned block of 256 elements): the handoff between the two radix-16
// passes of a length-256 transform is a 16x16 transpose, and the swizzle lets
// both its strided side and its contiguous side hit distinct LDS banks.
__host__ __device__ __forceinline__ int swz16(int i) { return i ^ ((i >> 4) & 15); }

// TST: the lines are sub-lines of lines 3x as long whose twiddle table
// (W_{6 * 2^LM}) serves them at stride 3 (lengths 3 2^a).
template <typename V, int R, bool INV, int LM, int LNS, int PADL = 0, int TWS = 0, bool SWR = false,
          bool SWW = false, int TST = 1>
struct PassCT {
    static constexpr int LR = (R == 2) ? 1 : (R == 4) ? 2 : (R == 8) ? 3 : 4;
    static constexpr int B = 16 / R;
    static constexpr int LQ = LM - LR, Q = 1 << LQ, NS = 1 << LNS, TSH = LM + 1 - LNS - LR + TWS;
    static_assert(LM <= 10 && LR <= LM - LNS, "pass does not fit the line");
    static_assert(PADL == 0 || PADL <= LM, "pad unit longer than a line");
    static_assert(!(SWR || SWW) || (PADL == 0 && LM >= 8), "swizzle needs dense lines of >= 256");
    static constexpr int po(int o) { return PADL ? o + (o >> PADL) : o; }

    __host__ __device__ static void read(const V* buf, int off0, int gl, const V* twl, int lane,
                                         V (&v)[B][R])
    {
        const int nbf = gl << LQ;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int g = lane | (b << 6);
            if (g < nbf) {
                const int line = g >> LQ, j = g & (Q - 1), k = j & (NS - 1);
                if constexpr (SWR) {
                    const int i0 = off0 + (line << LM) + j;
#pragma unroll
                    for (int r = 0; r < R; ++r) v[b][r] = buf[swz16(i0 + r * Q)];
                } else {
                    const V* base = buf + padx<PADL>(off0 + (line << LM) + j);
#pragma unroll
                    for (int r = 0; r < R; ++r) v[b][r] = base[po(r * Q)];
                }
                if (LNS > 0) {
#pragma unroll
                    for (int r = 1; r < R; ++r) v[b][r] = twm<INV>(v[b][r], twl[TST * ((r * k) << TSH)]);
                }
                dft_reg<V, R, INV>(v[b]);
            }
        }
    }

    __host__ __device__ static void write(V* buf, int off0, int gl, int lane, const V (&v)[B][R])
    {
        const int nbf = gl << LQ;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int g = lane | (b << 6);
            if (g < nbf) {
                const int line = g >> LQ, j = g & (Q - 1), k = j & (NS - 1);
                if constexpr (SWW) {
                    const int i0 = off0 + (line << LM) + ((j >> LNS) << (LNS + LR)) + k;
#pragma unroll
                    for (int r = 0; r < R; ++r) buf[swz16(i0 + r * NS)] = v[b][r];
                } else {
                    V* base = buf + padx<PADL>(off0 + (line << LM) + ((j >> LNS) << (LNS + LR)) + k);
#pragma unroll
                    for (int r = 0; r < R; ++r) base[po(r * NS)] = v[b][r];
                }
            }
        }
    }
};

// log2 radix of the next pass when rem bits of the length are left and
// passes are capped at maxb bits: the widest allowed radix, except that a
// remainder that would end in a lone radix-2 pass is split more evenly
// (e.g. 2^5 = 8*4, 2^9 = 8*8*8 with maxb 3; 4*4*2 for 2^5 with maxb 2).
__host__ __device__ constexpr int fft_next_bits(int rem, int maxb)
{
    if (rem <= maxb) return rem;
    if (maxb >= 4) return (rem == 5) ? 3 : (rem == 9 ? 3 : 4);
    if (maxb == 3) return (rem == 4) ? 2 : 3;
    return 2;
}

// lines per wavefront group: 1024 elements per group
__host__ __device__ constexpr int fft_group_lines(int lm) { return lm >= 10 ? 1 : (1 << (10 - lm)); }

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename V, int R, bool INV, int TST = 1>
__device__ __forceinline__ void run_pass(V* buf, int off0, int ls, int lm, int lns, int gl,
                                         const V* twl, int lane)
{
    using P = Pass<V, R, INV, TST>;
    V v[P::B][R];
    P::read(buf, off0, ls, lm, lns, gl, twl, lane, v);
    wave_sync();
    P::write(buf, off0, ls, lm, lns, gl, lane, v);
    wave_sync();
}

// Transform nl lines of length 2^lm at buf (stride ls, padded layout) in
// LDS; forward
// (exp(-2 pi i jk/m)) or unnormalised inverse.  twl: the LDS table of
// exp(-2 pi i e/(2m)), e < 2m.  MAXB (2 or 3) caps the pass radix at 2^MAXB;
// fewer pass kinds keep the register footprint of the caller small.  Call
// between workgroup barriers.
template <typename V, bool INV, int MAXB = 2, int TST = 1>
__device__ __forceinline__ void fft_lines(V* buf, int nl, int ls, int lm, const V* twl)
{
    if (lm == 0) return;
    int lane = threadIdx.x & 63;
    // opaque copy: per-lane addresses are recomputed at each call instead of
    // being hoisted (and kept live) across the caller's loops
    asm volatile("" : "+v"(lane));
    const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int lpg = fft_group_lines(lm);
    for (int g0 = wave * lpg; g0 < nl; g0 += nw * lpg) {
        const int gl = min(lpg, nl - g0);
        const int off0 = g0 * ls;
        int lns = 0, rem = lm;
        while (rem > 0) {
            const int bits = fft_next_bits(rem, MAXB);
            if (bits == 4) run_pass<V, 16, INV, TST>(buf, off0, ls, lm, lns, gl, twl, lane);
            else if (bits == 3) run_pass<V, 8, INV, TST>(buf, off0, ls, lm, lns, gl, twl, lane);
            else if (bits == 2) run_pass<V, 4, INV, TST>(buf, off0, ls, lm, lns, gl, twl, lane);
            else run_pass<V, 2, INV, TST>(buf, off0, ls, lm, lns, gl, twl, lane);
            lns += bits;
            rem -= bits;
        }
    }
}

// Passes from sub-length 2^LNS while the sub-length stays below 2^LEND
// (so passes [LNS, LEND) of the schedule; LEND = LM runs all the rest).
// SW: the swizzled handoff (swz16) between the passes starting at LNS = 0
// and LNS = 4: the first pass writes swizzled, the second reads swizzled.
template <typename V, bool INV, int LM, int MAXB, int LNS, int LEND, int PADL = 0, int TWS = 0, bool SW = false,
          int TST = 1>
__device__ __forceinline__ void fft_passes_ct_to(V* buf, int off0, int gl, const V* twl, int lane)
{
    static_assert(!SW || fft_next_bits(LM, MAXB) == 4, "swizzled handoff needs a radix-16 first pass");
    if constexpr (LNS < LEND) {
        constexpr int bits = fft_next_bits(LM - LNS, MAXB);
        constexpr int R = 1 << bits;
        using P = PassCT<V, R, INV, LM, LNS, PADL, TWS, SW && LNS == 4, SW && LNS == 0, TST>;
        V v[16 / R][R];
        P::read(buf, off0, gl, twl, lane, v);
        wave_sync();
        P::write(buf, off0, gl, lane, v);
        wave_sync();
        fft_passes_ct_to<V, INV, LM, MAXB, LNS + bits, LEND, PADL, TWS, SW, TST>(buf, off0, gl, twl, lane);
    }
}

// Passes from sub-length 2^LNS to exactly 2^LEND, scheduled on the
// LEND - LNS bits of that span (fft_next_bits), for a caller that runs the
// passes beyond LEND itself.
template <typename V, bool INV, int LM, int MAXB, int LNS, int LEND, int PADL = 0, int TST = 1>
__device__ __forceinline__ void fft_passes_ct_span(V* buf, int off0, int gl, const V* twl, int lane)
{
    if constexpr (LNS < LEND) {
        constexpr int bits = fft_next_bits(LEND - LNS, MAXB);
        constexpr int R = 1 << bits;
        using P = PassCT<V, R, INV, LM, LNS, PADL, 0, false, false, TST>;
        V v[16 / R][R];
        P::read(buf, off0, gl, twl, lane, v);
        wave_sync();
        P::write(buf, off0, gl, lane, v);
        wave_sync();
        fft_passes_ct_span<V, INV, LM, MAXB, LNS + bits, LEND, PADL, TST>(buf, off0, gl, twl, lane);
    }
}

// log2 sub-length at which the last pass of the schedule starts
__host__ __device__ constexpr int fft_last_lns(int lm, int maxb)
{
    int lns = 0;
    while (lns + fft_next_bits(lm - lns, maxb) < lm) lns += fft_next_bits(lm - lns, maxb);
    return lns;
}

// fft_lines for a line length 2^LM known at compile time (line stride 2^LM
// in the pad-PADL layout).  Same result as fft_lines up to rounding order.
template <typename V, bool INV, int LM, int MAXB, int PADL = 0, int TST = 1>
__device__ __forceinline__ void fft_lines_ct(V* buf, int nl, const V* twl)
{
    if constexpr (LM > 0) {
        int lane = threadIdx.x;
        // opaque copy (no per-lane address hoisting across the caller's
        // loops), then the mask restores the known range 0..63
        asm volatile("" : "+v"(lane));
        lane &= 63;
        const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
        constexpr int LPG = fft_group_lines(LM);
        for (int g0 = wave * LPG; g0 < nl; g0 += nw * LPG)
            fft_passes_ct_to<V, INV, LM, MAXB, 0, LM, PADL, 0, false, TST>(buf, g0 << LM, min(LPG, nl - g0), twl, lane);
    }
}

// ---------------------------------------------------------------------------
// Lengths m = 3 M, M = 2^lm (padded lengths 2m = 3 2^(lm+1): any padded
// length >= 2n - 1 gives the same convolution, and 3 2^a is often the
// smaller one).  A line of length m is three sub-lines of length M,
// sub-line r occupying positions [r M, (r + 1) M).
//
// Forward, decimation in frequency on natural-order input: for k < M the
// inputs x[k], x[k + M], x[k + 2M] become
//   y_r = sum_j x[k + j M] w^{j r} * W_m^{r k},  w = exp(-2 pi i / 3),
// stored at r M + k; the length-M transform of sub-line r then holds
// X[3 n + r] at position r M + n (output order permuted).
// Inverse, decimation in time: sub-line r holds at position n the input of
// frequency 3 n + r; after the length-M inverse transforms G_r of the
// sub-lines, x[k + j M] = sum_r G_r[k] W_m^{-r k} w^{-r j} in natural order.
// twl[e] = exp(-2 pi i e / (2m)), e < 2m, so W_m^{r k} = twl[2 r k].
// ---------------------------------------------------------------------------
// position of frequency q (forward output, inverse input) and its inverse
__host__ __device__ __forceinline__ int perm3(int q, int lm)
{
    // q / 3 for 0 <= q < 98304 by a multiply and shift
    const int d = (q * 43691) >> 17;
    return ((q - 3 * d) << lm) + d;
}
__host__ __device__ __forceinline__ int unperm3(int pos, int lm)
{
    return 3 * (pos & ((1 << lm) - 1)) + (pos >> lm);
}

template <bool INV, typename V>
__host__ __device__ __forceinline__ void radix3_bfly(V& a, V& b, V& c, V w1, V w2)
{
    using S = decltype(V::x);
    const S h = S(0.5), s3 = S(0.86602540378443864676);  // sqrt(3)/2
    if (INV) {
        b = cmulc(b, w1);
        c = cmulc(c, w2);
    }
    const V t1 = cadd(b, c), t2 = csub(b, c);
    const V m1 = mk<V>(a.x - h * t1.x, a.y - h * t1.y);
    // -i s3 t2 (forward), +i s3 t2 (inverse)
    const V rot = INV ? mk<V>(-s3 * t2.y, s3 * t2.x) : mk<V>(s3 * t2.y, -s3 * t2.x);
    a = cadd(a, t1);
    b = cadd(m1, rot);
    c = csub(m1, rot);
    if (!INV) {
        b = cmul(b, w1);
        c = cmul(c, w2);
    }
}

// The radix-3 step over nl lines of length 3M (stride ls) by all threads of
// the workgroup; in place, each butterfly on its own three elements.
template <typename V, bool INV>
__device__ __forceinline__ void radix3_step(V* buf, int nl, int ls, int lm, const V* twl)
{
    const int M = 1 << lm;
    for (int i = threadIdx.x; i < (nl << lm); i += blockDim.x) {
        const int line = i >> lm, k = i & (M - 1);
        const int i0 = line * ls + k;
        V a = buf[lds_pad(i0)], b = buf[lds_pad(i0 + M)], c = buf[lds_pad(i0 + 2 * M)];
        radix3_bfly<INV>(a, b, c, twl[2 * k], twl[4 * k]);
        buf[lds_pad(i0)] = a;
        buf[lds_pad(i0 + M)] = b;
        buf[lds_pad(i0 + 2 * M)] = c;
    }
}

// Transform of nl contiguous lines of length 3 2^lm (dense layout): forward
// with permuted output, inverse from permuted input (see above).  Call
// between workgroup barriers.
template <typename V, bool INV, int MAXB = 2>
__device__ __forceinline__ void fft_lines3(V* buf, int nl, int lm, const V* twl)
{
    if (!INV) {
        radix3_step<V, false>(buf, nl, 3 << lm, lm, twl);
        __syncthreads();
    }
    fft_lines<V, INV, MAXB, 3>(buf, 3 * nl, 1 << lm, lm, twl);
    if (INV) {
        __syncthreads();
        radix3_step<V, true>(buf, nl, 3 << lm, lm, twl);
    }
}

}  // namespace ssm
