// Host check of the LDS FFT passes (paper_1804_07135_amd/csrc/ssm_fft.hpp):
// runs the same pass code with the 64 lanes of a wavefront emulated in
// lockstep (every lane reads, then every lane writes) and compares with a
// naive DFT in long double, for the runtime-length passes (Pass) and the
// compile-time ones (PassCT).  Prints the worst relative error per length.
#include "ssm_fft.hpp"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <type_traits>
#include <vector>

using namespace ssm;

template <typename V, int R, bool INV, int TST = 1>
static void emulate_pass(V* buf, int off0, int ls, int lm, int lns, int gl, const V* twl)
{
    using P = Pass<V, R, INV, TST>;
    std::vector<V> regs(64 * P::B * R);
    for (int lane = 0; lane < 64; ++lane)
        P::read(buf, off0, ls, lm, lns, gl, twl, lane, *reinterpret_cast<V(*)[P::B][R]>(&regs[lane * P::B * R]));
    for (int lane = 0; lane < 64; ++lane)
        P::write(buf, off0, ls, lm, lns, gl, lane, *reinterpret_cast<V(*)[P::B][R]>(&regs[lane * P::B * R]));
}

template <typename V, bool INV, int TST = 1>
static void host_fft_lines(V* buf, int nl, int ls, int lm, const V* twl, int maxb)
{
    if (lm == 0) return;
    const int lpg = fft_group_lines(lm);
    for (int g0 = 0; g0 < nl; g0 += lpg) {
        const int gl = nl - g0 < lpg ? nl - g0 : lpg;
        int lns = 0;
        for (int rem = lm; rem > 0;) {
            const int bits = fft_next_bits(rem, maxb);
            rem -= bits;
            if (bits == 4) emulate_pass<V, 16, INV, TST>(buf, g0 * ls, ls, lm, lns, gl, twl);
            else if (bits == 3) emulate_pass<V, 8, INV, TST>(buf, g0 * ls, ls, lm, lns, gl, twl);
            else if (bits == 2) emulate_pass<V, 4, INV, TST>(buf, g0 * ls, ls, lm, lns, gl, twl);
            else emulate_pass<V, 2, INV, TST>(buf, g0 * ls, ls, lm, lns, gl, twl);
            lns += bits;
        }
    }
}

// the compile-time passes (PassCT), same lockstep emulation
template <typename V, bool INV, int LM, int MAXB, int LNS, int PADL, int TWS, bool SW = false, int TST = 1>
static void host_passes_ct(V* buf, int off0, int gl, const V* twl)
{
    if constexpr (LNS < LM) {
        constexpr int bits = fft_next_bits(LM - LNS, MAXB);
        constexpr int R = 1 << bits;
        using P = PassCT<V, R, INV, LM, LNS, PADL, TWS, SW && LNS == 4, SW && LNS == 0, TST>;
        std::vector<V> regs(64 * P::B * R);
        for (int lane = 0; lane < 64; ++lane)
            P::read(buf, off0, gl, twl, lane, *reinterpret_cast<V(*)[P::B][R]>(&regs[lane * P::B * R]));
        for (int lane = 0; lane < 64; ++lane)
            P::write(buf, off0, gl, lane, *reinterpret_cast<V(*)[P::B][R]>(&regs[lane * P::B * R]));
        host_passes_ct<V, INV, LM, MAXB, LNS + bits, PADL, TWS, SW, TST>(buf, off0, gl, twl);
    }
}

// naive DFT of every line of buf (element (l, j) at idx(l * m + j))
template <typename V, bool INV, typename F>
static std::vector<V> naive(const std::vector<V>& buf, int nl, int lm, F idx)
{
    using S = decltype(V::x);
    const int m = 1 << lm;
    std::vector<V> ref((size_t)nl * m);
    std::vector<long double> cs(m), sn(m);
    for (int e = 0; e < m; ++e) {
        const long double th = (INV ? 2.0L : -2.0L) * 3.14159265358979323846264338327950288L * e / m;
        cs[e] = cosl(th);
        sn[e] = sinl(th);
    }
    for (int l = 0; l < nl; ++l)
        for (int k = 0; k < m; ++k) {
            long double sr = 0, si = 0;
            for (int j = 0; j < m; ++j) {
                const int e = (int)((long long)j * k % m);
                const V x = buf[idx(l * m + j)];
                sr += x.x * cs[e] - x.y * sn[e];
                si += x.x * sn[e] + x.y * cs[e];
            }
            ref[(size_t)l * m + k] = mk<V>((S)sr, (S)si);
        }
    return ref;
}

// compile-time passes over nl lines of 2^LM in the pad-PADL layout, with the
// twiddles read at stride 2^TWS from a longer table
template <typename V, bool INV, int LM, int MAXB, int PADL, int TWS, bool SW = false>
static double check_ct(int nl, unsigned seed)
{
    using S = decltype(V::x);
    const int m = 1 << LM;
    const int nt = (2 * m) << TWS;
    std::vector<V> twl(nt);
    for (int e = 0; e < nt; ++e) {
        const long double th = 2.0L * 3.14159265358979323846264338327950288L * e / nt;
        twl[e] = mk<V>((S)cosl(th), (S)-sinl(th));
    }
    std::mt19937 rng(seed);
    std::normal_distribution<double> nd;
    const int n = nl * m;
    // sentinel-filled buffer: pad slots must stay untouched
    std::vector<V> buf(padx<PADL>(n - 1) + 1, mk<V>((S)1e30, (S)1e30));
    for (int i = 0; i < n; ++i) buf[padx<PADL>(i)] = mk<V>((S)nd(rng), (S)nd(rng));
    const std::vector<V> ref = naive<V, INV>(buf, nl, LM, [](int i) { return padx<PADL>(i); });
    constexpr int lpg = fft_group_lines(LM);
    for (int g0 = 0; g0 < nl; g0 += lpg)
        host_passes_ct<V, INV, LM, MAXB, 0, PADL, TWS, SW>(buf.data(), g0 << LM, nl - g0 < lpg ? nl - g0 : lpg,
                                                          twl.data());
    double worst = 0, nrm = 0;
    for (int i = 0; i < n; ++i) {
        const V a = buf[padx<PADL>(i)], b = ref[i];
        worst = fmax(worst, fabs((double)a.x - (double)b.x));
        worst = fmax(worst, fabs((double)a.y - (double)b.y));
        nrm = fmax(nrm, fabs((double)b.x) + fabs((double)b.y));
    }
    for (int i = 0; i < (int)buf.size(); ++i) {
        bool data = false;
        // a slot is data iff it is padx of some element; pads keep the sentinel
        if (PADL == 0) data = true;
        else {
            const int e = i - i / ((1 << PADL) + 1);
            data = padx<PADL>(e) == i;
        }
        if (!data && buf[i].x != (S)1e30) return 1e30;
    }
    return worst / (nrm > 0 ? nrm : 1);
}

template <int LM, int MAXB, int PADL, int TWS, bool SW = false>
static int run_ct()
{
    int bad = 0;
    const int nls[3] = {1, 3, fft_group_lines(LM) + (LM < 10 ? 3 : 1)};
    for (int t = 0; t < 3; ++t) {
        const int nl = nls[t];
        if ((long long)nl << (2 * LM) > (1LL << 22)) continue;
        const double e1 = check_ct<double2, false, LM, MAXB, PADL, TWS, SW>(nl, 11 + LM);
        const double e2 = check_ct<double2, true, LM, MAXB, PADL, TWS, SW>(nl, 13 + LM);
        const double e3 = check_ct<float2, false, LM, MAXB, PADL, TWS, SW>(nl, 17 + LM);
        const double e4 = check_ct<float2, true, LM, MAXB, PADL, TWS, SW>(nl, 19 + LM);
        std::printf("ct maxb=%d pad=%d tws=%d sw=%d m=%5d lines=%5d fp64 %.2e %.2e fp32 %.2e %.2e\n", MAXB, PADL,
                    TWS, (int)SW, 1 << LM, nl, e1, e2, e3, e4);
        if (e1 > 1e-14 || e2 > 1e-14 || e3 > 2e-6 || e4 > 2e-6) bad = 1;
    }
    return bad;
}

template <int LM, int MAXB>
static int run_ct_pads()
{
    int bad = run_ct<LM, MAXB, 0, 0>();
    bad |= run_ct<LM, MAXB, pad_for(4, LM), 0>();
    bad |= run_ct<LM, MAXB, pad_for(5, LM), 0>();
    bad |= run_ct<LM, MAXB, pad_for(6, LM), 2>();
    return bad;
}

template <int MAXB, int LM = 1>
static int run_ct_all()
{
    if constexpr (LM <= 10) return run_ct_pads<LM, MAXB>() | run_ct_all<MAXB, LM + 1>();
    else return 0;
}

template <typename V, bool INV>
static double check(int lm, int nl, int pad, unsigned seed, int maxb)
{
    using S = decltype(V::x);
    const int m = 1 << lm, ls = m + pad;
    std::vector<V> twl(2 * m);
    for (int e = 0; e < 2 * m; ++e) {
        const long double th = 2.0L * 3.14159265358979323846264338327950288L * e / (2.0L * m);
        twl[e] = mk<V>((S)cosl(th), (S)-sinl(th));
    }
    std::mt19937 rng(seed);
    std::normal_distribution<double> nd;
    std::vector<V> buf(lds_padded_size(nl * ls)), ref(nl * ls);
    for (int i = 0; i < nl * ls; ++i) buf[lds_pad(i)] = mk<V>((S)nd(rng), (S)nd(rng));
    std::vector<long double> xr(m), xi(m), cs(m), sn(m);
    for (int e = 0; e < m; ++e) {
        const long double th = (INV ? 2.0L : -2.0L) * 3.14159265358979323846264338327950288L * e / m;
        cs[e] = cosl(th);
        sn[e] = sinl(th);
    }
    double worst = 0;
    for (int l = 0; l < nl; ++l) {
        for (int j = 0; j < m; ++j) {
            xr[j] = buf[lds_pad(l * ls + j)].x;
            xi[j] = buf[lds_pad(l * ls + j)].y;
        }
        for (int k = 0; k < m; ++k) {
            long double sr = 0, si = 0;
            for (int j = 0; j < m; ++j) {
                const int e = (int)((long long)j * k % m);
                sr += xr[j] * cs[e] - xi[j] * sn[e];
                si += xr[j] * sn[e] + xi[j] * cs[e];
            }
            ref[l * ls + k] = mk<V>((S)sr, (S)si);
        }
    }
    host_fft_lines<V, INV>(buf.data(), nl, ls, lm, twl.data(), maxb);
    double nrm = 0;
    for (int l = 0; l < nl; ++l)
        for (int k = 0; k < m; ++k) {
            const V a = buf[lds_pad(l * ls + k)], b = ref[l * ls + k];
            worst = fmax(worst, fabs((double)a.x - (double)b.x));
            worst = fmax(worst, fabs((double)a.y - (double)b.y));
            nrm = fmax(nrm, fabs((double)b.x) + fabs((double)b.y));
        }
    return worst / (nrm > 0 ? nrm : 1);
}

// the compile-time passes over the 3 nl sub-lines of length 2^LM with the
// parent lines' table at stride 3 (the x kernels and the compile-time
// 3 2^a convolution body), groups as on the device,
// lines in the pad-PADL layout
template <typename V, bool INV, int LM, int MAXB, int PADL>
static void host_lines3_ct(V* buf, int nsub, const V* twl)
{
    constexpr int LPG = fft_group_lines(LM);
    for (int g0 = 0; g0 < nsub; g0 += LPG)
        host_passes_ct<V, INV, LM, MAXB, 0, PADL, 0, false, 3>(buf, g0 << LM, std::min(LPG, nsub - g0), twl);
}

template <typename V, bool INV, int MAXB, int PADL>
static bool host_lines3_ct_lm(V* buf, int nsub, int lm, const V* twl)
{
    switch (lm) {
    case 4: host_lines3_ct<V, INV, 4, MAXB, PADL>(buf, nsub, twl); return true;
    case 5: host_lines3_ct<V, INV, 5, MAXB, PADL>(buf, nsub, twl); return true;
    case 6: host_lines3_ct<V, INV, 6, MAXB, PADL>(buf, nsub, twl); return true;
    case 7: host_lines3_ct<V, INV, 7, MAXB, PADL>(buf, nsub, twl); return true;
    default: return false;
    }
}

template <typename V, bool INV, int MAXB>
static bool host_lines3_ct_any(V* buf, int nsub, int lm, int padl, const V* twl)
{
    return padl ? host_lines3_ct_lm<V, INV, MAXB, 4>(buf, nsub, lm, twl)
                : host_lines3_ct_lm<V, INV, MAXB, 0>(buf, nsub, lm, twl);
}

// Lines of length m = 3 2^lm (fft_lines3): the radix-3 step of every
// (line, k) butterfly (independent, so any order), and the power-of-two
// passes over the 3 nl sub-lines with the length-2m table at stride 3
// (runtime passes, or with ct the compile-time ones, in the dense layout or
// with padl = 4 the pad-4 layout).
// Forward: natural input, frequency q at position perm3(q); inverse: input
// of frequency q at perm3(q), natural output.
template <typename V, bool INV>
static double check3(int lm, int nl, unsigned seed, int maxb, bool ct = false, int padl = 0)
{
    using S = decltype(V::x);
    const int M = 1 << lm, m = 3 * M;
    std::vector<V> twl(2 * m);
    for (int e = 0; e < 2 * m; ++e) {
        const long double th = 2.0L * 3.14159265358979323846264338327950288L * e / (2.0L * m);
        twl[e] = mk<V>((S)cosl(th), (S)-sinl(th));
    }
    std::mt19937 rng(seed);
    std::normal_distribution<double> nd;
    std::vector<V> x((size_t)nl * m), buf((size_t)nl * m);
    for (auto& v : x) v = mk<V>((S)nd(rng), (S)nd(rng));
    // reference DFT of length m, natural order in and out
    std::vector<V> ref((size_t)nl * m);
    std::vector<long double> cs(m), sn(m);
    for (int e = 0; e < m; ++e) {
        const long double th = (INV ? 2.0L : -2.0L) * 3.14159265358979323846264338327950288L * e / m;
        cs[e] = cosl(th);
        sn[e] = sinl(th);
    }
    for (int l = 0; l < nl; ++l)
        for (int k = 0; k < m; ++k) {
            long double sr = 0, si = 0;
            for (int j = 0; j < m; ++j) {
                const int e = (int)((long long)j * k % m);
                const V v = x[(size_t)l * m + j];
                sr += v.x * cs[e] - v.y * sn[e];
                si += v.x * sn[e] + v.y * cs[e];
            }
            ref[(size_t)l * m + k] = mk<V>((S)sr, (S)si);
        }
    // physical position of element i of the lines
    auto P = [&](size_t i) { return padl ? i + (i >> padl) : i; };
    buf.assign(P((size_t)nl * m) + 1, mk<V>((S)0, (S)0));
    for (int l = 0; l < nl; ++l)
        for (int q = 0; q < m; ++q) buf[P((size_t)l * m + (INV ? perm3(q, lm) : q))] = x[(size_t)l * m + q];
    auto step = [&](auto inv) {
        for (int i = 0; i < nl * M; ++i) {
            const int line = i >> lm, k = i & (M - 1);
            const size_t i0 = (size_t)line * m + k;
            radix3_bfly<decltype(inv)::value>(buf[P(i0)], buf[P(i0 + M)], buf[P(i0 + 2 * M)], twl[2 * k],
                                              twl[4 * k]);
        }
    };
    if (!INV) step(std::false_type{});
    if (!ct) host_fft_lines<V, INV, 3>(buf.data(), 3 * nl, M, lm, twl.data(), maxb);
    else if (maxb == 2) host_lines3_ct_any<V, INV, 2>(buf.data(), 3 * nl, lm, padl, twl.data());
    else if (maxb == 3) host_lines3_ct_any<V, INV, 3>(buf.data(), 3 * nl, lm, padl, twl.data());
    else host_lines3_ct_any<V, INV, 4>(buf.data(), 3 * nl, lm, padl, twl.data());
    if (INV) step(std::true_type{});
    double worst = 0, nrm = 0;
    for (int l = 0; l < nl; ++l)
        for (int q = 0; q < m; ++q) {
            const V a = buf[P((size_t)l * m + (INV ? q : perm3(q, lm)))], b = ref[(size_t)l * m + q];
            worst = fmax(worst, fabs((double)a.x - (double)b.x));
            worst = fmax(worst, fabs((double)a.y - (double)b.y));
            nrm = fmax(nrm, fabs((double)b.x) + fabs((double)b.y));
        }
    return worst / (nrm > 0 ? nrm : 1);
}

int main()
{
    int bad = 0;
    // the position map of the 3 2^lm order and its inverse
    for (int lm = 0; lm <= 15; ++lm)
        for (int q = 0; q < (3 << lm) && q < 98304; q += (lm > 10 ? 7 : 1)) {
            const int pos = perm3(q, lm);
            if (pos != (q % 3) * (1 << lm) + q / 3 || unperm3(pos, lm) != q) {
                std::printf("perm3 wrong at lm=%d q=%d\n", lm, q);
                bad = 1;
                break;
            }
        }
    for (int maxb = 2; maxb <= 4; ++maxb)
        for (int lm = 0; lm <= 8; ++lm) {
            const int nls[3] = {1, 2, 1024 / (3 << lm) + 2};
            for (int t = 0; t < 3; ++t) {
                const int nl = nls[t];
                if ((long long)nl * (9LL << (2 * lm)) > (1LL << 22)) continue;
                const double e64f = check3<double2, false>(lm, nl, 23 + lm, maxb);
                const double e64i = check3<double2, true>(lm, nl, 29 + lm, maxb);
                const double e32f = check3<float2, false>(lm, nl, 31 + lm, maxb);
                const double e32i = check3<float2, true>(lm, nl, 37 + lm, maxb);
                std::printf("radix3 maxb=%d m=%5d lines=%5d fp64 %.2e %.2e fp32 %.2e %.2e\n", maxb, 3 << lm, nl,
                            e64f, e64i, e32f, e32i);
                if (e64f > 1e-14 || e64i > 1e-14 || e32f > 2e-6 || e32i > 2e-6) bad = 1;
            }
        }
    // the same with the compile-time sub-line passes (lengths 48 .. 384),
    // dense and pad-4 layouts
    for (int maxb = 2; maxb <= 4; ++maxb)
        for (int lm = 4; lm <= 7; ++lm) {
            const int nls[2] = {1, 1024 / (1 << lm) + 1};
            for (int t = 0; t < 4; ++t) {
                const int nl = nls[t & 1], padl = t < 2 ? 0 : 4;
                const double e64f = check3<double2, false>(lm, nl, 41 + lm, maxb, true, padl);
                const double e64i = check3<double2, true>(lm, nl, 43 + lm, maxb, true, padl);
                const double e32f = check3<float2, false>(lm, nl, 47 + lm, maxb, true, padl);
                const double e32i = check3<float2, true>(lm, nl, 53 + lm, maxb, true, padl);
                std::printf("radix3 ct maxb=%d m=%5d lines=%5d pad %d fp64 %.2e %.2e fp32 %.2e %.2e\n", maxb,
                            3 << lm, nl, padl, e64f, e64i, e32f, e32i);
                if (e64f > 1e-14 || e64i > 1e-14 || e32f > 2e-6 || e32i > 2e-6) bad = 1;
            }
        }
    for (int maxb = 2; maxb <= 4; ++maxb)
    for (int lm = 0; lm <= 10; ++lm) {
        // one line, an odd count, and a full group plus a partial one
        const int nls[3] = {1, 3, (1 << (10 - lm)) + (lm < 10 ? 3 : 1)};
        for (int t = 0; t < 3; ++t) {
            const int nl = nls[t];
            if ((long long)nl << (2 * lm) > (1LL << 22)) continue;  // naive DFT cost cap
            const int pad = t == 1 ? 1 : 0;
            const double e64f = check<double2, false>(lm, nl, pad, 11 + lm, maxb);
            const double e64i = check<double2, true>(lm, nl, pad, 13 + lm, maxb);
            const double e32f = check<float2, false>(lm, nl, pad, 17 + lm, maxb);
            const double e32i = check<float2, true>(lm, nl, pad, 19 + lm, maxb);
            std::printf("maxb=%d m=%5d lines=%5d fp64 %.2e %.2e fp32 %.2e %.2e\n", maxb, 1 << lm, nl,
                        e64f, e64i, e32f, e32i);
            if (e64f > 1e-14 || e64i > 1e-14 || e32f > 2e-6 || e32i > 2e-6) bad = 1;
        }
    }
    bad |= run_ct_all<2>();
    bad |= run_ct_all<3>();
    bad |= run_ct_all<4>();
    // swizzled handoff between radix-16 passes
    bad |= run_ct<8, 4, 0, 0, true>();
    bad |= run_ct<10, 4, 0, 0, true>();
    std::printf(bad ? "FAIL\n" : "OK\n");
    return bad;
}
