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
#include <vector>

using namespace ssm;

template <typename V, int R, bool INV>
static void emulate_pass(V* buf, int off0, int ls, int lm, int lns, int gl, const V* twl)
{
    using P = Pass<V, R, INV>;
    std::vector<V> regs(64 * P::B * R);
    for (int lane = 0; lane < 64; ++lane)
        P::read(buf, off0, ls, lm, lns, gl, twl, lane, *reinterpret_cast<V(*)[P::B][R]>(&regs[lane * P::B * R]));
    for (int lane = 0; lane < 64; ++lane)
        P::write(buf, off0, ls, lm, lns, gl, lane, *reinterpret_cast<V(*)[P::B][R]>(&regs[lane * P::B * R]));
}

template <typename V, bool INV>
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
            if (bits == 4) emulate_pass<V, 16, INV>(buf, g0 * ls, ls, lm, lns, gl, twl);
            else if (bits == 3) emulate_pass<V, 8, INV>(buf, g0 * ls, ls, lm, lns, gl, twl);
            else if (bits == 2) emulate_pass<V, 4, INV>(buf, g0 * ls, ls, lm, lns, gl, twl);
            else emulate_pass<V, 2, INV>(buf, g0 * ls, ls, lm, lns, gl, twl);
            lns += bits;
        }
    }
}

// the compile-time passes (PassCT), same lockstep emulation
template <typename V, bool INV, int LM, int MAXB, int LNS>
static void host_passes_ct(V* buf, int off0, int gl, const V* twl)
{
    if constexpr (LNS < LM) {
        constexpr int bits = fft_next_bits(LM - LNS, MAXB);
        constexpr int R = 1 << bits;
        using P = PassCT<V, R, INV, LM, LNS>;
        std::vector<V> regs(64 * P::B * R);
        for (int lane = 0; lane < 64; ++lane)
            P::read(buf, off0, gl, twl, lane, *reinterpret_cast<V(*)[P::B][R]>(&regs[lane * P::B * R]));
        for (int lane = 0; lane < 64; ++lane)
            P::write(buf, off0, gl, lane, *reinterpret_cast<V(*)[P::B][R]>(&regs[lane * P::B * R]));
        host_passes_ct<V, INV, LM, MAXB, LNS + bits>(buf, off0, gl, twl);
    }
}

template <typename V, bool INV, int LM, int MAXB>
static void host_fft_lines_ct(V* buf, int nl, const V* twl)
{
    constexpr int lpg = fft_group_lines(LM);
    for (int g0 = 0; g0 < nl; g0 += lpg)
        host_passes_ct<V, INV, LM, MAXB, 0>(buf, g0 << LM, nl - g0 < lpg ? nl - g0 : lpg, twl);
}

template <typename V, bool INV, int MAXB, int LM = 1>
static void host_fft_ct_dispatch(V* buf, int nl, int lm, const V* twl)
{
    if constexpr (LM <= 10) {
        if (lm == LM) host_fft_lines_ct<V, INV, LM, MAXB>(buf, nl, twl);
        else host_fft_ct_dispatch<V, INV, MAXB, LM + 1>(buf, nl, lm, twl);
    }
}

// maxb < 0: the compile-time passes with cap -maxb (dense layout only)
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
    if (maxb > 0) host_fft_lines<V, INV>(buf.data(), nl, ls, lm, twl.data(), maxb);
    else if (maxb == -2) host_fft_ct_dispatch<V, INV, 2>(buf.data(), nl, lm, twl.data());
    else if (maxb == -3) host_fft_ct_dispatch<V, INV, 3>(buf.data(), nl, lm, twl.data());
    else host_fft_ct_dispatch<V, INV, 4>(buf.data(), nl, lm, twl.data());
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

int main()
{
    int bad = 0;
    for (int maxb : {2, 3, 4, -2, -3, -4})
    for (int lm = 0; lm <= 10; ++lm) {
        // one line, an odd count, and a full group plus a partial one
        const int nls[3] = {1, 3, (1 << (10 - lm)) + (lm < 10 ? 3 : 1)};
        for (int t = 0; t < 3; ++t) {
            const int nl = nls[t];
            if ((long long)nl << (2 * lm) > (1LL << 22)) continue;  // naive DFT cost cap
            const int pad = (t == 1 && maxb > 0) ? 1 : 0;
            const double e64f = check<double2, false>(lm, nl, pad, 11 + lm, maxb);
            const double e64i = check<double2, true>(lm, nl, pad, 13 + lm, maxb);
            const double e32f = check<float2, false>(lm, nl, pad, 17 + lm, maxb);
            const double e32i = check<float2, true>(lm, nl, pad, 19 + lm, maxb);
            std::printf("maxb=%d m=%5d lines=%5d fp64 %.2e %.2e fp32 %.2e %.2e\n", maxb, 1 << lm, nl,
                        e64f, e64i, e32f, e32i);
            if (e64f > 1e-14 || e64i > 1e-14 || e32f > 2e-6 || e32i > 2e-6) bad = 1;
        }
    }
    std::printf(bad ? "FAIL\n" : "OK\n");
    return bad;
}
