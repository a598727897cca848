// Host runtime and C ABI of the gfx950 simplified-string-method library.
// See include/ssm.h for the contract of every entry point.
#include "ssm.h"
#include "ssm_fft.hpp"
#include "ssm_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

using namespace ssm;

namespace {

constexpr int kVersion = 1;
constexpr size_t kAlign = 256;
constexpr size_t kLdsMax = 160 * 1024;
// work maps: forward / inverse x per length kind (2 + 2), convolution per
// build slot, arc, site, image, per-problem site, 4-site
constexpr int kNumMaps = 4 + kConvSlots + 5;

thread_local std::string g_create_error;

const char* const kKernelNames[SSM_N_KERNELS] = {
    "k_xfwd", "k_conv", "k_xinv", "k_arc", "k_reduce", "k_interp",
    "k_tan1", "k_tan2", "k_tanred", "k_spec", "k_util", "graph", "k_rk"};

int pow2ceil(int n)
{
    int m = 1;
    while (m < n) m <<= 1;
    return m;
}

int ilog2(int m)
{
    int l = 0;
    while ((1 << l) < m) ++l;
    return l;
}

size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Half padded transform length m >= n of an x or y axis.  Any padded
// length 2m >= 2n - 1 gives the same zero-padded convolution, so this only
// chooses the cheaper transform: the power of two >= n, or the length
// 3 2^a >= n (a >= 4, m <= 768) when that is smaller and not a slower kind
// of transform: fast(lg, f3) says whether the length 2^lg (f3 = 0) or
// 3 2^lg (f3 = 1) takes the compile-time-length transforms, which run faster
// than the runtime-length ones.  lg = log2 of the power-of-two factor,
// f3 = 1 for 3 2^a.
#ifndef SSM_LEN3
#define SSM_LEN3 1
#endif
// 1: the spline step in one pass where the image counts allow
#ifndef SSM_SPLW
#define SSM_SPLW 1
#endif
#ifndef SSM_LEN3_CT_X
#define SSM_LEN3_CT_X 3
#endif
#ifndef SSM_LEN3_CT_Y
#define SSM_LEN3_CT_Y 3
#endif
template <typename Fast>
void transform_len(int n, Fast fast, int& m, int& lg, int& f3)
{
    m = pow2ceil(n);
    lg = ilog2(m);
    f3 = 0;
    if (!SSM_LEN3 || n <= 32) return;
    int t = 48, a = 4;
    while (t < n) { t *= 2; ++a; }
    if (t < m && t <= 768 && (fast(a, 1) || !fast(lg, 0))) { m = t; lg = a; f3 = 1; }
}

struct Tiles {
    int ytf;    // rows per tile, forward x kernel
    int yt;     // rows per tile, inverse x kernel + epilogue
    int gconv;  // slices per convolution workgroup
};

// Everything about a batch that follows from the problem list: descriptors,
// work maps and the carve-up of the workspace.
struct Plan {
    int prec = 0;
    int np = 0;
    int mz = 1;
    int red_kinds = 0;                // reduction kernels in use (launch_reduce)
    bool rk = false;                  // workspace of the adaptive integrator reserved
    int kmax = 0;                     // largest image count of the batch
    int kmax_le16 = 0, kmax_le32 = 0; // largest image counts <= 16 and <= 32 (0: none)
    size_t tsize = 8;                 // bytes of one spin component
    std::vector<Prob> P;
    std::vector<Tiles> tiles;         // tile shapes in use, per problem
    std::vector<int> geo;             // problem -> distinct-shape index
    std::vector<std::tuple<int, int, int>> shapes;
    std::vector<long long> nh_size;   // elements per distinct shape
    std::vector<int> wm_xf[2], wm_xi[2], wm_conv[kConvSlots];  // per kind
    std::vector<int> wm_arc, wm_site, wm_img, wm_sitep, wm_site4;
    long long n_img = 0, n_spin = 0, n_x = 0, n_nh = 0, n_ep = 0, n_ap = 0, n_fp = 0, n_fm = 0;
    size_t lds_xf = 0, lds_xi = 0, lds_conv = 0;
    size_t scratch_bytes = 0;
    // workspace offsets
    size_t o_P, o_wm, o_tw, o_tw64, o_s, o_ss, o_h, o_nh, o_big, o_ep, o_ap, o_fp, o_E, o_T,
        o_alpha, o_w, o_tc, o_fn, o_fm, o_j, o_done, o_iters, o_skip, o_flags, o_seg, o_cnt, total;
    // adaptive integrator (when rk): 7 slopes + stage input (string-sized),
    // per-image state
    size_t o_rk_k = 0, o_rk_y = 0, o_rk_t = 0, o_rk_dtp = 0, o_rk_dtu = 0, o_rk_cap = 0, o_rk_act = 0,
           o_rk_acc = 0, o_rk_cnt = 0, o_rk_nact = 0;
    // step-2 options: spline arrays, climbing image per problem, spline
    // validity per problem, climbing coefficient per problem
    size_t o_s2 = 0, o_kci = 0, o_splok = 0, o_cic = 0;
};

// LDS bytes of the FFT kernels: twiddle table (2m complex) + line buffer in
// the padded layout of ssm_fft.hpp (+ the tile's real field for k_xinv).
size_t lds_xfwd(const Prob& p, int yt, size_t tsize)
{
    const int n = yt * p.mx;
    const int pl = x_padl(p.lmx, p.f3x, (int)tsize);
    const int lines = pl ? padded_len(n, pl) : lds_padded_size(n);
    return (size_t)(2 * p.mx + lines) * 2 * tsize;
}

size_t lds_xinv(const Prob& p, int yt, size_t tsize)
{
    const int n = yt * p.mx;
    const int pl = x_padl(p.lmx, p.f3x, (int)tsize);
    const int lines = pl ? padded_len(n, pl) : lds_padded_size(n);
    return (size_t)(2 * p.mx + lines) * 2 * tsize + (size_t)3 * yt * p.nx * tsize;
}

size_t lds_convg(const Prob& p, int G, size_t tsize)
{
    const int n = G * 3 * p.nz * p.my;
    if (conv_ct_shape(p.mz, p.lmy, p.f3y) || conv_ct3_shape(p.mz, p.lmy, p.f3y))
        return (size_t)(2 * p.my + padded_len(n, conv_padl(p.mz, p.lmy, p.f3y, (int)tsize))) * 2 * tsize;
    return (size_t)(2 * p.my + lds_padded_size(n)) * 2 * tsize;
}

ssm_status check_problems(const ssm_problem* pr, int np, int prec, std::string& err)
{
    if (!pr || np < 1) { err = "no problems"; return SSM_EINVAL; }
    if (np > 256) { err = "more than 256 problems"; return SSM_EUNSUPPORTED; }
    if (prec != SSM_FP64 && prec != SSM_FP32_MIXED) { err = "unknown precision"; return SSM_EINVAL; }
    int mz0 = -1;
    for (int i = 0; i < np; ++i) {
        const ssm_problem& q = pr[i];
        if (q.nx < 1 || q.ny < 1 || q.nz < 1 || q.n_images < 2) {
            err = "problem " + std::to_string(i) + ": dims must be >= 1 and n_images >= 2";
            return SSM_EINVAL;
        }
        if (!std::isfinite(q.J) || !std::isfinite(q.d) || !std::isfinite(q.ku) || !std::isfinite(q.dip)) {
            err = "problem " + std::to_string(i) + ": non-finite parameter";
            return SSM_EINVAL;
        }
        // (the inverse-x epilogue addresses an image with 32-bit byte
        // offsets, which these limits keep below 2^32)
        if (q.nx > 1024 || q.ny > 1024 || q.nz > 16 || q.n_images > 1024) {
            err = "problem " + std::to_string(i) + ": size beyond the supported limits";
            return SSM_EUNSUPPORTED;
        }
        const int mz = q.nz > 1 ? pow2ceil(q.nz) : 1;
        if (mz0 >= 0 && mz != mz0) {
            err = "all problems of a context need nz rounding to the same power of two";
            return SSM_EUNSUPPORTED;
        }
        mz0 = mz;
        const long long elems = (long long)q.n_images * 3 * q.nx * q.ny * q.nz;
        if (elems > (1LL << 40)) { err = "string too large"; return SSM_EUNSUPPORTED; }
    }
    return SSM_OK;
}

// Default tile shapes; autotuning may replace them.  Workgroups should fit
// three to a CU (LDS <= 52 KiB) and write or read >= 64-byte runs of the
// [img][kx][c][z][y] spectra.
constexpr size_t kLdsTarget = 52 * 1024;

// batch_rows: image rows (K nz ny), batch_slices: convolution slices
// (K (m_x + 1)) of every problem of the context, for the occupancy of a
// launch covering them all
Tiles default_tiles(const Prob& p, size_t tsize, long long batch_rows, long long batch_slices)
{
    Tiles t;
    const int cs = (int)(2 * tsize);
    const int ycap = std::max(2, pow2ceil(p.ny));
    int yf = std::max(2, 128 / cs);
    while (yf * p.mx < 4096 && yf < ycap && lds_xfwd(p, 2 * yf, tsize) <= kLdsTarget) yf *= 2;
    yf = std::min(yf, ycap);
    while (yf > 2 && lds_xfwd(p, yf, tsize) > kLdsTarget) yf /= 2;
    // small batches: more, shorter tiles (down to 64-byte runs) until a
    // launch has about four workgroups per CU
    while (yf * cs > 64 && batch_rows / yf < 1024) yf /= 2;
    t.ytf = yf;
    int yi = std::max(2, 128 / cs);
    while (yi * p.mx < 4096 && yi < ycap && lds_xinv(p, 2 * yi, tsize) <= kLdsTarget) yi *= 2;
    yi = std::min(yi, ycap);
    while (yi > 2 && lds_xinv(p, yi, tsize) > kLdsTarget) yi /= 2;
    t.yt = yi;
    const int per = 3 * p.nz * p.ny;
    int gmax = std::max(1, kConvElems / per);
    while (gmax > 1 && lds_convg(p, gmax, tsize) > kLdsTarget) --gmax;
    // as many slices per workgroup as keep about 1024 workgroups in a
    // launch over the whole batch (small lattices: several wavefronts' line
    // groups per workgroup)
    t.gconv = (int)std::max<long long>(1, std::min<long long>(gmax, batch_slices / 1024));
    return t;
}

int pad8(int n) { return (n + 7) / 8 * 8; }

void apply_tiles(Prob& p, const Tiles& t)
{
    p.ytf = t.ytf;
    p.ntyf = (p.ny + p.ytf - 1) / p.ytf;
    p.tilesf = p.nz * p.ntyf;
    p.wgf = pad8(p.K * p.tilesf);
    p.yt = t.yt;
    p.nty = (p.ny + p.yt - 1) / p.yt;
    p.tiles = p.nz * p.nty;
    p.wgi = pad8(p.K * p.tiles);
    p.gconv = t.gconv;
    p.xcd_remap = (t.gconv == 1) ? 1 : 0;
}

int conv_wgs(const Prob& p)
{
    if (p.xcd_remap) return ((p.mx + 1 + 7) / 8) * 8 * p.K;
    const long long slices = (long long)p.K * (p.mx + 1);
    const int w = (int)((slices + p.gconv - 1) / p.gconv);
    return (w + 7) / 8 * 8;
}

ssm_status build_plan(const ssm_problem* pr, int np, int prec_flags, const std::vector<Tiles>* tiles,
                      Plan& pl, std::string& err)
{
    const bool rk = (prec_flags & SSM_WITH_RK) != 0;
    const int prec = prec_flags & ~SSM_WITH_RK;
    ssm_status st = check_problems(pr, np, prec, err);
    if (st != SSM_OK) return st;
    pl = Plan();
    pl.prec = prec;
    pl.rk = rk;
    pl.np = np;
    pl.tsize = prec == SSM_FP64 ? 8 : 4;
    pl.P.resize(np);
    pl.geo.resize(np);
    std::map<std::tuple<int, int, int>, int> shape_id;
    long long img = 0, spin = 0, xo = 0, ep = 0, ap = 0, fp = 0, fm = 0;
    long long batch_rows = 0, batch_slices = 0;
    // SSM_LEN3_CT_X / _Y: precisions (bit 0 FP32-mixed, bit 1 FP64) in
    // which a compile-time 3 2^a length is preferred to a compile-time power
    // of two
    const int pbit = pl.tsize == 8 ? 2 : 1;
    const auto x_fast = [&](int lg, int f3) {
        return f3 ? x_ct3_len(lg, f3) && (SSM_LEN3_CT_X & pbit) : x_ct_len(lg, f3);
    };
    for (int i = 0; i < np; ++i) {
        batch_rows += (long long)pr[i].n_images * pr[i].nz * pr[i].ny;
        int mx, lg, f3;
        transform_len(pr[i].nx, x_fast, mx, lg, f3);
        batch_slices += (long long)pr[i].n_images * (mx + 1);
    }
    for (int i = 0; i < np; ++i) {
        const ssm_problem& q = pr[i];
        Prob& p = pl.P[i];
        std::memset(&p, 0, sizeof(p));
        p.nx = q.nx; p.ny = q.ny; p.nz = q.nz; p.K = q.n_images;
        p.mz = q.nz > 1 ? pow2ceil(q.nz) : 1;
        p.lmz = ilog2(p.mz);
        transform_len(q.nx, x_fast, p.mx, p.lmx, p.f3x);
        transform_len(q.ny, [&](int lg, int f3) { return conv_build(p.mz, lg, f3) > 0 && (!f3 || (SSM_LEN3_CT_Y & pbit)); },
                      p.my, p.lmy, p.f3y);
        p.pz = q.nz > 1 ? 2 * p.mz : 1;
        p.nhz = q.nz > 1 ? 2 : 1;
        p.N = (long long)q.nx * q.ny * q.nz;
        const Tiles t = tiles ? (*tiles)[i] : default_tiles(p, pl.tsize, batch_rows, batch_slices);
        apply_tiles(p, t);
        pl.tiles.push_back(t);
        if (lds_xfwd(p, p.ytf, pl.tsize) > kLdsMax || lds_xinv(p, p.yt, pl.tsize) > kLdsMax ||
            lds_convg(p, p.gconv, pl.tsize) > kLdsMax) {
            err = "problem " + std::to_string(i) + ": lattice too large for one workgroup's LDS";
            return SSM_EUNSUPPORTED;
        }
        p.img0 = (int)img;
        p.s_off = spin;
        p.x_off = xo;
        p.ep_off = ep;
        p.ap_off = ap;
        p.arc_chunks = (int)((3 * p.N + kNT * kArcEPT - 1) / (kNT * kArcEPT));
        // image groups: in FP32 groups of about three images (short groups
        // balance better than one long round, and the image each group
        // re-reads is mostly an L2 hit: the same chunk of neighbouring
        // groups lands on the same XCD; single images leave small lattices
        // with workgroups too short to pay for their start), at most 12288
        // workgroups per problem; in FP64 at least 512 workgroups (FP64
        // chunks carry twice the bytes and stream best ungrouped on large
        // lattices)
        const int arc_ng = pl.tsize == 4 ? std::min(12288 / p.arc_chunks, (p.K - 1 + 2) / 3)
                                         : (512 + p.arc_chunks - 1) / p.arc_chunks;
        p.arc_ng = std::max(1, std::min(p.K - 1, arc_ng));
        p.arc_g = (p.K - 1 + p.arc_ng - 1) / p.arc_ng;
        p.arc_ng = (p.K - 1 + p.arc_g - 1) / p.arc_g;
        // few images with few partials each: the whole reduction in one
        // workgroup (no hand-off between workgroups)
        p.red1 = (p.K <= kRed1MaxK && p.tiles * kNTerm + 4 * p.arc_chunks <= kRed1MaxPart) ? 1 : 0;
        p.ichunks = (int)((p.N + kNT - 1) / kNT);
        // spin buffers are 256-byte aligned, so an image is 16-byte aligned
        // when its element offset is a multiple of 4
        p.vec4 = (pl.tsize == 4 && p.N % 4 == 0 && spin % 4 == 0) ? 1 : 0;
        p.vec2 = (pl.tsize == 8 && p.N % 2 == 0 && spin % 2 == 0) ? 1 : 0;
        p.ichunks4 = p.vec4 ? (int)((p.N + 4 * kNT - 1) / (4 * kNT))
                            : p.vec2 ? (int)((p.N + 2 * kNT - 1) / (2 * kNT)) : p.ichunks;
        p.fp_off = fp;
        p.fm_off = fm;
        p.J = q.J; p.d = q.d; p.ku = q.ku; p.D = q.dip;
        img += p.K;
        spin += (long long)p.K * 3 * p.N;
        xo += (long long)p.K * (p.mx + 1) * 3 * p.nz * p.ny;
        xo = (xo + 31) & ~31LL;  // every problem's spectra start 256-byte aligned (paired 16-byte accesses)
        // sized for the smallest inverse tile (2 rows) so that retuned tiles
        // keep the workspace layout
        ep += (long long)p.K * p.nz * ((p.ny + 1) / 2) * kNTerm;
        ap += (long long)p.K * p.arc_chunks * 4;
        fp += (long long)p.K * p.ichunks * 2;
        fm += (long long)p.K * p.ichunks;
        const auto key = std::make_tuple(p.nx, p.ny, p.nz);
        auto it = shape_id.find(key);
        if (it == shape_id.end()) {
            const int id = (int)pl.shapes.size();
            shape_id[key] = id;
            pl.shapes.push_back(key);
            pl.nh_size.push_back(6LL * (p.mx + 1) * (2 * p.my) * p.pz);
            pl.geo[i] = id;
            // F1 + F2 scratch of the spectrum setup
            const long long f = 6LL * (p.mx + 1) * (2 * p.nz - 1) * ((2 * p.ny - 1) + 2 * p.my);
            pl.scratch_bytes = std::max(pl.scratch_bytes, (size_t)f * 8);
        } else {
            pl.geo[i] = it->second;
        }
        pl.mz = p.mz;
        pl.red_kinds |= p.red1 ? 2 : 1;
        pl.lds_xf = std::max(pl.lds_xf, lds_xfwd(p, p.ytf, pl.tsize));
        pl.lds_xi = std::max(pl.lds_xi, lds_xinv(p, p.yt, pl.tsize));
        pl.lds_conv = std::max(pl.lds_conv, lds_convg(p, p.gconv, pl.tsize));
    }
    // kernel-spectrum offsets per shape
    std::vector<long long> nh_off(pl.shapes.size());
    long long nh = 0;
    for (size_t g = 0; g < pl.shapes.size(); ++g) {
        nh_off[g] = nh;
        nh += (pl.nh_size[g] + 63) / 64 * 64;
    }
    for (int i = 0; i < np; ++i) pl.P[i].nh_off = nh_off[pl.geo[i]];
    pl.n_img = img; pl.n_spin = spin; pl.n_x = xo; pl.n_nh = nh;
    for (const Prob& q : pl.P) {
        pl.kmax = std::max(pl.kmax, q.K);
        if (q.K <= 16) pl.kmax_le16 = std::max(pl.kmax_le16, q.K);
        if (q.K <= 32) pl.kmax_le32 = std::max(pl.kmax_le32, q.K);
    }
    pl.n_ep = ep; pl.n_ap = ap; pl.n_fp = fp; pl.n_fm = fm;
    // work maps
    auto prefix = [&](std::vector<int>& v, auto count) {
        v.assign(np + 1, 0);
        for (int i = 0; i < np; ++i) v[i + 1] = v[i] + count(pl.P[i]);
    };
    // the FFT kernels per kind: other kinds' problems get no workgroups
    for (int k = 0; k < 2; ++k) {
        prefix(pl.wm_xf[k], [k](const Prob& p) { return p.f3x == k ? p.wgf : 0; });
        prefix(pl.wm_xi[k], [k](const Prob& p) { return p.f3x == k ? p.wgi : 0; });
    }
    for (int j = 0; j < kConvSlots; ++j)
        prefix(pl.wm_conv[j], [j](const Prob& p) {
            return conv_slot(conv_build(p.mz, p.lmy, p.f3y)) == j ? (int)conv_wgs(p) : 0;
        });
    prefix(pl.wm_arc, [](const Prob& p) { return p.arc_chunks * p.arc_ng; });
    prefix(pl.wm_site, [](const Prob& p) { return p.K * p.ichunks; });
    prefix(pl.wm_img, [](const Prob& p) { return p.K; });
    prefix(pl.wm_sitep, [](const Prob& p) { return p.ichunks; });
    prefix(pl.wm_site4, [](const Prob& p) { return p.K * p.ichunks4; });
    // workspace layout
    const size_t ts = pl.tsize, cs = 2 * ts;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = up(o + std::max<size_t>(bytes, 1)); return r; };
    pl.o_P = take(sizeof(Prob) * np);
    pl.o_wm = take(sizeof(int) * kNumMaps * (np + 1));
    pl.o_tw = take(cs * kTwCompact);
    pl.o_tw64 = take(16 * kTwM);
    pl.o_s = take(ts * spin);
    pl.o_ss = take(ts * spin);
    pl.o_h = take(ts * spin);
    pl.o_nh = take(ts * nh);
    // the convolution's last y pass reads whole transform lines of the
    // second spectrum buffer (up to m_y - 1 past a ragged line's end): one
    // line of slack after it keeps those reads inside the workspace
    int my_max = 1;
    for (const Prob& q : pl.P) my_max = std::max(my_max, q.my);
    pl.o_big = take(std::max((size_t)(2 * cs * xo + cs * my_max), pl.scratch_bytes));
    pl.o_ep = take(8 * ep);
    pl.o_ap = take(8 * ap);
    pl.o_fp = take(8 * fp);
    pl.o_E = take(8 * img);
    pl.o_T = take(8 * 4 * img);
    pl.o_alpha = take(8 * img);
    pl.o_w = take(8 * img);
    pl.o_tc = take(8 * 2 * img);
    pl.o_fn = take(8 * np);
    pl.o_fm = take(8 * fm);
    pl.o_j = take(4 * img);
    pl.o_done = take(4 * np);
    pl.o_iters = take(4 * np);
    pl.o_skip = take(4 * np);
    pl.o_flags = take(4);
    pl.o_seg = take(8 * img);
    pl.o_cnt = take(4 * np);
    pl.o_s2 = take(8 * (7 + kWRow) * img);  // spline: hh, sa, den, cp, A, B, H, operator row per image
    pl.o_kci = take(4 * np);
    pl.o_splok = take(4 * np);
    pl.o_cic = take(8 * np);
    if (rk) {
        pl.o_rk_k = take(7 * ts * spin);
        pl.o_rk_y = take(ts * spin);
        pl.o_rk_t = take(8 * img);
        pl.o_rk_dtp = take(8 * img);
        pl.o_rk_dtu = take(8 * img);
        pl.o_rk_cap = take(4 * img);
        pl.o_rk_act = take(4 * img);
        pl.o_rk_acc = take(4 * img);
        pl.o_rk_cnt = take(8 * img);
        pl.o_rk_nact = take(4);
    }
    pl.total = o;
    return SSM_OK;
}

}  // namespace

struct ssm_ctx {
    Plan pl;
    std::vector<ssm_problem> probs;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    unsigned char* ws = nullptr;
    size_t ws_bytes = 0;
    std::string err;
    bool have_string = false;
    bool have_eval = false;
    int check_every = 10;
    int graph_chunk = 0;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    double graph_tau = 0;
    int graph_n = 0;
    bool profiling = false;
    // step 1 method (ssm_set_integrator)
    int rk_method = SSM_STEP_EULER;
    double rk_rtol = 1e-6, rk_atol = 1e-6, rk_dt0 = 0.1;
    long long rk_nfe = 0;             // field evaluations by the integrator
    int interp = SSM_INTERP_LINEAR;   // step 2 (ssm_set_reparam)
    int climb = 0;
    struct Ev { int kind; hipEvent_t a, b; };
    std::vector<Ev> events;
    std::vector<hipEvent_t> pool;
    double prof_ms[SSM_N_KERNELS] = {0};
    int prof_cnt[SSM_N_KERNELS] = {0};

    template <typename X> X* at(size_t off) const { return reinterpret_cast<X*>(ws + off); }
    const Prob* P() const { return at<Prob>(pl.o_P); }
    WorkMap wm(int which, const std::vector<int>& v) const
    {
        WorkMap w;
        w.start = at<int>(pl.o_wm) + which * (pl.np + 1);
        w.total = v.back();
        return w;
    }
    struct XMaps { WorkMap m[2]; };
    struct ConvMaps { WorkMap m[kConvSlots]; };
    XMaps wm_xf() const { return {{wm(0, pl.wm_xf[0]), wm(1, pl.wm_xf[1])}}; }
    XMaps wm_xi() const { return {{wm(2, pl.wm_xi[0]), wm(3, pl.wm_xi[1])}}; }
    ConvMaps wm_conv() const
    {
        ConvMaps r;
        for (int j = 0; j < kConvSlots; ++j) r.m[j] = wm(4 + j, pl.wm_conv[j]);
        return r;
    }
    WorkMap wm_arc() const { return wm(4 + kConvSlots, pl.wm_arc); }
    WorkMap wm_site() const { return wm(5 + kConvSlots, pl.wm_site); }
    WorkMap wm_img() const { return wm(6 + kConvSlots, pl.wm_img); }
    WorkMap wm_sitep() const { return wm(7 + kConvSlots, pl.wm_sitep); }
    WorkMap wm_site4() const { return wm(8 + kConvSlots, pl.wm_site4); }
    Step2 step2() const
    {
        Step2 r;
        r.opts = (interp == SSM_INTERP_SPLINE ? 1 : 0) | (climb ? 2 : 0);
        r.E = at<double>(pl.o_E);
        r.kci = at<int>(pl.o_kci);
        r.spl_ok = at<int>(pl.o_splok);
        double* b = at<double>(pl.o_s2);
        const long long n = pl.n_img;
        r.hh = b; r.sa = b + n; r.den = b + 2 * n; r.cp = b + 3 * n;
        r.A = b + 4 * n; r.B = b + 5 * n; r.H = b + 6 * n;
        r.Wm = b + 7 * n;
        r.wmax = SSM_SPLW ? (pl.tsize == 4 ? kSplwMax<float> : kSplwMax<double>) : 0;
        return r;
    }
    void* X() const { return ws + pl.o_big; }
    void* Xp() const { return ws + pl.o_big + 2 * pl.tsize * pl.n_x; }
};

namespace {

ssm_status fail(ssm_ctx* c, ssm_status st, const std::string& msg)
{
    if (c) c->err = msg; else g_create_error = msg;
    return st;
}

ssm_status hipfail(ssm_ctx* c, hipError_t e, const char* where)
{
    return fail(c, SSM_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(c, expr, where)                                  \
    do {                                                        \
        hipError_t e_ = (expr);                                 \
        if (e_ != hipSuccess) return hipfail((c), e_, (where)); \
    } while (0)

hipEvent_t get_event(ssm_ctx* c)
{
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Run one launch, bracketed by events when profiling.
template <typename F>
hipError_t timed(ssm_ctx* c, hipStream_t st, int kind, F&& f)
{
    if (!c->profiling) return f();
    hipEvent_t a = get_event(c), b = get_event(c);
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, st);
    if (e != hipSuccess) return e;
    e = f();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, st);
    c->events.push_back({kind, a, b});
    return e;
}

template <typename T>
struct Ops {
    // x transform -> convolution -> inverse x transform + epilogue
    static hipError_t field(ssm_ctx* c, hipStream_t st, const T* src, T* s_star, T* hdst, int mode,
                            double tau, const int* done, double fcp = 0.0, double fcd = 1.0)
    {
        const Plan& pl = c->pl;
        const void* tw = c->at<void>(pl.o_tw);
        hipError_t e;
        e = timed(c, st, KK_XFWD, [&] {
            return launch_xfwd<T>(c->P(), pl.np, c->wm_xf().m, src, c->X(), tw, done, pl.lds_xf, st);
        });
        if (e != hipSuccess) return e;
        e = timed(c, st, KK_CONV, [&] {
            return launch_conv<T>(pl.mz, c->P(), pl.np, c->wm_conv().m, c->X(), c->Xp(),
                                  c->at<T>(pl.o_nh), tw, done, pl.lds_conv, st);
        });
        if (e != hipSuccess) return e;
        return timed(c, st, KK_XINV, [&] {
            return launch_xinv<T>(c->P(), pl.np, c->wm_xi().m, c->Xp(), src, s_star, hdst,
                                  c->at<double>(pl.o_ep), tw, done, mode, tau, fcp, fcd, pl.lds_xi, st);
        });
    }

    // Step 2: arc lengths of ss, the reduction (energies into E when
    // write_E; the options' targets and spline factors in its last
    // workgroup), interpolation into s: linear, or the natural cubic spline
    // with its second derivatives in the field buffer (problems whose
    // spline is degenerate fall back to linear)
    static hipError_t step2(ssm_ctx* c, hipStream_t st, const T* ss, T* s, const int* done, bool write_E)
    {
        const Plan& pl = c->pl;
        const Step2 o = c->step2();
        int* flags = c->at<int>(pl.o_flags);
        hipError_t e = timed(c, st, KK_ARC, [&] {
            return launch_arc<T>(c->P(), pl.np, c->wm_arc(), ss, c->at<double>(pl.o_ap), done, st);
        });
        if (e != hipSuccess) return e;
        e = timed(c, st, KK_REDUCE, [&] {
            return launch_reduce(c->P(), pl.np, (int)pl.n_img, pl.red_kinds, c->wm_img().start,
                                 c->at<double>(pl.o_ep), c->at<double>(pl.o_ap),
                                 write_E ? c->at<double>(pl.o_E) : nullptr, nullptr, nullptr, nullptr,
                                 c->at<double>(pl.o_seg), c->at<double>(pl.o_alpha),
                                 c->at<int>(pl.o_j), c->at<double>(pl.o_w), c->at<int>(pl.o_skip),
                                 const_cast<int*>(done), c->at<int>(pl.o_iters), c->at<int>(pl.o_cnt),
                                 flags, 1, st, o);
        });
        if (e != hipSuccess) return e;
        // the spline: problems of at most kSplwMax images in one pass, the
        // others by second derivatives then evaluation (per problem, so a
        // problem's path does not depend on the rest of the batch)
        const int kw = SSM_SPLW ? (kSplwMax<T> >= 32 ? pl.kmax_le32 : pl.kmax_le16) : 0;
        const int kskip = SSM_SPLW ? kSplwMax<T> : 0;
        if ((o.opts & 1) && kw > 0) {
            e = timed(c, st, KK_INTERP, [&] {
                return launch_interp_splw<T>(c->P(), pl.np, c->wm_sitep(), kw, ss, s, c->at<int>(pl.o_j),
                                             c->at<double>(pl.o_w), o, done, flags, st);
            });
            if (e != hipSuccess) return e;
        }
        if ((o.opts & 1) && pl.kmax > kskip) {
            T* M = c->at<T>(pl.o_h);
            e = timed(c, st, KK_INTERP, [&] {
                return launch_spline_m<T>(c->P(), pl.np, c->wm_sitep(), ss, M, o, done, kskip, st);
            });
            if (e != hipSuccess) return e;
            e = timed(c, st, KK_INTERP, [&] {
                return launch_interp_spline<T>(c->P(), pl.np, c->wm_site(), ss, M, s, c->at<int>(pl.o_j),
                                               c->at<double>(pl.o_w), o, done, flags, kskip, st);
            });
            if (e != hipSuccess) return e;
        }
        return timed(c, st, KK_INTERP, [&] {
            return launch_interp<T>(c->P(), pl.np, c->wm_site4(), ss, s, c->at<int>(pl.o_j),
                                    c->at<double>(pl.o_w), c->at<int>(pl.o_skip), done, flags, st,
                                    (o.opts & 2) ? o.kci : nullptr, (o.opts & 1) ? o.spl_ok : nullptr);
        });
    }

    static hipError_t iteration(ssm_ctx* c, hipStream_t st, double tau)
    {
        const Plan& pl = c->pl;
        T* s = c->at<T>(pl.o_s);
        T* ss = c->at<T>(pl.o_ss);
        int* done = c->at<int>(pl.o_done);
        const bool ci = c->climb != 0;
        T* h = ci ? c->at<T>(pl.o_h) : nullptr;
        hipError_t e = field(c, st, s, ss, h, EPI_STEP | (ci ? EPI_FIELD : 0), tau, done);
        if (e != hipSuccess) return e;
        if (ci) {
            // energies of the current string, then the climbing image's step
            const Step2 o = c->step2();
            e = timed(c, st, KK_REDUCE, [&] {
                return launch_reduce(c->P(), pl.np, (int)pl.n_img, pl.red_kinds, c->wm_img().start, c->at<double>(pl.o_ep),
                                     nullptr, c->at<double>(pl.o_E), nullptr, nullptr, nullptr, nullptr, nullptr,
                                     nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, c->at<int>(pl.o_flags), 0,
                                     st);
            });
            if (e != hipSuccess) return e;
            e = timed(c, st, KK_TAN1, [&] {
                return launch_ci_part<T>(c->P(), pl.np, c->wm_sitep(), s, h, c->at<double>(pl.o_E),
                                         c->at<double>(pl.o_fp), o.kci, done, st);
            });
            if (e != hipSuccess) return e;
            e = timed(c, st, KK_TANRED, [&] {
                return launch_ci_red(c->P(), pl.np, c->at<double>(pl.o_fp), o.kci, c->at<double>(pl.o_cic), done,
                                     st);
            });
            if (e != hipSuccess) return e;
            e = timed(c, st, KK_TAN2, [&] {
                return launch_ci_step<T>(c->P(), pl.np, c->wm_sitep(), s, h, ss, o.kci, c->at<double>(pl.o_cic), tau,
                                         done, st);
            });
            if (e != hipSuccess) return e;
        }
        return step2(c, st, ss, s, done, !ci);
    }

    // Adaptive Dormand-Prince integration of every image of the current
    // string over Tint: ds/dt = -fcp (s x h) + fcd ((s.s) h - (s.h) s).  The
    // result (not renormalised) replaces the string.  With energies, the
    // energies of the string before the interval are reduced into E from
    // the first slope's evaluation.  The attempts are driven from the host:
    // after each one the number of images still integrating is read back.
    static ssm_status rk_interval(ssm_ctx* c, double Tint, double fcp, double fcd, bool energies)
    {
        const Plan& pl = c->pl;
        hipStream_t st = c->stream;
        T* s = c->at<T>(pl.o_s);
        T* y = c->at<T>(pl.o_rk_y);
        int* done = c->at<int>(pl.o_done);
        int* flags = c->at<int>(pl.o_flags);
        RkSlopes<T> ks;
        for (int j = 0; j < 7; ++j) ks.k[j] = c->at<T>(pl.o_rk_k) + (size_t)j * pl.n_spin;
        RkState rs{c->at<double>(pl.o_rk_t), c->at<double>(pl.o_rk_dtp), c->at<double>(pl.o_rk_dtu),
                   c->at<int>(pl.o_rk_cap), c->at<int>(pl.o_rk_act), c->at<int>(pl.o_rk_acc),
                   c->at<int>(pl.o_rk_cnt), c->at<int>(pl.o_rk_nact)};
        const int nimg = (int)pl.n_img;
        const int* istart = c->wm_img().start;
        HIPCHK(c, timed(c, st, KK_RK, [&] { return launch_rk_init(c->P(), pl.np, nimg, istart, rs, Tint, done, st); }),
               "integrator");
        HIPCHK(c, field(c, st, s, nullptr, ks.k[0], EPI_FORCE, 0.0, done, fcp, fcd), "integrator");
        if (energies)
            HIPCHK(c, timed(c, st, KK_REDUCE, [&] {
                       return launch_reduce(c->P(), pl.np, nimg, pl.red_kinds, istart, c->at<double>(pl.o_ep), nullptr,
                                            c->at<double>(pl.o_E), nullptr, nullptr, nullptr, nullptr, nullptr,
                                            nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, flags, 0, st);
                   }), "integrator");
        c->rk_nfe += 1;
        constexpr int kMaxAttempts = 100000;
        int hnact = 0;
        for (int att = 0;; ++att) {
            if (att >= kMaxAttempts)
                return fail(c, SSM_ENONFINITE, "adaptive integrator: interval not completed within the attempt limit");
            for (int i = 1; i < 7; ++i) {
                HIPCHK(c, timed(c, st, KK_RK, [&] {
                           return launch_rk_stage<T>(c->P(), pl.np, c->wm_site(), s, ks, i, rs, y, done, st);
                       }), "integrator");
                HIPCHK(c, field(c, st, y, nullptr, ks.k[i], EPI_FORCE, 0.0, done, fcp, fcd), "integrator");
            }
            c->rk_nfe += 6;
            HIPCHK(c, launch_fill_int(rs.nact, 1, 0, st), "integrator");
            HIPCHK(c, timed(c, st, KK_RK, [&] {
                       return launch_rk_err<T>(c->P(), pl.np, c->wm_site(), s, y, ks, rs, c->rk_rtol, c->rk_atol,
                                               c->at<double>(pl.o_fm), done, st);
                   }), "integrator");
            HIPCHK(c, timed(c, st, KK_RK, [&] {
                       return launch_rk_ctrl(c->P(), pl.np, nimg, istart, c->at<double>(pl.o_fm), rs, Tint, done,
                                             flags, st);
                   }), "integrator");
            HIPCHK(c, timed(c, st, KK_RK, [&] {
                       return launch_rk_apply<T>(c->P(), pl.np, c->wm_site(), s, y, ks, rs, done, st);
                   }), "integrator");
            HIPCHK(c, hipMemcpyAsync(&hnact, rs.nact, sizeof(int), hipMemcpyDeviceToHost, st), "integrator");
            HIPCHK(c, hipStreamSynchronize(st), "integrator");
            if (hnact == 0) break;
        }
        return SSM_OK;
    }

    // Step 1 by the adaptive integrator (damping term alone) over Tint, then
    // renormalisation, arc length, reduction and interpolation as in
    // iteration().
    static ssm_status rk_iteration(ssm_ctx* c, double Tint)
    {
        const Plan& pl = c->pl;
        hipStream_t st = c->stream;
        T* s = c->at<T>(pl.o_s);
        T* ss = c->at<T>(pl.o_ss);
        int* done = c->at<int>(pl.o_done);
        int* flags = c->at<int>(pl.o_flags);
        ssm_status r = rk_interval(c, Tint, 0.0, 1.0, true);
        if (r != SSM_OK) return r;
        HIPCHK(c, timed(c, st, KK_RK, [&] {
                   return launch_rk_norm<T>(c->P(), pl.np, c->wm_site(), s, ss, done, flags, st);
               }), "integrator");
        HIPCHK(c, step2(c, st, ss, s, done, false), "integrator");
        return SSM_OK;
    }

    // eq. (9) over T for every image (no reparametrisation), renormalised
    static ssm_status llg(ssm_ctx* c, double T_, double alpha)
    {
        const Plan& pl = c->pl;
        T* s = c->at<T>(pl.o_s);
        const double cp = 1.0 / (1.0 + alpha * alpha), cd = alpha / (1.0 + alpha * alpha);
        ssm_status r = rk_interval(c, T_, cp, cd, false);
        if (r != SSM_OK) return r;
        T* ss = c->at<T>(pl.o_ss);
        HIPCHK(c, timed(c, c->stream, KK_RK, [&] {
                   return launch_rk_norm<T>(c->P(), pl.np, c->wm_site(), s, ss, c->at<int>(pl.o_done),
                                            c->at<int>(pl.o_flags), c->stream);
               }), "llg");
        HIPCHK(c, hipMemcpyAsync(s, ss, pl.tsize * pl.n_spin, hipMemcpyDeviceToDevice, c->stream), "llg");
        return SSM_OK;
    }

    // evaluation of `src` (current string when store)
    static hipError_t eval(ssm_ctx* c, hipStream_t st, const T* src, T* hdst, double* E_out,
                           double* T_out, bool store)
    {
        const Plan& pl = c->pl;
        const int mode = (hdst ? EPI_FIELD : 0) | EPI_TERMS;
        hipError_t e = field(c, st, src, nullptr, hdst, mode, 0.0, nullptr);
        if (e != hipSuccess) return e;
        return timed(c, st, KK_REDUCE, [&] {
            return launch_reduce(c->P(), pl.np, (int)pl.n_img, pl.red_kinds, c->wm_img().start,
                                 c->at<double>(pl.o_ep), nullptr,
                                 store ? c->at<double>(pl.o_E) : nullptr,
                                 store ? c->at<double>(pl.o_T) : nullptr, E_out, T_out, nullptr,
                                 nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                 c->at<int>(pl.o_flags), 0, st);
        });
    }

    // tangents of the current string, force norm; uses ss as scratch
    static hipError_t tangents(ssm_ctx* c, hipStream_t st, T* t_out, double* norm_out, double tol)
    {
        const Plan& pl = c->pl;
        T* s = c->at<T>(pl.o_s);
        T* h = c->at<T>(pl.o_h);
        T* tt = c->at<T>(pl.o_ss);
        hipError_t e = timed(c, st, KK_TAN1, [&] {
            return launch_tan1<T>(c->P(), pl.np, c->wm_site(), s, h, tt, c->at<double>(pl.o_fp), st);
        });
        if (e != hipSuccess) return e;
        e = timed(c, st, KK_TANRED, [&] {
            return launch_tanred(c->P(), pl.np, c->at<double>(pl.o_fp), c->at<double>(pl.o_tc), st);
        });
        if (e != hipSuccess) return e;
        e = timed(c, st, KK_TAN2, [&] {
            return launch_tan2<T>(c->P(), pl.np, c->wm_site(), s, h, tt, t_out,
                                  c->at<double>(pl.o_tc), c->at<double>(pl.o_fm), st);
        });
        if (e != hipSuccess) return e;
        return timed(c, st, KK_TANRED, [&] {
            return launch_fmax(c->P(), pl.np, c->at<double>(pl.o_fm), c->at<double>(pl.o_fn),
                               c->at<int>(pl.o_done), tol, norm_out, st);
        });
    }
};

template <typename F>
hipError_t dispatch(ssm_ctx* c, F&& f)
{
    if (c->pl.prec == SSM_FP64) return f(Ops<double>());
    return f(Ops<float>());
}

void drop_graph(ssm_ctx* c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->graph_n = 0;
}

ssm_status ensure_graph(ssm_ctx* c, double tau, int n)
{
    if (c->gexec && c->graph_tau == tau && c->graph_n == n) return SSM_OK;
    drop_graph(c);
    HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
    hipError_t e = hipSuccess;
    for (int i = 0; i < n && e == hipSuccess; ++i)
        e = dispatch(c, [&](auto ops) { return ops.iteration(c, c->cap_stream, tau); });
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
    if (e != hipSuccess) { if (g) (void)hipGraphDestroy(g); return hipfail(c, e, "graph capture"); }
    if (e2 != hipSuccess) return hipfail(c, e2, "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) { (void)hipGraphDestroy(g); return hipfail(c, e, "hipGraphInstantiate"); }
    c->graph = g;
    c->gexec = ex;
    c->graph_tau = tau;
    c->graph_n = n;
    return SSM_OK;
}

void twiddles(std::vector<double>& tw64)
{
    tw64.resize(2 * kTwM);
    for (int e = 0; e < kTwM; ++e) {
        const long double th = 2.0L * 3.14159265358979323846264338327950288L * (long double)e /
                               (long double)kTwM;
        tw64[2 * e] = (double)cosl(th);
        tw64[2 * e + 1] = (double)-sinl(th);
    }
}

}  // namespace

static ssm_status upload_plan(ssm_ctx* c)
{
    const Plan& pl = c->pl;
    HIPCHK(c, hipMemcpyAsync(c->ws + pl.o_P, pl.P.data(), sizeof(Prob) * pl.np,
                             hipMemcpyHostToDevice, c->stream), "upload descriptors");
    std::vector<int> wm;
    std::vector<const std::vector<int>*> maps = {&pl.wm_xf[0], &pl.wm_xf[1], &pl.wm_xi[0], &pl.wm_xi[1]};
    for (int j = 0; j < kConvSlots; ++j) maps.push_back(&pl.wm_conv[j]);
    for (const auto* v : {&pl.wm_arc, &pl.wm_site, &pl.wm_img, &pl.wm_sitep, &pl.wm_site4}) maps.push_back(v);
    for (const auto* v : maps) wm.insert(wm.end(), v->begin(), v->end());
    HIPCHK(c, hipMemcpyAsync(c->ws + pl.o_wm, wm.data(), sizeof(int) * wm.size(),
                             hipMemcpyHostToDevice, c->stream), "upload work maps");
    HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    return SSM_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: candidate tile shapes per kernel, timed on the live context.
// ---------------------------------------------------------------------------
namespace {

// Rebuild descriptors and work maps for new tile shapes; the workspace
// layout does not depend on them.
ssm_status retile(ssm_ctx* c, const std::vector<Tiles>& tiles)
{
    Plan pl;
    std::string err;
    ssm_status st = build_plan(c->probs.data(), (int)c->probs.size(), c->pl.prec, &tiles, pl, err);
    if (st != SSM_OK) return fail(c, st, err);
    if (pl.total != c->pl.total) return fail(c, SSM_EUNSUPPORTED, "retiling changed the workspace layout");
    // keep the parameters set since creation
    for (size_t i = 0; i < pl.P.size(); ++i) {
        pl.P[i].J = c->pl.P[i].J;
        pl.P[i].d = c->pl.P[i].d;
        pl.P[i].ku = c->pl.P[i].ku;
        pl.P[i].D = c->pl.P[i].D;
    }
    c->pl = pl;
    drop_graph(c);
    return upload_plan(c);
}

// Median time (ms) of `reps` launches of one evaluation kernel kind.
template <typename T>
double time_kernel(ssm_ctx* c, int kind, int reps)
{
    const Plan& pl = c->pl;
    const void* tw = c->at<void>(pl.o_tw);
    const T* s = c->at<T>(pl.o_s);
    std::vector<float> ts;
    hipEvent_t a = get_event(c), b = get_event(c);
    for (int r = 0; r < reps + 1; ++r) {
        if (hipEventRecord(a, c->stream) != hipSuccess) return 1e30;
        hipError_t e = hipSuccess;
        if (kind == KK_XFWD)
            e = launch_xfwd<T>(c->P(), pl.np, c->wm_xf().m, s, c->X(), tw, nullptr, pl.lds_xf, c->stream);
        else if (kind == KK_CONV)
            e = launch_conv<T>(pl.mz, c->P(), pl.np, c->wm_conv().m, c->X(), c->Xp(), c->at<T>(pl.o_nh), tw,
                               nullptr, pl.lds_conv, c->stream);
        else
            e = launch_xinv<T>(c->P(), pl.np, c->wm_xi().m, c->Xp(), s, nullptr, nullptr,
                               c->at<double>(pl.o_ep), tw, nullptr, EPI_TERMS, 0.0, 0.0, 1.0, pl.lds_xi,
                               c->stream);
        if (e != hipSuccess || hipEventRecord(b, c->stream) != hipSuccess) return 1e30;
        if (hipEventSynchronize(b) != hipSuccess) return 1e30;
        float ms = 0;
        if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 1e30;
        if (r > 0) ts.push_back(ms);  // first launch warms caches
    }
    c->pool.push_back(a);
    c->pool.push_back(b);
    std::sort(ts.begin(), ts.end());
    return ts[ts.size() / 2];
}

std::string device_name()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string n = prop.gcnArchName;
    for (auto& ch : n) if (ch == ' ') ch = '_';
    return n;
}

std::string cache_key(const std::string& dev, int prec, const ssm_problem& q)
{
    std::ostringstream os;
    os << dev << " " << prec << " " << q.nx << "x" << q.ny << "x" << q.nz << " " << q.n_images;
    return os.str();
}

ssm_status autotune(ssm_ctx* c, const char* cache_path)
{
    const int np = c->pl.np;
    const size_t ts = c->pl.tsize;
    const std::string dev = device_name();
    std::vector<Tiles> cur = c->pl.tiles;
    std::vector<bool> known(np, false);
    // cache lookup: "<device> <prec> <nx>x<ny>x<nz> <K> ytf yt gconv"
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        std::map<std::string, Tiles> cache;
        while (std::getline(in, line)) {
            std::istringstream is(line);
            std::string d, shape;
            int pr, K, a, b, g;
            // row tiles are powers of two >= 2 (the x kernels index with
            // shifts); anything else in the file is ignored
            auto pow2ok = [](int v) { return v >= 2 && v <= 1024 && (v & (v - 1)) == 0; };
            if ((is >> d >> pr >> shape >> K >> a >> b >> g) && pow2ok(a) && pow2ok(b) && g >= 1 && g <= 64) {
                std::ostringstream k;
                k << d << " " << pr << " " << shape << " " << K;
                cache[k.str()] = Tiles{a, b, g};
            }
        }
        for (int i = 0; i < np; ++i) {
            auto it = cache.find(cache_key(dev, c->pl.prec, c->probs[i]));
            if (it != cache.end()) { cur[i] = it->second; known[i] = true; }
        }
    }
    bool all_known = true;
    for (bool k : known) all_known = all_known && k;
    if (!all_known) {
        // candidates are applied to every problem at once (clamped to what
        // each problem's LDS admits); kernels are timed one kind at a time
        auto fits = [&](const Prob& p, const Tiles& t) {
            return lds_xfwd(p, t.ytf, ts) <= kLdsMax && lds_xinv(p, t.yt, ts) <= kLdsMax &&
                   lds_convg(p, t.gconv, ts) <= kLdsMax;
        };
        auto timed_kind = [&](int kind) {
            return c->pl.prec == SSM_FP64 ? time_kernel<double>(c, kind, 5) : time_kernel<float>(c, kind, 5);
        };
        const int rows[] = {2, 4, 8, 16, 32, 64};
        for (int kind : {KK_XFWD, KK_XINV, KK_CONV}) {
            std::vector<Tiles> best = cur;
            ssm_status st = retile(c, cur);
            if (st != SSM_OK) return st;
            double tbest = timed_kind(kind);
            const int ncand = kind == KK_CONV ? 6 : 6;
            for (int ci = 0; ci < ncand; ++ci) {
                std::vector<Tiles> cand = cur;
                bool any = false;
                for (int i = 0; i < np; ++i) {
                    if (known[i]) continue;
                    Prob p = c->pl.P[i];
                    Tiles t = cur[i];
                    const int ycap = std::max(2, pow2ceil(p.ny));
                    if (kind == KK_XFWD) t.ytf = std::min(rows[ci], ycap);
                    else if (kind == KK_XINV) t.yt = std::min(rows[ci], ycap);
                    else t.gconv = 1 << ci;
                    if (kind == KK_CONV && (long long)t.gconv * 3 * p.nz * p.ny > kConvElems && t.gconv > 1) continue;
                    if (!fits(p, t)) continue;
                    if (t.ytf != cur[i].ytf || t.yt != cur[i].yt || t.gconv != cur[i].gconv) any = true;
                    cand[i] = t;
                }
                if (!any) continue;
                st = retile(c, cand);
                if (st != SSM_OK) return st;
                const double tc = timed_kind(kind);
                if (tc < tbest) { tbest = tc; best = cand; }
            }
            cur = best;
        }
    }
    ssm_status st = retile(c, cur);
    if (st != SSM_OK) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream), "autotune");
    c->have_eval = false;  // the scratch buffers were overwritten
    if (cache_path && !all_known) {
        std::ofstream out(cache_path, std::ios::app);
        for (int i = 0; i < np; ++i)
            if (!known[i])
                out << cache_key(dev, c->pl.prec, c->probs[i]) << " " << cur[i].ytf << " " << cur[i].yt << " "
                    << cur[i].gconv << "\n";
    }
    return SSM_OK;
}

}  // namespace

// Twiddle tables, descriptors and work maps, and the FFT of the point-dipole
// tensor (eq. (7)) on the padded grid of every distinct lattice shape, in the
// context's workspace.  Synchronises the stream (the host copies' sources
// are locals).
static ssm_status setup_tables(ssm_ctx* c)
{
    const Plan& pl = c->pl;
    std::vector<double> tw64;
    twiddles(tw64);
    // the compact table: W_{2m}^e = full-table entry e kTwM / (2m)
    std::vector<double> cpt(2 * kTwCompact);
    for (int f3 = 0; f3 < 2; ++f3)
        for (int lg = 0; lg <= (f3 ? 8 : kMaxLogM); ++lg) {
            const int n2 = (f3 ? 6 : 2) << lg, stride = kTwM / n2;
            for (int e = 0; e < n2; ++e) {
                cpt[2 * (tw_off(lg, f3) + e)] = tw64[2 * e * stride];
                cpt[2 * (tw_off(lg, f3) + e) + 1] = tw64[2 * e * stride + 1];
            }
        }
    std::vector<unsigned char> twt(2 * pl.tsize * kTwCompact);
    if (pl.tsize == 8) {
        std::memcpy(twt.data(), cpt.data(), twt.size());
    } else {
        float* f = reinterpret_cast<float*>(twt.data());
        for (int i = 0; i < 2 * kTwCompact; ++i) f[i] = (float)cpt[i];
    }
    hipError_t e = hipMemcpyAsync(c->ws + pl.o_tw, twt.data(), twt.size(), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->ws + pl.o_tw64, tw64.data(), 16 * kTwM, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) { return hipfail(c, e, "upload twiddles"); }
    ssm_status st = upload_plan(c);
    if (st != SSM_OK) return st;
    // dipole-kernel spectrum of every distinct shape (FP64, then stored as T)
    for (size_t g = 0; g < pl.shapes.size(); ++g) {
        int i = 0;
        while (pl.geo[i] != (int)g) ++i;
        const Prob& pr = pl.P[i];
        double* f1 = c->at<double>(pl.o_big);
        double* f2 = f1 + 6LL * (pr.mx + 1) * (2 * pr.ny - 1) * (2 * pr.nz - 1);
        if (pl.prec == SSM_FP64)
            e = launch_spectrum<double>(pr, c->at<double>(pl.o_nh) + pr.nh_off, f1, f2,
                                        c->at<double>(pl.o_tw64), c->stream);
        else
            e = launch_spectrum<float>(pr, c->at<float>(pl.o_nh) + pr.nh_off, f1, f2,
                                       c->at<double>(pl.o_tw64), c->stream);
        if (e != hipSuccess) { return hipfail(c, e, "kernel spectrum"); }
        // scratch reuse by the next shape needs this one finished
        e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) { return hipfail(c, e, "kernel spectrum"); }
    }
    return SSM_OK;
}

// ---------------------------------------------------------------------------
// Evaluation without any device allocation (ssm_eval_noalloc).  Its scratch
// (descriptors, twiddles, kernel spectra, x half-spectra, energy partials,
// flags) is one file-scope device array; every GPU the library runs on holds
// its own copy until the process ends.  Host code never uses the array's
// name as an address: the device address comes from hipGetSymbolAddress, once
// per device, with that device current.
// ---------------------------------------------------------------------------
constexpr size_t kStaticScratchBytes = size_t(SSM_NOALLOC_SCRATCH_MIB) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
constexpr int kStaticMaxProblems = 16;

// Offsets of the evaluation's buffers packed into the static scratch (the
// string buffers of a context are the caller's inputs and outputs here).
void carve_static(Plan& pl)
{
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = up(o + std::max<size_t>(bytes, 1)); return r; };
    const size_t ts = pl.tsize, cs = 2 * ts;
    int my_max = 1;
    for (const Prob& q : pl.P) my_max = std::max(my_max, q.my);
    // buffers the evaluation never touches share offset 0
    pl.o_s = pl.o_ss = pl.o_h = pl.o_ap = pl.o_fp = pl.o_E = pl.o_T = pl.o_alpha = pl.o_w = pl.o_tc = 0;
    pl.o_fn = pl.o_fm = pl.o_j = pl.o_done = pl.o_iters = pl.o_skip = pl.o_seg = pl.o_cnt = 0;
    pl.o_s2 = pl.o_kci = pl.o_splok = pl.o_cic = 0;
    pl.o_P = take(sizeof(Prob) * pl.np);
    pl.o_wm = take(sizeof(int) * kNumMaps * (pl.np + 1));
    pl.o_tw = take(cs * kTwCompact);
    pl.o_tw64 = take(16 * kTwM);
    pl.o_nh = take(ts * pl.n_nh);
    pl.o_big = take(std::max((size_t)(2 * cs * pl.n_x + cs * my_max), pl.scratch_bytes));
    pl.o_ep = take(8 * pl.n_ep);
    pl.o_flags = take(4);
    pl.total = o;
}

// Per device: the scratch's device address and the layout (problem shapes,
// image counts, precision) whose tables it currently holds.
struct StaticDev {
    unsigned char* ptr = nullptr;
    bool have_tables = false;
    int prec = -1;
    int np = 0;
    int shape[kStaticMaxProblems][4] = {};
    ssm_ctx ctx;  // host description of the layout (no workspace of its own)
};
StaticDev g_static[kMaxDevices];
std::mutex g_static_mu;

bool same_layout(const StaticDev& d, const ssm_problem* p, int np, int prec)
{
    if (!d.have_tables || d.prec != prec || d.np != np) return false;
    for (int i = 0; i < np; ++i)
        if (d.shape[i][0] != p[i].nx || d.shape[i][1] != p[i].ny || d.shape[i][2] != p[i].nz ||
            d.shape[i][3] != p[i].n_images)
            return false;
    return true;
}

// Copy host bytes to device memory through kernel arguments (no host buffer
// has to outlive the call).
hipError_t put_bytes(void* dst, const void* src, size_t n, hipStream_t st)
{
    const unsigned char* b = static_cast<const unsigned char*>(src);
    for (size_t o = 0; o < n; o += kBlobBytes) {
        Blob blob;
        blob.n = (int)std::min<size_t>(kBlobBytes, n - o);
        std::memcpy(blob.b, b + o, blob.n);
        hipError_t e = launch_put(static_cast<unsigned char*>(dst) + o, blob, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int32_t ssm_version(void) { return kVersion; }

const char* ssm_kernel_name(int32_t i)
{
    if (i < 0 || i >= SSM_N_KERNELS) return nullptr;
    return kKernelNames[i];
}

const char* ssm_last_error(const ssm_ctx* ctx)
{
    if (!ctx) return g_create_error.c_str();
    return ctx->err.c_str();
}

ssm_status ssm_workspace_size(const ssm_problem* p, int32_t n_problems, int32_t precision,
                              size_t* bytes)
{
    if (!bytes) return fail(nullptr, SSM_EINVAL, "bytes is NULL");
    Plan pl;
    std::string err;
    ssm_status st = build_plan(p, n_problems, precision, nullptr, pl, err);
    if (st != SSM_OK) return fail(nullptr, st, err);
    *bytes = pl.total;
    return SSM_OK;
}

ssm_status ssm_create(const ssm_problem* p, int32_t n_problems, int32_t precision,
                      void* d_workspace, size_t ws_bytes, void* stream, ssm_ctx** out)
{
    if (!out) return fail(nullptr, SSM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d_workspace) return fail(nullptr, SSM_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(d_workspace) % kAlign)
        return fail(nullptr, SSM_EINVAL, "workspace not 256-byte aligned");
    ssm_ctx* c = new ssm_ctx();
    std::string err;
    ssm_status st = build_plan(p, n_problems, precision, nullptr, c->pl, err);
    if (st != SSM_OK) { delete c; return fail(nullptr, st, err); }
    if (ws_bytes < c->pl.total) {
        const size_t need = c->pl.total;
        delete c;
        return fail(nullptr, SSM_EINVAL, "workspace too small: need " + std::to_string(need));
    }
    c->probs.assign(p, p + n_problems);
    c->stream = (hipStream_t)stream;
    c->ws = (unsigned char*)d_workspace;
    c->ws_bytes = ws_bytes;
    auto bail = [&](ssm_status s) {
        g_create_error = c->err;
        if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
        delete c;
        return s;
    };
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        c->err = "hipStreamCreateWithFlags failed";
        return bail(SSM_EHIP);
    }
    if ((st = setup_tables(c)) != SSM_OK) return bail(st);
    const Plan& pl = c->pl;
    hipError_t e;
    e = launch_fill_int(c->at<int>(pl.o_done), pl.np, 0, c->stream);
    if (e == hipSuccess) e = launch_fill_int(c->at<int>(pl.o_iters), pl.np, 0, c->stream);
    if (e == hipSuccess) e = launch_fill_int(c->at<int>(pl.o_skip), pl.np, 0, c->stream);
    if (e == hipSuccess) e = launch_fill_int(c->at<int>(pl.o_flags), 1, 0, c->stream);
    if (e == hipSuccess) e = launch_fill_int(c->at<int>(pl.o_cnt), pl.np, 0, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) { hipfail(c, e, "create"); return bail(SSM_EHIP); }
    *out = c;
    return SSM_OK;
}

ssm_status ssm_destroy(ssm_ctx* ctx)
{
    if (!ctx) return SSM_OK;
    (void)hipStreamSynchronize(ctx->stream);
    drop_graph(ctx);
    for (auto& ev : ctx->events) { (void)hipEventDestroy(ev.a); (void)hipEventDestroy(ev.b); }
    for (auto e : ctx->pool) (void)hipEventDestroy(e);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    delete ctx;
    return SSM_OK;
}

ssm_status ssm_set_params(ssm_ctx* ctx, int32_t problem, double J, double d, double ku, double dip)
{
    if (!ctx) return SSM_EINVAL;
    if (problem < 0 || problem >= ctx->pl.np) return fail(ctx, SSM_EINVAL, "problem index out of range");
    if (!std::isfinite(J) || !std::isfinite(d) || !std::isfinite(ku) || !std::isfinite(dip))
        return fail(ctx, SSM_EINVAL, "non-finite parameter");
    Prob& p = ctx->pl.P[problem];
    p.J = J; p.d = d; p.ku = ku; p.D = dip;
    ctx->have_eval = false;  // energies and fields depend on the parameters
    HIPCHK(ctx, hipMemcpyAsync(ctx->ws + ctx->pl.o_P + sizeof(Prob) * problem, &p, sizeof(Prob),
                               hipMemcpyHostToDevice, ctx->stream), "set params");
    // the source must stay valid until the copy has run
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "set params");
    return SSM_OK;
}

ssm_status ssm_set_string(ssm_ctx* ctx, const void* d_spins)
{
    if (!ctx || !d_spins) return ctx ? fail(ctx, SSM_EINVAL, "d_spins is NULL") : SSM_EINVAL;
    HIPCHK(ctx, hipMemcpyAsync(ctx->ws + ctx->pl.o_s, d_spins, ctx->pl.tsize * ctx->pl.n_spin,
                               hipMemcpyDeviceToDevice, ctx->stream), "set string");
    ctx->have_string = true;
    ctx->have_eval = false;
    return SSM_OK;
}

ssm_status ssm_get_string(ssm_ctx* ctx, void* d_spins)
{
    if (!ctx || !d_spins) return ctx ? fail(ctx, SSM_EINVAL, "d_spins is NULL") : SSM_EINVAL;
    if (!ctx->have_string) return fail(ctx, SSM_ESTATE, "no string set");
    HIPCHK(ctx, hipMemcpyAsync(d_spins, ctx->ws + ctx->pl.o_s, ctx->pl.tsize * ctx->pl.n_spin,
                               hipMemcpyDeviceToDevice, ctx->stream), "get string");
    return SSM_OK;
}

ssm_status ssm_set_reparam(ssm_ctx* ctx, int32_t interp, int32_t climbing)
{
    if (!ctx) return SSM_EINVAL;
    if (interp != SSM_INTERP_LINEAR && interp != SSM_INTERP_SPLINE)
        return fail(ctx, SSM_EINVAL, "unknown interpolation");
    if (climbing != 0 && climbing != 1) return fail(ctx, SSM_EINVAL, "climbing must be 0 or 1");
    if (interp != ctx->interp || climbing != ctx->climb) drop_graph(ctx);
    ctx->interp = interp;
    ctx->climb = climbing;
    return SSM_OK;
}

ssm_status ssm_set_integrator(ssm_ctx* ctx, int32_t method, double rtol, double atol, double dt0)
{
    if (!ctx) return SSM_EINVAL;
    if (method != SSM_STEP_EULER && method != SSM_STEP_DOPRI54)
        return fail(ctx, SSM_EINVAL, "unknown step method");
    if (method == SSM_STEP_EULER) {
        ctx->rk_method = method;
        return SSM_OK;
    }
    if (!ctx->pl.rk) return fail(ctx, SSM_EUNSUPPORTED, "context created without SSM_WITH_RK");
    if (!(rtol >= 0.0) || !(atol > 0.0) || !(dt0 > 0.0) || !std::isfinite(rtol) || !std::isfinite(atol) ||
        !std::isfinite(dt0))
        return fail(ctx, SSM_EINVAL, "rtol >= 0, atol > 0 and dt0 > 0 (finite) required");
    ctx->rk_method = method;
    ctx->rk_rtol = rtol;
    ctx->rk_atol = atol;
    ctx->rk_dt0 = dt0;
    ctx->rk_nfe = 0;
    const Plan& pl = ctx->pl;
    HIPCHK(ctx, launch_fill_double(ctx->at<double>(pl.o_rk_dtp), (int)pl.n_img, dt0, ctx->stream), "set integrator");
    HIPCHK(ctx, launch_fill_int(ctx->at<int>(pl.o_rk_cnt), (int)(2 * pl.n_img), 0, ctx->stream), "set integrator");
    return SSM_OK;
}

static ssm_status run_eval_current(ssm_ctx* c);

ssm_status ssm_llg(ssm_ctx* ctx, double t_total, double alpha)
{
    if (!ctx) return SSM_EINVAL;
    ssm_ctx* c = ctx;
    const Plan& pl = c->pl;
    if (!pl.rk) return fail(c, SSM_EUNSUPPORTED, "context created without SSM_WITH_RK");
    if (!c->have_string) return fail(c, SSM_ESTATE, "no string set");
    if (!(t_total > 0.0) || !std::isfinite(t_total) || !(alpha >= 0.0) || !std::isfinite(alpha))
        return fail(c, SSM_EINVAL, "t_total > 0 and alpha >= 0 (finite) required");
    HIPCHK(c, launch_fill_int(c->at<int>(pl.o_done), pl.np, 0, c->stream), "llg");
    c->have_eval = false;
    return pl.prec == SSM_FP64 ? Ops<double>::llg(c, t_total, alpha) : Ops<float>::llg(c, t_total, alpha);
}

ssm_status ssm_get_rk_stats(ssm_ctx* ctx, int32_t* d_counts, double* d_dt, int64_t* h_evals)
{
    if (!ctx) return SSM_EINVAL;
    const Plan& pl = ctx->pl;
    if (!pl.rk) return fail(ctx, SSM_EUNSUPPORTED, "context created without SSM_WITH_RK");
    if (d_counts)
        HIPCHK(ctx, hipMemcpyAsync(d_counts, ctx->ws + pl.o_rk_cnt, 8 * pl.n_img, hipMemcpyDeviceToDevice,
                                   ctx->stream), "rk stats");
    if (d_dt)
        HIPCHK(ctx, hipMemcpyAsync(d_dt, ctx->ws + pl.o_rk_dtp, 8 * pl.n_img, hipMemcpyDeviceToDevice,
                                   ctx->stream), "rk stats");
    if (h_evals) *h_evals = ctx->rk_nfe;
    return SSM_OK;
}

ssm_status ssm_set_options(ssm_ctx* ctx, int32_t check_every, int32_t graph_chunk)
{
    if (!ctx) return SSM_EINVAL;
    if (check_every < 1 || graph_chunk < 0 || graph_chunk > 100000)
        return fail(ctx, SSM_EINVAL, "check_every >= 1 and 0 <= graph_chunk <= 100000");
    ctx->check_every = check_every;
    if (graph_chunk != ctx->graph_chunk) drop_graph(ctx);
    ctx->graph_chunk = graph_chunk;
    return SSM_OK;
}

static ssm_status run_eval_current(ssm_ctx* c)
{
    const Plan& pl = c->pl;
    hipError_t e;
    if (pl.prec == SSM_FP64)
        e = Ops<double>::eval(c, c->stream, c->at<double>(pl.o_s), c->at<double>(pl.o_h), nullptr,
                              nullptr, true);
    else
        e = Ops<float>::eval(c, c->stream, c->at<float>(pl.o_s), c->at<float>(pl.o_h), nullptr,
                             nullptr, true);
    if (e != hipSuccess) return hipfail(c, e, "evaluation");
    c->have_eval = true;
    return SSM_OK;
}

// The getters' view of the current string: evaluated on first use after the
// string or the parameters changed (enqueued on the context's stream).
static ssm_status ensure_eval(ssm_ctx* c)
{
    if (c->have_eval) return SSM_OK;
    if (!c->have_string) return fail(c, SSM_ESTATE, "no string set");
    return run_eval_current(c);
}

ssm_status ssm_iterate(ssm_ctx* ctx, int32_t max_iter, double tau, double tol_force,
                       int32_t* d_iters_done)
{
    if (!ctx) return SSM_EINVAL;
    if (!ctx->have_string) return fail(ctx, SSM_ESTATE, "no string set");
    if (max_iter < 0 || !std::isfinite(tau) || !(tol_force >= 0.0))
        return fail(ctx, SSM_EINVAL, "max_iter >= 0, finite tau and tol_force >= 0 required");
    if (ctx->climb && ctx->rk_method == SSM_STEP_DOPRI54)
        return fail(ctx, SSM_EUNSUPPORTED, "the climbing image needs the explicit step");
    ssm_ctx* c = ctx;
    const Plan& pl = c->pl;
    HIPCHK(c, launch_fill_int(c->at<int>(pl.o_done), pl.np, 0, c->stream), "iterate");
    HIPCHK(c, launch_fill_int(c->at<int>(pl.o_iters), pl.np, 0, c->stream), "iterate");
    const bool check = tol_force > 0.0;
    const bool use_graph = c->graph_chunk > 0 && !c->profiling;
    std::vector<int> hdone(pl.np);
    int it = 0;
    for (;;) {
        if (check && it % c->check_every == 0) {
            ssm_status st = run_eval_current(c);
            if (st != SSM_OK) return st;
            hipError_t e = dispatch(c, [&](auto ops) {
                return decltype(ops)::tangents(c, c->stream, nullptr, nullptr, tol_force);
            });
            if (e != hipSuccess) return hipfail(c, e, "convergence check");
            HIPCHK(c, hipMemcpyAsync(hdone.data(), c->at<int>(pl.o_done), 4 * pl.np,
                                     hipMemcpyDeviceToHost, c->stream), "convergence check");
            HIPCHK(c, hipStreamSynchronize(c->stream), "convergence check");
            bool all = true;
            for (int v : hdone) all = all && v;
            if (all) break;
        }
        if (it >= max_iter) break;
        int n = max_iter - it;
        if (check) n = std::min(n, c->check_every - it % c->check_every);
        c->have_eval = false;  // the string changes from here on
        if (c->rk_method == SSM_STEP_DOPRI54) {
            for (int i = 0; i < n; ++i) {
                ssm_status st = pl.prec == SSM_FP64 ? Ops<double>::rk_iteration(c, tau)
                                                    : Ops<float>::rk_iteration(c, tau);
                if (st != SSM_OK) return st;
            }
            it += n;
            continue;
        }
        if (use_graph && n >= c->graph_chunk) {
            const int reps = n / c->graph_chunk;
            ssm_status st = ensure_graph(c, tau, c->graph_chunk);
            if (st != SSM_OK) return st;
            for (int r = 0; r < reps; ++r)
                HIPCHK(c, hipGraphLaunch(c->gexec, c->stream), "hipGraphLaunch");
            it += reps * c->graph_chunk;
            continue;
        }
        hipError_t e = hipSuccess;
        for (int i = 0; i < n && e == hipSuccess; ++i)
            e = dispatch(c, [&](auto ops) { return decltype(ops)::iteration(c, c->stream, tau); });
        if (e != hipSuccess) return hipfail(c, e, "iteration");
        it += n;
    }
    // the final string is evaluated when a getter first needs it
    if (d_iters_done)
        HIPCHK(c, launch_iters_out(pl.np, c->at<int>(pl.o_iters), nullptr, d_iters_done, c->stream),
               "iterate");
    return SSM_OK;
}

ssm_status ssm_eval(ssm_ctx* ctx, const void* d_spins, void* d_field_or_null, double* d_energy,
                    double* d_terms_or_null)
{
    if (!ctx) return SSM_EINVAL;
    ssm_ctx* c = ctx;
    const Plan& pl = c->pl;
    if (!d_spins) {
        if (!c->have_string) return fail(c, SSM_ESTATE, "no string set");
        ssm_status st = run_eval_current(c);
        if (st != SSM_OK) return st;
        const size_t nb = pl.tsize * pl.n_spin;
        if (d_field_or_null)
            HIPCHK(c, hipMemcpyAsync(d_field_or_null, c->ws + pl.o_h, nb, hipMemcpyDeviceToDevice, c->stream), "eval");
        if (d_energy)
            HIPCHK(c, hipMemcpyAsync(d_energy, c->ws + pl.o_E, 8 * pl.n_img, hipMemcpyDeviceToDevice, c->stream), "eval");
        if (d_terms_or_null)
            HIPCHK(c, hipMemcpyAsync(d_terms_or_null, c->ws + pl.o_T, 32 * pl.n_img, hipMemcpyDeviceToDevice, c->stream), "eval");
        return SSM_OK;
    }
    hipError_t e;
    if (pl.prec == SSM_FP64)
        e = Ops<double>::eval(c, c->stream, (const double*)d_spins, (double*)d_field_or_null, d_energy,
                              d_terms_or_null, false);
    else
        e = Ops<float>::eval(c, c->stream, (const float*)d_spins, (float*)d_field_or_null, d_energy,
                             d_terms_or_null, false);
    if (e != hipSuccess) return hipfail(c, e, "eval");
    return SSM_OK;
}

ssm_status ssm_get_energies(ssm_ctx* ctx, double* d_energy)
{
    if (!ctx || !d_energy) return ctx ? fail(ctx, SSM_EINVAL, "d_energy is NULL") : SSM_EINVAL;
    ssm_status st = ensure_eval(ctx);
    if (st != SSM_OK) return st;
    HIPCHK(ctx, hipMemcpyAsync(d_energy, ctx->ws + ctx->pl.o_E, 8 * ctx->pl.n_img,
                               hipMemcpyDeviceToDevice, ctx->stream), "get energies");
    return SSM_OK;
}

ssm_status ssm_get_fields(ssm_ctx* ctx, void* d_field)
{
    if (!ctx || !d_field) return ctx ? fail(ctx, SSM_EINVAL, "d_field is NULL") : SSM_EINVAL;
    ssm_status st = ensure_eval(ctx);
    if (st != SSM_OK) return st;
    HIPCHK(ctx, hipMemcpyAsync(d_field, ctx->ws + ctx->pl.o_h, ctx->pl.tsize * ctx->pl.n_spin,
                               hipMemcpyDeviceToDevice, ctx->stream), "get fields");
    return SSM_OK;
}

ssm_status ssm_get_tangents(ssm_ctx* ctx, void* d_tangent, double* d_force_norm_or_null)
{
    if (!ctx) return SSM_EINVAL;
    ssm_status st = ensure_eval(ctx);
    if (st != SSM_OK) return st;
    hipError_t e;
    if (ctx->pl.prec == SSM_FP64)
        e = Ops<double>::tangents(ctx, ctx->stream, (double*)d_tangent, d_force_norm_or_null, 0.0);
    else
        e = Ops<float>::tangents(ctx, ctx->stream, (float*)d_tangent, d_force_norm_or_null, 0.0);
    if (e != hipSuccess) return hipfail(ctx, e, "tangents");
    return SSM_OK;
}

ssm_status ssm_get_barrier(ssm_ctx* ctx, double* d_out)
{
    if (!ctx || !d_out) return ctx ? fail(ctx, SSM_EINVAL, "d_out is NULL") : SSM_EINVAL;
    ssm_status st = ensure_eval(ctx);
    if (st != SSM_OK) return st;
    HIPCHK(ctx, launch_barrier(ctx->P(), ctx->pl.np, ctx->at<double>(ctx->pl.o_E),
                               ctx->at<double>(ctx->pl.o_T), d_out, ctx->stream), "barrier");
    return SSM_OK;
}

ssm_status ssm_check(ssm_ctx* ctx, int32_t* h_flags)
{
    if (!ctx || !h_flags) return ctx ? fail(ctx, SSM_EINVAL, "h_flags is NULL") : SSM_EINVAL;
    int f = 0;
    HIPCHK(ctx, hipMemcpyAsync(&f, ctx->ws + ctx->pl.o_flags, 4, hipMemcpyDeviceToHost, ctx->stream), "check");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "check");
    HIPCHK(ctx, launch_fill_int(ctx->at<int>(ctx->pl.o_flags), 1, 0, ctx->stream), "check");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "check");
    *h_flags = f;
    if (f & (SSM_FLAG_NONFINITE_ENERGY | SSM_FLAG_NONFINITE_SPIN))
        return fail(ctx, SSM_ENONFINITE, "non-finite energy or spin");
    return SSM_OK;
}

ssm_status ssm_profile(ssm_ctx* ctx, int32_t enable)
{
    if (!ctx) return SSM_EINVAL;
    ctx->profiling = enable != 0;
    return SSM_OK;
}

ssm_status ssm_profile_read(ssm_ctx* ctx, double* h_ms, int32_t* h_counts)
{
    if (!ctx) return SSM_EINVAL;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream), "profile read");
    for (auto& ev : ctx->events) {
        float ms = 0;
        HIPCHK(ctx, hipEventElapsedTime(&ms, ev.a, ev.b), "hipEventElapsedTime");
        ctx->prof_ms[ev.kind] += ms;
        ctx->prof_cnt[ev.kind] += 1;
        ctx->pool.push_back(ev.a);
        ctx->pool.push_back(ev.b);
    }
    ctx->events.clear();
    for (int i = 0; i < SSM_N_KERNELS; ++i) {
        if (h_ms) h_ms[i] = ctx->prof_ms[i];
        if (h_counts) h_counts[i] = ctx->prof_cnt[i];
        ctx->prof_ms[i] = 0;
        ctx->prof_cnt[i] = 0;
    }
    return SSM_OK;
}

ssm_status ssm_autotune(ssm_ctx* ctx, const char* cache_path)
{
    if (!ctx) return SSM_EINVAL;
    if (!ctx->have_string) return fail(ctx, SSM_ESTATE, "no string set");
    return autotune(ctx, cache_path);
}

ssm_status ssm_eval_noalloc(const ssm_problem* p, int32_t n_problems, int32_t precision, const void* d_spins,
                            void* d_field_or_null, double* d_energy, double* d_terms_or_null, void* stream)
{
    if (!p || !d_spins || !d_energy) return fail(nullptr, SSM_EINVAL, "p, d_spins and d_energy are required");
    if (n_problems < 1 || n_problems > kStaticMaxProblems)
        return fail(nullptr, SSM_EUNSUPPORTED, "ssm_eval_noalloc takes 1 to 16 problems");
    if (precision != SSM_FP64 && precision != SSM_FP32_MIXED)
        return fail(nullptr, SSM_EINVAL, "precision must be SSM_FP64 or SSM_FP32_MIXED");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(nullptr, SSM_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, SSM_EUNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_static_mu);
    StaticDev& sd = g_static[dev];
    ssm_ctx* c = &sd.ctx;
    const hipStream_t st = (hipStream_t)stream;
    if (!sd.ptr) {
        // once per device, with that device current: the device address of
        // this device's copy of the scratch array
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(nullptr, SSM_EHIP, std::string("hipGetSymbolAddress(scratch): ") +
                                                (e != hipSuccess ? hipGetErrorString(e) : "null address"));
        sd.ptr = static_cast<unsigned char*>(ptr);
    }
    if (!same_layout(sd, p, n_problems, precision)) {
        Plan pl;
        std::string err;
        ssm_status s = build_plan(p, n_problems, precision, nullptr, pl, err);
        if (s != SSM_OK) return fail(nullptr, s, err);
        carve_static(pl);
        if (pl.total > kStaticScratchBytes)
            return fail(nullptr, SSM_EUNSUPPORTED,
                        "ssm_eval_noalloc: these problems need " + std::to_string(pl.total) +
                            " bytes of scratch, more than its fixed " + std::to_string(kStaticScratchBytes));
        sd.have_tables = false;
        c->pl = pl;
        c->probs.assign(p, p + n_problems);
        c->ws = sd.ptr;
        c->ws_bytes = kStaticScratchBytes;
        c->stream = st;
        c->err.clear();
        s = setup_tables(c);
        if (s != SSM_OK) return fail(nullptr, s, c->err);
        sd.prec = precision;
        sd.np = n_problems;
        for (int i = 0; i < n_problems; ++i) {
            sd.shape[i][0] = p[i].nx; sd.shape[i][1] = p[i].ny;
            sd.shape[i][2] = p[i].nz; sd.shape[i][3] = p[i].n_images;
        }
        sd.have_tables = true;
    }
    c->stream = st;
    // this call's parameters into the descriptors, then the evaluation
    Plan& pl = c->pl;
    for (int i = 0; i < n_problems; ++i) {
        if (!std::isfinite(p[i].J) || !std::isfinite(p[i].d) || !std::isfinite(p[i].ku) || !std::isfinite(p[i].dip))
            return fail(nullptr, SSM_EINVAL, "non-finite parameter");
        pl.P[i].J = p[i].J; pl.P[i].d = p[i].d; pl.P[i].ku = p[i].ku; pl.P[i].D = p[i].dip;
    }
    e = put_bytes(sd.ptr + pl.o_P, pl.P.data(), sizeof(Prob) * pl.np, st);
    // the flags must start at zero: the scratch keeps the last call's contents
    if (e == hipSuccess) e = launch_fill_int(c->at<int>(pl.o_flags), 1, 0, st);
    if (e == hipSuccess) {
        if (pl.prec == SSM_FP64)
            e = Ops<double>::eval(c, st, (const double*)d_spins, (double*)d_field_or_null, d_energy,
                                  d_terms_or_null, false);
        else
            e = Ops<float>::eval(c, st, (const float*)d_spins, (float*)d_field_or_null, d_energy,
                                 d_terms_or_null, false);
    }
    if (e != hipSuccess) return fail(nullptr, SSM_EHIP, std::string("ssm_eval_noalloc: ") + hipGetErrorString(e));
    return SSM_OK;
}

}  // extern "C"
