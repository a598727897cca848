// HIP kernels (gfx950) of the simplified string method for atomistic spin
// lattices (Heistracher et al., arXiv:1804.07135).
//
// One string iteration is six kernels over every image of every problem:
//   k_xfwd   zero-padded real-to-complex FFT along x of the three spin
//            components (Sec. II.A: the dipolar field of eq. (6) is a
//            circular convolution once the lattice is padded);
//   k_conv   for each x-frequency: FFTs along y (and z), multiplication by
//            the FFT of the point-dipole tensor of eq. (7), inverse FFTs;
//   k_xinv   inverse FFT along x, then per site: exchange, DMI and
//            anisotropy stencils (eqs. (3)-(5)), the energy -1/2 h.s of
//            eq. (8) reduced in FP64, and the projected descent step with
//            renormalisation (eq. (10), Appendix force);
//   k_arc    FP64 partial sums of |phi*_k - phi*_{k-1}|^2 (eq. (11));
//   k_reduce per problem: energies, arc lengths, alpha* (eq. (12)) and the
//            interpolation interval/weight of every image (one workgroup
//            per image, or k_reduce1: one per small problem);
//   k_interp linear interpolation onto alpha_k = k/(K-1) + renormalisation
//            (or the spline step of the options).
//
// Padded lengths are P = 2m with m >= n a power of two, or 3 2^a where that
// is smaller.  A zero-padded length-P transform of n <= m inputs is two
// length-m transforms: the even outputs are the FFT of the inputs, the odd
// outputs the FFT of the inputs times W_P^j.  The inverse restricted to the
// first n outputs is the sum of the two inverse length-m transforms, the
// odd one times W_P^{-j}.  So no transform ever runs on a buffer of zeros,
// and only the x-spectra (m+1 complex values per row of n reals) travel
// through HBM.
//
// Length-m transforms run in LDS as Stockham passes (radix 16 first at the
// compile-time lengths, radix 4 and 2 otherwise; a radix-3 step for 3 2^a);
// every line belongs to one wavefront, which needs no workgroup barrier
// between passes.
#include "ssm_fft.hpp"
#include "ssm_internal.hpp"

namespace ssm {

// Tuning constants (compile-time): widest FFT pass (log2 radix) of the x
// kernels and of the convolution kernel, and the occupancy the FP32
// convolution kernel is compiled for (waves per SIMD; fewer waves leave more
// registers for its accumulator).
#ifndef SSM_X_RADIX_BITS
#define SSM_X_RADIX_BITS 2
#endif
#ifndef SSM_CONV_RADIX_BITS
#define SSM_CONV_RADIX_BITS 2
#endif
// 1: the 3 2^a forward x loads read 16 bytes per load where rows allow
#ifndef SSM_XFWD3_VEC
#define SSM_XFWD3_VEC 0
#endif
#ifndef SSM_XINV_WAVES_F32
#define SSM_XINV_WAVES_F32 3
#endif
#ifndef SSM_CONV_WAVES_F32
#define SSM_CONV_WAVES_F32 3
#endif
// Workgroup order of the convolution kernel when it takes one slice per
// workgroup: 1 = the images of one kx on one XCD back to back (kx spread
// over XCDs); 0 = kx-major, images innermost.
#ifndef SSM_CONV_XCD_REMAP
#define SSM_CONV_XCD_REMAP 1
#endif
// 1: load the kernel-spectrum coefficients of one z frequency at a time
// (fewer live registers in the z-phase).
#ifndef SSM_CONV_NH_SERIAL
#define SSM_CONV_NH_SERIAL 0
#endif
// widest pass of the compile-time-length x transforms (x lengths 32..512)
#ifndef SSM_X_CT_RADIX_BITS
#define SSM_X_CT_RADIX_BITS 4
#endif
// 1: swizzled LDS handoff between the radix-16 passes (y length 256)
#ifndef SSM_CONV_SWZ
#define SSM_CONV_SWZ 1
#endif
// 1: inverse-x tiles ordered with z fastest (0: y tile fastest)
#ifndef SSM_XINV_ZFAST
#define SSM_XINV_ZFAST 1
#endif
// 1: the convolution reads each kernel-spectrum row once per mirror pair
// of z frequencies (kz and -kz differ only in the sign of xz, yz)
#ifndef SSM_CONV_NH_MIRROR
#define SSM_CONV_NH_MIRROR 1
#endif
// 1: x-neighbour exchange of the inverse-x epilogue by DPP wavefront shifts
// (0: LDS permutes)
#ifndef SSM_XINV_DPP
#define SSM_XINV_DPP 1
#endif
// widest pass of the compile-time-length convolution bodies
#ifndef SSM_CONV_CT_RADIX_BITS
#define SSM_CONV_CT_RADIX_BITS 4
#endif
template <typename T> constexpr int kConvRadixBits = SSM_CONV_RADIX_BITS;

template <typename T> struct CT;
template <> struct CT<float> { using type = float2; };
template <> struct CT<double> { using type = double2; };
template <typename T> using cplx = typename CT<T>::type;

// The problem of item b: the last one whose first item (start, prefix
// sums) is <= b.  find_problem_lane takes any b per lane; find_problem a b
// that is the same on every lane of a full wavefront.
__device__ __forceinline__ int find_problem_lane(const int* __restrict__ start, int np, int b)
{
    int lo = 0, hi = np - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int find_problem(const int* __restrict__ start, int np, int b)
{
    if (np > 1 && np <= 64) {
        // one load per lane and a ballot instead of a chain of dependent loads
        const int lane = threadIdx.x & 63;
        const int v = start[lane < np ? lane : 0];
        return __popcll(__ballot(lane < np && v <= b)) - 1;
    }
    return find_problem_lane(start, np, b);
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Give each XCD a contiguous run of work items so that neighbouring
// items (adjacent rows, shared halo) are processed by one L2 back to back.
// w: workgroup index within the problem, n8: item count padded to 8.
__device__ __forceinline__ int xcd_item(int w, int n8) { return (w & 7) * (n8 >> 3) + (w >> 3); }

// Load exp(-2 pi i e/(2m)), e < 2m, into LDS from the compact table;
// m = 2^lm, or 3 2^lm when f3.
template <typename V>
__device__ __forceinline__ void load_twiddles(V* twl, int lm, int f3, const V* __restrict__ tw)
{
    const int n = (f3 ? 6 : 2) << lm;
    const V* src = tw + tw_off(lm, f3);
    for (int e = threadIdx.x; e < n; e += blockDim.x) twl[e] = src[e];
}

// q = i / L and r = i % L for a transform length L = 2^lg (f3 = 0) or
// 3 2^lg (f3 = 1); i < 3 2^17
__device__ __forceinline__ void divlen(int i, int lg, int f3, int& q, int& r)
{
    if (f3) {
        q = ((i >> lg) * 43691) >> 17;  // / 3
        r = i - ((q * 3) << lg);
    } else {
        q = i >> lg;
        r = i & ((1 << lg) - 1);
    }
}

// position in a transformed line of length m of x frequency q (within a
// half transform): lengths 3 2^lm leave the forward transform's output and
// take the inverse transform's input in the permuted order of fft_lines3
__device__ __forceinline__ int fpos(int q, int lm, int f3) { return f3 ? perm3(q, lm) : q; }

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// Transform of nl lines of length 2^lm stored contiguously: compile-time-
// length passes for 32..512 (pad layout x_padl), runtime-length passes
// (dense layout) otherwise.  f3: lines of length 3 2^lm, of which this runs
// only the power-of-two transforms of the 3 nl sub-lines (the x kernels do
// the radix-3 step as they load or store the lines): compile-time passes for
// 48..384.
template <typename V, bool INV>
__device__ __forceinline__ void fft_lines_x(V* lines, int nl, int lm, int f3, const V* twl)
{
    if (f3) {
        switch (SSM_X_CT ? lm : 0) {
        case 4: fft_lines_ct<V, INV, 4, SSM_X_CT_RADIX_BITS, x_padl(4, 1, sizeof(V) / 2), 3>(lines, 3 * nl, twl); break;
        case 5: fft_lines_ct<V, INV, 5, SSM_X_CT_RADIX_BITS, x_padl(5, 1, sizeof(V) / 2), 3>(lines, 3 * nl, twl); break;
        case 6: fft_lines_ct<V, INV, 6, SSM_X_CT_RADIX_BITS, x_padl(6, 1, sizeof(V) / 2), 3>(lines, 3 * nl, twl); break;
        case 7: fft_lines_ct<V, INV, 7, SSM_X_CT_RADIX_BITS, x_padl(7, 1, sizeof(V) / 2), 3>(lines, 3 * nl, twl); break;
        default: fft_lines<V, INV, SSM_X_RADIX_BITS, 3>(lines, 3 * nl, 1 << lm, lm, twl); break;
        }
        return;
    }
    switch (SSM_X_CT ? lm : 0) {
    case 5: fft_lines_ct<V, INV, 5, SSM_X_CT_RADIX_BITS, pad_for(SSM_X_PADL, 5)>(lines, nl, twl); break;
    case 6: fft_lines_ct<V, INV, 6, SSM_X_CT_RADIX_BITS, pad_for(SSM_X_PADL, 6)>(lines, nl, twl); break;
    case 7: fft_lines_ct<V, INV, 7, SSM_X_CT_RADIX_BITS, pad_for(SSM_X_PADL, 7)>(lines, nl, twl); break;
    case 8: fft_lines_ct<V, INV, 8, SSM_X_CT_RADIX_BITS, pad_for(SSM_X_PADL, 8)>(lines, nl, twl); break;
    case 9: fft_lines_ct<V, INV, 9, SSM_X_CT_RADIX_BITS, pad_for(SSM_X_PADL, 9)>(lines, nl, twl); break;
    default: fft_lines<V, INV, SSM_X_RADIX_BITS>(lines, nl, 1 << lm, lm, twl); break;
    }
}

// Two adjacent complex values p[0], p[1] with one 16-byte access in FP32
// (p 16-byte aligned: the spectra of an even ny, at an even y); in FP64 each
// value is a 16-byte access already.
template <typename V>
__device__ __forceinline__ void load2(const V* p, V& a, V& b)
{
    if constexpr (sizeof(V) == 8) {
        const float4 q = *reinterpret_cast<const float4*>(p);
        a = mk<V>(q.x, q.y);
        b = mk<V>(q.z, q.w);
    } else {
        a = p[0];
        b = p[1];
    }
}
template <typename V>
__device__ __forceinline__ void store2(V* p, V a, V b)
{
    if constexpr (sizeof(V) == 8) {
        *reinterpret_cast<float4*>(p) = make_float4(a.x, a.y, b.x, b.y);
    } else {
        p[0] = a;
        p[1] = b;
    }
}

// 16 bytes of T at p (16-byte aligned) into v, or zeros when !ok
template <typename T>
__device__ __forceinline__ void load16(const T* p, bool ok, T (&v)[16 / sizeof(T)])
{
    if constexpr (sizeof(T) == 4) {
        const float4 q = ok ? *reinterpret_cast<const float4*>(p) : make_float4(0.f, 0.f, 0.f, 0.f);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
        const double2 q = ok ? *reinterpret_cast<const double2*>(p) : make_double2(0.0, 0.0);
        v[0] = q.x; v[1] = q.y;
    }
}

// Loads of k_xfwd for power-of-two x lengths m = 2^lm: row pair rp, site j
// goes to position j of the even half line 2 rp and, twiddled by W_{2m}^j,
// of the odd half line 2 rp + 1; zero beyond the lattice.  kXfwdU items
// per thread per round: their loads, from positions clamped into the
// lattice, are issued together (no load sits under a branch), then the
// zeros are selected and the LDS writes done.  vecw: rows are read VW
// sites per 16-byte load.
#ifndef SSM_XFWD_U
#define SSM_XFWD_U 4
#endif
constexpr int kXfwdU = SSM_XFWD_U;
template <typename T>
__device__ __forceinline__ void xfwd_load_lines(const T* __restrict__ sc, cplx<T>* lines, const cplx<T>* twl,
                                                bool vecw, int hp, int m, int lm, int y0, int nx, int ny, int psh)
{
    using V = cplx<T>;
    constexpr int VW = 16 / sizeof(T), LVW = VW == 4 ? 2 : 1;
    auto put = [&](int rp, int j, V v) {
        const int i0 = (2 * rp) * m + j, i1 = i0 + m;
        lines[i0 + (i0 >> psh)] = v;
        lines[i1 + (i1 >> psh)] = cmul(v, twl[j]);
    };
    if (vecw) {
        const int lmv = lm - LVW;  // a line is m / VW chunks of VW sites
        const int total = hp << lmv;
#pragma unroll 1
        for (int idx0 = threadIdx.x; idx0 < total; idx0 += kXfwdU * kNT) {
            T av[kXfwdU][VW], bv[kXfwdU][VW];
#pragma unroll
            for (int u = 0; u < kXfwdU; ++u) {
                const int idx = min(idx0 + u * kNT, total - 1);
                const int rp = idx >> lmv, j = min((idx & ((1 << lmv) - 1)) << LVW, nx - VW);
                const int ya = y0 + 2 * rp;
                load16<T>(sc + (long long)min(ya, ny - 1) * nx + j, true, av[u]);
                load16<T>(sc + (long long)min(ya + 1, ny - 1) * nx + j, true, bv[u]);
            }
#pragma unroll
            for (int u = 0; u < kXfwdU; ++u) {
                const int idx = idx0 + u * kNT;
                if (idx >= total) break;
                const int rp = idx >> lmv, j = (idx & ((1 << lmv) - 1)) << LVW;
                const int ya = y0 + 2 * rp;
                const bool oka = j < nx && ya < ny, okb = j < nx && ya + 1 < ny;
#pragma unroll
                for (int k = 0; k < VW; ++k) put(rp, j + k, mk<V>(oka ? av[u][k] : T(0), okb ? bv[u][k] : T(0)));
            }
        }
    } else {
        const int total = hp << lm;
#pragma unroll 1
        for (int idx0 = threadIdx.x; idx0 < total; idx0 += kXfwdU * kNT) {
            T a[kXfwdU], b[kXfwdU];
#pragma unroll
            for (int u = 0; u < kXfwdU; ++u) {
                const int idx = min(idx0 + u * kNT, total - 1);
                const int rp = idx >> lm, j = min(idx & (m - 1), nx - 1);
                const int ya = y0 + 2 * rp;
                a[u] = sc[(long long)min(ya, ny - 1) * nx + j];
                b[u] = sc[(long long)min(ya + 1, ny - 1) * nx + j];
            }
#pragma unroll
            for (int u = 0; u < kXfwdU; ++u) {
                const int idx = idx0 + u * kNT;
                if (idx >= total) break;
                const int rp = idx >> lm, j = idx & (m - 1);
                const int ya = y0 + 2 * rp;
                const bool in = j < nx;
                put(rp, j, mk<V>(in && ya < ny ? a[u] : T(0), in && ya + 1 < ny ? b[u] : T(0)));
            }
        }
    }
}

// Loads of k_xfwd for x lengths m = 3 M (M = 2^lm) with the radix-3 step of
// the forward transform (decimation in frequency, ssm_fft.hpp) applied on the
// way: the thread of row pair rp and position k < M reads the sites k, k + M,
// k + 2M of both rows, and writes the three butterfly outputs of the even
// half line, and of the odd half line (input twiddled by W_{2m}^x first), to
// positions k, k + M, k + 2M of those lines, where the sub-line transforms
// take them.  vecw: rows are read VW sites per 16-byte load.
template <typename T>
__device__ __forceinline__ void xfwd_load3(const T* __restrict__ sc, cplx<T>* lines, const cplx<T>* twl, bool vecw,
                                           int hp, int lm, int y0, int nx, int ny, int psh)
{
    using V = cplx<T>;
    constexpr int VW = 16 / sizeof(T), LVW = VW == 4 ? 2 : 1;
    const int M = 1 << lm, m = 3 * M;
    auto put = [&](int rp, int k, V (&e)[3]) {
        V o[3];
#pragma unroll
        for (int t = 0; t < 3; ++t) o[t] = cmul(e[t], twl[k + t * M]);
        const V w1 = twl[2 * k], w2 = twl[4 * k];
        radix3_bfly<false>(e[0], e[1], e[2], w1, w2);
        radix3_bfly<false>(o[0], o[1], o[2], w1, w2);
        const int i0 = (2 * rp) * m + k, i1 = i0 + m;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const int a = i0 + t * M, b = i1 + t * M;
            lines[a + (a >> psh)] = e[t];
            lines[b + (b >> psh)] = o[t];
        }
    };
    if (SSM_XFWD3_VEC && vecw) {
        const int lmv = lm - LVW;  // a sub-line is M / VW chunks of VW sites
#pragma unroll 1
        for (int idx = threadIdx.x; idx < (hp << lmv); idx += kNT) {
            const int rp = idx >> lmv, k0 = (idx & ((1 << lmv) - 1)) << LVW;
            const int ya = y0 + 2 * rp;
            T av[3][VW], bv[3][VW];
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                const int j = k0 + t * M;
                load16<T>(sc + (long long)ya * nx + j, j < nx && ya < ny, av[t]);
                load16<T>(sc + (long long)(ya + 1) * nx + j, j < nx && ya + 1 < ny, bv[t]);
            }
#pragma unroll
            for (int q = 0; q < VW; ++q) {
                V e[3];
#pragma unroll
                for (int t = 0; t < 3; ++t) e[t] = mk<V>(av[t][q], bv[t][q]);
                put(rp, k0 + q, e);
            }
        }
    } else {
#pragma unroll 1
        for (int idx = threadIdx.x; idx < (hp << lm); idx += kNT) {
            const int rp = idx >> lm, k = idx & (M - 1);
            const int ya = y0 + 2 * rp;
            // rows and columns clamped into the lattice for the loads (all
            // issued before any is used), zero outside it
            const T* ra = sc + (long long)min(ya, ny - 1) * nx;
            const T* rb = sc + (long long)min(ya + 1, ny - 1) * nx;
            V e[3];
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                const int j = min(k + t * M, nx - 1);
                e[t] = mk<V>(ra[j], rb[j]);
            }
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                const bool in = k + t * M < nx;
                e[t] = mk<V>(in && ya < ny ? e[t].x : T(0), in && ya + 1 < ny ? e[t].y : T(0));
            }
            put(rp, k, e);
        }
    }
}

// ---------------------------------------------------------------------------
// k_xfwd: rows of a tile (image, z, ytf rows) -> x half-spectra, one spin
// component at a time.  Two real rows of one component form one complex
// signal a + i b; its length-2m spectrum Z gives A(k) = (Z(k) + conj Z(-k))/2
// and B(k) = -i (Z(k) - conj Z(-k))/2 for k = 0..m.
// Output layout X[img][kx][c][z][y]: a tile writes ytf consecutive y values.
// LDS: twiddles (2m) + ytf lines of m (padded layout).
// ---------------------------------------------------------------------------
// F3: x length 3 2^lmx (the kernel serves the problems of that length kind
// only, so the length arithmetic is fixed at compile time)
template <typename T, int F3>
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 3, 8))) void k_xfwd(const Prob* __restrict__ P, int np,
                                              const int* __restrict__ wstart,
                                              const T* __restrict__ s, cplx<T>* __restrict__ X,
                                              const cplx<T>* __restrict__ tw,
                                              const int* __restrict__ done)
{
    using V = cplx<T>;
    extern __shared__ double2 smem_[];
    const int pi = find_problem(wstart, np, blockIdx.x);
    if (done && done[pi]) return;
    const Prob& p = P[pi];
    if (p.f3x != F3) return;  // served by the other length kind's launch
    const int t = xcd_item(blockIdx.x - wstart[pi], p.wgf);
    if (t >= p.K * p.tilesf) return;
    const int ty = t % p.ntyf, rest = t / p.ntyf;
    const int z = rest % p.nz, img = rest / p.nz;
    const int yt = p.ytf, hp = yt >> 1, nx = p.nx, ny = p.ny, nz = p.nz, m = p.mx, lm = p.lmx;
    constexpr int f3 = F3;
    const int lhp = __ffs(hp) - 1;  // tiles are powers of two
    const int psh = x_padl(lm, f3, sizeof(T)) ? x_padl(lm, f3, sizeof(T)) : 31;  // pad layout of the lines
    // line index of position q (< m) of line l: l m + q, m = 2^lm or 3 2^lm
    auto lidx = [&](int l, int q) { return (F3 ? (l + (l << 1)) << lm : l << lm) + q; };
    V* twl = reinterpret_cast<V*>(smem_);
    V* lines = twl + 2 * m;
    load_twiddles(twl, lm, f3, tw);
    const long long N = p.N;
    const T* si = s + p.s_off + (long long)img * 3 * N + (long long)z * ny * nx;
    // the image's spectra as a uniform base and 32-bit byte offsets (they
    // span at most 1025 * 3 * 16 * 1024 complex values, under 2^32 bytes)
    char* const Xi = reinterpret_cast<char*>(X + p.x_off + (long long)img * (m + 1) * 3 * nz * ny);
    const int y0 = ty * yt, P2 = 2 * m;
    __syncthreads();
    // rows of a length divisible by VW = 16 / sizeof(T) from a 16-byte
    // aligned image are read VW sites per 16-byte load
    constexpr int VW = 16 / sizeof(T);
    const bool vecw = !(nx & (VW - 1)) && !(reinterpret_cast<size_t>(si) & 15);
#pragma unroll 1
    for (int c = 0; c < 3; ++c) {
        const T* sc = si + (long long)c * N;
        if constexpr (F3) {
            xfwd_load3<T>(sc, lines, twl, vecw, hp, lm, y0, nx, ny, psh);
        } else {
            xfwd_load_lines<T>(sc, lines, twl, vecw, hp, m, lm, y0, nx, ny, psh);
        }
        __syncthreads();
        fft_lines_x<V, false>(lines, yt, lm, f3, twl);
        __syncthreads();
        for (int idx = threadIdx.x; idx < (m + 1) * hp; idx += kNT) {
            const int rp = idx & (hp - 1), kx = idx >> lhp;
            const int kr = kx ? P2 - kx : 0;
            // the two halves (even, odd frequencies) are separate lines
            const int iz = lidx(2 * rp + (kx & 1), fpos(kx >> 1, lm, f3));
            const int ir = lidx(2 * rp + (kr & 1), fpos(kr >> 1, lm, f3));
            const V Z = lines[iz + (iz >> psh)];
            const V Zr = lines[ir + (ir >> psh)];
            const T hlf = T(0.5);
            const V A = mk<V>((Z.x + Zr.x) * hlf, (Z.y - Zr.y) * hlf);
            const V B = mk<V>((Z.y + Zr.y) * hlf, (Zr.x - Z.x) * hlf);
            const int ya = y0 + 2 * rp;
            const unsigned o = (unsigned)(((kx * 3 + c) * nz + z) * ny + ya) * (unsigned)sizeof(V);
            V* dst = reinterpret_cast<V*>(Xi + o);  // row ya
            if (!(ny & 1)) {
                if (ya < ny) store2(dst, A, B);
            } else {
                if (ya < ny) dst[0] = A;
                if (ya + 1 < ny) *reinterpret_cast<V*>(Xi + o + (unsigned)sizeof(V)) = B;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// k_conv: for G consecutive (image, kx) slices [c][z][y], the convolution in
// (y, z) with the dipole-kernel spectrum.  The padded y transform (length
// 2 m_y) is split into its even and odd halves hy (twiddle W^{hy*y}, then a
// length-m_y FFT in LDS).  The z twiddle of the padded z transform is a
// per-line constant, so it commutes with the y FFT: the register z-phase
// applies it and runs both z halves hz itself (length-mz DFTs), multiplies
// by the real symmetric kernel spectrum (xx, xy, xz, yy, yz, zz), inverts
// and sums the halves.  Then inverse y FFT and un-twiddle; the y half 0
// result goes to the output slice and the y half 1 result is added onto it
// (each thread adds onto the values it stored itself).  The kernel
// spectrum carries 1/(Px Py Pz).
// LDS: twiddles (2 m_y) + G*3*nz lines of m_y.
// ---------------------------------------------------------------------------



// multiply by the padded-z twiddle exp(-2 pi i zz / (2 MZ)) (conjugate for
// INV); zz is a compile-time constant after unrolling
template <bool INV, typename V, int MZ>
__device__ __forceinline__ V twz(V v, int zz, const V* __restrict__ tw)
{
    if (MZ <= 8) return twc16<INV>(v, zz * (8 / MZ));
    const V w = tw[tw_off(4, 0) + zz];  // W_32^zz
    return INV ? cmulc(v, w) : cmul(v, w);
}

// y transform of the runtime-length convolution body; lengths 3 2^lmy
// (f3y) in the permuted order of fft_lines3
template <typename V, bool INV>
__device__ __forceinline__ void conv_fft_y(V* lines, int nlines, int lmy, int f3y, const V* twl)
{
    if (f3y) fft_lines3<V, INV, SSM_CONV_RADIX_BITS>(lines, nlines, lmy, twl);
    else fft_lines<V, INV, SSM_CONV_RADIX_BITS>(lines, nlines, 1 << lmy, lmy, twl);
}

// z-phase of the compile-time-length convolution bodies: for every column
// (slice g, position py, y frequency qy) of the G slices in LDS, both z
// halves of the padded z transform (length-MZ DFTs), the 3x3 kernel-
// spectrum multiply, the inverse and the sum of the halves.  NZ > 0 fixes
// nz at compile time.  y length MY = 2^LMY, or 3 2^LMY (F3) with the
// permuted frequency order of the 3 2^a transforms.
template <typename T, int MZ, int LMY, int NZ, int PADL, int F3 = 0>
__device__ __forceinline__ void conv_zphase(const Prob& p, int G, int kx0, int hy, cplx<T>* lines,
                                            const T* __restrict__ nhat, const cplx<T>* __restrict__ tw)
{
    using V = cplx<T>;
    constexpr int MY = (F3 ? 3 : 1) << LMY;
    const int nz = NZ > 0 ? NZ : p.nz, nhz = p.nhz, nsl_img = p.mx + 1;
    int col0 = threadIdx.x;
    asm volatile("" : "+v"(col0));
    for (int col = col0; col < G * MY; col += kNT) {
        const int g = col / MY, py = col - g * MY;
        const int qy = F3 ? unperm3(py, LMY) : py;
        int kx = kx0 + g;
        while (kx >= nsl_img) kx -= nsl_img;
        // padded offsets: cbase % 2^PADL = py % 2^PADL and the line offsets
        // are multiples of the line length, so padx distributes
        const int cbase = padx<PADL>(g * 3 * nz * MY + py);
        V b[3][MZ];
        // the two z halves as separate bodies (hz a compile-time constant:
        // the even half has no twiddles, and no selects between the halves)
        auto zhalf = [&](auto hzc) {
            constexpr int hz = decltype(hzc)::value;
            const T* nh = nhat + p.nh_off + (((((long long)kx * nhz + hz) * 2 + hy) * MZ) * 6 * MY) + qy;
            // the column's kernel-spectrum rows, loaded before its LDS reads
            // and z transforms so that their latency overlaps that work.
            // z frequency kz = 2r + hz and its mirror -kz (mod 2 MZ) hold
            // the same spectrum up to the sign of the z-odd components xz
            // and yz (the tensor is even in z except for those), so each
            // column reads only the rows r <= mirror (9 of 16 for MZ = 8)
            // and the unrolled loop folds the repeated loads (not for 8
            // layers with y lengths below 256, where keeping the shared rows
            // live costs more registers than it saves)
            constexpr bool kMir = SSM_CONV_NH_MIRROR && (MZ <= 4 || LMY >= 8);
            T nv[MZ][6];
#pragma unroll
            for (int r = 0; r < MZ; ++r) {
                const bool mir = kMir && (hz == 0 ? 2 * r > MZ : 2 * r >= MZ);
                const int rs = mir ? (hz == 0 ? MZ - r : MZ - 1 - r) : r;
                const T* q6 = nh + rs * 6 * MY;
                nv[r][0] = q6[0];
                nv[r][1] = q6[MY];
                nv[r][2] = mir ? -q6[2 * MY] : q6[2 * MY];
                nv[r][3] = q6[3 * MY];
                nv[r][4] = mir ? -q6[4 * MY] : q6[4 * MY];
                nv[r][5] = q6[5 * MY];
            }
            V a[3][MZ];
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int zz = 0; zz < MZ; ++zz) {
                    V v = (zz < nz) ? lines[cbase + padx<PADL>((c * nz + zz) * MY)] : mk<V>(0, 0);
                    if constexpr (hz == 1) v = twz<false, V, MZ>(v, zz, tw);
                    a[c][zz] = v;
                }
#pragma unroll
            for (int c = 0; c < 3; ++c) dft_reg<V, MZ, false>(a[c]);
#pragma unroll
            for (int r = 0; r < MZ; ++r) {
                const T nxx = nv[r][0], nxy = nv[r][1], nxz = nv[r][2];
                const T nyy = nv[r][3], nyz = nv[r][4], nzz = nv[r][5];
                const V sx = a[0][r], sy = a[1][r], sz = a[2][r];
                a[0][r] = mk<V>(nxx * sx.x + nxy * sy.x + nxz * sz.x, nxx * sx.y + nxy * sy.y + nxz * sz.y);
                a[1][r] = mk<V>(nxy * sx.x + nyy * sy.x + nyz * sz.x, nxy * sx.y + nyy * sy.y + nyz * sz.y);
                a[2][r] = mk<V>(nxz * sx.x + nyz * sy.x + nzz * sz.x, nxz * sx.y + nyz * sy.y + nzz * sz.y);
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) dft_reg<V, MZ, true>(a[c]);
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int zz = 0; zz < MZ; ++zz) {
                    V v = a[c][zz];
                    if constexpr (hz == 1) {
                        v = twz<true, V, MZ>(v, zz, tw);
                        b[c][zz] = cadd(b[c][zz], v);
                    } else {
                        b[c][zz] = v;
                    }
                }
        };
        zhalf(std::integral_constant<int, 0>{});
        if (nhz > 1) zhalf(std::integral_constant<int, 1>{});
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int zz = 0; zz < MZ; ++zz)
                if (zz < nz) lines[cbase + padx<PADL>((c * nz + zz) * MY)] = b[c][zz];
    }
}

// Compile-time-length body (m_y = 2^LMY) of the convolution of G slices.
// The forward y transform takes its first pass straight from the slice in
// global memory (zero beyond ny, the odd-half twiddle W^{hy*y} applied on
// the way) and the inverse writes its last pass straight to the output
// slice, so the lines visit LDS only between passes and in the z-phase.
// Lines belong to wavefronts (groups of 1024 elements), so only the z-phase,
// which reads every line of a column, needs workgroup barriers.
template <typename T, int MZ, int LMY>
__device__ __forceinline__ void conv_body_ct(const Prob& p, int s0, int G, cplx<T>* __restrict__ X,
                                             cplx<T>* __restrict__ Xp, const T* __restrict__ nhat,
                                             const cplx<T>* __restrict__ tw, cplx<T>* smem)
{
    using V = cplx<T>;
    constexpr int MB = SSM_CONV_CT_RADIX_BITS;
    constexpr int MY = 1 << LMY;
    constexpr int LPG = fft_group_lines(LMY);
    // first pass (from global) and last pass (to global) of the schedule
    constexpr int B0 = fft_next_bits(LMY, MB), R0 = 1 << B0;
    constexpr int LNSL = fft_last_lns(LMY, MB);
    constexpr int BL = LMY - LNSL, RL = 1 << BL;
    static_assert(LNSL >= B0, "the y schedule needs at least two passes");
    // pad layout; twiddles W_{2 m_y} from an LDS copy
    constexpr int PADL = conv_padl(MZ, LMY, 0, sizeof(T));
    constexpr int TWS = 0;
    // swizzled handoff between the two radix-16 passes of length 256
    constexpr bool SW = SSM_CONV_SWZ && PADL == 0 && LMY == 8 && MB == 4;
    using P0 = PassCT<V, R0, false, LMY, 0, PADL, TWS, false, SW>;
    using PL = PassCT<V, RL, true, LMY, LNSL, PADL, TWS, SW, false>;
    const int nsl_img = p.mx + 1;
    const int nz = p.nz, ny = p.ny;
    const int per = 3 * nz * ny, nlines = G * 3 * nz;
    load_twiddles(smem, LMY, 0, tw);
    const V* twl = smem;
    V* lines = smem + 2 * MY;
    V* in = X + p.x_off + (long long)s0 * per;
    V* out = Xp + p.x_off + (long long)s0 * per;
    const int kx0 = s0 % nsl_img;
    const int wave = threadIdx.x >> 6;
    constexpr int NW = kNT / 64;
    __syncthreads();

#pragma unroll 1
    for (int hy = 0; hy < 2; ++hy) {
        // per-lane indices are recomputed in every phase (opaque copy) so
        // that no address stays live across the register-heavy z-phase
        int lane = threadIdx.x;
        asm volatile("" : "+v"(lane));
        lane &= 63;
        // forward y transform, wavefront-owned line groups
        for (int g0 = wave * LPG; g0 < nlines; g0 += NW * LPG) {
            const int gl = min(LPG, nlines - g0);
            {
                V v[P0::B][R0];
#pragma unroll
                for (int b = 0; b < P0::B; ++b) {
                    const int g = lane | (b << 6);
                    if (g < (gl << P0::LQ)) {
                        const int line = g >> P0::LQ, j = g & (P0::Q - 1);
                        const V* src = in + (long long)(g0 + line) * ny;
                        if (ny == MY) {
#pragma unroll
                            for (int r = 0; r < R0; ++r) v[b][r] = src[j + r * P0::Q];
                        } else {
                            // loads from inside the line first, then zeros
#pragma unroll
                            for (int r = 0; r < R0; ++r) v[b][r] = src[min(j + r * P0::Q, ny - 1)];
#pragma unroll
                            for (int r = 0; r < R0; ++r)
                                if (j + r * P0::Q >= ny) v[b][r] = mk<V>(0, 0);
                        }
                        if (hy) {
#pragma unroll
                            for (int r = 0; r < R0; ++r) v[b][r] = cmul(v[b][r], twl[(j + r * P0::Q) << TWS]);
                        }
                        dft_reg<V, R0, false>(v[b]);
                    }
                }
                P0::write(lines, g0 << LMY, gl, lane, v);
                wave_sync();
            }
            fft_passes_ct_to<V, false, LMY, MB, B0, LMY, PADL, TWS, SW>(lines, g0 << LMY, gl, twl, lane);
        }
        __syncthreads();

        // z-phase: per column (slice, qy), z DFT halves, 3x3 multiply,
        // inverse (nz at run time: compile-time offsets make the scheduler
        // hoist every load of the column and run out of registers)
        conv_zphase<T, MZ, LMY, 0, PADL>(p, G, kx0, hy, lines, nhat, tw);
        __syncthreads();

        // inverse y transform; the last pass writes y half hy = 0 to the
        // output slice and adds hy = 1 (un-twiddled) onto it
        lane = threadIdx.x;
        asm volatile("" : "+v"(lane));
        lane &= 63;
        for (int g0 = wave * LPG; g0 < nlines; g0 += NW * LPG) {
            const int gl = min(LPG, nlines - g0);
            fft_passes_ct_to<V, true, LMY, MB, 0, LNSL, PADL, TWS, SW>(lines, g0 << LMY, gl, twl, lane);
            V v[PL::B][RL];
            PL::read(lines, g0 << LMY, gl, twl, lane, v);
#pragma unroll
            for (int b = 0; b < PL::B; ++b) {
                const int g = lane | (b << 6);
                if (g < (gl << PL::LQ)) {
                    // last pass: j < NS, so the outputs are y = j + r NS
                    const int line = g >> PL::LQ, j = g & (PL::Q - 1);
                    V* dst = out + (long long)(g0 + line) * ny;
                    if (hy) {
                        // half 1, un-twiddled, added onto half 0, which this
                        // thread stored to the same places before the
                        // z-phase barriers of this half (all loads issued
                        // before any add)
#pragma unroll
                        for (int r = 0; r < RL; ++r) v[b][r] = cmulc(v[b][r], twl[(j + r * PL::NS) << TWS]);
                        // (a ragged line also reads the positions past ny:
                        // the next line's values, or the slack the
                        // workspace keeps after the buffer; those sums are
                        // never stored)
                        V h0[RL];
#pragma unroll
                        for (int r = 0; r < RL; ++r) h0[r] = dst[j + r * PL::NS];
#pragma unroll
                        for (int r = 0; r < RL; ++r) v[b][r] = cadd(v[b][r], h0[r]);
                    }
                    if (ny == MY) {
#pragma unroll
                        for (int r = 0; r < RL; ++r) dst[j + r * PL::NS] = v[b][r];
                    } else {
#pragma unroll
                        for (int r = 0; r < RL; ++r) {
                            const int y = j + r * PL::NS;
                            if (y < ny) dst[y] = v[b][r];
                        }
                    }
                }
            }
            // the next forward pass of this group rewrites these lines
            wave_sync();
        }
    }
}

// The convolution of G slices starting at s0, y length from the problem
// (the runtime-length body).
constexpr int kConvU = 4;
template <typename T, int MZ>
__device__ __forceinline__ void conv_body(const Prob& p, int s0, int G, cplx<T>* __restrict__ X,
                                          cplx<T>* __restrict__ Xp, const T* __restrict__ nhat,
                                          const cplx<T>* __restrict__ tw, cplx<T>* smem)
{
    using V = cplx<T>;
    const int nsl_img = p.mx + 1;
    const int nz = p.nz, ny = p.ny, nhz = p.nhz;
    const int lmy = p.lmy, f3y = p.f3y, my = p.my;
    const int per = 3 * nz * ny, nel = G * per, nlines = G * 3 * nz;
    V* twl = smem;
    V* lines = twl + 2 * my;
    load_twiddles(twl, lmy, f3y, tw);
    V* in = X + p.x_off + (long long)s0 * per;
    V* out = Xp + p.x_off + (long long)s0 * per;
    const int dy = kNT % ny, dr = kNT / ny;
    const int yb = threadIdx.x % ny, rb = threadIdx.x / ny;
    const int kx0 = s0 % nsl_img;

    __syncthreads();

#pragma unroll 1
    for (int hy = 0; hy < 2; ++hy) {
        {
            // kConvU elements per thread per round, their loads issued
            // together (an element past the end loads the last one)
            int y = yb, r = rb;
            asm volatile("" : "+v"(y), "+v"(r));
#pragma unroll 1
            for (int e0 = threadIdx.x; e0 < nel; e0 += kConvU * kNT) {
                V v[kConvU];
#pragma unroll
                for (int u = 0; u < kConvU; ++u) v[u] = in[min(e0 + u * kNT, nel - 1)];
#pragma unroll
                for (int u = 0; u < kConvU; ++u) {
                    if (e0 + u * kNT < nel) lines[lds_pad(r * my + y)] = hy ? cmul(v[u], twl[y]) : v[u];
                    y += dy;
                    r += dr;
                    if (y >= ny) { y -= ny; r += 1; }
                }
            }
        }
        if (my > ny) {
            const int tail = my - ny;
            for (int e = threadIdx.x; e < nlines * tail; e += kNT) {
                const int r = e / tail, y = ny + e % tail;
                lines[lds_pad(r * my + y)] = mk<V>(0, 0);
            }
        }
        __syncthreads();
        conv_fft_y<V, false>(lines, nlines, lmy, f3y, twl);
        __syncthreads();

        int col0 = threadIdx.x;
        asm volatile("" : "+v"(col0));
        for (int col = col0; col < G * my; col += kNT) {
            // column at position py of slice g holds y frequency qy
            int g, py;
            divlen(col, lmy, f3y, g, py);
            const int qy = f3y ? unperm3(py, lmy) : py;
            int kx = kx0 + g;
            while (kx >= nsl_img) kx -= nsl_img;
            const int cbase = g * 3 * nz * my + py;
            V b[3][MZ];
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int zz = 0; zz < MZ; ++zz) b[c][zz] = mk<V>(0, 0);
#pragma unroll 1
            for (int hz = 0; hz < nhz; ++hz) {
                V a[3][MZ];
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int zz = 0; zz < MZ; ++zz) {
                        V v = (zz < nz) ? lines[lds_pad(cbase + (c * nz + zz) * my)] : mk<V>(0, 0);
                        if (hz) v = twz<false, V, MZ>(v, zz, tw);
                        a[c][zz] = v;
                    }
#pragma unroll
                for (int c = 0; c < 3; ++c) dft_reg<V, MZ, false>(a[c]);
                const T* nh = nhat + p.nh_off + ((((long long)kx * nhz + hz) * 2 + hy) * MZ) * 6 * my + qy;
#pragma unroll
                for (int r = 0; r < MZ; ++r) {
                    const T* q6 = nh + (long long)r * 6 * my;
                    if (SSM_CONV_NH_SERIAL) asm volatile("" : "+v"(q6));
                    const T nxx = q6[0], nxy = q6[my], nxz = q6[2 * my];
                    const T nyy = q6[3 * my], nyz = q6[4 * my], nzz = q6[5 * my];
                    const V sx = a[0][r], sy = a[1][r], sz = a[2][r];
                    a[0][r] = mk<V>(nxx * sx.x + nxy * sy.x + nxz * sz.x, nxx * sx.y + nxy * sy.y + nxz * sz.y);
                    a[1][r] = mk<V>(nxy * sx.x + nyy * sy.x + nyz * sz.x, nxy * sx.y + nyy * sy.y + nyz * sz.y);
                    a[2][r] = mk<V>(nxz * sx.x + nyz * sy.x + nzz * sz.x, nxz * sx.y + nyz * sy.y + nzz * sz.y);
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) dft_reg<V, MZ, true>(a[c]);
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int zz = 0; zz < MZ; ++zz) {
                        V v = a[c][zz];
                        if (hz) v = twz<true, V, MZ>(v, zz, tw);
                        b[c][zz] = cadd(b[c][zz], v);
                    }
            }
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int zz = 0; zz < MZ; ++zz)
                    if (zz < nz) lines[lds_pad(cbase + (c * nz + zz) * my)] = b[c][zz];
        }
        __syncthreads();
        conv_fft_y<V, true>(lines, nlines, lmy, f3y, twl);
        __syncthreads();
        {
            // y half hy = 0 goes to the output slice, hy = 1 (un-twiddled)
            // over this workgroup's input slice, which is no longer read
            // (half 1: the half-0 values of a round's elements, which this
            // thread stored itself, are loaded together first)
            int y = yb, r = rb;
            asm volatile("" : "+v"(y), "+v"(r));
            V* dst = out;
#pragma unroll 1
            for (int e0 = threadIdx.x; e0 < nel; e0 += kConvU * kNT) {
                V h0[kConvU];
                if (hy) {
#pragma unroll
                    for (int u = 0; u < kConvU; ++u) h0[u] = dst[min(e0 + u * kNT, nel - 1)];
                }
#pragma unroll
                for (int u = 0; u < kConvU; ++u) {
                    const int e = e0 + u * kNT;
                    if (e < nel) {
                        V v = lines[lds_pad(r * my + y)];
                        if (hy) v = cadd(cmulc(v, twl[y]), h0[u]);
                        dst[e] = v;
                    }
                    y += dy;
                    r += dr;
                    if (y >= ny) { y -= ny; r += 1; }
                }
            }
        }
        __syncthreads();
    }
}

// Compile-time-length body for y lengths m_y = 3 M, M = 2^LMY (48, 96,
// 192).  As conv_body_ct, with the radix-3 steps of the y transform
// (ssm_fft.hpp) fused into the global-memory side: the forward one reads
// the slice (zero beyond ny, the odd-half twiddle applied), does the radix-3
// butterflies and the first, radix-4 pass of the three sub-lines, and
// writes to LDS; the inverse one does the last, radix-4 pass of the three
// sub-lines and the inverse radix-3 butterflies, and writes the slice.  A
// wavefront owns whole lines (PLG of them, 3 PLG sub-lines), so only the
// z-phase needs workgroup barriers.
template <typename T, int MZ, int LMY>
__device__ __forceinline__ void conv_body_ct3(const Prob& p, int s0, int G, cplx<T>* __restrict__ X,
                                              cplx<T>* __restrict__ Xp, const T* __restrict__ nhat,
                                              const cplx<T>* __restrict__ tw, cplx<T>* smem)
{
    using V = cplx<T>;
    constexpr int MB = SSM_CONV_CT_RADIX_BITS;
    constexpr int M = 1 << LMY, MY = 3 * M;
    constexpr int PLG = 1024 / MY;      // lines per wavefront group
    constexpr int BF = 2, RF = 1 << BF;  // fused sub-line passes: radix 4
    constexpr int QF = M / RF;           // their butterflies per sub-line
    constexpr int LQF = LMY - BF;
    constexpr int PADL = conv_padl(MZ, LMY, 1, sizeof(T));
    static_assert(PLG >= 1 && LMY - BF >= 2, "length outside the compile-time 3 2^a set");
    const int nsl_img = p.mx + 1;
    const int nz = p.nz, ny = p.ny;
    const int per = 3 * nz * ny, nlines = G * 3 * nz;
    load_twiddles(smem, LMY, 1, tw);
    const V* twl = smem;
    V* lines = smem + 2 * MY;
    V* in = X + p.x_off + (long long)s0 * per;
    V* out = Xp + p.x_off + (long long)s0 * per;
    const int kx0 = s0 % nsl_img;
    const int wave = threadIdx.x >> 6;
    constexpr int NW = kNT / 64;
    __syncthreads();

#pragma unroll 1
    for (int hy = 0; hy < 2; ++hy) {
        int lane = threadIdx.x;
        asm volatile("" : "+v"(lane));
        lane &= 63;
        for (int g0 = wave * PLG; g0 < nlines; g0 += NW * PLG) {
            const int gl = min(PLG, nlines - g0);
            // item (line, j): inputs y = j + r QF + t M (r < 4, t < 3), all
            // loaded (from inside the line) before any is used, then zeroed
            // beyond ny
            for (int it = lane; it < (gl << LQF); it += 64) {
                const int line = it >> LQF, j = it & (QF - 1);
                const V* src = in + (long long)(g0 + line) * ny;
                V v[3][RF];
#pragma unroll
                for (int t = 0; t < 3; ++t)
#pragma unroll
                    for (int r = 0; r < RF; ++r) v[t][r] = src[min(j + r * QF + t * M, ny - 1)];
                if (hy) {
#pragma unroll
                    for (int t = 0; t < 3; ++t)
#pragma unroll
                        for (int r = 0; r < RF; ++r) v[t][r] = cmul(v[t][r], twl[j + r * QF + t * M]);
                }
#pragma unroll
                for (int t = 0; t < 3; ++t)
#pragma unroll
                    for (int r = 0; r < RF; ++r)
                        if (j + r * QF + t * M >= ny) v[t][r] = mk<V>(0, 0);
#pragma unroll
                for (int r = 0; r < RF; ++r) {
                    const int k = j + r * QF;
                    radix3_bfly<false>(v[0][r], v[1][r], v[2][r], twl[2 * k], twl[4 * k]);
                }
                // first pass (sub-length 1) of sub-line t: outputs at j RF + r
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                    dft_reg<V, RF, false>(v[t]);
                    const int b = (((g0 + line) * 3 + t) << LMY) + j * RF;
#pragma unroll
                    for (int r = 0; r < RF; ++r) lines[padx<PADL>(b + r)] = v[t][r];
                }
            }
            wave_sync();
            fft_passes_ct_to<V, false, LMY, MB, BF, LMY, PADL, 0, false, 3>(lines, (3 * g0) << LMY, 3 * gl, twl,
                                                                           lane);
        }
        __syncthreads();

        conv_zphase<T, MZ, LMY, 0, PADL, 1>(p, G, kx0, hy, lines, nhat, tw);
        __syncthreads();

        lane = threadIdx.x;
        asm volatile("" : "+v"(lane));
        lane &= 63;
        for (int g0 = wave * PLG; g0 < nlines; g0 += NW * PLG) {
            const int gl = min(PLG, nlines - g0);
            fft_passes_ct_span<V, true, LMY, MB, 0, LMY - BF, PADL, 3>(lines, (3 * g0) << LMY, 3 * gl, twl, lane);
            // item (line, j): the last pass (sub-length M / 4) of the three
            // sub-lines gives their values at k = j + r QF, the inverse
            // radix-3 butterflies turn them into y = k + t M
            for (int it = lane; it < (gl << LQF); it += 64) {
                const int line = it >> LQF, j = it & (QF - 1);
                V v[3][RF];
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                    const int b = (((g0 + line) * 3 + t) << LMY) + j;
#pragma unroll
                    for (int r = 0; r < RF; ++r) {
                        V a = lines[padx<PADL>(b + r * QF)];
                        // twiddle W_{4 QF}^{r j} = twl[3 (2 r j)] of the 3 M table
                        if (r > 0) a = cmulc(a, twl[6 * r * j]);
                        v[t][r] = a;
                    }
                    dft_reg<V, RF, true>(v[t]);
                }
                V* dst = out + (long long)(g0 + line) * ny;
#pragma unroll
                for (int r = 0; r < RF; ++r) {
                    const int k = j + r * QF;
                    radix3_bfly<true>(v[0][r], v[1][r], v[2][r], twl[2 * k], twl[4 * k]);
                }
                // y half hy = 0 to the output slice; hy = 1 (un-twiddled) added
                // onto it (this thread stored those half-0 values itself; all
                // are loaded, from inside the line, before any is stored)
                if (hy) {
                    V h0[3][RF];
#pragma unroll
                    for (int t = 0; t < 3; ++t)
#pragma unroll
                        for (int r = 0; r < RF; ++r) h0[t][r] = dst[min(j + r * QF + t * M, ny - 1)];
#pragma unroll
                    for (int t = 0; t < 3; ++t)
#pragma unroll
                        for (int r = 0; r < RF; ++r) {
                            const int y = j + r * QF + t * M;
                            v[t][r] = cadd(cmulc(v[t][r], twl[y]), h0[t][r]);
                        }
                }
#pragma unroll
                for (int t = 0; t < 3; ++t)
#pragma unroll
                    for (int r = 0; r < RF; ++r) {
                        const int y = j + r * QF + t * M;
                        if (y < ny) dst[y] = v[t][r];
                    }
            }
            // the next forward pass of this group rewrites these lines
            wave_sync();
        }
    }
}

template <typename T, int MZ, int BUILD>
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && MZ <= 8 ? SSM_CONV_WAVES_F32 : 1, 8))) void k_conv(const Prob* __restrict__ P, int np,
                                              const int* __restrict__ wstart,
                                              cplx<T>* __restrict__ X,
                                              cplx<T>* __restrict__ Xp, const T* __restrict__ nhat,
                                              const cplx<T>* __restrict__ tw,
                                              const int* __restrict__ done)
{
    extern __shared__ double2 smem_[];
    const int pi = find_problem(wstart, np, blockIdx.x);
    if (done && done[pi]) return;
    const Prob& p = P[pi];
    if (conv_build(MZ, p.lmy, p.f3y) != BUILD) return;  // served by another build
    const int w = blockIdx.x - wstart[pi];
    const int nsl_img = p.mx + 1, nsl = p.K * nsl_img;
    int s0, G;
    if (p.xcd_remap) {
        int kx, img;
        if (SSM_CONV_XCD_REMAP) {
            const int xcd = w & 7, j = w >> 3;
            kx = (j / p.K) * 8 + xcd;
            img = j % p.K;
        } else {
            kx = w / p.K;
            img = w % p.K;
        }
        if (kx > p.mx || img >= p.K) return;
        s0 = img * nsl_img + kx;
        G = 1;
    } else {
        s0 = w * p.gconv;
        if (s0 >= nsl) return;
        G = min(p.gconv, nsl - s0);
    }
    cplx<T>* sm = reinterpret_cast<cplx<T>*>(smem_);
    if constexpr (BUILD >= 16) conv_body_ct3<T, MZ, BUILD - 16>(p, s0, G, X, Xp, nhat, tw, sm);
    else if constexpr (BUILD > 0) conv_body_ct<T, MZ, BUILD>(p, s0, G, X, Xp, nhat, tw, sm);
    else conv_body<T, MZ>(p, s0, G, X, Xp, nhat, tw, sm);
}

// The value of the next (previous) lane of the wavefront: DPP wavefront
// shifts by one lane (one VALU move, no LDS permute); the last (first) lane
// receives 0, which callers replace.
__device__ __forceinline__ int dpp_next(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, false); }
__device__ __forceinline__ int dpp_prev(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false); }
template <typename T>
__device__ __forceinline__ T lane_next(T v)
{
    if constexpr (!SSM_XINV_DPP) {
        return __shfl_down(v, 1);
    } else if constexpr (sizeof(T) == 4) {
        return __int_as_float(dpp_next(__float_as_int(v)));
    } else {
        const long long b = __double_as_longlong(v);
        const int lo = dpp_next((int)(b & 0xffffffffLL)), hi = dpp_next((int)(b >> 32));
        return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    }
}
template <typename T>
__device__ __forceinline__ T lane_prev(T v)
{
    if constexpr (!SSM_XINV_DPP) {
        return __shfl_up(v, 1);
    } else if constexpr (sizeof(T) == 4) {
        return __int_as_float(dpp_prev(__float_as_int(v)));
    } else {
        const long long b = __double_as_longlong(v);
        const int lo = dpp_prev((int)(b & 0xffffffffLL)), hi = dpp_prev((int)(b >> 32));
        return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    }
}

// The convolved x half-spectra of component c of a k_xinv tile into its
// LDS lines: item (kx, row pair rp) reads rows ya, ya + 1 of frequency kx
// and writes Z(kx) = A + iB and, for 0 < kx < m, Z(2m - kx) = conj(A) +
// i conj(B), each into the line of its half (even, odd frequencies).  A row
// past the lattice reads a row inside it instead (rows transform
// independently, and no field of a row past the lattice is used); even ny
// reads the pair as one 16-byte load.
// items per thread per round: 8 in FP32 at power-of-two lengths; 4 at
// lengths 3 2^a, whose radix-3 step holds more registers, and in FP64,
// whose 16-byte complex values hold twice the registers per item
#ifndef SSM_XINV_U
#define SSM_XINV_U 8
#endif
#ifndef SSM_XINV_U_F3
#define SSM_XINV_U_F3 4
#endif
#ifndef SSM_XINV_U_F64
#define SSM_XINV_U_F64 4
#endif
template <typename T, int F3>
constexpr int kXinvU = sizeof(T) == 4 ? (F3 ? SSM_XINV_U_F3 : SSM_XINV_U) : SSM_XINV_U_F64;
template <typename T, int F3>
__device__ __forceinline__ void xinv_load_lines(const char* __restrict__ Xi, cplx<T>* lines, int c, int z, int y0,
                                                int hp, int lhp, int m, int lm, int nz, int ny, int psh)
{
    using V = cplx<T>;
    constexpr int f3 = F3;
    const int total = (m + 1) * hp;
    // line index of position q (< m) of line l: l m + q, m = 2^lm or 3 2^lm
    auto lidx = [&](int l, int q) { return (F3 ? (l + (l << 1)) << lm : l << lm) + q; };
    auto rounds = [&](auto oddc) {
        constexpr bool ODD = decltype(oddc)::value;
        // the items of a thread share rp (kNT is a multiple of hp) and step
        // kx by dk = kNT / hp, so their offsets step by a uniform stride;
        // items past the end read kx = m
        const int dk = kNT >> lhp;
        const unsigned kstr = (unsigned)(dk * 3 * nz * ny) * (unsigned)sizeof(V);
        const unsigned cbm = (unsigned)(((m * 3 + c) * nz + z) * ny) * (unsigned)sizeof(V);
#pragma unroll 1
        for (int idx0 = threadIdx.x; idx0 < total; idx0 += kXinvU<T, F3> * kNT) {
            const int rp = idx0 & (hp - 1), kx0 = idx0 >> lhp;
            const int ya = y0 + 2 * rp;
            const unsigned cb0 = (unsigned)(((kx0 * 3 + c) * nz + z) * ny) * (unsigned)sizeof(V);
            const unsigned ya0 = (unsigned)min(ya, ny - (ODD ? 1 : 2)) * (unsigned)sizeof(V);
            const unsigned ya1 = (unsigned)min(ya + 1, ny - 1) * (unsigned)sizeof(V);
            V A[kXinvU<T, F3>], B[kXinvU<T, F3>];
#pragma unroll
            for (int u = 0; u < kXinvU<T, F3>; ++u) {
                const unsigned cb = min(cb0 + (unsigned)u * kstr, cbm);
                if constexpr (!ODD) {
                    load2(reinterpret_cast<const V*>(Xi + cb + ya0), A[u], B[u]);
                } else {
                    A[u] = *reinterpret_cast<const V*>(Xi + cb + ya0);
                    B[u] = *reinterpret_cast<const V*>(Xi + cb + ya1);
                }
            }
            if constexpr (ODD) {
                if (ya >= ny)
#pragma unroll
                    for (int u = 0; u < kXinvU<T, F3>; ++u) A[u] = mk<V>(0, 0);
                if (ya + 1 >= ny)
#pragma unroll
                    for (int u = 0; u < kXinvU<T, F3>; ++u) B[u] = mk<V>(0, 0);
            }
#pragma unroll
            for (int u = 0; u < kXinvU<T, F3>; ++u) {
                if (idx0 + u * kNT >= total) break;
                const int kx = kx0 + u * dk;
                const V a = A[u], b = B[u];
                // the two halves (even, odd frequencies) are separate lines
                const int i0 = lidx(2 * rp + (kx & 1), fpos(kx >> 1, lm, f3));
                lines[i0 + (i0 >> psh)] = mk<V>(a.x - b.y, a.y + b.x);
                if (kx > 0 && kx < m) {
                    const int km = 2 * m - kx;
                    const int i1 = lidx(2 * rp + (km & 1), fpos(km >> 1, lm, f3));
                    lines[i1 + (i1 >> psh)] = mk<V>(a.x + b.y, b.x - a.y);
                }
            }
        }
    };
    if (ny & 1) rounds(std::true_type{});
    else rounds(std::false_type{});
}

// ---------------------------------------------------------------------------
// k_xinv: x half-spectra of the convolved field -> unit-strength dipolar
// field of a tile (one component at a time), then the per-site epilogue.
// Two half-spectra A, B of real rows form Z = A + i B on k = 0..m and
// conj(A) + i conj(B) on k = m+1..2m-1; the inverse transform gives row a
// in the real part and row b in the imaginary part.
// LDS: twiddles (2m) + yt lines of m + the tile's dipolar field (3 yt nx).
// ---------------------------------------------------------------------------
template <typename T, int F3>
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? SSM_XINV_WAVES_F32 : 3, 8))) void k_xinv(const Prob* __restrict__ P, int np,
                                              const int* __restrict__ wstart,
                                              const cplx<T>* __restrict__ Xp,
                                              const T* __restrict__ s, T* __restrict__ ss,
                                              T* __restrict__ hout, double* __restrict__ epart,
                                              const cplx<T>* __restrict__ tw,
                                              const int* __restrict__ done, int mode, double tau,
                                              double fcp, double fcd)
{
    using V = cplx<T>;
    extern __shared__ double2 smem_[];
    __shared__ double red[kNT / 64][kNTerm];
    const int pi = find_problem(wstart, np, blockIdx.x);
    if (done && done[pi]) return;
    const Prob& p = P[pi];
    if (p.f3x != F3) return;  // served by the other length kind's launch
    const int t = xcd_item(blockIdx.x - wstart[pi], p.wgi);
    if (t >= p.K * p.tiles) return;
    // z fastest: the tiles that read a plane's rows as z neighbours run
    // back to back on one XCD, while the plane is still in its L2
    const int z = SSM_XINV_ZFAST ? t % p.nz : (t / p.nty) % p.nz;
    const int ty = SSM_XINV_ZFAST ? (t / p.nz) % p.nty : t % p.nty;
    const int img = t / (p.nz * p.nty);
    const int yt = p.yt, hp = yt >> 1, nx = p.nx, ny = p.ny, nz = p.nz, m = p.mx, lm = p.lmx;
    constexpr int f3 = F3;
    const int lhp = __ffs(hp) - 1;  // tiles are powers of two
    const int psh = x_padl(lm, f3, sizeof(T)) ? x_padl(lm, f3, sizeof(T)) : 31;  // pad layout of the lines
    const int y0 = ty * yt;
    const long long N = p.N;
    V* twl = reinterpret_cast<V*>(smem_);
    V* lines = twl + 2 * m;
    T* hd = reinterpret_cast<T*>(lines + padded_len(yt * m, x_padl(lm, f3, sizeof(T))));
    load_twiddles(twl, lm, f3, tw);
    // the convolved x half-spectra of the image
    // (as a uniform base and 32-bit byte offsets: an image's spectra span
    // at most 1025 * 3 * 16 * 1024 complex values, under 2^32 bytes)
    const char* const Xi = reinterpret_cast<const char*>(Xp + p.x_off + (long long)img * (m + 1) * 3 * nz * ny);
    __syncthreads();
#pragma unroll 1
    for (int c = 0; c < 3; ++c) {
        // kXinvU items per thread per round: their loads are issued
        // together (no load sits under a branch; an item past the end loads
        // the values at kx = m and stores nothing), then their LDS writes
        xinv_load_lines<T, F3>(Xi, lines, c, z, y0, hp, lhp, m, lm, nz, ny, psh);
        __syncthreads();
        fft_lines_x<V, true>(lines, yt, lm, f3, twl);
        __syncthreads();
        if constexpr (F3) {
            // the inverse radix-3 step (decimation in time) on the way out:
            // sub-line positions k of both half lines give x = k + t 2^lm
            const int M = 1 << lm;
            for (int idx = threadIdx.x; idx < (hp << lm); idx += kNT) {
                const int rp = idx >> lm, k = idx & (M - 1);
                if (k >= nx) continue;
                const int ie = (2 * rp) * m + k, io = ie + m;
                V e[3], o[3];
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                    const int a = ie + t * M, b = io + t * M;
                    e[t] = lines[a + (a >> psh)];
                    o[t] = lines[b + (b >> psh)];
                }
                const V w1 = twl[2 * k], w2 = twl[4 * k];
                radix3_bfly<true>(e[0], e[1], e[2], w1, w2);
                radix3_bfly<true>(o[0], o[1], o[2], w1, w2);
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                    const int x = k + t * M;
                    if (x < nx) {
                        const V ot = cmulc(o[t], twl[x]);
                        hd[(c * yt + 2 * rp) * nx + x] = e[t].x + ot.x;
                        hd[(c * yt + 2 * rp + 1) * nx + x] = e[t].y + ot.y;
                    }
                }
            }
        } else {
            for (int idx = threadIdx.x; idx < hp * m; idx += kNT) {
                const int rp = idx >> lm, x = idx & (m - 1);
                if (x >= nx) continue;
                const int ie = (2 * rp) * m + x, io = ie + m;
                const V e = lines[ie + (ie >> psh)];
                const V o = cmulc(lines[io + (io >> psh)], twl[x]);
                hd[(c * yt + 2 * rp) * nx + x] = e.x + o.x;
                hd[(c * yt + 2 * rp + 1) * nx + x] = e.y + o.y;
            }
        }
        __syncthreads();
    }

    // Per-site epilogue.  Each thread owns one column x and walks a run of
    // the tile's rows keeping rows y-1, y, y+1 in registers; x neighbours come
    // from the adjacent lanes (the lanes of a wave hold consecutive x), so
    // only the z neighbours and the wave-edge lanes read global memory.  The
    // loads a row needs are issued one row ahead, so their latency overlaps
    // the arithmetic of the row before.
    const double J = p.J, dm = p.d, ku = p.ku, D = p.D;
    // Global accesses take the image's first element (uniform) plus a 32-bit
    // byte offset: an image spans at most 3 * 2^24 sites, under 2^32 bytes.
    const long long ib = p.s_off + (long long)img * 3 * N;
    const char* const sb = reinterpret_cast<const char*>(s + ib);
    const unsigned cb = (unsigned)N * sizeof(T), plb = (unsigned)(nx * ny) * sizeof(T), xb = sizeof(T);
    const unsigned zb = (unsigned)z * plb;
    auto at = [&](unsigned o) -> T { return *reinterpret_cast<const T*>(sb + o); };
    int nxp = 1;
    while (nxp < nx && nxp < kNT) nxp <<= 1;
    // row groups of nxp lanes: the power of two >= nx, or nx itself where
    // that gives each thread fewer rows (lanes past the last group idle)
    if (nx < nxp && (yt + kNT / nx - 1) / (kNT / nx) < (yt + kNT / nxp - 1) / (kNT / nxp)) nxp = nx;
    const int rgs = kNT / nxp;                    // row groups
    const int rg = threadIdx.x / nxp, xl = threadIdx.x - rg * nxp;
    const int rper = (yt + rgs - 1) / rgs;
    const int ra = rg * rper, rb = min(yt, ra + rper);
    const int lane = threadIdx.x & 63;
    const bool redge = (xl == nxp - 1 || lane == 63), ledge = (xl == 0 || lane == 0);
    double acc[kNTerm] = {0, 0, 0, 0, 0};
    for (int xc = 0; xc < nx; xc += nxp) {
        const int x = xc + xl;
        const bool xin = x < nx;
        // a lane at the edge of its wavefront or row group loads its one
        // neighbour outside it that lies in the lattice: the right one at a
        // right edge, else the left one at a left edge (with row groups of
        // nx lanes a lane can end a row group and start a wavefront; it is
        // then at the lattice's right end and needs only the left one)
        const bool needR = redge && x + 1 < nx, needL = ledge && x > 0;
        const bool egok = needR || needL;
        const int xcl = min(x, nx - 1);
        // spin component c at (x, y0 + rr), zero outside the lattice in y
        // (loaded from the site clamped into the lattice, then selected: the
        // values of lanes outside it in x reach no site that is updated)
        auto rowv = [&](int rr, int c) -> T {
            const int y = y0 + rr;
            const T v = at(c * cb + zb + (unsigned)(min(max(y, 0), ny - 1) * nx + xcl) * xb);
            return (y >= 0 && y < ny) ? v : T(0);
        };
        // the z neighbours and (wave-edge lanes) x neighbours of row rr.  A
        // lane outside the lattice or past its run uses none of them, so the
        // z neighbours are loaded by every lane from the site clamped into
        // the lattice, with no per-lane predicate
        auto fetch = [&](int rr, T (&zu)[3], T (&zd)[3], T (&eg)[3]) {
            const int y = y0 + rr;
            const bool a = xin && rr < rb && y < ny;
            const unsigned o = zb + (unsigned)(min(y, ny - 1) * nx + xcl) * xb;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const unsigned oc = o + c * cb;
                zu[c] = (z + 1 < nz) ? at(oc + plb) : T(0);
                zd[c] = (z > 0) ? at(oc - plb) : T(0);
                eg[c] = (a && egok) ? at(needR ? oc + xb : oc - xb) : T(0);
            }
        };
        T cm[3], cc[3], cp[3], zu[3], zd[3], eg[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            cm[c] = rowv(ra - 1, c);
            cc[c] = rowv(ra, c);
            cp[c] = rowv(ra + 1, c);
        }
        fetch(ra, zu, zd, eg);
        for (int r = ra; r < ra + rper; ++r) {
            const int y = y0 + r;
            const bool act = xin && r < rb && y < ny;
            const unsigned o = zb + (unsigned)(y * nx + x) * xb;
            // next row's loads first
            T cn[3], zu2[3], zd2[3], eg2[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) cn[c] = rowv(r + 2, c);
            fetch(r + 1, zu2, zd2, eg2);
            double sv[3], xp[3], xm[3], nb[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                T right = lane_next(cc[c]);
                T left = lane_prev(cc[c]);
                if (redge) right = eg[c];
                if (ledge) left = needL ? eg[c] : T(0);
                if (x + 1 >= nx) right = T(0);
                sv[c] = (double)cc[c];
                xp[c] = (double)right;
                xm[c] = (double)left;
                nb[c] = xp[c] + xm[c] + (double)cp[c] + (double)cm[c] + ((double)zu[c] + (double)zd[c]);
            }
            if (act) {
                // unit-strength DMI field, eq. (4)
                const double dmx = -(xp[2] - xm[2]);
                const double dmy = -((double)cp[2] - (double)cm[2]);
                const double dmz = -(-xp[0] + xm[0] - (double)cp[1] + (double)cm[1]);
                const double hu[3] = {(double)hd[(0 * yt + r) * nx + x], (double)hd[(1 * yt + r) * nx + x],
                                      (double)hd[(2 * yt + r) * nx + x]};
                double h[3];
                h[0] = J * nb[0] + dm * dmx + D * hu[0];
                h[1] = J * nb[1] + dm * dmy + D * hu[1];
                h[2] = J * nb[2] + dm * dmz + 2.0 * ku * sv[2] + D * hu[2];
                const double sh = sv[0] * h[0] + sv[1] * h[1] + sv[2] * h[2];
                acc[0] += -0.5 * sh;
                if (mode & EPI_TERMS) {
                    acc[1] += -0.5 * (sv[0] * nb[0] + sv[1] * nb[1] + sv[2] * nb[2]);
                    acc[2] += -0.5 * (sv[0] * dmx + sv[1] * dmy + sv[2] * dmz);
                    acc[3] += -sv[2] * sv[2];
                    acc[4] += -0.5 * (sv[0] * hu[0] + sv[1] * hu[1] + sv[2] * hu[2]);
                }
                if (mode & EPI_FORCE) {
                    // eq. (9) in reduced time: -cp (s x h) + cd ((s.s) h - (s.h) s)
                    const double s2 = sv[0] * sv[0] + sv[1] * sv[1] + sv[2] * sv[2];
                    const double x[3] = {sv[1] * h[2] - sv[2] * h[1], sv[2] * h[0] - sv[0] * h[2],
                                         sv[0] * h[1] - sv[1] * h[0]};
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        *reinterpret_cast<T*>(reinterpret_cast<char*>(hout + ib) + o + c * cb) =
                            (T)(fcd * (s2 * h[c] - sh * sv[c]) - fcp * x[c]);
                } else if (mode & EPI_FIELD) {
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        *reinterpret_cast<T*>(reinterpret_cast<char*>(hout + ib) + o + c * cb) = (T)h[c];
                }
                if (mode & EPI_STEP) {
                    double wv[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) wv[c] = sv[c] + tau * (h[c] - sh * sv[c]);
                    const double inv = rsqrt(wv[0] * wv[0] + wv[1] * wv[1] + wv[2] * wv[2]);
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        *reinterpret_cast<T*>(reinterpret_cast<char*>(ss + ib) + o + c * cb) = (T)(wv[c] * inv);
                }
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                cm[c] = cc[c];
                cc[c] = cp[c];
                cp[c] = cn[c];
                zu[c] = zu2[c];
                zd[c] = zd2[c];
                eg[c] = eg2[c];
            }
        }
    }
    const int nterm = (mode & EPI_TERMS) ? kNTerm : 1;
    const int wave = threadIdx.x >> 6;
    for (int j = 0; j < nterm; ++j) {
        const double v = wave_sum(acc[j]);
        if (lane == 0) red[wave][j] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < nterm) {
        double v = 0;
        for (int wv = 0; wv < kNT / 64; ++wv) v += red[wv][threadIdx.x];
        epart[p.ep_off + ((long long)img * p.tiles + (z * p.nty + ty)) * kNTerm + threadIdx.x] = v;
    }
}

// ---------------------------------------------------------------------------
// k_arc: per flat chunk of the 3N components and group of consecutive
// images, partial sums of (phi*_k - phi*_{k-1})^2 for the group's k, one
// value per wavefront (the same values whatever the grouping).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kNT) void k_arc(const Prob* __restrict__ P, int np,
                                             const int* __restrict__ wstart,
                                             const T* __restrict__ ss, double* __restrict__ apart,
                                             const int* __restrict__ done)
{
    const int pi = find_problem(wstart, np, blockIdx.x);
    if (done && done[pi]) return;
    const Prob& p = P[pi];
    const int w = blockIdx.x - wstart[pi];
    const int chunk = w % p.arc_chunks, grp = w / p.arc_chunks;
    // images k0..k1-1 of this workgroup's group, against image k0 - 1
    const int k0 = 1 + grp * p.arc_g, k1 = min(p.K, k0 + p.arc_g);
    if (k0 >= p.K) return;
    const long long M = 3 * p.N;
    const T* src = ss + p.s_off;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // the chunk's kNT * kArcEPT elements in groups of 4 consecutive ones
    // (thread t: 4t + 4 kNT j + q), summed in the same order whether a group
    // is one 16-byte load (FP32, N divisible by 4, aligned) or four loads
    constexpr int NV = kArcEPT / 4;
    static_assert(kArcEPT % 4 == 0, "arc elements per thread come in groups of 4");
    const long long b4 = (long long)chunk * (kNT * kArcEPT) + 4 * threadIdx.x;
    const bool v4 = sizeof(T) == 4 && p.vec4;
    auto load4 = [&](const T* im, long long e, T (&v)[4]) {
        if constexpr (sizeof(T) == 4) {
            if (v4) {
                const float4 q = (e < M) ? *reinterpret_cast<const float4*>(im + e) : make_float4(0.f, 0.f, 0.f, 0.f);
                v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
                return;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = (e + q < M) ? im[e + q] : T(0);
    };
    T pv[NV][4], cv[NV][4];
#pragma unroll
    for (int j = 0; j < NV; ++j) load4(src + (long long)(k0 - 1) * M, b4 + (long long)j * 4 * kNT, pv[j]);
    for (int k = k0; k < k1; ++k) {
        const T* im = src + (long long)k * M;
#pragma unroll
        for (int j = 0; j < NV; ++j) load4(im, b4 + (long long)j * 4 * kNT, cv[j]);
        double a = 0;
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const double d0 = (double)cv[j][0] - (double)pv[j][0], d1 = (double)cv[j][1] - (double)pv[j][1];
            const double d2 = (double)cv[j][2] - (double)pv[j][2], d3 = (double)cv[j][3] - (double)pv[j][3];
            a += d0 * d0 + d1 * d1 + d2 * d2 + d3 * d3;
#pragma unroll
            for (int q = 0; q < 4; ++q) pv[j][q] = cv[j][q];
        }
        a = wave_sum(a);
        if (lane == 0)
            apart[p.ap_off + ((long long)k * p.arc_chunks + chunk) * 4 + wave] = a;
    }
}

// ---------------------------------------------------------------------------
// The end of step 2 for problem pi, by one workgroup.  al[0..K) (LDS) holds
// the segment lengths |phi*_k - phi*_{k-1}| (al[0] = 0); el is LDS for K
// energies.  Scans them in a fixed order into S_k, alpha*_k = S_k/S_{K-1}
// and, for every interior image, the interval
// j = max{j <= K-2 : alpha*_j <= target} and its weight; with the options,
// the climbing image and the spline factors.
// ---------------------------------------------------------------------------
__device__ void reduce_final(const Prob& p, int pi, double* al, double* el, double* bc, int* s_kci,
                             double* alpha, int* jidx, double* wgt, int* skip, int* iters, const Step2& s2)
{
    const int K = p.K, g0 = p.img0;
    // S_k = al[1] + ... + al[k]: an inclusive scan by the first wavefront,
    // 64 images at a time with the running total carried over (a fixed
    // order, so reruns are bitwise identical)
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        double carry = 0.0;
        for (int base = 0; base < K; base += 64) {
            const int kk = base + lane;
            const bool in = kk >= 1 && kk < K;
            double v = in ? al[kk] : 0.0;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const double u = __shfl_up(v, o);
                if (lane >= o) v += u;
            }
            v += carry;
            if (in) al[kk] = v;
            carry = __shfl(v, 63);
        }
        if (lane == 0) {
            *bc = carry;
            skip[pi] = (carry > 0.0) ? 0 : 1;
            atomicAdd(&iters[pi], 1);  // the problem's only writer in this launch
        }
    }
    __syncthreads();
    const double L = *bc;
    if (!(L > 0.0)) {
        for (int kk = threadIdx.x; kk < K; kk += kNT) {
            alpha[g0 + kk] = 0;
            jidx[g0 + kk] = kk;
            wgt[g0 + kk] = 0;
        }
        if (threadIdx.x == 0) {
            if (s2.kci) s2.kci[pi] = -1;
            if (s2.spl_ok) s2.spl_ok[pi] = 0;
        }
        return;
    }
    for (int kk = 1 + threadIdx.x; kk < K; kk += kNT) al[kk] = al[kk] / L;
    if (s2.opts & 2) {
        const volatile double* Ev = s2.E;
        for (int kk = threadIdx.x; kk < K; kk += kNT) el[kk] = Ev[g0 + kk];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // climbing image: the image of highest energy (smallest index on
        // ties) when it is interior
        int kci = -1;
        if (s2.opts & 2) {
            int km = 0;
            double em = el[0];
            for (int kk = 1; kk < K; ++kk) {
                const double e = el[kk];
                if (e > em) { em = e; km = kk; }
            }
            if (km > 0 && km < K - 1) kci = km;
        }
        *s_kci = kci;
        if (s2.kci) s2.kci[pi] = kci;
    }
    __syncthreads();
    const int kci = *s_kci;
    // target of image kk: k/(K-1), or equal spacing within 0..kci and
    // within kci..K-1 around a climbing image
    auto target = [&](int kk) {
        if (kci < 0) return (double)kk / (double)(K - 1);
        if (kk <= kci) return al[kci] * (double)kk / (double)kci;
        return al[kci] + (1.0 - al[kci]) * (double)(kk - kci) / (double)(K - 1 - kci);
    };
    // interval of target t >= 0: the largest j <= K-2 with al[j] <= t, by
    // bisection (al is non-decreasing from al[0] = 0; with non-finite
    // lengths j still lies in 0..K-2)
    auto interval = [&](double t) {
        int lo = 0, hi = K - 2;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (al[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    };
    for (int kk = threadIdx.x; kk < K; kk += kNT) {
        alpha[g0 + kk] = al[kk];
        if (kk == 0 || kk == K - 1 || kk == kci) {
            jidx[g0 + kk] = kk;
            wgt[g0 + kk] = 0;
            continue;
        }
        const double tk = target(kk);
        const int j = interval(tk);
        const double width = al[j + 1] - al[j];
        jidx[g0 + kk] = j;
        wgt[g0 + kk] = (width > 0.0) ? (tk - al[j]) / width : 0.0;
    }
    if (!(s2.opts & 1)) return;
    // the one-pass spline step's operator is formed here for K <= wmax
    // (copies of the factors and targets kept in LDS for it)
    const bool wop = K <= s2.wmax;
    __shared__ double fsa[kWRow], fden[kWRow], fcp[kWRow], tA[kWRow], tB[kWRow], tH[kWRow];
    __shared__ double Zs[kWRow][kWRow + 1];
    __shared__ int tj[kWRow], s_ok;
    // natural cubic spline in alpha: interval widths and the Thomas factors
    // of the tridiagonal system for the interior second derivatives
    if (threadIdx.x == 0) {
        int ok = K > 2;
        for (int j = 0; j + 1 < K; ++j) {
            const double hw = al[j + 1] - al[j];
            s2.hh[g0 + j] = hw;
            if (!(hw > 0.0)) ok = 0;
        }
        if (ok) {
            double cpp = 0.0;
            for (int i = 1; i <= K - 2; ++i) {
                const double hl = al[i] - al[i - 1], hr = al[i + 1] - al[i];
                const double a = hl / 6.0, b = (hl + hr) / 3.0, c = hr / 6.0;
                const double den = b - (i > 1 ? a * cpp : 0.0);
                cpp = c / den;
                s2.sa[g0 + i] = a;
                s2.den[g0 + i] = den;
                s2.cp[g0 + i] = cpp;
                if (wop) { fsa[i] = a; fden[i] = den; fcp[i] = cpp; }
            }
        }
        s2.spl_ok[pi] = ok;
        s_ok = ok;
    }
    for (int kk = threadIdx.x; kk < K; kk += kNT) {
        if (kk == 0 || kk == K - 1 || kk == kci) continue;
        const double tk = target(kk);
        const int j = interval(tk);
        const double h = al[j + 1] - al[j];
        const double A = (al[j + 1] - tk) / h;
        s2.A[g0 + kk] = A;
        s2.B[g0 + kk] = 1.0 - A;
        s2.H[g0 + kk] = h;
        if (wop) { tA[kk] = A; tB[kk] = 1.0 - A; tH[kk] = h; tj[kk] = j; }
    }
    if (!wop) return;
    __syncthreads();
    if (!s_ok) return;
    // the interpolated value at target k is linear in the K images of a
    // site, s(t_k) = sum_i W_ki f_i: column i of the second-derivative map
    // by the Thomas recurrences on the unit image e_i (M_0 = M_{K-1} = 0),
    // then the spline formula; rows of the endpoints and of the climbing
    // image are zero (they are copied)
    if ((int)threadIdx.x < K) {
        const int i = threadIdx.x;
        double dpp = 0.0;
        Zs[0][i] = 0.0;
        Zs[K - 1][i] = 0.0;
        for (int k = 1; k <= K - 2; ++k) {
            const double r = ((i == k + 1 ? 1.0 : 0.0) - (i == k ? 1.0 : 0.0)) / (al[k + 1] - al[k]) -
                             ((i == k ? 1.0 : 0.0) - (i == k - 1 ? 1.0 : 0.0)) / (al[k] - al[k - 1]);
            const double dp = (r - (k > 1 ? fsa[k] * dpp : 0.0)) / fden[k];
            Zs[k][i] = dp;
            dpp = dp;
        }
        double mn = Zs[K - 2][i];
        for (int k = K - 3; k >= 1; --k) {
            const double mk = Zs[k][i] - fcp[k] * mn;
            Zs[k][i] = mk;
            mn = mk;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < K * K; e += kNT) {
        const int k = e / K, i = e - k * K;
        double w = 0.0;
        if (k > 0 && k < K - 1 && k != kci) {
            const int j = tj[k];
            const double A = tA[k], B = tB[k], h = tH[k];
            w = (i == j ? A : 0.0) + (i == j + 1 ? B : 0.0) +
                ((A * A * A - A) * Zs[j][i] + (B * B * B - B) * Zs[j + 1][i]) * h * h / 6.0;
        }
        s2.Wm[(long long)(g0 + k) * kWRow + i] = w;
    }
}

// ---------------------------------------------------------------------------
// k_reduce: one workgroup per image of the problems without red1.
// Fixed-order sums of the image's energy partials (E and the four
// unit-parameter terms) and, with_arc, of its arc partials (segment length
// |phi*_k - phi*_{k-1}|).  With with_arc the last workgroup of a problem to
// finish (atomic counter) ends step 2 (reduce_final).  Every sum has a
// fixed order, so results do not depend on which workgroup finishes last.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kNT) void k_reduce(const Prob* __restrict__ P, int np,
                                                const int* __restrict__ istart,
                                                const double* __restrict__ epart,
                                                const double* __restrict__ apart,
                                                double* E, double* Tm, double* E_out,
                                                double* T_out, double* seg, double* alpha,
                                                int* jidx, double* wgt, int* skip, int* done,
                                                int* iters, int* count, int* flags, int with_arc,
                                                Step2 s2)
{
    __shared__ double red[kNT / 64][kNTerm + 1];
    __shared__ double al[kMaxImages], el[kMaxImages];
    __shared__ double bc;
    __shared__ int last, s_kci;
    const int gimg = blockIdx.x;
    const int pi = find_problem(istart, np, gimg);
    if (with_arc && done && done[pi]) return;
    const Prob& p = P[pi];
    if (p.red1) return;  // reduced by k_reduce1
    const int k = gimg - p.img0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double v[kNTerm + 1] = {0, 0, 0, 0, 0, 0};
    const double* ep = epart + p.ep_off + (long long)k * p.tiles * kNTerm;
    // partials in rounds: a round's loads (past the end: the last partial)
    // are issued together, then added in the same order as one at a time
    constexpr int RE = 4, RA = 8;
    const int nt = p.tiles;
    for (int t0 = threadIdx.x; t0 < nt; t0 += RE * kNT) {
        double q[RE][kNTerm];
#pragma unroll
        for (int u = 0; u < RE; ++u) {
            const long long t = min(t0 + u * kNT, nt - 1);
#pragma unroll
            for (int j = 0; j < kNTerm; ++j) q[u][j] = ep[t * kNTerm + j];
        }
#pragma unroll
        for (int u = 0; u < RE; ++u)
            if (t0 + u * kNT < nt)
#pragma unroll
                for (int j = 0; j < kNTerm; ++j) v[j] += q[u][j];
    }
    if (with_arc && k > 0) {
        const double* ap = apart + p.ap_off + (long long)k * p.arc_chunks * 4;
        const int na = p.arc_chunks * 4;
        for (int t0 = threadIdx.x; t0 < na; t0 += RA * kNT) {
            double q[RA];
#pragma unroll
            for (int u = 0; u < RA; ++u) q[u] = ap[min(t0 + u * kNT, na - 1)];
#pragma unroll
            for (int u = 0; u < RA; ++u)
                if (t0 + u * kNT < na) v[kNTerm] += q[u];
        }
    }
    for (int j = 0; j <= kNTerm; ++j) {
        const double s = wave_sum(v[j]);
        if (lane == 0) red[wave][j] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double r[kNTerm + 1];
        for (int j = 0; j <= kNTerm; ++j) {
            r[j] = 0;
            for (int wv = 0; wv < kNT / 64; ++wv) r[j] += red[wv][j];
        }
        if (E) E[gimg] = r[0];
        if (E_out) E_out[gimg] = r[0];
        for (int j = 0; j < 4; ++j) {
            if (Tm) Tm[(long long)gimg * 4 + j] = r[j + 1];
            if (T_out) T_out[(long long)gimg * 4 + j] = r[j + 1];
        }
        if (!isfinite(r[0])) atomicOr(flags, 1);
        if (with_arc) {
            seg[gimg] = sqrt(r[kNTerm]);
            __threadfence();
            last = (atomicAdd(&count[pi], 1) == p.K - 1);
        }
    }
    if (!with_arc) return;
    __syncthreads();
    if (!last) return;
    // last workgroup of the problem: every image's segment length is
    // visible (written before the counter increment); fetch them in
    // parallel, then end step 2
    __threadfence();
    const int K = p.K, g0 = p.img0;
    const volatile double* sg = seg;
    for (int kk = threadIdx.x; kk < K; kk += kNT) al[kk] = (kk == 0) ? 0.0 : sg[g0 + kk];
    if (threadIdx.x == 0) count[pi] = 0;
    __syncthreads();
    reduce_final(p, pi, al, el, &bc, &s_kci, alpha, jidx, wgt, skip, iters, s2);
}

// ---------------------------------------------------------------------------
// k_reduce1: the whole reduction of one problem with red1 (few images and
// few partials per image) in one workgroup, so that no result passes
// between workgroups: the device-scope fences of that hand-off cost more
// than these sums.  kRedLanes lanes per image sum its partials in rounds,
// then combine them in a fixed butterfly order (4 lanes: the 64 images of
// the largest such problem in one pass, so the partials' loads wait on
// memory once); with_arc, reduce_final ends step 2 from the segment
// lengths kept in LDS.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kNT) void k_reduce1(const Prob* __restrict__ P, int np,
                                                 const double* __restrict__ epart,
                                                 const double* __restrict__ apart,
                                                 double* E, double* Tm, double* E_out,
                                                 double* T_out, double* seg, double* alpha,
                                                 int* jidx, double* wgt, int* skip, int* done,
                                                 int* iters, int* flags, int with_arc, Step2 s2)
{
    __shared__ double al[kMaxImages], el[kMaxImages];
    __shared__ double bc;
    __shared__ int s_kci;
    const int pi = blockIdx.x;
    if (pi >= np) return;
    if (with_arc && done && done[pi]) return;
    const Prob& p = P[pi];
    if (!p.red1) return;  // reduced by k_reduce
    const int K = p.K, g0 = p.img0, nt = p.tiles, na = p.arc_chunks * 4;
    constexpr int IPP = kNT / kRedLanes;  // images per pass
    constexpr int RE = 4, RA = 8;
    const int sub = threadIdx.x & (kRedLanes - 1);
    for (int k0 = 0; k0 < K; k0 += IPP) {
        const int k = k0 + (int)threadIdx.x / kRedLanes;
        const int kc = min(k, K - 1);  // lanes past the last image repeat it and store nothing
        double v[kNTerm + 1] = {0, 0, 0, 0, 0, 0};
        const double* ep = epart + p.ep_off + (long long)kc * nt * kNTerm;
        for (int t0 = sub; t0 < nt; t0 += RE * kRedLanes) {
            double q[RE][kNTerm];
#pragma unroll
            for (int u = 0; u < RE; ++u) {
                const long long t = min(t0 + u * kRedLanes, nt - 1);
#pragma unroll
                for (int j = 0; j < kNTerm; ++j) q[u][j] = ep[t * kNTerm + j];
            }
#pragma unroll
            for (int u = 0; u < RE; ++u)
                if (t0 + u * kRedLanes < nt)
#pragma unroll
                    for (int j = 0; j < kNTerm; ++j) v[j] += q[u][j];
        }
        if (with_arc && kc > 0) {
            const double* ap = apart + p.ap_off + (long long)kc * na;
            for (int t0 = sub; t0 < na; t0 += RA * kRedLanes) {
                double q[RA];
#pragma unroll
                for (int u = 0; u < RA; ++u) q[u] = ap[min(t0 + u * kRedLanes, na - 1)];
#pragma unroll
                for (int u = 0; u < RA; ++u)
                    if (t0 + u * kRedLanes < na) v[kNTerm] += q[u];
            }
        }
#pragma unroll
        for (int off = kRedLanes / 2; off > 0; off >>= 1)
#pragma unroll
            for (int j = 0; j <= kNTerm; ++j) v[j] += __shfl_xor(v[j], off, kRedLanes);
        if (sub == 0 && k < K) {
            const int g = g0 + k;
            if (E) E[g] = v[0];
            if (E_out) E_out[g] = v[0];
            for (int j = 0; j < 4; ++j) {
                if (Tm) Tm[(long long)g * 4 + j] = v[j + 1];
                if (T_out) T_out[(long long)g * 4 + j] = v[j + 1];
            }
            if (!isfinite(v[0])) atomicOr(flags, 1);
            if (with_arc) {
                const double sl = sqrt(v[kNTerm]);
                seg[g] = sl;
                al[k] = (k == 0) ? 0.0 : sl;
            }
        }
    }
    if (!with_arc) return;
    __syncthreads();
    reduce_final(p, pi, al, el, &bc, &s_kci, alpha, jidx, wgt, skip, iters, s2);
}

// One site of the linear interpolation: (1 - w) a + w b renormalised in
// FP64 by the device library's reciprocal square root (within an ulp or two
// of sqrt and division); a norm below 1e-12 takes the nearer source's spin.
// Flags: 4 a non-finite norm, 2 a degenerate one.  Every path of k_interp
// calls it, so a problem's result does not depend on which path its place
// in a batch selects.
template <typename T>
__device__ __forceinline__ void interp_site(const T (&a)[3], const T (&b)[3], double wt, T (&o)[3], int* flags)
{
    double v[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = (1.0 - wt) * (double)a[c] + wt * (double)b[c];
    const double n2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    if (!isfinite(n2)) atomicOr(flags, 4);
    if (n2 < 1e-24) {
        atomicOr(flags, 2);
#pragma unroll
        for (int c = 0; c < 3; ++c) o[c] = (wt < 0.5) ? a[c] : b[c];
    } else {
        const double inv = rsqrt(n2);
#pragma unroll
        for (int c = 0; c < 3; ++c) o[c] = (T)(v[c] * inv);
    }
}

// ---------------------------------------------------------------------------
// k_interp: s_k = normalise((1-w) s*_j + w s*_{j+1}); endpoints (and every
// image when the reparametrisation is skipped) are copied.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kNT) void k_interp(const Prob* __restrict__ P, int np,
                                                const int* __restrict__ wstart,
                                                const T* __restrict__ ss, T* __restrict__ s,
                                                const int* __restrict__ jidx,
                                                const double* __restrict__ wgt,
                                                const int* __restrict__ skip,
                                                const int* __restrict__ done, int* flags,
                                                const int* __restrict__ kci,
                                                const int* __restrict__ skip_if)
{
    const int pi = find_problem(wstart, np, blockIdx.x);
    if (done && done[pi]) return;
    if (skip_if && skip_if[pi]) return;
    const Prob& p = P[pi];
    const int w = blockIdx.x - wstart[pi];
    const int k = w / p.ichunks4, chunk = w - k * p.ichunks4;
    const long long N = p.N, M = 3 * N;
    const T* src = ss + p.s_off;
    T* dst = s + p.s_off + (long long)k * M;
    const bool copy = skip[pi] || k == 0 || k == p.K - 1 || (kci && k == kci[pi]);
    if constexpr (sizeof(T) == 4) {
        if (p.vec4) {
            // four consecutive sites per thread, 16-byte accesses
            const long long i = ((long long)chunk * kNT + threadIdx.x) * 4;
            if (i >= N) return;
            if (copy) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    *reinterpret_cast<float4*>(dst + c * N + i) =
                        *reinterpret_cast<const float4*>(src + (long long)k * M + c * N + i);
                return;
            }
            const int j = jidx[p.img0 + k];
            const double wt = wgt[p.img0 + k];
            const T* a = src + (long long)j * M;
            const T* b = a + M;
            float av[3][4], bv[3][4];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float4 x = *reinterpret_cast<const float4*>(a + c * N + i);
                const float4 y = *reinterpret_cast<const float4*>(b + c * N + i);
                av[c][0] = x.x; av[c][1] = x.y; av[c][2] = x.z; av[c][3] = x.w;
                bv[c][0] = y.x; bv[c][1] = y.y; bv[c][2] = y.z; bv[c][3] = y.w;
            }
            float o[3][4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float ta[3] = {av[0][q], av[1][q], av[2][q]}, tb[3] = {bv[0][q], bv[1][q], bv[2][q]}, to[3];
                interp_site<float>(ta, tb, wt, to, flags);
#pragma unroll
                for (int c = 0; c < 3; ++c) o[c][q] = to[c];
            }
#pragma unroll
            for (int c = 0; c < 3; ++c)
                *reinterpret_cast<float4*>(dst + c * N + i) = make_float4(o[c][0], o[c][1], o[c][2], o[c][3]);
            return;
        }
    } else {
        if (p.vec2) {
            // two consecutive sites per thread, 16-byte accesses
            const long long i = ((long long)chunk * kNT + threadIdx.x) * 2;
            if (i >= N) return;
            if (copy) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    *reinterpret_cast<double2*>(dst + c * N + i) =
                        *reinterpret_cast<const double2*>(src + (long long)k * M + c * N + i);
                return;
            }
            const int j = jidx[p.img0 + k];
            const double wt = wgt[p.img0 + k];
            const T* a = src + (long long)j * M;
            const T* b = a + M;
            double av[3][2], bv[3][2];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double2 x = *reinterpret_cast<const double2*>(a + c * N + i);
                const double2 y = *reinterpret_cast<const double2*>(b + c * N + i);
                av[c][0] = x.x; av[c][1] = x.y;
                bv[c][0] = y.x; bv[c][1] = y.y;
            }
            double o[3][2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                double ta[3] = {av[0][q], av[1][q], av[2][q]}, tb[3] = {bv[0][q], bv[1][q], bv[2][q]}, to[3];
                interp_site<double>(ta, tb, wt, to, flags);
#pragma unroll
                for (int c = 0; c < 3; ++c) o[c][q] = to[c];
            }
#pragma unroll
            for (int c = 0; c < 3; ++c)
                *reinterpret_cast<double2*>(dst + c * N + i) = make_double2(o[c][0], o[c][1]);
            return;
        }
    }
    const long long i = (long long)chunk * kNT + threadIdx.x;
    if (i >= N) return;
    if (copy) {
#pragma unroll
        for (int c = 0; c < 3; ++c) dst[c * N + i] = src[(long long)k * M + c * N + i];
        return;
    }
    const int j = jidx[p.img0 + k];
    const double wt = wgt[p.img0 + k];
    const T* a = src + (long long)j * M;
    const T* b = a + M;
    T ta[3], tb[3], to[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        ta[c] = a[c * N + i];
        tb[c] = b[c * N + i];
    }
    interp_site<T>(ta, tb, wt, to, flags);
#pragma unroll
    for (int c = 0; c < 3; ++c) dst[c * N + i] = to[c];
}

// ---------------------------------------------------------------------------
// Tangents and perpendicular force.
// k_tan1: t~ = (phi_{k+1} - phi_{k-1}) projected per spin onto the tangent
//         plane, stored to tt; partial sums of |t~|^2 and h_perp . t~.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kNT) void k_tan1(const Prob* __restrict__ P, int np,
                                              const int* __restrict__ wstart,
                                              const T* __restrict__ s, const T* __restrict__ h,
                                              T* __restrict__ tt, double* __restrict__ fpart)
{
    __shared__ double red[kNT / 64][2];
    const int pi = find_problem(wstart, np, blockIdx.x);
    const Prob& p = P[pi];
    const int w = blockIdx.x - wstart[pi];
    const int k = w / p.ichunks, chunk = w - k * p.ichunks;
    const long long N = p.N, M = 3 * N;
    const long long i = (long long)chunk * kNT + threadIdx.x;
    double a0 = 0, a1 = 0;
    if (i < N) {
        const int kp = (k + 1 < p.K) ? k + 1 : k, km = (k > 0) ? k - 1 : k;
        const T* sk = s + p.s_off + (long long)k * M;
        const T* sp = s + p.s_off + (long long)kp * M;
        const T* sm = s + p.s_off + (long long)km * M;
        const T* hk = h + p.s_off + (long long)k * M;
        double v[3], f[3], d[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
            v[c] = (double)sk[c * N + i];
            f[c] = (double)hk[c * N + i];
            d[c] = (double)sp[c * N + i] - (double)sm[c * N + i];
        }
        const double sh = v[0] * f[0] + v[1] * f[1] + v[2] * f[2];
        const double sd = v[0] * d[0] + v[1] * d[1] + v[2] * d[2];
        T* to = tt + p.s_off + (long long)k * M;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
            const double tc = d[c] - sd * v[c];
            const double hc = f[c] - sh * v[c];
            to[c * N + i] = (T)tc;
            a0 += tc * tc;
            a1 += hc * tc;
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    if (lane == 0) { red[wave][0] = a0; red[wave][1] = a1; }
    __syncthreads();
    if (threadIdx.x < 2) {
        double v = 0;
        for (int wv = 0; wv < kNT / 64; ++wv) v += red[wv][threadIdx.x];
        fpart[p.fp_off + ((long long)k * p.ichunks + chunk) * 2 + threadIdx.x] = v;
    }
}

// per problem, wave per image: tcoef[g] = {1/|t~|, projection coefficient}
__global__ __launch_bounds__(kNT) void k_tanred(const Prob* __restrict__ P, int np,
                                                const double* __restrict__ fpart,
                                                double* __restrict__ tcoef)
{
    const int pi = blockIdx.x;
    if (pi >= np) return;
    const Prob& p = P[pi];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = wave; k < p.K; k += kNT / 64) {
        const double* fp = fpart + p.fp_off + (long long)k * p.ichunks * 2;
        double n2 = 0, ht = 0;
        for (int t = lane; t < p.ichunks; t += 64) {
            n2 += fp[2 * t];
            ht += fp[2 * t + 1];
        }
        n2 = wave_sum(n2);
        ht = wave_sum(ht);
        if (lane == 0) {
            const double tn = sqrt(n2);
            const double inv = (tn > 0.0) ? 1.0 / tn : 0.0;
            const bool interior = (k > 0 && k < p.K - 1);
            const int g = p.img0 + k;
            tcoef[2 * g] = inv;
            tcoef[2 * g + 1] = interior ? ht * inv * inv : 0.0;
        }
    }
}

// k_tan2: F_perp = h_perp - c t~; per-workgroup max |F_perp|; tangents out.
template <typename T>
__global__ __launch_bounds__(kNT) void k_tan2(const Prob* __restrict__ P, int np,
                                              const int* __restrict__ wstart,
                                              const T* __restrict__ s, const T* __restrict__ h,
                                              const T* __restrict__ tt, T* __restrict__ t_out,
                                              const double* __restrict__ tcoef,
                                              double* __restrict__ fmx)
{
    __shared__ double red[kNT / 64];
    const int pi = find_problem(wstart, np, blockIdx.x);
    const Prob& p = P[pi];
    const int w = blockIdx.x - wstart[pi];
    const int k = w / p.ichunks, chunk = w - k * p.ichunks;
    const long long N = p.N, M = 3 * N;
    const long long i = (long long)chunk * kNT + threadIdx.x;
    const int g = p.img0 + k;
    double fm = 0;
    if (i < N) {
        const double inv = tcoef[2 * g], cf = tcoef[2 * g + 1];
        const T* sk = s + p.s_off + (long long)k * M;
        const T* hk = h + p.s_off + (long long)k * M;
        const T* tk = tt + p.s_off + (long long)k * M;
        double v[3], f[3], tc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
            v[c] = (double)sk[c * N + i];
            f[c] = (double)hk[c * N + i];
            tc[c] = (double)tk[c * N + i];
        }
        const double sh = v[0] * f[0] + v[1] * f[1] + v[2] * f[2];
        double n2 = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
            const double fc = f[c] - sh * v[c] - cf * tc[c];
            n2 += fc * fc;
        }
        // a non-finite force counts as infinitely large, so that a diverged
        // problem can never pass the convergence test (fmax would drop NaN)
        fm = isfinite(n2) ? sqrt(n2) : (double)INFINITY;
        if (t_out) {
            T* to = t_out + p.s_off + (long long)k * M;
#pragma unroll
            for (int c = 0; c < 3; ++c) to[c * N + i] = (T)(tc[c] * inv);
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    fm = wave_max(fm);
    if (lane == 0) red[wave] = fm;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0;
        for (int wv = 0; wv < kNT / 64; ++wv) v = fmax(v, red[wv]);
        fmx[p.fm_off + (long long)k * p.ichunks + chunk] = v;
    }
}

__global__ __launch_bounds__(kNT) void k_fmax(const Prob* __restrict__ P, int np,
                                              const double* __restrict__ fm,
                                              double* __restrict__ fnorm, int* done, double tol,
                                              double* out)
{
    __shared__ double red[kNT / 64];
    const int pi = blockIdx.x;
    if (pi >= np) return;
    const Prob& p = P[pi];
    const long long n = (long long)p.K * p.ichunks;
    const double* f = fm + p.fm_off;
    double v = 0;
    for (long long t = threadIdx.x; t < n; t += kNT) v = fmax(v, f[t]);
    v = wave_max(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0;
        for (int wv = 0; wv < kNT / 64; ++wv) r = fmax(r, red[wv]);
        fnorm[pi] = r;
        if (out) out[pi] = r;
        if (tol > 0.0 && r < tol && done) done[pi] = 1;
    }
}

// B = max_k E_k - E_0, smallest argmax, envelope derivatives.
__global__ void k_barrier(const Prob* __restrict__ P, int np, const double* __restrict__ E,
                          const double* __restrict__ Tm, double* __restrict__ out)
{
    const int pi = blockIdx.x * blockDim.x + threadIdx.x;
    if (pi >= np) return;
    const Prob& p = P[pi];
    const int g0 = p.img0;
    int km = 0;
    for (int k = 1; k < p.K; ++k)
        if (E[g0 + k] > E[g0 + km]) km = k;
    double* o = out + (long long)pi * 6;
    o[0] = E[g0 + km] - E[g0];
    o[1] = (double)km;
    for (int j = 0; j < 4; ++j) o[2 + j] = Tm[(long long)(g0 + km) * 4 + j] - Tm[(long long)g0 * 4 + j];
}

__global__ void k_fill_int(int* p, int n, int v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_copy_int(const int* a, int* b, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// ---------------------------------------------------------------------------
// Dipole-kernel spectrum, FP64, once per lattice shape.
// N_ab(r) = 3 r_a r_b / |r|^5 - delta_ab / |r|^3 (4 pi times eq. (7), r in
// lattice units, r != 0, |r_x| < nx, |r_y| < ny, |r_z| < nz).  Each
// component is even or odd along each axis, so its DFT on the padded grid is
// real: products of cosine sums (even axes) and sine sums (odd axes), with
// sign -1 for the off-diagonal components (two odd axes).  Three separable
// direct passes; the result carries 1/(Px Py Pz).
// Component c: 0 xx, 1 xy, 2 xz, 3 yy, 4 yz, 5 zz.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void comp_ab(int c, int& a, int& b)
{
    const int A[6] = {0, 0, 0, 1, 1, 2}, B[6] = {0, 1, 2, 1, 2, 2};
    a = A[c];
    b = B[c];
}

__device__ __forceinline__ double trig(const double* __restrict__ tw64, long long kd, int Pn,
                                       bool odd)
{
    long long e = kd % Pn;
    if (e < 0) e += Pn;
    const long long idx = e * (kTwM / Pn);
    return odd ? -tw64[2 * idx + 1] : tw64[2 * idx];
}

// F1[c][kx][dyi][dzi] = sum_dx N_c(dx,dy,dz) f(kx dx)
__global__ void k_spec1(Prob p, double* __restrict__ F1, const double* __restrict__ tw64)
{
    const int nyo = 2 * p.ny - 1, nzo = 2 * p.nz - 1;
    const long long total = 6LL * (p.mx + 1) * nyo * nzo;
    const long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= total) return;
    const int dzi = o % nzo;
    long long r = o / nzo;
    const int dyi = r % nyo;
    r /= nyo;
    const int kx = r % (p.mx + 1);
    const int c = r / (p.mx + 1);
    int a, b;
    comp_ab(c, a, b);
    const int dy = dyi - (p.ny - 1), dz = dzi - (p.nz - 1);
    const bool oddx = ((a == 0) + (b == 0)) == 1;
    const int Px = 2 * p.mx;
    double acc = 0;
    for (int dx = -(p.nx - 1); dx <= p.nx - 1; ++dx) {
        if (dx == 0 && dy == 0 && dz == 0) continue;
        const double r2 = (double)dx * dx + (double)dy * dy + (double)dz * dz;
        const double rr = sqrt(r2);
        const double r3 = r2 * rr, r5 = r3 * r2;
        const double v[3] = {(double)dx, (double)dy, (double)dz};
        const double n = 3.0 * v[a] * v[b] / r5 - ((a == b) ? 1.0 / r3 : 0.0);
        acc += n * trig(tw64, (long long)kx * dx, Px, oddx);
    }
    F1[o] = acc;
}

// F2[c][kx][ky][dzi] = sum_dy F1[c][kx][dyi][dzi] f(ky dy)
__global__ void k_spec2(Prob p, const double* __restrict__ F1, double* __restrict__ F2,
                        const double* __restrict__ tw64)
{
    const int nyo = 2 * p.ny - 1, nzo = 2 * p.nz - 1, Py = 2 * p.my;
    const long long total = 6LL * (p.mx + 1) * Py * nzo;
    const long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= total) return;
    const int dzi = o % nzo;
    long long r = o / nzo;
    const int ky = r % Py;
    r /= Py;
    const int kx = r % (p.mx + 1);
    const int c = r / (p.mx + 1);
    int a, b;
    comp_ab(c, a, b);
    const bool oddy = ((a == 1) + (b == 1)) == 1;
    const double* f = F1 + (((long long)c * (p.mx + 1) + kx) * nyo) * nzo + dzi;
    double acc = 0;
    for (int dyi = 0; dyi < nyo; ++dyi)
        acc += f[(long long)dyi * nzo] * trig(tw64, (long long)ky * (dyi - (p.ny - 1)), Py, oddy);
    F2[o] = acc;
}

// final pass along z, scaling and storage in the convolution kernel's layout
template <typename T>
__global__ void k_spec3(Prob p, const double* __restrict__ F2, T* __restrict__ nh,
                        const double* __restrict__ tw64)
{
    const int nzo = 2 * p.nz - 1, Py = 2 * p.my, Pz = p.pz;
    const long long total = 6LL * (p.mx + 1) * Py * Pz;
    const long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= total) return;
    const int kz = o % Pz;
    long long r = o / Pz;
    const int ky = r % Py;
    r /= Py;
    const int kx = r % (p.mx + 1);
    const int c = r / (p.mx + 1);
    int a, b;
    comp_ab(c, a, b);
    const bool oddz = ((a == 2) + (b == 2)) == 1;
    const double* f = F2 + (((long long)c * (p.mx + 1) + kx) * Py + ky) * nzo;
    double acc = 0;
    for (int dzi = 0; dzi < nzo; ++dzi)
        acc += f[dzi] * trig(tw64, (long long)kz * (dzi - (p.nz - 1)), Pz, oddz);
    const double sign = (a == b) ? 1.0 : -1.0;
    const double scale = sign / ((double)(2 * p.mx) * (double)Py * (double)Pz);
    const int hy = ky & 1, qy = ky >> 1;
    const int hz = (p.nhz == 2) ? (kz & 1) : 0, rz = (p.nhz == 2) ? (kz >> 1) : 0;
    const long long idx = ((((long long)kx * p.nhz + hz) * 2 + hy) * p.mz + rz) * 6 * p.my;
    nh[idx + (long long)c * p.my + qy] = (T)(acc * scale);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_xfwd(const Prob* P, int np, const WorkMap* wm, const T* s, void* X,
                       const void* tw, const int* done, size_t lds, hipStream_t st)
{
    if (wm[0].total)
        hipLaunchKernelGGL((k_xfwd<T, 0>), dim3(wm[0].total), dim3(kNT), lds, st, P, np, wm[0].start, s,
                           (cplx<T>*)X, (const cplx<T>*)tw, done);
    if (wm[1].total)
        hipLaunchKernelGGL((k_xfwd<T, 1>), dim3(wm[1].total), dim3(kNT), lds, st, P, np, wm[1].start, s,
                           (cplx<T>*)X, (const cplx<T>*)tw, done);
    return hipGetLastError();
}

template <typename T, int MZ, int BUILD>
static void launch_conv_b(const Prob* P, int np, const WorkMap* wm, cplx<T>* x, cplx<T>* xp,
                          const T* nhat, const cplx<T>* t, const int* done, size_t lds, hipStream_t st)
{
    const WorkMap& w = wm[conv_slot(BUILD)];
    if (w.total)
        hipLaunchKernelGGL((k_conv<T, MZ, BUILD>), dim3(w.total), dim3(kNT), lds, st, P, np, w.start, x, xp,
                           nhat, t, done);
}

template <typename T, int MZ>
static hipError_t launch_conv_mz(const Prob* P, int np, const WorkMap* wm, cplx<T>* x,
                                 cplx<T>* xp, const T* nhat, const cplx<T>* t, const int* done, size_t lds,
                                 hipStream_t st)
{
    launch_conv_b<T, MZ, 0>(P, np, wm, x, xp, nhat, t, done, lds, st);
    if constexpr (MZ <= 8 && SSM_CONV_CT) {
        launch_conv_b<T, MZ, 5>(P, np, wm, x, xp, nhat, t, done, lds, st);
        launch_conv_b<T, MZ, 6>(P, np, wm, x, xp, nhat, t, done, lds, st);
        launch_conv_b<T, MZ, 7>(P, np, wm, x, xp, nhat, t, done, lds, st);
        launch_conv_b<T, MZ, 8>(P, np, wm, x, xp, nhat, t, done, lds, st);
        launch_conv_b<T, MZ, 20>(P, np, wm, x, xp, nhat, t, done, lds, st);
        launch_conv_b<T, MZ, 21>(P, np, wm, x, xp, nhat, t, done, lds, st);
        launch_conv_b<T, MZ, 22>(P, np, wm, x, xp, nhat, t, done, lds, st);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_conv(int mz, const Prob* P, int np, const WorkMap* wm, void* X, void* Xp,
                       const T* nhat, const void* tw, const int* done, size_t lds, hipStream_t st)
{
    cplx<T>* x = (cplx<T>*)X;
    cplx<T>* xp = (cplx<T>*)Xp;
    const cplx<T>* t = (const cplx<T>*)tw;
    switch (mz) {
    case 1: return launch_conv_mz<T, 1>(P, np, wm, x, xp, nhat, t, done, lds, st);
    case 2: return launch_conv_mz<T, 2>(P, np, wm, x, xp, nhat, t, done, lds, st);
    case 4: return launch_conv_mz<T, 4>(P, np, wm, x, xp, nhat, t, done, lds, st);
    case 8: return launch_conv_mz<T, 8>(P, np, wm, x, xp, nhat, t, done, lds, st);
    case 16: return launch_conv_mz<T, 16>(P, np, wm, x, xp, nhat, t, done, lds, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_xinv(const Prob* P, int np, const WorkMap* wm, const void* Xp, const T* s,
                       T* s_star, T* h, double* epart, const void* tw, const int* done, int mode,
                       double tau, double fcp, double fcd, size_t lds, hipStream_t st)
{
    if (wm[0].total)
        hipLaunchKernelGGL((k_xinv<T, 0>), dim3(wm[0].total), dim3(kNT), lds, st, P, np, wm[0].start,
                           (const cplx<T>*)Xp, s, s_star, h, epart, (const cplx<T>*)tw, done, mode, tau, fcp, fcd);
    if (wm[1].total)
        hipLaunchKernelGGL((k_xinv<T, 1>), dim3(wm[1].total), dim3(kNT), lds, st, P, np, wm[1].start,
                           (const cplx<T>*)Xp, s, s_star, h, epart, (const cplx<T>*)tw, done, mode, tau, fcp, fcd);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_arc(const Prob* P, int np, const WorkMap& wm, const T* ss, double* apart,
                      const int* done, hipStream_t st)
{
    if (wm.total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_arc<T>, dim3(wm.total), dim3(kNT), 0, st, P, np, wm.start, ss, apart, done);
    return hipGetLastError();
}

hipError_t launch_reduce(const Prob* P, int np, int nimg, int kinds, const int* istart, const double* epart,
                         const double* apart, double* E, double* Tm, double* E_out, double* T_out,
                         double* seg, double* alpha, int* jidx, double* wgt, int* skip, int* done,
                         int* iters, int* count, int* flags, int with_arc, hipStream_t st, Step2 s2)
{
    if (kinds & 1)
        hipLaunchKernelGGL(k_reduce, dim3(nimg), dim3(kNT), 0, st, P, np, istart, epart, apart, E, Tm,
                           E_out, T_out, seg, alpha, jidx, wgt, skip, done, iters, count, flags, with_arc, s2);
    if (kinds & 2)
        hipLaunchKernelGGL(k_reduce1, dim3(np), dim3(kNT), 0, st, P, np, epart, apart, E, Tm, E_out, T_out,
                           seg, alpha, jidx, wgt, skip, done, iters, flags, with_arc, s2);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_interp(const Prob* P, int np, const WorkMap& wm, const T* ss, T* s,
                         const int* jidx, const double* wgt, const int* skip, const int* done,
                         int* flags, hipStream_t st, const int* kci, const int* skip_if)
{
    if (wm.total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_interp<T>, dim3(wm.total), dim3(kNT), 0, st, P, np, wm.start, ss, s, jidx,
                       wgt, skip, done, flags, kci, skip_if);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_tan1(const Prob* P, int np, const WorkMap& wm, const T* s, const T* h, T* tt,
                       double* fpart, hipStream_t st)
{
    hipLaunchKernelGGL(k_tan1<T>, dim3(wm.total), dim3(kNT), 0, st, P, np, wm.start, s, h, tt, fpart);
    return hipGetLastError();
}

hipError_t launch_tanred(const Prob* P, int np, const double* fpart, double* tcoef, hipStream_t st)
{
    hipLaunchKernelGGL(k_tanred, dim3(np), dim3(kNT), 0, st, P, np, fpart, tcoef);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_tan2(const Prob* P, int np, const WorkMap& wm, const T* s, const T* h,
                       const T* tt, T* t_out, const double* tcoef, double* fmax, hipStream_t st)
{
    hipLaunchKernelGGL(k_tan2<T>, dim3(wm.total), dim3(kNT), 0, st, P, np, wm.start, s, h, tt, t_out,
                       tcoef, fmax);
    return hipGetLastError();
}

hipError_t launch_fmax(const Prob* P, int np, const double* fmax, double* fnorm, int* done,
                       double tol, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_fmax, dim3(np), dim3(kNT), 0, st, P, np, fmax, fnorm, done, tol, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_spectrum(const Prob& p, T* nhat, double* f1, double* f2, const double* tw64,
                           hipStream_t st)
{
    const int nyo = 2 * p.ny - 1, nzo = 2 * p.nz - 1, Py = 2 * p.my;
    const long long n1 = 6LL * (p.mx + 1) * nyo * nzo;
    const long long n2 = 6LL * (p.mx + 1) * Py * nzo;
    const long long n3 = 6LL * (p.mx + 1) * Py * p.pz;
    hipLaunchKernelGGL(k_spec1, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, st, p, f1, tw64);
    hipLaunchKernelGGL(k_spec2, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, p, f1, f2, tw64);
    hipLaunchKernelGGL(k_spec3<T>, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, st, p, f2, nhat, tw64);
    return hipGetLastError();
}

hipError_t launch_barrier(const Prob* P, int np, const double* E, const double* Tm, double* out,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_barrier, dim3((np + 63) / 64), dim3(64), 0, st, P, np, E, Tm, out);
    return hipGetLastError();
}

hipError_t launch_iters_out(int np, const int* iters, const int* iters0, int* out, hipStream_t st)
{
    (void)iters0;
    hipLaunchKernelGGL(k_copy_int, dim3((np + 255) / 256), dim3(256), 0, st, iters, out, np);
    return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int n, int v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Step 1 by the adaptive Dormand-Prince 5(4) pair (Sec. III: each image is
// evolved over an interval by explicit embedded Runge-Kutta with adaptive
// step size; right-hand side the damping term of eq. (9), f = (s.s) h -
// (s.h) s, evaluated by the field kernels in EPI_FORCE mode).  Coefficients
// of Dormand and Prince (1980): stage rows, and the difference of the
// fifth- and fourth-order weights for the error estimate.  The last stage's
// input is the fifth-order solution (its row equals the weights).
// ---------------------------------------------------------------------------
__constant__ double kDopriA[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
__constant__ double kDopriE[7] = {35.0 / 384 - 5179.0 / 57600, 0.0, 500.0 / 1113 - 7571.0 / 16695,
                                  125.0 / 192 - 393.0 / 640, -2187.0 / 6784 + 92097.0 / 339200,
                                  11.0 / 84 - 187.0 / 2100, -1.0 / 40};

// per-image start of an interval: t = 0, first attempt's step
__global__ void k_rk_init(const Prob* __restrict__ P, int np, int nimg, const int* __restrict__ istart,
                          RkState rs, double Tint, const int* __restrict__ done)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nimg) return;
    const int pi = find_problem_lane(istart, np, g);
    rs.t[g] = 0.0;
    rs.acc[g] = 0;
    const bool on = !(done && done[pi]);
    rs.act[g] = on ? 1 : 0;
    const int cap = rs.dtp[g] >= Tint;
    rs.capped[g] = cap;
    rs.dtu[g] = cap ? Tint : rs.dtp[g];
}

// stage input y = s + dtu * sum_{j < STAGE} a[STAGE][j] k_j (FP64 sums);
// images that are not integrating get y = s.  STAGE at compile time: the
// slope loads of a site are all in flight together.
template <typename T, int STAGE>
__global__ __launch_bounds__(kNT) void k_rk_stage(const Prob* __restrict__ P, int np,
                                                  const int* __restrict__ wstart, const T* __restrict__ s,
                                                  RkSlopes<T> ks, RkState rs, T* __restrict__ y,
                                                  const int* __restrict__ done)
{
    const int pi = find_problem(wstart, np, blockIdx.x);
    if (done && done[pi]) return;
    const Prob& p = P[pi];
    const int w = blockIdx.x - wstart[pi];
    const int img = w / p.ichunks, chunk = w - img * p.ichunks;
    const long long N = p.N;
    const long long i = (long long)chunk * kNT + threadIdx.x;
    if (i >= N) return;
    const int g = p.img0 + img;
    const double h = rs.act[g] ? rs.dtu[g] : 0.0;
    const long long base = p.s_off + (long long)img * 3 * N + i;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const long long o = base + c * N;
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < STAGE; ++j) acc += kDopriA[STAGE][j] * (double)ks.k[j][o];
        y[o] = (T)((double)s[o] + h * acc);
    }
}

// error partials: sum over the workgroup's sites of (e_c / sc_c)^2, e the
// difference of the fifth- and fourth-order solutions, sc = atol + rtol
// max(|s|, |y5|); y holds y5 (the last stage's input)
template <typename T>
__global__ __launch_bounds__(kNT) void k_rk_err(const Prob* __restrict__ P, int np,
                                                const int* __restrict__ wstart, const T* __restrict__ s,
                                                const T* __restrict__ y, RkSlopes<T> ks, RkState rs,
                                                double rtol, double atol, double* __restrict__ part,
                                                const int* __restrict__ done)
{
    __shared__ double red[kNT / 64];
    const int pi = find_problem(wstart, np, blockIdx.x);
    if (done && done[pi]) return;
    const Prob& p = P[pi];
    const int w = blockIdx.x - wstart[pi];
    const int img = w / p.ichunks, chunk = w - img * p.ichunks;
    const long long N = p.N;
    const long long i = (long long)chunk * kNT + threadIdx.x;
    const int g = p.img0 + img;
    const double h = rs.dtu[g];
    double q = 0.0;
    if (i < N && rs.act[g]) {
        const long long base = p.s_off + (long long)img * 3 * N + i;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const long long o = base + c * N;
            double e = 0.0;
#pragma unroll
            for (int j = 0; j < 7; ++j) e += kDopriE[j] * (double)ks.k[j][o];
            e *= h;
            const double sc = atol + rtol * fmax(fabs((double)s[o]), fabs((double)y[o]));
            q += (e / sc) * (e / sc);
        }
    }
    q = wave_sum(q);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = q;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int wv = 0; wv < kNT / 64; ++wv) v += red[wv];
        part[p.fm_off + (long long)img * p.ichunks + chunk] = v;
    }
}

// step control, one workgroup per image: err = sqrt(mean of the partials);
// accept iff err <= 1; next step = step * clamp(0.9 err^(-1/5), 0.2, 5) (at
// most 1 after a rejection); the next attempt is shortened to end at Tint
__global__ __launch_bounds__(kNT) void k_rk_ctrl(const Prob* __restrict__ P, int np,
                                                 const int* __restrict__ istart, const double* __restrict__ part,
                                                 RkState rs, double Tint, const int* __restrict__ done,
                                                 int* flags)
{
    __shared__ double red[kNT / 64];
    const int g = blockIdx.x;
    const int pi = find_problem(istart, np, g);
    const Prob& p = P[pi];
    const int img = g - p.img0;
    if ((done && done[pi]) || !rs.act[g]) {
        if (threadIdx.x == 0) rs.acc[g] = 0;
        return;
    }
    double v = 0.0;
    const double* pp = part + p.fm_off + (long long)img * p.ichunks;
    for (int t = threadIdx.x; t < p.ichunks; t += kNT) v += pp[t];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x != 0) return;
    double sum = 0.0;
    for (int wv = 0; wv < kNT / 64; ++wv) sum += red[wv];
    const double err = sqrt(sum / (double)(3 * p.N));
    double fac = 0.9 * pow(fmax(err, 1e-10), -0.2);
    fac = fmin(5.0, fmax(0.2, fac));
    const double hs = rs.dtu[g];
    if (!(err <= 1.0) && !isfinite(err)) {
        // a non-finite error estimate cannot be controlled: stop this image
        atomicOr(flags, 8);
        rs.acc[g] = 0;
        rs.act[g] = 0;
        return;
    }
    if (err <= 1.0) {
        rs.acc[g] = 1;
        rs.cnt[2 * g] += 1;
        if (rs.capped[g]) rs.act[g] = 0;
        else rs.t[g] += hs;
    } else {
        rs.acc[g] = 0;
        fac = fmin(fac, 1.0);
        rs.cnt[2 * g + 1] += 1;
    }
    rs.dtp[g] = hs * fac;
    if (rs.act[g]) {
        const double rem = Tint - rs.t[g];
        const int cap = rs.dtp[g] >= rem;
        rs.capped[g] = cap;
        rs.dtu[g] = cap ? rem : rs.dtp[g];
        atomicAdd(rs.nact, 1);
    }
}

// accepted images: s = y5, first slope of the next attempt = last slope
template <typename T>
__global__ __launch_bounds__(kNT) void k_rk_apply(const Prob* __restrict__ P, int np,
                                                  const int* __restrict__ wstart, T* __restrict__ s,
                                                  const T* __restrict__ y, RkSlopes<T> ks, RkState rs,
                                                  const int* __restrict__ done)
{
    const int pi = find_problem(wstart, np, blockIdx.x);
    if (done && done[pi]) return;
    const Prob& p = P[pi];
    const int w = blockIdx.x - wstart[pi];
    const int img = w / p.ichunks, chunk = w - img * p.ichunks;
    const long long N = p.N;
    const long long i = (long long)chunk * kNT + threadIdx.x;
    if (i >= N || !rs.acc[p.img0 + img]) return;
    const long long base = p.s_off + (long long)img * 3 * N + i;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        s[base + c * N] = y[base + c * N];
        ks.k[0][base + c * N] = ks.k[6][base + c * N];
    }
}

// end of the interval: s* = s / |s| per spin
template <typename T>
__global__ __launch_bounds__(kNT) void k_rk_norm(const Prob* __restrict__ P, int np,
                                                 const int* __restrict__ wstart, const T* __restrict__ s,
                                                 T* __restrict__ ss, const int* __restrict__ done, int* flags)
{
    const int pi = find_problem(wstart, np, blockIdx.x);
    if (done && done[pi]) return;
    const Prob& p = P[pi];
    const int w = blockIdx.x - wstart[pi];
    const int img = w / p.ichunks, chunk = w - img * p.ichunks;
    const long long N = p.N;
    const long long i = (long long)chunk * kNT + threadIdx.x;
    if (i >= N) return;
    const long long base = p.s_off + (long long)img * 3 * N + i;
    const double v[3] = {(double)s[base], (double)s[base + N], (double)s[base + 2 * N]};
    const double nrm = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    if (!isfinite(nrm)) atomicOr(flags, 4);
    else if (nrm < 1e-12) atomicOr(flags, 2);
#pragma unroll
    for (int c = 0; c < 3; ++c) ss[base + c * N] = (T)(v[c] / nrm);
}

hipError_t launch_rk_init(const Prob* P, int np, int nimg, const int* istart, RkState rs, double Tint,
                          const int* done, hipStream_t st)
{
    if (nimg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rk_init, dim3((nimg + 255) / 256), dim3(256), 0, st, P, np, nimg, istart, rs, Tint,
                       done);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_rk_stage(const Prob* P, int np, const WorkMap& wm, const T* s, RkSlopes<T> ks, int stage,
                           RkState rs, T* y, const int* done, hipStream_t st)
{
    if (wm.total == 0) return hipSuccess;
    switch (stage) {
#define SSM_RK_STAGE(S)                                                                                     \
    case S:                                                                                                 \
        hipLaunchKernelGGL((k_rk_stage<T, S>), dim3(wm.total), dim3(kNT), 0, st, P, np, wm.start, s, ks, rs, y, \
                           done);                                                                           \
        break;
        SSM_RK_STAGE(1)
        SSM_RK_STAGE(2)
        SSM_RK_STAGE(3)
        SSM_RK_STAGE(4)
        SSM_RK_STAGE(5)
        SSM_RK_STAGE(6)
#undef SSM_RK_STAGE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_rk_err(const Prob* P, int np, const WorkMap& wm, const T* s, const T* y, RkSlopes<T> ks,
                         RkState rs, double rtol, double atol, double* part, const int* done, hipStream_t st)
{
    if (wm.total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rk_err<T>, dim3(wm.total), dim3(kNT), 0, st, P, np, wm.start, s, y, ks, rs, rtol, atol,
                       part, done);
    return hipGetLastError();
}

hipError_t launch_rk_ctrl(const Prob* P, int np, int nimg, const int* istart, const double* part, RkState rs,
                          double Tint, const int* done, int* flags, hipStream_t st)
{
    if (nimg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rk_ctrl, dim3(nimg), dim3(kNT), 0, st, P, np, istart, part, rs, Tint, done, flags);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_rk_apply(const Prob* P, int np, const WorkMap& wm, T* s, const T* y, RkSlopes<T> ks,
                           RkState rs, const int* done, hipStream_t st)
{
    if (wm.total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rk_apply<T>, dim3(wm.total), dim3(kNT), 0, st, P, np, wm.start, s, y, ks, rs, done);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_rk_norm(const Prob* P, int np, const WorkMap& wm, const T* s, T* ss, const int* done,
                          int* flags, hipStream_t st)
{
    if (wm.total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rk_norm<T>, dim3(wm.total), dim3(kNT), 0, st, P, np, wm.start, s, ss, done, flags);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Step-2 variants (Sec. III).  Natural cubic spline in alpha through the
// images, per site and spin component: k_spline_m solves the tridiagonal
// system for the second derivatives M (M_0 = M_{K-1} = 0) with the Thomas
// factors of the reduction's last workgroup; k_interp_spline evaluates
// A f_j + B f_{j+1} + ((A^3 - A) M_j + (B^3 - B) M_{j+1}) h^2/6 at every
// target and renormalises.  Climbing image k*: force F - 2 (F.t) t with F
// the perpendicular field and t the normalised per-spin-projected central
// difference of its neighbours.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kNT) void k_spline_m(const Prob* __restrict__ P, int np,
                                                  const int* __restrict__ wstart, const T* __restrict__ ss,
                                                  T* __restrict__ M, Step2 s2, const int* __restrict__ done,
                                                  int kskip)
{
    const int pi = find_problem(wstart, np, blockIdx.x);
    if ((done && done[pi]) || !s2.spl_ok[pi]) return;
    const Prob& p = P[pi];
    if (p.K <= kskip) return;  // served by k_interp_splw
    const long long N = p.N, Ms = 3 * N;
    const long long i = (long long)(blockIdx.x - wstart[pi]) * kNT + threadIdx.x;
    if (i >= N) return;
    const int K = p.K, g0 = p.img0;
#pragma unroll 1
    for (int c = 0; c < 3; ++c) {
        const long long o = p.s_off + c * N + i;
        double fm = (double)ss[o], f0 = (double)ss[o + Ms], dpp = 0.0;
        M[o] = T(0);
        M[o + (long long)(K - 1) * Ms] = T(0);
        for (int k = 1; k <= K - 2; ++k) {
            const double fp = (double)ss[o + (long long)(k + 1) * Ms];
            const double r = (fp - f0) / s2.hh[g0 + k] - (f0 - fm) / s2.hh[g0 + k - 1];
            const double dp = (r - (k > 1 ? s2.sa[g0 + k] * dpp : 0.0)) / s2.den[g0 + k];
            M[o + (long long)k * Ms] = (T)dp;
            dpp = dp;
            fm = f0;
            f0 = fp;
        }
        double mn = (double)M[o + (long long)(K - 2) * Ms];
        for (int k = K - 3; k >= 1; --k) {
            const double mk = (double)M[o + (long long)k * Ms] - s2.cp[g0 + k] * mn;
            M[o + (long long)k * Ms] = (T)mk;
            mn = mk;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kNT) void k_interp_spline(const Prob* __restrict__ P, int np,
                                                       const int* __restrict__ wstart, const T* __restrict__ ss,
                                                       const T* __restrict__ M, T* __restrict__ s,
                                                       const int* __restrict__ jidx,
                                                       const double* __restrict__ wgt, Step2 s2,
                                                       const int* __restrict__ done, int* flags, int kskip)
{
    const int pi = find_problem(wstart, np, blockIdx.x);
    if ((done && done[pi]) || !s2.spl_ok[pi]) return;
    const Prob& p = P[pi];
    if (p.K <= kskip) return;  // served by k_interp_splw
    const int w = blockIdx.x - wstart[pi];
    const int k = w / p.ichunks, chunk = w - k * p.ichunks;
    const long long N = p.N, Ms = 3 * N;
    const long long i = (long long)chunk * kNT + threadIdx.x;
    if (i >= N) return;
    const T* src = ss + p.s_off;
    T* dst = s + p.s_off + (long long)k * Ms;
    if (k == 0 || k == p.K - 1 || k == s2.kci[pi]) {
#pragma unroll
        for (int c = 0; c < 3; ++c) dst[c * N + i] = src[(long long)k * Ms + c * N + i];
        return;
    }
    const int g = p.img0 + k;
    const int j = jidx[g];
    const double A = s2.A[g], B = s2.B[g], h = s2.H[g];
    const long long oa = (long long)j * Ms + i, ob = oa + Ms;
    double v[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const long long q = c * N;
        v[c] = A * (double)src[oa + q] + B * (double)src[ob + q];
        v[c] += ((A * A * A - A) * (double)M[p.s_off + oa + q] + (B * B * B - B) * (double)M[p.s_off + ob + q]) *
                h * h / 6.0;
    }
    const double nrm = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    if (!isfinite(nrm)) atomicOr(flags, 4);
    if (nrm < 1e-12) {
        atomicOr(flags, 2);
        const long long on = (wgt[g] < 0.5) ? oa : ob;
#pragma unroll
        for (int c = 0; c < 3; ++c) dst[c * N + i] = src[on + c * N];
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) dst[c * N + i] = (T)(v[c] / nrm);
    }
}

// The same spline step in one pass for K <= KMAX: the interpolated value at
// a target is linear in the K images of its site, s(t_k) = sum_i W_ki f_i.
// The problem's K x K operator W (the columns of the second-derivative map
// by the Thomas recurrences of k_spline_m applied to unit right-hand sides,
// then the spline formula of k_interp_spline) is formed once by the end of
// step 2 (reduce_final); each workgroup loads it into LDS, and each thread
// then reads its site's K images once and writes the K targets.  Endpoints
// and the climbing image are copied.
template <typename T, int KMAX>
__global__ __launch_bounds__(kNT) void k_interp_splw(const Prob* __restrict__ P, int np,
                                                     const int* __restrict__ wstart, const T* __restrict__ ss,
                                                     T* __restrict__ s, const int* __restrict__ jidx,
                                                     const double* __restrict__ wgt, Step2 s2,
                                                     const int* __restrict__ done, int* flags)
{
    __shared__ double W[KMAX][KMAX];
    const int pi = find_problem(wstart, np, blockIdx.x);
    if ((done && done[pi]) || !s2.spl_ok[pi]) return;
    const Prob& p = P[pi];
    if (p.K > KMAX) return;  // served by k_spline_m and k_interp_spline
    const int K = p.K, g0 = p.img0, kci = s2.kci ? s2.kci[pi] : -1;
    // the problem's operator, formed by the end of step 2
    for (int e = threadIdx.x; e < KMAX * KMAX; e += kNT) {
        const int k = e / KMAX, i = e % KMAX;
        W[k][i] = (k < K && i < K) ? s2.Wm[(long long)(g0 + k) * kWRow + i] : 0.0;
    }
    __syncthreads();
    const long long N = p.N, Ms = 3 * N;
    const long long i = (long long)(blockIdx.x - wstart[pi]) * kNT + threadIdx.x;
    if (i >= N) return;
    const T* src = ss + p.s_off + i;
    T* dst = s + p.s_off + i;
    T f[3][KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) f[c][k] = (k < K) ? src[k * Ms + c * N] : T(0);
#pragma unroll 1
    for (int k = 0; k < K; ++k) {
        if (k == 0 || k == K - 1 || k == kci) {
            // copied like the endpoints (the same bits)
#pragma unroll
            for (int c = 0; c < 3; ++c) dst[k * Ms + c * N] = src[k * Ms + c * N];
            continue;
        }
        double v[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < KMAX; ++q) {
            const double w = W[k][q];
#pragma unroll
            for (int c = 0; c < 3; ++c) v[c] += w * (double)f[c][q];
        }
        // renormalised by the device library's FP64 reciprocal square root
        // (within an ulp or two of sqrt and division); the norm below 1e-12
        // takes the nearer source's spin
        const double n2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        if (!isfinite(n2)) atomicOr(flags, 4);
        if (n2 < 1e-24) {
            atomicOr(flags, 2);
            const int g = g0 + k, j = jidx[g];
            const int jn = (wgt[g] < 0.5) ? j : j + 1;
#pragma unroll
            for (int c = 0; c < 3; ++c) dst[k * Ms + c * N] = src[jn * Ms + c * N];
        } else {
            const double inv = rsqrt(n2);
#pragma unroll
            for (int c = 0; c < 3; ++c) dst[k * Ms + c * N] = (T)(v[c] * inv);
        }
    }
}

// one workgroup per (problem, site chunk): the image of highest energy
// (every workgroup finds the same one) and, when interior, partial sums of
// |t~|^2 and F.t~ over the chunk
template <typename T>
__global__ __launch_bounds__(kNT) void k_ci_part(const Prob* __restrict__ P, int np,
                                                 const int* __restrict__ wstart, const T* __restrict__ s,
                                                 const T* __restrict__ h, const double* __restrict__ E,
                                                 double* __restrict__ part, int* __restrict__ kci,
                                                 const int* __restrict__ done)
{
    __shared__ double red[kNT / 64][2];
    __shared__ int s_km;
    const int pi = find_problem(wstart, np, blockIdx.x);
    if (done && done[pi]) return;
    const Prob& p = P[pi];
    const int chunk = blockIdx.x - wstart[pi];
    const int K = p.K, g0 = p.img0;
    if (threadIdx.x < 64) {
        // the first index of the largest energy (NaN energies never count;
        // a NaN first energy gives 0), by the first wavefront in parallel:
        // each lane scans its own images in order, then the lanes combine
        // (larger value, else smaller index)
        const int lane = threadIdx.x;
        double bv = 0.0;
        int bi = -1;
        for (int kk = lane; kk < K; kk += 64) {
            const double e = E[g0 + kk];
            if (e == e && (bi < 0 || e > bv)) { bv = e; bi = kk; }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(bv, o);
            const int oi = __shfl_xor(bi, o);
            if (oi >= 0 && (bi < 0 || ov > bv || (ov == bv && oi < bi))) { bv = ov; bi = oi; }
        }
        if (lane == 0) {
            const double e0 = E[g0];
            const int km = (e0 == e0) ? bi : 0;
            s_km = km;
            if (chunk == 0) kci[pi] = (km > 0 && km < K - 1) ? km : -1;
        }
    }
    __syncthreads();
    const int km = s_km;
    if (km == 0 || km == K - 1) return;
    const long long N = p.N, Ms = 3 * N;
    const long long i = (long long)chunk * kNT + threadIdx.x;
    double q1 = 0.0, q2 = 0.0;
    if (i < N) {
        const long long o = p.s_off + (long long)km * Ms + i;
        double v[3], f[3], dl[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            v[c] = (double)s[o + c * N];
            f[c] = (double)h[o + c * N];
            dl[c] = (double)s[o + Ms + c * N] - (double)s[o - Ms + c * N];
        }
        const double sh = v[0] * f[0] + v[1] * f[1] + v[2] * f[2];
        const double sd = v[0] * dl[0] + v[1] * dl[1] + v[2] * dl[2];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double F = f[c] - sh * v[c], t = dl[c] - sd * v[c];
            q1 += t * t;
            q2 += F * t;
        }
    }
    q1 = wave_sum(q1);
    q2 = wave_sum(q2);
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6][0] = q1;
        red[threadIdx.x >> 6][1] = q2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int wv = 0; wv < kNT / 64; ++wv) {
            a += red[wv][0];
            b += red[wv][1];
        }
        part[p.fp_off + (long long)chunk * 2] = a;
        part[p.fp_off + (long long)chunk * 2 + 1] = b;
    }
}

__global__ __launch_bounds__(kNT) void k_ci_red(const Prob* __restrict__ P, int np,
                                                const double* __restrict__ part, const int* __restrict__ kci,
                                                double* __restrict__ coef, const int* __restrict__ done)
{
    __shared__ double red[kNT / 64][2];
    const int pi = blockIdx.x;
    if ((done && done[pi]) || kci[pi] < 0) return;
    const Prob& p = P[pi];
    double a = 0.0, b = 0.0;
    for (int t = threadIdx.x; t < p.ichunks; t += kNT) {
        a += part[p.fp_off + (long long)t * 2];
        b += part[p.fp_off + (long long)t * 2 + 1];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6][0] = a;
        red[threadIdx.x >> 6][1] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tn2 = 0.0, ft = 0.0;
        for (int wv = 0; wv < kNT / 64; ++wv) {
            tn2 += red[wv][0];
            ft += red[wv][1];
        }
        coef[pi] = (tn2 > 0.0) ? ft / tn2 : 0.0;
    }
}

template <typename T>
__global__ __launch_bounds__(kNT) void k_ci_step(const Prob* __restrict__ P, int np,
                                                 const int* __restrict__ wstart, const T* __restrict__ s,
                                                 const T* __restrict__ h, T* __restrict__ ss,
                                                 const int* __restrict__ kci, const double* __restrict__ coef,
                                                 double tau, const int* __restrict__ done)
{
    const int pi = find_problem(wstart, np, blockIdx.x);
    if (done && done[pi]) return;
    const int km = kci[pi];
    if (km < 0) return;
    const Prob& p = P[pi];
    const long long N = p.N, Ms = 3 * N;
    const long long i = (long long)(blockIdx.x - wstart[pi]) * kNT + threadIdx.x;
    if (i >= N) return;
    const long long o = p.s_off + (long long)km * Ms + i;
    const double cc = coef[pi];
    double v[3], f[3], dl[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        v[c] = (double)s[o + c * N];
        f[c] = (double)h[o + c * N];
        dl[c] = (double)s[o + Ms + c * N] - (double)s[o - Ms + c * N];
    }
    const double sh = v[0] * f[0] + v[1] * f[1] + v[2] * f[2];
    const double sd = v[0] * dl[0] + v[1] * dl[1] + v[2] * dl[2];
    double w[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) w[c] = v[c] + tau * ((f[c] - sh * v[c]) - 2.0 * cc * (dl[c] - sd * v[c]));
    const double nrm = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
#pragma unroll
    for (int c = 0; c < 3; ++c) ss[o + c * N] = (T)(w[c] / nrm);
}

template <typename T>
hipError_t launch_spline_m(const Prob* P, int np, const WorkMap& wm_sitep, const T* ss, T* M, Step2 s2,
                           const int* done, int kskip, hipStream_t st)
{
    if (wm_sitep.total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_spline_m<T>, dim3(wm_sitep.total), dim3(kNT), 0, st, P, np, wm_sitep.start, ss, M, s2,
                       done, kskip);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_interp_spline(const Prob* P, int np, const WorkMap& wm, const T* ss, const T* M, T* s,
                                const int* jidx, const double* wgt, Step2 s2, const int* done, int* flags,
                                int kskip, hipStream_t st)
{
    if (wm.total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_interp_spline<T>, dim3(wm.total), dim3(kNT), 0, st, P, np, wm.start, ss, M, s, jidx, wgt,
                       s2, done, flags, kskip);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_interp_splw(const Prob* P, int np, const WorkMap& wm_sitep, int kmax, const T* ss, T* s,
                              const int* jidx, const double* wgt, Step2 s2, const int* done, int* flags,
                              hipStream_t st)
{
    if (wm_sitep.total == 0) return hipSuccess;
    if (kmax > kSplwMax<T>) return hipErrorInvalidValue;
    if (kmax <= 16) {
        hipLaunchKernelGGL((k_interp_splw<T, 16>), dim3(wm_sitep.total), dim3(kNT), 0, st, P, np, wm_sitep.start,
                           ss, s, jidx, wgt, s2, done, flags);
    } else if constexpr (kSplwMax<T> >= 32) {
        hipLaunchKernelGGL((k_interp_splw<T, 32>), dim3(wm_sitep.total), dim3(kNT), 0, st, P, np, wm_sitep.start,
                           ss, s, jidx, wgt, s2, done, flags);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ci_part(const Prob* P, int np, const WorkMap& wm, const T* s, const T* h, const double* E,
                          double* part, int* kci, const int* done, hipStream_t st)
{
    if (wm.total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ci_part<T>, dim3(wm.total), dim3(kNT), 0, st, P, np, wm.start, s, h, E, part, kci, done);
    return hipGetLastError();
}

hipError_t launch_ci_red(const Prob* P, int np, const double* part, const int* kci, double* coef,
                         const int* done, hipStream_t st)
{
    hipLaunchKernelGGL(k_ci_red, dim3(np), dim3(kNT), 0, st, P, np, part, kci, coef, done);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ci_step(const Prob* P, int np, const WorkMap& wm, const T* s, const T* h, T* ss,
                          const int* kci, const double* coef, double tau, const int* done, hipStream_t st)
{
    if (wm.total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ci_step<T>, dim3(wm.total), dim3(kNT), 0, st, P, np, wm.start, s, h, ss, kci, coef, tau,
                       done);
    return hipGetLastError();
}

// Copy of a small host blob passed by value as the kernel argument (the
// launch itself carries the bytes, so the host copy needs no lifetime and the
// call allocates nothing).
__global__ void k_put(unsigned char* dst, Blob b)
{
    for (int i = threadIdx.x; i < b.n; i += blockDim.x) dst[i] = b.b[i];
}

hipError_t launch_put(void* dst, const Blob& b, hipStream_t st)
{
    hipLaunchKernelGGL(k_put, dim3(1), dim3(256), 0, st, static_cast<unsigned char*>(dst), b);
    return hipGetLastError();
}

__global__ void k_fill_double(double* p, int n, double v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_double(double* p, int n, double v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_double, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

// explicit instantiations
#define SSM_INST(T)                                                                                \
    template hipError_t launch_xfwd<T>(const Prob*, int, const WorkMap*, const T*, void*,         \
                                       const void*, const int*, size_t, hipStream_t);             \
    template hipError_t launch_conv<T>(int, const Prob*, int, const WorkMap*, void*, void*,            \
                                       const T*, const void*, const int*, size_t, hipStream_t);   \
    template hipError_t launch_xinv<T>(const Prob*, int, const WorkMap*, const void*,              \
                                       const T*,                                                    \
                                       T*, T*, double*, const void*, const int*, int, double,     \
                                       double, double, size_t, hipStream_t);                       \
    template hipError_t launch_arc<T>(const Prob*, int, const WorkMap&, const T*, double*,        \
                                      const int*, hipStream_t);                                    \
    template hipError_t launch_interp<T>(const Prob*, int, const WorkMap&, const T*, T*,          \
                                         const int*, const double*, const int*, const int*, int*, \
                                         hipStream_t, const int*, const int*);                     \
    template hipError_t launch_spline_m<T>(const Prob*, int, const WorkMap&, const T*, T*, Step2,  \
                                           const int*, int, hipStream_t);                          \
    template hipError_t launch_interp_splw<T>(const Prob*, int, const WorkMap&, int, const T*, T*, \
                                              const int*, const double*, Step2, const int*, int*,  \
                                              hipStream_t);                                        \
    template hipError_t launch_interp_spline<T>(const Prob*, int, const WorkMap&, const T*,        \
                                                const T*, T*, const int*, const double*, Step2,    \
                                                const int*, int*, int, hipStream_t);               \
    template hipError_t launch_ci_part<T>(const Prob*, int, const WorkMap&, const T*, const T*,   \
                                          const double*, double*, int*, const int*, hipStream_t);  \
    template hipError_t launch_ci_step<T>(const Prob*, int, const WorkMap&, const T*, const T*,   \
                                          T*, const int*, const double*, double, const int*,       \
                                          hipStream_t);                                            \
    template hipError_t launch_tan1<T>(const Prob*, int, const WorkMap&, const T*, const T*, T*,  \
                                       double*, hipStream_t);                                      \
    template hipError_t launch_tan2<T>(const Prob*, int, const WorkMap&, const T*, const T*,      \
                                       const T*, T*, const double*, double*, hipStream_t);         \
    template hipError_t launch_spectrum<T>(const Prob&, T*, double*, double*, const double*,      \
                                           hipStream_t);                                           \
    template hipError_t launch_rk_stage<T>(const Prob*, int, const WorkMap&, const T*, RkSlopes<T>, \
                                           int, RkState, T*, const int*, hipStream_t);             \
    template hipError_t launch_rk_err<T>(const Prob*, int, const WorkMap&, const T*, const T*,    \
                                         RkSlopes<T>, RkState, double, double, double*,           \
                                         const int*, hipStream_t);                                 \
    template hipError_t launch_rk_apply<T>(const Prob*, int, const WorkMap&, T*, const T*,        \
                                           RkSlopes<T>, RkState, const int*, hipStream_t);         \
    template hipError_t launch_rk_norm<T>(const Prob*, int, const WorkMap&, const T*, T*,         \
                                          const int*, int*, hipStream_t);
SSM_INST(float)
SSM_INST(double)

}  // namespace ssm
