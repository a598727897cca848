// Internal declarations shared by the kernels and the host runtime of the
// gfx950 simplified-string-method library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ssm_fft.hpp"

namespace ssm {

// Twiddle table: tw[e] = exp(-2 pi i e / kTwM).  A length-L root W_L^e is
// tw[e * (kTwM / L)]; every padded length 2m (m = 2^a <= 1024 or
// m = 3 2^a <= 768) and every sub-length divides kTwM = 3 * 2^11.
constexpr int kTwM = 3 << 11;
constexpr int kMaxLogM = 10;   // half padded length m <= 1024, padded P = 2m <= 2048
// The FFT kernels read their twiddles from a compact table: for every half
// length m = 2^lg (lg <= 10) and m = 3 2^lg (lg <= 8), the 2m values
// W_{2m}^e, e < 2m, contiguous, starting at tw_off(lg, f3).
__host__ __device__ constexpr int tw_off(int lg, int f3)
{
    return f3 ? (4 << kMaxLogM) - 2 + 6 * ((1 << lg) - 1) : (2 << lg) - 2;
}
constexpr int kTwCompact = tw_off(9, 1);  // entries of the compact table
constexpr int kNT = 256;       // threads per workgroup for every kernel
constexpr int kConvElems = 24 * kNT;  // complex values per convolution workgroup (slice batching cap)
constexpr int kArcEPT = 8;     // flat elements per thread in the arc-length kernel
constexpr int kNTerm = 5;      // energy partial slots: E, T_J, T_d, T_ku, T_dip
constexpr int kMaxImages = 1024;  // images per problem (the ABI's limit)
// Reduction in one workgroup per problem (k_reduce1) for problems of at
// most kRed1MaxK images with at most kRed1MaxPart energy and arc partials
// per image; kRedLanes lanes sum one image's partials there.
#ifndef SSM_RED_LANES
#define SSM_RED_LANES 4
#endif
constexpr int kRed1MaxK = 64, kRed1MaxPart = 256, kRedLanes = SSM_RED_LANES;

// The convolution kernel comes in two builds: one with compile-time-length
// bodies for y lengths 32..256 and up to 8 layers, one with a runtime-length
// body for every other shape.  They are separate kernels so that each gets
// its own register allocation; a launch covers a problem with whichever
// build serves its shape.
#ifndef SSM_CONV_CT
#define SSM_CONV_CT 1
#endif
__host__ __device__ constexpr bool conv_ct_shape(int mz, int lmy, int f3y)
{
    return SSM_CONV_CT && !f3y && mz <= 8 && lmy >= 5 && lmy <= 8;
}
// y lengths 3 2^lmy with compile-time sub-line passes (48, 96, 192)
__host__ __device__ constexpr bool conv_ct3_shape(int mz, int lmy, int f3y)
{
    return SSM_CONV_CT && f3y && mz <= 8 && lmy >= 4 && lmy <= 6;
}
// build serving a problem: the y length's log2 (5..8) for the compile-time
// power-of-two builds, 16 + log2 of the power-of-two factor (20..22) for the
// compile-time 3 2^a builds, 0 for the runtime-length one
__host__ __device__ constexpr int conv_build(int mz, int lmy, int f3y)
{
    return conv_ct_shape(mz, lmy, f3y) ? lmy : conv_ct3_shape(mz, lmy, f3y) ? 16 + lmy : 0;
}

// LDS layout of the line buffers (pad_for, padx in ssm_fft.hpp).  The
// compile-time-length transforms can store lines with one pad element per
// 2^PADL (PADL = 0: dense), which spreads their strided accesses over the
// banks; the runtime-length ones use the dense layout.
#ifndef SSM_X_CT
#define SSM_X_CT 1
#endif
#ifndef SSM_X_PADL
#define SSM_X_PADL 4
#endif
#ifndef SSM_CONV_PADL
#define SSM_CONV_PADL 0
#endif
#ifndef SSM_CONV3_PADL
#define SSM_CONV3_PADL 4
#endif
// the 3 2^a layouts of the FP32 form: one pad per 8 elements (fewer bank
// conflicts on its 8-byte elements; FP64 keeps one per 16)
#ifndef SSM_X3_PADL_F32
#define SSM_X3_PADL_F32 3
#endif
#ifndef SSM_CONV3_PADL_F32
#define SSM_CONV3_PADL_F32 3
#endif
// x lengths with compile-time passes: powers of two 32..512 (lm = log2 m)
// and 3 2^lm for 48..384, in the pad-SSM_X_PADL layout (3 2^lm in FP32:
// pad-SSM_X3_PADL_F32); tsize: bytes per real value
__host__ __device__ constexpr bool x_ct_len(int lm, int f3) { return SSM_X_CT && !f3 && lm >= 5 && lm <= 9; }
__host__ __device__ constexpr bool x_ct3_len(int lm, int f3) { return SSM_X_CT && f3 && lm >= 4 && lm <= 7; }
__host__ __device__ constexpr int x_padl(int lm, int f3, int tsize)
{
    return x_ct_len(lm, f3)    ? pad_for(SSM_X_PADL, lm)
           : x_ct3_len(lm, f3) ? pad_for(tsize == 4 ? SSM_X3_PADL_F32 : SSM_X_PADL, lm)
                               : 0;
}
__host__ __device__ constexpr int conv_padl(int mz, int lmy, int f3y, int tsize)
{
    return conv_ct_shape(mz, lmy, f3y)    ? pad_for(SSM_CONV_PADL, lmy)
           : conv_ct3_shape(mz, lmy, f3y) ? pad_for(tsize == 4 ? SSM_CONV3_PADL_F32 : SSM_CONV3_PADL, lmy)
                                          : 0;
}
// elements of a buffer of n elements in the pad-padl layout
__host__ __device__ constexpr int padded_len(int n, int padl) { return padl ? n + (n >> padl) + 1 : n; }

// Kernel kinds (profiling slots; names in the runtime).
enum KernelKind {
    KK_XFWD = 0, KK_CONV, KK_XINV, KK_ARC, KK_REDUCE, KK_INTERP,
    KK_TAN1, KK_TAN2, KK_TANRED, KK_SPEC, KK_UTIL, KK_GRAPH, KK_RK, KK_COUNT_
};

// Per-problem descriptor, resident in device memory (read-only in kernels).
struct Prob {
    int nx, ny, nz, K;
    int mx, my, mz;        // half padded lengths >= nx, ny, nz: 2^a, or 3 2^a (a >= 4) along x and y
    int lmx, lmy, lmz;     // log2 of their power-of-two factor
    int f3x, f3y;          // 1: mx (my) = 3 2^lmx (3 2^lmy)
    int pz;                // padded z length: 2*mz when nz > 1, else 1
    int nhz;               // z halves of the padded z spectrum: 2 when nz > 1, else 1
    int yt;                // lattice rows per tile of the inverse-x / epilogue kernel
    int nty;               // ceil(ny / yt)
    int tiles;             // inverse-x tiles per image = nz * nty (energy partials)
    int ytf, ntyf, tilesf; // the same for the forward x kernel
    int wgf, wgi;          // forward / inverse x workgroups (K * tiles, padded to 8)
    int img0;              // index of this problem's first image in batch-wide arrays
    int gconv;             // consecutive (image, kx) slices per convolution workgroup
    int arc_chunks;        // arc-length workgroups (flat chunks of 3N) per image
    int xcd_remap;         // convolution kernel: group same-kx slices on one XCD
    long long N;           // sites per image
    long long s_off;       // element offset of image 0 in spin / field buffers
    long long x_off;       // complex-element offset in the x-spectrum buffers
    long long nh_off;      // element offset of this shape's dipole-kernel spectrum
    long long ep_off;      // offset (doubles) of energy partials: [K][tiles][kNTerm]
    long long ap_off;      // offset (doubles) of arc partials: [K][arc_chunks*4]
    long long fp_off;      // offset (doubles) of tangent partials: [K][ichunks][2]
    long long fm_off;      // offset (doubles) of per-workgroup force maxima: [K][ichunks]
    int ichunks;           // per-site workgroups per image (interp / tangents)
    int vec4;              // FP32 images of N divisible by 4, 16-byte aligned: 4 sites per thread
    int vec2;              // FP64 images of even N, 16-byte aligned: 2 sites per thread
    int ichunks4;          // interpolation workgroups per image (ichunks / 4 with vec4, / 2 with vec2)
    int arc_g;             // images per arc-length workgroup (image groups of arc_g)
    int arc_ng;            // image groups: arc-length workgroups = arc_chunks * arc_ng
    int red1;              // 1: reduced by one workgroup (k_reduce1), else one per image (k_reduce)
    double J, d, ku, D;    // eq. (1) parameters
};

// Work maps: workgroup ranges per problem for each kernel kind.
struct WorkMap {
    int* start;      // device: [nprob + 1] prefix sums of workgroup counts
    int total;
};

// ------------------------------------------------------------------------
// launchers (ssm_kernels.hip); all enqueue on `st` and return the HIP error
// ------------------------------------------------------------------------
// The FFT kernels come in kinds (x: power-of-two or 3 2^a length;
// convolution: one build per conv_build value) and each kind has a work map
// of its own, in which the problems of other kinds have no workgroups; a
// kind whose map is empty is not launched.  wm[0..1]: x length kinds
// (f3x); wm[conv_slot(b)]: convolution build b.
constexpr int kConvSlots = 8;
__host__ __device__ constexpr int conv_slot(int b) { return b == 0 ? 0 : (b <= 8 ? b - 4 : b - 15); }
template <typename T>
hipError_t launch_xfwd(const Prob* P, int np, const WorkMap* wm, const T* s, void* X,
                       const void* tw, const int* done, size_t lds, hipStream_t st);
// X' receives the convolved x half-spectra (X keeps the inputs)
template <typename T>
hipError_t launch_conv(int mz, const Prob* P, int np, const WorkMap* wm, void* X,
                       void* Xp, const T* nhat, const void* tw, const int* done, size_t lds,
                       hipStream_t st);
// mode bits for the inverse/epilogue kernel: EPI_STEP writes the stepped
// string, EPI_FIELD the field h, EPI_FORCE the damping right-hand side
// (s.s) h - (s.h) s in place of h, EPI_TERMS the four term partials
enum { EPI_STEP = 1, EPI_FIELD = 2, EPI_TERMS = 4, EPI_FORCE = 8 };
template <typename T>
// fcp, fcd: coefficients of EPI_FORCE (precession, damping)
hipError_t launch_xinv(const Prob* P, int np, const WorkMap* wm, const void* Xp, const T* s,
                       T* s_star, T* h, double* epart, const void* tw, const int* done,
                       int mode, double tau, double fcp, double fcd, size_t lds, hipStream_t st);
template <typename T>
hipError_t launch_arc(const Prob* P, int np, const WorkMap& wm, const T* ss, double* apart,
                      const int* done, hipStream_t st);
// Step-2 options of the reduction's last workgroup (ssm_set_reparam): bit 0
// natural cubic spline, bit 1 climbing image.  E: the current energies
// (climbing image choice); per problem: kci (climbing image or -1), spl_ok
// (spline factors valid); per image: interval widths hh, Thomas factors
// (sa, den, cp); per target image: spline weights A, B and interval width H.
struct Step2 {
    int opts = 0;
    const double* E = nullptr;
    int* kci = nullptr;
    int* spl_ok = nullptr;
    double* hh = nullptr;
    double* sa = nullptr;
    double* den = nullptr;
    double* cp = nullptr;
    double* A = nullptr;
    double* B = nullptr;
    double* H = nullptr;
    // the one-pass spline step's K x K operator of every problem of at most
    // wmax images (row k of problem pi at Wm + (img0 + k) kWRow), formed by
    // the end of step 2; wmax = 0: not formed
    double* Wm = nullptr;
    int wmax = 0;
};
constexpr int kWRow = 32;  // row stride of Step2::Wm (the largest one-pass image count)
// kinds: bit 0 problems reduced per image, bit 1 problems reduced by one
// workgroup (Prob::red1)
hipError_t launch_reduce(const Prob* P, int np, int nimg, int kinds, const int* istart, const double* epart,
                         const double* apart, double* E, double* Tm, double* E_out, double* T_out,
                         double* seg, double* alpha, int* jidx, double* wgt, int* skip, int* done,
                         int* iters, int* count, int* flags, int with_arc, hipStream_t st,
                         Step2 s2 = Step2{});
template <typename T>
// kci (or NULL): per-problem climbing image, copied like the endpoints;
// skip_if (or NULL): problems whose flag is set are left to the spline
hipError_t launch_interp(const Prob* P, int np, const WorkMap& wm, const T* ss, T* s,
                         const int* jidx, const double* wgt, const int* skip, const int* done,
                         int* flags, hipStream_t st, const int* kci = nullptr,
                         const int* skip_if = nullptr);
// natural cubic spline: second derivatives M of every site and component
// (M buffer in the spin layout), then the interpolation at the targets;
// problems of at most kskip images are left to launch_interp_splw
template <typename T>
hipError_t launch_spline_m(const Prob* P, int np, const WorkMap& wm_sitep, const T* ss, T* M, Step2 s2,
                           const int* done, int kskip, hipStream_t st);
template <typename T>
hipError_t launch_interp_spline(const Prob* P, int np, const WorkMap& wm, const T* ss, const T* M, T* s,
                                const int* jidx, const double* wgt, Step2 s2, const int* done, int* flags,
                                int kskip, hipStream_t st);
// the spline step in one pass for the problems of at most kSplwMax images
// (one thread per site, wm_sitep); kmax: the largest of their image
// counts; problems with more images are left to the two kernels above, so
// each problem takes the same path whatever else is in the batch
template <typename T>
constexpr int kSplwMax = sizeof(T) == 4 ? 32 : 16;
static_assert(kSplwMax<float> <= kWRow && kSplwMax<double> <= kWRow, "operator rows");
template <typename T>
hipError_t launch_interp_splw(const Prob* P, int np, const WorkMap& wm_sitep, int kmax, const T* ss, T* s,
                              const int* jidx, const double* wgt, Step2 s2, const int* done, int* flags,
                              hipStream_t st);
// climbing image: partial sums (|t~|^2, F.t~) over image kci, their
// per-problem reduction to c = F.t~ / |t~|^2, and the step
// normalise(s + tau (F - 2 c t~)) into ss
template <typename T>
hipError_t launch_ci_part(const Prob* P, int np, const WorkMap& wm, const T* s, const T* h, const double* E,
                          double* part, int* kci, const int* done, hipStream_t st);
hipError_t launch_ci_red(const Prob* P, int np, const double* part, const int* kci, double* coef,
                         const int* done, hipStream_t st);
template <typename T>
hipError_t launch_ci_step(const Prob* P, int np, const WorkMap& wm, const T* s, const T* h, T* ss,
                          const int* kci, const double* coef, double tau, const int* done, hipStream_t st);
template <typename T>
hipError_t launch_tan1(const Prob* P, int np, const WorkMap& wm, const T* s, const T* h,
                       T* tt, double* fpart, hipStream_t st);
hipError_t launch_tanred(const Prob* P, int np, const double* fpart, double* tcoef,
                         hipStream_t st);
template <typename T>
hipError_t launch_tan2(const Prob* P, int np, const WorkMap& wm, const T* s, const T* h,
                       const T* tt, T* t_out, const double* tcoef, double* fmax,
                       hipStream_t st);
hipError_t launch_fmax(const Prob* P, int np, const double* fmax, double* fnorm, int* done,
                       double tol, double* out, hipStream_t st);
template <typename T>
hipError_t launch_spectrum(const Prob& p, T* nhat, double* f1, double* f2, const double* tw64,
                           hipStream_t st);
hipError_t launch_barrier(const Prob* P, int np, const double* E, const double* Tm,
                          double* out, hipStream_t st);
hipError_t launch_iters_out(int np, const int* iters, const int* iters0, int* out,
                            hipStream_t st);
hipError_t launch_fill_int(int* p, int n, int v, hipStream_t st);
// up to kBlobBytes bytes copied to device memory by a kernel whose argument
// carries them
constexpr int kBlobBytes = 2048;
struct Blob {
    int n;
    unsigned char b[kBlobBytes];
};
hipError_t launch_put(void* dst, const Blob& b, hipStream_t st);
hipError_t launch_fill_double(double* p, int n, double v, hipStream_t st);

// Adaptive Dormand-Prince 5(4) step 1.  Per image (batch-wide index g):
// t[g] time reached in the interval, dtp[g] proposed step, dtu[g] step of
// the current attempt, capped[g] whether that attempt ends the interval,
// act[g] still integrating, acc[g] current attempt accepted, cnt[2g..]
// accepted / rejected steps; nact counts active images after control.
struct RkState {
    double* t;
    double* dtp;
    double* dtu;
    int* capped;
    int* act;
    int* acc;
    int* cnt;
    int* nact;
};
template <typename T>
struct RkSlopes {
    T* k[7];
};
hipError_t launch_rk_init(const Prob* P, int np, int nimg, const int* istart, RkState rs, double Tint,
                          const int* done, hipStream_t st);
template <typename T>
hipError_t launch_rk_stage(const Prob* P, int np, const WorkMap& wm, const T* s, RkSlopes<T> ks, int stage,
                           RkState rs, T* y, const int* done, hipStream_t st);
template <typename T>
hipError_t launch_rk_err(const Prob* P, int np, const WorkMap& wm, const T* s, const T* y, RkSlopes<T> ks,
                         RkState rs, double rtol, double atol, double* part, const int* done, hipStream_t st);
hipError_t launch_rk_ctrl(const Prob* P, int np, int nimg, const int* istart, const double* part, RkState rs,
                          double Tint, const int* done, int* flags, hipStream_t st);
template <typename T>
hipError_t launch_rk_apply(const Prob* P, int np, const WorkMap& wm, T* s, const T* y, RkSlopes<T> ks,
                           RkState rs, const int* done, hipStream_t st);
template <typename T>
hipError_t launch_rk_norm(const Prob* P, int np, const WorkMap& wm, const T* s, T* ss, const int* done,
                          int* flags, hipStream_t st);

}  // namespace ssm
