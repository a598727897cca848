/*
 * ssm.h -- C ABI of the MI355X (gfx950) simplified-string-method library.
 *
 * The library computes minimum energy paths and energy barriers of an
 * atomistic spin model with the simplified string method, following
 * Heistracher et al., "GPU Accelerated Atomistic Energy Barrier Calculations
 * of Skyrmion Annihilations" (arXiv:1804.07135):
 *   - Hamiltonian, eq. (1): nearest-neighbour exchange J, interfacial DMI d
 *     with DMI vector r_ij x z, uniaxial anisotropy k_u along z and the full
 *     dipole-dipole sum, on a simple cubic lattice with free boundaries;
 *   - effective field, eqs. (2)-(7): exchange/DMI/anisotropy stencils plus
 *     the dipolar field as a zero-padded FFT convolution with the
 *     point-dipole tensor (Sec. II.A);
 *   - energy from the field, eq. (8);
 *   - string iteration, Sec. III: every image takes one damping-only descent
 *     step along the force of the Appendix (the field component
 *     perpendicular to each spin, eq. (10)) and is renormalised; the string
 *     is then reparametrised to equal arc length, eqs. (11)-(12).
 *
 * Units.  Reduced units with the lattice constant as the length unit and
 * unit spins.  Fields are h = mu0 |S| H_eff = -dE/ds, so eq. (3) reads
 * h_ex = J sum_nn s_j, eq. (5) reads h_an = 2 k_u s_z z, and the dipolar
 * pair energy is -dip [3(s_i.r)(s_j.r) - s_i.s_j]/r^3 per unordered pair
 * with dip = mu0 |S|^2 / (4 pi a^3).  Every nearest-neighbour bond is
 * counted once.
 *
 * Layout.  A string of K images on an nx*ny*nz lattice is stored
 * structure-of-arrays, x fastest: element (k, c, z, y, x) sits at
 *   ((k*3 + c)*nz + z)*ny*nx + y*nx + x,
 * c = 0,1,2 for the x,y,z spin components.  A batch of problems stores the
 * strings of its problems one after another in creation order.  Spins,
 * fields and tangents are double for SSM_FP64 and float for SSM_FP32_MIXED;
 * energies, per-term energies, barriers and force norms are always double.
 *
 * Memory.  Every pointer argument named d_* is device memory owned by the
 * caller; the library only borrows it for the work it enqueues.  The
 * library never allocates device memory: all of its state lives in one
 * caller-provided workspace whose size ssm_workspace_size() returns.  The
 * context object itself is host memory owned by the library.
 *
 * Streams.  Every call enqueues its work on the stream given to
 * ssm_create() (a hipStream_t passed as void*; NULL = the default stream)
 * and returns without waiting, except ssm_workspace_size, ssm_check,
 * ssm_profile_read, ssm_autotune and ssm_iterate with tol_force > 0, which
 * synchronise that stream.
 *
 * Errors.  Functions return SSM_OK (0) or a negative status; nothing
 * throws across the ABI.  Argument errors are detected before anything is
 * enqueued.  HIP runtime failures return SSM_EHIP; ssm_last_error() then
 * holds the HIP error text.  A context is used by one host thread at a
 * time; distinct contexts are independent.
 *
 * Limits.  1 <= nx, ny <= 1024 and 1 <= nz <= 16; 2 <= n_images <= 1024;
 * at most 256 problems per context; every problem of a context has nz
 * values that round up to the same power of two; the convolution's
 * twiddles and one (y, z) plane of x-spectra, (2 + 3 * nz) * m_y complex
 * values with m_y the half padded y length (below), fit in 160 KiB of LDS,
 * i.e. m_y * (2 + 3 * nz) <= 10240 for SSM_FP64 and <= 20480 for
 * SSM_FP32_MIXED (m_y = 1024: nz <= 2 and <= 6; m_y = 512: nz <= 6 and
 * <= 12; m_y = 256: nz <= 12 and any nz).  Exceeding a limit returns
 * SSM_EUNSUPPORTED.
 *
 * Padding.  The dipolar convolution runs on a zero-padded grid of 2 m_x by
 * 2 m_y by (2 m_z, or 1 for nz = 1) sites; any padded length >= 2n - 1 per
 * axis gives the same field (Sec. II.A: circular sorting).  m_z is the
 * power of two >= nz; m_x and m_y are the power of two >= n or, for n > 32,
 * the length 3 * 2^a >= n (a >= 4, at most 768) when that is smaller, e.g.
 * m = 48 for n = 33..48, 96 for 65..96, 192 for 129..192, 384 for
 * 257..384 and 768 for 513..768.
 */
#ifndef SSM_H
#define SSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ssm_ctx ssm_ctx;
typedef int32_t ssm_status;

#define SSM_OK 0
#define SSM_EINVAL (-1)        /* bad argument (null pointer, K < 2, dim < 1, ...) */
#define SSM_ESTATE (-2)        /* call not valid in the current state */
#define SSM_EHIP (-3)          /* a HIP runtime call failed; see ssm_last_error */
#define SSM_ENONFINITE (-4)    /* ssm_check found a non-finite energy or spin */
#define SSM_EUNSUPPORTED (-5)  /* size or option outside the documented limits */

#define SSM_FP64 0        /* spins, FFTs, fields and all reductions in FP64 */
#define SSM_FP32_MIXED 1  /* spins, spectra and FFTs in FP32; per-site field
                             arithmetic, energies, arc lengths, weights and the
                             barrier in FP64 */

/* OR into the precision argument of ssm_workspace_size and ssm_create to
 * reserve the workspace of the adaptive integrator (8 more string-sized
 * buffers); needed for SSM_STEP_DOPRI54. */
#define SSM_WITH_RK 0x100

/* Step 1 of the string iteration (ssm_set_integrator) */
#define SSM_STEP_EULER 0    /* one explicit projected step of size tau (default) */
#define SSM_STEP_DOPRI54 1  /* adaptive Dormand-Prince 5(4) over an interval tau */

/* Interpolation of step 2 (ssm_set_reparam) */
#define SSM_INTERP_LINEAR 0  /* piecewise linear in alpha (default) */
#define SSM_INTERP_SPLINE 1  /* natural cubic spline in alpha */

/* ssm_check flag bits */
#define SSM_FLAG_NONFINITE_ENERGY 1
#define SSM_FLAG_ZERO_NORM_SPIN 2
#define SSM_FLAG_NONFINITE_SPIN 4
#define SSM_FLAG_RK_ERROR 8  /* the integrator's error estimate was not finite */

/* One lattice + parameter set (reduced units, see above).  K = n_images. */
typedef struct {
    int32_t nx, ny, nz;
    int32_t n_images;
    double J;    /* exchange, eq. (1) first term */
    double d;    /* interfacial DMI, eq. (1) second term */
    double ku;   /* uniaxial anisotropy, eq. (1) third term */
    double dip;  /* dipolar strength mu0 |S|^2/(4 pi a^3), eq. (1) last term */
} ssm_problem;

/* Library version (monotonic integer). */
int32_t ssm_version(void);

/* Bytes of device workspace a context for these problems needs.
 * p[n_problems]: problem descriptions (host memory).  precision: SSM_FP64
 * or SSM_FP32_MIXED, optionally | SSM_WITH_RK.  *bytes receives the size.
 * Pure host computation. */
ssm_status ssm_workspace_size(const ssm_problem* p, int32_t n_problems, int32_t precision,
                              size_t* bytes);

/* Create a context over a caller-owned workspace of ws_bytes bytes at
 * d_workspace (256-byte aligned, at least ssm_workspace_size bytes).
 * n_problems > 1 batches several lattices and parameter sets so that every
 * kernel of an iteration covers all of them in one launch.  Builds the FFT
 * of the point-dipole tensor of eq. (7) on the zero-padded grid of every
 * distinct lattice shape (Sec. II.A: the dipolar field as a circular
 * convolution) and synchronises the stream once.  *out receives the
 * context.  The string is undefined until ssm_set_string. */
ssm_status ssm_create(const ssm_problem* p, int32_t n_problems, int32_t precision,
                      void* d_workspace, size_t ws_bytes, void* stream, ssm_ctx** out);

/* Destroy a context (host memory and HIP graph objects only; the workspace
 * stays the caller's).  Waits for the context's stream.  NULL is a no-op. */
ssm_status ssm_destroy(ssm_ctx* ctx);

/* Change the parameters (eq. (1)) of one problem.  Applies to work enqueued
 * afterwards. */
ssm_status ssm_set_params(ssm_ctx* ctx, int32_t problem, double J, double d, double ku,
                          double dip);

/* Copy a whole string (all problems, layout above, spin dtype of the
 * context's precision) from d_spins into the context.  Spins are used as
 * given (not renormalised); they must be unit vectors. */
ssm_status ssm_set_string(ssm_ctx* ctx, const void* d_spins);

/* Copy the current string out to d_spins (same layout and dtype). */
ssm_status ssm_get_string(ssm_ctx* ctx, void* d_spins);

/* Run up to max_iter string iterations (Sec. III) with descent step tau
 * (reduced time units 1/J).  One iteration = field and energy of every image
 * (eqs. (2)-(8)), the projected descent step with renormalisation of every
 * image including both endpoints (eq. (10), Appendix), the arc lengths
 * (eq. (11)) and the interpolation onto alpha_k = k/(K-1) (eq. (12)).
 * tol_force > 0: the perpendicular-force norm (ssm_get_tangents) of the
 * current string is checked every check_every iterations (ssm_set_options)
 * before iterating, and a problem whose norm is below tol_force stops; the
 * call synchronises the stream at every check.  The energies, fields,
 * tangents and barrier of the final string are evaluated when first asked
 * for (ssm_get_energies/fields/tangents/barrier enqueue that evaluation on
 * the stream), so the work this call enqueues is its iterations and
 * convergence checks only.  d_iters_done (device int32[n_problems] or NULL)
 * receives the iterations each problem performed in this call. */
ssm_status ssm_iterate(ssm_ctx* ctx, int32_t max_iter, double tau, double tol_force,
                       int32_t* d_iters_done);

/* Options of step 2 of ssm_iterate (Sec. III: reparametrisation by equal
 * arc length; the paper interpolates linearly and omits the climbing-image
 * refinement of the saddle it mentions).  interp: SSM_INTERP_LINEAR, or
 * SSM_INTERP_SPLINE: every spin component of every site is interpolated by
 * the natural cubic spline through (alpha*_k, phi*_k) (second derivatives
 * zero at both ends) and renormalised; with K = 2 or an interval of zero
 * width a problem falls back to linear interpolation for that iteration.
 * climbing = 1: in every iteration the image k* of highest energy (smallest
 * index on ties), if interior, is stepped with F - 2 (F.t) t instead of F
 * (F = h - (s.h) s its perpendicular force, t the normalised per-spin
 * projection of phi_{k*+1} - phi_{k*-1}) and kept by the reparametrisation,
 * which spaces images 0..k* and k*..K-1 to equal arc length within their
 * own segment.  The climbing image needs SSM_STEP_EULER (ssm_iterate
 * returns SSM_EUNSUPPORTED otherwise).  Both options apply to all
 * problems of the context; the spline uses the field buffer as scratch
 * (ssm_iterate re-evaluates the fields at the end). */
ssm_status ssm_set_reparam(ssm_ctx* ctx, int32_t interp, int32_t climbing);

/* Choose step 1 of ssm_iterate.  SSM_STEP_EULER (default): one projected
 * step of size tau.  SSM_STEP_DOPRI54 (Sec. III: each image evolved over an
 * interval by an explicit embedded Runge-Kutta method with adaptive step
 * size): every image, endpoints included, evolves over the interval tau of
 * ds/dt = -s x (s x h(s)) (the damping term of eq. (9) with its prefactor
 * in the time unit; Appendix) with the Dormand-Prince 5(4) pair, fifth-order
 * solution propagated, first-same-as-last.  Per image: error norm
 * err = RMS over its 3N components of (y5 - y4) / (atol + rtol
 * max(|y|, |y5|)); a step is accepted iff err <= 1; the next step is the
 * attempted one times clamp(0.9 err^(-1/5), 0.2, 5) (at most 1 after a
 * rejection), shortened to end exactly at tau; the proposal carries over
 * to the next iteration.  Stage states are not normalised; every spin is
 * renormalised at the end of the interval.  The energies of an iteration
 * are those of the string before its step (as for the Euler step).  Needs a
 * context created with SSM_WITH_RK (else SSM_EUNSUPPORTED); rtol >= 0,
 * atol > 0, dt0 > 0 (initial step proposal of every image).  Resets the
 * proposals and the statistics of ssm_get_rk_stats.  ssm_iterate then runs
 * without graph replay and synchronises the stream after every attempt
 * (the number of attempts adapts). */
ssm_status ssm_set_integrator(ssm_ctx* ctx, int32_t method, double rtol, double atol, double dt0);

/* Landau-Lifshitz-Gilbert time integration (eq. (9), precession and
 * damping) of every image of the current string over t_total, without the
 * reparametrisation of the string method:
 *   ds/dt = -(s x h)/(1 + alpha^2) - alpha/(1 + alpha^2) s x (s x h)
 * in reduced time (unit mu0 |S| / (gamma J)), with the adaptive
 * Dormand-Prince pair of ssm_set_integrator (its rtol, atol and the
 * per-image step proposals, which carry over); spins are renormalised at
 * the end.  Then evaluates the new string (ssm_get_energies/fields).  Needs
 * SSM_WITH_RK; alpha >= 0 (0: pure precession), t_total > 0.  Synchronises
 * the stream after every attempted step.  The getters evaluate the new
 * string when first called. */
ssm_status ssm_llg(ssm_ctx* ctx, double t_total, double alpha);

/* Integrator statistics since ssm_set_integrator.  d_counts (device
 * int32[sum K][2] or NULL): accepted and rejected steps per image; d_dt
 * (device double[sum K] or NULL): current step proposal per image;
 * h_evals (host, or NULL): field evaluations (of all images at once) done
 * by the integrator.  SSM_EUNSUPPORTED without SSM_WITH_RK. */
ssm_status ssm_get_rk_stats(ssm_ctx* ctx, int32_t* d_counts, double* d_dt, int64_t* h_evals);

/* Evaluate field and energies of a string without changing the context's
 * string.  d_spins: a string in the context layout, or NULL for the
 * current string (which also refreshes what ssm_get_energies/fields/barrier
 * return).  d_field_or_null receives h = -dE/ds (spin layout and dtype).
 * d_energy receives E_k = -1/2 sum h.s per image (eq. (8)), double[sum K].
 * d_terms_or_null receives, per image, the unit-parameter term energies
 * (T_J, T_d, T_ku, T_dip) with E = J T_J + d T_d + ku T_ku + dip T_dip
 * (eq. (1) is linear in each parameter), double[sum K][4]. */
ssm_status ssm_eval(ssm_ctx* ctx, const void* d_spins, void* d_field_or_null,
                    double* d_energy, double* d_terms_or_null);

/* Allocation-free evaluation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same field and energies as ssm_eval, for
 * n_problems (1..16) problems in the batch layout above, with no context
 * and no workspace.  Its scratch (descriptors, twiddles, the kernel spectra
 * of eq. (7), x half-spectra, energy partials) is a fixed device array of
 * SSM_NOALLOC_SCRATCH_MIB MiB inside the library, one per GPU, held until
 * the process ends; the call makes no hipMalloc, hipFree or other allocating
 * call.  d_spins (spin layout and dtype of the precision), d_energy
 * (double[sum K]) and the optional d_field_or_null and d_terms_or_null are
 * the caller's, as in ssm_eval.  Work is enqueued on `stream` (a
 * hipStream_t as void*, NULL = default stream) on the current device.
 * When the problem shapes, image counts or precision differ from the
 * previous call on this device, the call first rebuilds the tables (kernel
 * spectra) and synchronises the stream once; later calls with the same
 * layout are asynchronous, whatever their parameters.  Calls on one device
 * share its scratch: calls that overlap in time on that device (other
 * streams, other host threads' work still running) race and give undefined
 * results.  Returns SSM_EUNSUPPORTED if the problems need more scratch than
 * the fixed size (ssm_workspace_size-sized contexts have no such limit) or
 * n_problems is outside 1..16, SSM_EINVAL for bad arguments; errors are
 * reported by ssm_last_error(NULL). */
#define SSM_NOALLOC_SCRATCH_MIB 64
ssm_status ssm_eval_noalloc(const ssm_problem* p, int32_t n_problems, int32_t precision, const void* d_spins,
                            void* d_field_or_null, double* d_energy, double* d_terms_or_null, void* stream);

/* Energies of the current string (double[sum K]).  Every getter below
 * returns the evaluation of the current string and parameters: if the
 * string or a parameter changed since the last evaluation, the getter first
 * enqueues one (field, energies and term energies of every image).
 * SSM_ESTATE before any ssm_set_string. */
ssm_status ssm_get_energies(ssm_ctx* ctx, double* d_energy);

/* Field h of the current string (spin layout). */
ssm_status ssm_get_fields(ssm_ctx* ctx, void* d_field);

/* Path tangents of the current string and the perpendicular-force norm.
 * An MEP has the potential force parallel to the path (Sec. III).  Tangent
 * t_k: phi_{k+1} - phi_{k-1} (one-sided at the endpoints), each spin's part
 * projected onto that spin's tangent plane, normalised in R^{3N}.  Force:
 * h_perp = h - (s.h)s per spin (Appendix); F_perp = h_perp - (h_perp.t)t
 * for interior images and h_perp at the endpoints.  Uses the field of the
 * current string (evaluated first if needed).  A force that is not finite
 * counts as +infinity, so a diverged problem never passes tol_force.
 * d_tangent (spin layout, or NULL) receives t;
 * d_force_norm_or_null (double[n_problems]) receives
 * max_k max_i |F_perp,k,i| per problem. */
ssm_status ssm_get_tangents(ssm_ctx* ctx, void* d_tangent, double* d_force_norm_or_null);

/* Barrier of every problem for the current string (Sec. III: the energy of
 * the highest image relative to the first).  d_out: double[n_problems][6] =
 * {B = max_k E_k - E_0, argmax k (smallest on ties),
 *  dB/dJ, dB/dd, dB/dku, dB/ddip}; the derivatives are the envelope-theorem
 * values T_theta(k*) - T_theta(0), valid at a converged path. */
ssm_status ssm_get_barrier(ssm_ctx* ctx, double* d_out);

/* Options.  check_every >= 1: iterations between convergence checks
 * (default 10).  graph_chunk >= 0: when > 0, ssm_iterate replays a HIP
 * graph holding graph_chunk iterations instead of launching kernels one by
 * one (default 0). */
ssm_status ssm_set_options(ssm_ctx* ctx, int32_t check_every, int32_t graph_chunk);

/* Time the candidate tile shapes of the x-transform and convolution kernels
 * on this context's problems and keep the fastest.  Uses the current string
 * as input and leaves it unchanged; synchronises the stream.  cache_path
 * (or NULL): a text file of previous results keyed by device name, precision
 * and lattice shape; read if present, appended with new results. */
ssm_status ssm_autotune(ssm_ctx* ctx, const char* cache_path);

/* Synchronise the stream and read the sticky failure flags into *h_flags,
 * then clear them.  Kernels set SSM_FLAG_NONFINITE_ENERGY on a non-finite
 * image energy; SSM_FLAG_NONFINITE_SPIN when a spin they renormalise (an
 * interpolated spin, or an image at the end of an integrator interval) has
 * a non-finite norm; SSM_FLAG_ZERO_NORM_SPIN when that norm is below 1e-12
 * (an interpolated spin then takes the nearer source image's spin);
 * SSM_FLAG_RK_ERROR when the integrator's error estimate is not finite.
 * Returns SSM_ENONFINITE when SSM_FLAG_NONFINITE_ENERGY or
 * SSM_FLAG_NONFINITE_SPIN is set. */
ssm_status ssm_check(ssm_ctx* ctx, int32_t* h_flags);

/* Text of the last error on this context ("" if none).  ctx may be NULL for
 * errors of ssm_create. */
const char* ssm_last_error(const ssm_ctx* ctx);

/* Kernel timing.  enable != 0: every kernel launch is bracketed by HIP
 * events on the context's stream (graph replay is then replaced by direct
 * launches).  ssm_profile_read synchronises, adds the elapsed times per
 * kernel kind since enabling into h_ms[SSM_N_KERNELS] (milliseconds) and
 * h_counts[SSM_N_KERNELS] (launches), and resets the accumulators. */
#define SSM_N_KERNELS 13
ssm_status ssm_profile(ssm_ctx* ctx, int32_t enable);
ssm_status ssm_profile_read(ssm_ctx* ctx, double* h_ms, int32_t* h_counts);

/* Name of kernel kind i (0 <= i < SSM_N_KERNELS), or NULL. */
const char* ssm_kernel_name(int32_t i);

#ifdef __cplusplus
}
#endif

#endif /* SSM_H */
