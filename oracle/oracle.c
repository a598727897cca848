/*
 * FP64 CPU oracle for the simplified string method on an atomistic spin
 * lattice (Heistracher et al., "GPU Accelerated Atomistic Energy Barrier
 * Calculations of Skyrmion Annihilations", arXiv:1804.07135).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so, which
 * only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load.  The product library never links, loads or calls it, and it shares
 * no source with the HIP path.
 *
 * Plain, slow, obviously correct: every quantity is FP64, the dipolar field
 * and energy are direct O(N^2) sums over all site pairs (no FFT), and every
 * sum over sites is a fixed-order pairwise sum so results do not depend on
 * the OpenMP thread count.
 *
 * Units and conventions (reduced units; lattice constant 1, unit spins):
 *   - spins of one image are stored SoA: s[c*N + (z*ny + y)*nx + x],
 *     c = 0,1,2 for the x,y,z components, N = nx*ny*nz; images follow each
 *     other with stride 3N.
 *   - the field is h = mu0*|S|*H_eff = -dE/ds (Sec. II.A, eq. (2)), so the
 *     paper's prefactors 1/(mu0 |S|) disappear.
 *   - D = mu0 |S|^2 / (4 pi a^3) is the reduced dipolar strength, so one
 *     unordered pair contributes -D [3(s_i.r)(s_j.r) - s_i.s_j]/r^3
 *     (last term of eq. (1); the 1/(8 pi) over ordered pairs is 1/(4 pi)
 *     over unordered ones).
 *   - nearest-neighbour bonds <i,j> are counted once each; open boundaries,
 *     missing neighbours contribute nothing (Sec. II: free boundaries).
 *
 * Parity unpinned by the paper: the adaptive step controller's constants
 * (safety factor 0.9, step-factor bounds 0.2 and 5, exponent -1/5; the
 * paper names Dormand-Prince with step control but no controller) and every
 * barrier value (the paper prints none).  They are pinned only by behaviour
 * (tableau order conditions, step response, single-spin closed forms) and
 * through the pinned parts they are built from.
 *
 * Every function below names the passage of the paper it follows.
 * Parity pins for each function live in tests/test_oracle_pins.py (field,
 * energy, step, reparametrisation, tangents), test_oracle_rk_pins.py and
 * test_oracle_llg_pins.py (integrators) and test_oracle_reparam_pins.py
 * (spline and climbing image).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_VERSION 4

int oracle_version(void) { return ORACLE_VERSION; }

/* ------------------------------------------------------------------ */
/* fixed-order pairwise summation                                       */
/* ------------------------------------------------------------------ */
static double psum(const double* a, int64_t n)
{
    if (n <= 0) return 0.0;
    if (n <= 16) {
        double t = 0.0;
        for (int64_t i = 0; i < n; ++i) t += a[i];
        return t;
    }
    int64_t h = n / 2;
    return psum(a, h) + psum(a + h, n - h);
}

static inline int64_t site(int nx, int ny, int x, int y, int z)
{
    return ((int64_t)z * ny + y) * nx + x;
}

/* ------------------------------------------------------------------ */
/* Term energies, written as the bond and pair sums of eq. (1).         */
/* T[0] = -sum_bonds s_i.s_j                       (exchange, per unit J)
 * T[1] =  sum_bonds (r_ij x z).(s_i x s_j)        (DMI, per unit d)
 * T[2] = -sum_i (s_i.z)^2                         (anisotropy, per unit k)
 * T[3] = -sum_{i<j} [3(s_i.r)(s_j.r) - s_i.s_j]/r^3 (dipolar, per unit D)
 * E = J*T[0] + d*T[1] + k*T[2] + D*T[3].
 * These never touch the field code, so they pin it by finite differences. */
/* ------------------------------------------------------------------ */
void oracle_energy_terms(int nx, int ny, int nz, const double* s, double* T)
{
    const int64_t N = (int64_t)nx * ny * nz;
    const double* sx = s;
    const double* sy = s + N;
    const double* sz = s + 2 * N;
    double* ex = (double*)calloc((size_t)N, sizeof(double));
    double* dm = (double*)calloc((size_t)N, sizeof(double));
    double* an = (double*)calloc((size_t)N, sizeof(double));
    double* dd = (double*)calloc((size_t)N, sizeof(double));

    /* local terms: each site owns the bonds to its +x, +y, +z neighbour */
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        int x = (int)(i % nx);
        int y = (int)((i / nx) % ny);
        int z = (int)(i / ((int64_t)nx * ny));
        double e_ex = 0.0, e_dm = 0.0;
        const int dx[3] = {1, 0, 0}, dy[3] = {0, 1, 0}, dz[3] = {0, 0, 1};
        for (int b = 0; b < 3; ++b) {
            int xj = x + dx[b], yj = y + dy[b], zj = z + dz[b];
            if (xj >= nx || yj >= ny || zj >= nz) continue;
            int64_t j = site(nx, ny, xj, yj, zj);
            e_ex -= sx[i] * sx[j] + sy[i] * sy[j] + sz[i] * sz[j];
            /* DMI vector r_ij x z: x-bond -> (0,-1,0), y-bond -> (1,0,0),
             * z-bond -> 0.  (s_i x s_j) written out component by component. */
            double cx = sy[i] * sz[j] - sz[i] * sy[j];
            double cy = sz[i] * sx[j] - sx[i] * sz[j];
            double rx = (double)dx[b], ry = (double)dy[b];
            /* (r x z) = (ry, -rx, 0) */
            e_dm += ry * cx - rx * cy;
        }
        ex[i] = e_ex;
        dm[i] = e_dm;
        an[i] = -sz[i] * sz[i];
    }

    /* dipolar: unordered pairs i<j, charged to the lower site */
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < N; ++i) {
        int xi = (int)(i % nx);
        int yi = (int)((i / nx) % ny);
        int zi = (int)(i / ((int64_t)nx * ny));
        double acc = 0.0;
        for (int64_t j = i + 1; j < N; ++j) {
            int xj = (int)(j % nx);
            int yj = (int)((j / nx) % ny);
            int zj = (int)(j / ((int64_t)nx * ny));
            double rx = xj - xi, ry = yj - yi, rz = zj - zi;
            double r2 = rx * rx + ry * ry + rz * rz;
            double r = sqrt(r2);
            double ux = rx / r, uy = ry / r, uz = rz / r;
            double si_u = sx[i] * ux + sy[i] * uy + sz[i] * uz;
            double sj_u = sx[j] * ux + sy[j] * uy + sz[j] * uz;
            double si_sj = sx[i] * sx[j] + sy[i] * sy[j] + sz[i] * sz[j];
            acc -= (3.0 * si_u * sj_u - si_sj) / (r2 * r);
        }
        dd[i] = acc;
    }

    T[0] = psum(ex, N);
    T[1] = psum(dm, N);
    T[2] = psum(an, N);
    T[3] = psum(dd, N);
    free(ex); free(dm); free(an); free(dd);
}

double oracle_energy(int nx, int ny, int nz, double J, double d, double k,
                     double D, const double* s)
{
    double T[4];
    oracle_energy_terms(nx, ny, nz, s, T);
    return J * T[0] + d * T[1] + k * T[2] + D * T[3];
}

/* ------------------------------------------------------------------ */
/* Effective field h_i = -dE/ds_i at one site.                          */
/*   exchange   eq. (3):  J * sum over nearest neighbours of s_j
 *   DMI        eq. (4):  -d (s^z_{+x}-s^z_{-x}, s^z_{+y}-s^z_{-y},
 *                            -s^x_{+x}+s^x_{-x}-s^y_{+y}+s^y_{-y})
 *   anisotropy eq. (5):  2k s^z z
 *   dipolar    eqs. (6)-(7): D sum_{j != i} (3 r r^T/r^5 - I/r^3) s_j
 * Missing neighbours (open boundary) contribute 0.                     */
/* ------------------------------------------------------------------ */
static void field_at(int nx, int ny, int nz, double J, double d, double k,
                     double D, const double* s, int64_t i, double* hout)
{
    const int64_t N = (int64_t)nx * ny * nz;
    const double* sx = s;
    const double* sy = s + N;
    const double* sz = s + 2 * N;
    int x = (int)(i % nx);
    int y = (int)((i / nx) % ny);
    int z = (int)(i / ((int64_t)nx * ny));

    /* neighbour values, 0 where the neighbour is outside the sample */
    double px[3] = {0, 0, 0}, mx[3] = {0, 0, 0};
    double py[3] = {0, 0, 0}, my[3] = {0, 0, 0};
    double pz[3] = {0, 0, 0}, mz[3] = {0, 0, 0};
    int64_t j;
    if (x + 1 < nx) { j = site(nx, ny, x + 1, y, z); px[0] = sx[j]; px[1] = sy[j]; px[2] = sz[j]; }
    if (x - 1 >= 0) { j = site(nx, ny, x - 1, y, z); mx[0] = sx[j]; mx[1] = sy[j]; mx[2] = sz[j]; }
    if (y + 1 < ny) { j = site(nx, ny, x, y + 1, z); py[0] = sx[j]; py[1] = sy[j]; py[2] = sz[j]; }
    if (y - 1 >= 0) { j = site(nx, ny, x, y - 1, z); my[0] = sx[j]; my[1] = sy[j]; my[2] = sz[j]; }
    if (z + 1 < nz) { j = site(nx, ny, x, y, z + 1); pz[0] = sx[j]; pz[1] = sy[j]; pz[2] = sz[j]; }
    if (z - 1 >= 0) { j = site(nx, ny, x, y, z - 1); mz[0] = sx[j]; mz[1] = sy[j]; mz[2] = sz[j]; }

    double h[3];
    for (int c = 0; c < 3; ++c)
        h[c] = J * (px[c] + mx[c] + py[c] + my[c] + pz[c] + mz[c]);

    h[0] += -d * (px[2] - mx[2]);
    h[1] += -d * (py[2] - my[2]);
    h[2] += -d * (-px[0] + mx[0] - py[1] + my[1]);

    h[2] += 2.0 * k * sz[i];

    if (D != 0.0) {
        double ax = 0.0, ay = 0.0, az = 0.0;
        for (int64_t jj = 0; jj < N; ++jj) {
            if (jj == i) continue;
            int xj = (int)(jj % nx);
            int yj = (int)((jj / nx) % ny);
            int zj = (int)(jj / ((int64_t)nx * ny));
            double rx = xj - x, ry = yj - y, rz = zj - z;
            double r2 = rx * rx + ry * ry + rz * rz;
            double r = sqrt(r2);
            double r3 = r2 * r, r5 = r3 * r2;
            double rs = rx * sx[jj] + ry * sy[jj] + rz * sz[jj];
            ax += 3.0 * rx * rs / r5 - sx[jj] / r3;
            ay += 3.0 * ry * rs / r5 - sy[jj] / r3;
            az += 3.0 * rz * rs / r5 - sz[jj] / r3;
        }
        h[0] += D * ax;
        h[1] += D * ay;
        h[2] += D * az;
    }
    hout[0] = h[0];
    hout[1] = h[1];
    hout[2] = h[2];
}

/* Field of one image, all sites; h has the spin layout. */
void oracle_field(int nx, int ny, int nz, double J, double d, double k,
                  double D, const double* s, double* h)
{
    const int64_t N = (int64_t)nx * ny * nz;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < N; ++i) {
        double hi[3];
        field_at(nx, ny, nz, J, d, k, D, s, i, hi);
        h[i] = hi[0];
        h[N + i] = hi[1];
        h[2 * N + i] = hi[2];
    }
}

/* Field at a list of sites only (for sampled checks on large lattices);
 * hout is [nsites][3]. */
void oracle_field_at(int nx, int ny, int nz, double J, double d, double k,
                     double D, const double* s, const int64_t* sites,
                     int64_t nsites, double* hout)
{
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < nsites; ++q)
        field_at(nx, ny, nz, J, d, k, D, s, sites[q], hout + 3 * q);
}

/* E = -1/2 sum_i h_i . s_i  (eq. (8); exact for this Hamiltonian, whose
 * terms are all homogeneous quadratic in the spins). */
double oracle_energy_from_field(int64_t N, const double* s, const double* h)
{
    double* e = (double*)malloc((size_t)N * sizeof(double));
    for (int64_t i = 0; i < N; ++i)
        e[i] = -0.5 * (h[i] * s[i] + h[N + i] * s[N + i] + h[2 * N + i] * s[2 * N + i]);
    double E = psum(e, N);
    free(e);
    return E;
}

/* ------------------------------------------------------------------ */
/* String method step 1 (Sec. III, eq. (10); force from the Appendix):  */
/* the potential force on a unit spin is the field's component          */
/* perpendicular to the spin, h - (s.h)s = -s x (s x h).  One explicit  */
/* Euler step of length tau followed by renormalisation to |s| = 1.     */
/* ------------------------------------------------------------------ */
void oracle_step(int64_t N, int K, const double* s, const double* h,
                 double tau, double* s_star)
{
    #pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < (int64_t)K * N; ++q) {
        int64_t kk = q / N, i = q % N;
        const double* sk = s + kk * 3 * N;
        const double* hk = h + kk * 3 * N;
        double* ok = s_star + kk * 3 * N;
        double v[3] = {sk[i], sk[N + i], sk[2 * N + i]};
        double f[3] = {hk[i], hk[N + i], hk[2 * N + i]};
        double sh = v[0] * f[0] + v[1] * f[1] + v[2] * f[2];
        double w[3];
        for (int c = 0; c < 3; ++c) w[c] = v[c] + tau * (f[c] - sh * v[c]);
        double nrm = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        for (int c = 0; c < 3; ++c) ok[c * N + i] = w[c] / nrm;
    }
}

/* ------------------------------------------------------------------ */
/* String method step 2 (Sec. III, eqs. (11)-(12)): arc length,         */
/* normalised parameters, interpolation onto the uniform grid.          */
/* Readings where the text is garbled or silent:                        */
/*   - eq. (12) divides by the last arc length S_{K-1};                 */
/*   - the uniform grid is alpha_k = k/(K-1), so both endpoints stay;   */
/*   - interpolation is piecewise linear in alpha, component by         */
/*     component, followed by per-spin renormalisation; a spin whose    */
/*     interpolated norm is below 1e-12 takes the nearer source spin;   */
/*   - a zero-width interval gives weight 0; S_{K-1} = 0 skips the      */
/*     reparametrisation (s_out = s_star).                              */
/* alpha_star[K], jidx[K], wts[K] receive the parameters used.          */
/* Returns 1 if the reparametrisation was applied, 0 if skipped.        */
/* ------------------------------------------------------------------ */
int oracle_reparam(int K, int64_t N, const double* s_star, double* s_out,
                   double* alpha_star, int32_t* jidx, double* wts)
{
    const int64_t M = 3 * N;
    double* seg = (double*)malloc((size_t)K * sizeof(double));
    double* sq = (double*)malloc((size_t)M * sizeof(double));
    seg[0] = 0.0;
    for (int kk = 1; kk < K; ++kk) {
        const double* a = s_star + (int64_t)kk * M;
        const double* b = s_star + (int64_t)(kk - 1) * M;
        for (int64_t q = 0; q < M; ++q) {
            double t = a[q] - b[q];
            sq[q] = t * t;
        }
        seg[kk] = sqrt(psum(sq, M));
    }
    double* S = (double*)malloc((size_t)K * sizeof(double));
    S[0] = 0.0;
    for (int kk = 1; kk < K; ++kk) S[kk] = S[kk - 1] + seg[kk];
    double L = S[K - 1];
    if (!(L > 0.0)) {
        for (int kk = 0; kk < K; ++kk) {
            alpha_star[kk] = 0.0;
            jidx[kk] = kk;
            wts[kk] = 0.0;
        }
        memcpy(s_out, s_star, (size_t)K * M * sizeof(double));
        free(seg); free(sq); free(S);
        return 0;
    }
    for (int kk = 0; kk < K; ++kk) alpha_star[kk] = S[kk] / L;

    for (int kk = 0; kk < K; ++kk) {
        if (kk == 0 || kk == K - 1) {
            jidx[kk] = kk;
            wts[kk] = 0.0;
            memcpy(s_out + (int64_t)kk * M, s_star + (int64_t)kk * M, (size_t)M * sizeof(double));
            continue;
        }
        double t = (double)kk / (double)(K - 1);
        int j = 0;
        for (int jj = 0; jj <= K - 2; ++jj)
            if (alpha_star[jj] <= t) j = jj;
        double width = alpha_star[j + 1] - alpha_star[j];
        double w = (width > 0.0) ? (t - alpha_star[j]) / width : 0.0;
        jidx[kk] = j;
        wts[kk] = w;
        const double* a = s_star + (int64_t)j * M;
        const double* b = s_star + (int64_t)(j + 1) * M;
        double* o = s_out + (int64_t)kk * M;
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            double v[3];
            for (int c = 0; c < 3; ++c) v[c] = (1.0 - w) * a[c * N + i] + w * b[c * N + i];
            double nrm = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            if (nrm < 1e-12) {
                const double* src = (w < 0.5) ? a : b;
                for (int c = 0; c < 3; ++c) o[c * N + i] = src[c * N + i];
            } else {
                for (int c = 0; c < 3; ++c) o[c * N + i] = v[c] / nrm;
            }
        }
    }
    free(seg); free(sq); free(S);
    return 1;
}

/* ------------------------------------------------------------------ */
/* Path tangents and the perpendicular-force norm.  An MEP is a path    */
/* along which the potential force is parallel to the path (Sec. III),  */
/* so convergence is measured by the force component perpendicular to   */
/* it:                                                                  */
/*   h_perp = h - (s.h)s per spin (Appendix, force equation);           */
/*   tangent t_k: phi_{k+1}-phi_{k-1} (one-sided at the ends), each     */
/*     spin's part projected onto that spin's tangent plane, then       */
/*     normalised in R^{3N} (t = 0 if its norm is 0);                   */
/*   F_perp = h_perp - (h_perp . t) t for interior images, h_perp at    */
/*     the endpoints;                                                   */
/*   norm = max over images and sites of |F_perp| per spin.             */
/* s, h: [K][3N]; tangents_or_null: [K][3N].                            */
/* ------------------------------------------------------------------ */
double oracle_force_norm(int K, int64_t N, const double* s, const double* h,
                         double* tangents_or_null)
{
    const int64_t M = 3 * N;
    double* tt = (double*)malloc((size_t)M * sizeof(double));
    double* hp = (double*)malloc((size_t)M * sizeof(double));
    double* buf = (double*)malloc((size_t)N * sizeof(double));
    double worst = 0.0;
    for (int kk = 0; kk < K; ++kk) {
        const double* sk = s + (int64_t)kk * M;
        const double* hk = h + (int64_t)kk * M;
        int kp = (kk + 1 < K) ? kk + 1 : kk;
        int km = (kk - 1 >= 0) ? kk - 1 : kk;
        const double* sp = s + (int64_t)kp * M;
        const double* sm = s + (int64_t)km * M;
        for (int64_t i = 0; i < N; ++i) {
            double v[3] = {sk[i], sk[N + i], sk[2 * N + i]};
            double f[3] = {hk[i], hk[N + i], hk[2 * N + i]};
            double dlt[3];
            for (int c = 0; c < 3; ++c) dlt[c] = sp[c * N + i] - sm[c * N + i];
            double sh = v[0] * f[0] + v[1] * f[1] + v[2] * f[2];
            double sd = v[0] * dlt[0] + v[1] * dlt[1] + v[2] * dlt[2];
            for (int c = 0; c < 3; ++c) {
                hp[c * N + i] = f[c] - sh * v[c];
                tt[c * N + i] = dlt[c] - sd * v[c];
            }
        }
        for (int64_t i = 0; i < N; ++i)
            buf[i] = tt[i] * tt[i] + tt[N + i] * tt[N + i] + tt[2 * N + i] * tt[2 * N + i];
        double tn = sqrt(psum(buf, N));
        double inv = (tn > 0.0) ? 1.0 / tn : 0.0;
        for (int64_t q = 0; q < M; ++q) tt[q] *= inv;
        int interior = (kk > 0 && kk < K - 1);
        double proj = 0.0;
        if (interior) {
            for (int64_t i = 0; i < N; ++i)
                buf[i] = hp[i] * tt[i] + hp[N + i] * tt[N + i] + hp[2 * N + i] * tt[2 * N + i];
            proj = psum(buf, N);
        }
        for (int64_t i = 0; i < N; ++i) {
            double fx = hp[i] - proj * tt[i];
            double fy = hp[N + i] - proj * tt[N + i];
            double fz = hp[2 * N + i] - proj * tt[2 * N + i];
            double n = sqrt(fx * fx + fy * fy + fz * fz);
            if (n > worst) worst = n;
        }
        if (tangents_or_null)
            memcpy(tangents_or_null + (int64_t)kk * M, tt, (size_t)M * sizeof(double));
    }
    free(tt); free(hp); free(buf);
    return worst;
}

/* ------------------------------------------------------------------ */
/* The two-step string iteration of Sec. III, repeated.                 */
/*   for each iteration: field and energy of every image (eqs. (2)-(8)),*/
/*   descent step of every image including the endpoints (eq. (10)),    */
/*   reparametrisation (eqs. (11)-(12)).                                */
/* Convergence (tol > 0): before iterations 0, every, 2*every, ... the  */
/* perpendicular-force norm of the current string is computed; the run  */
/* stops when it is below tol.  After the loop the final string is      */
/* evaluated once more: E[K] and (optionally) h[K][3N] are its energies */
/* and fields.  s[K][3N] is updated in place.  Returns iterations done. */
/* ------------------------------------------------------------------ */
int oracle_iterate(int nx, int ny, int nz, double J, double d, double k,
                   double D, int K, int max_iter, double tau, double tol,
                   int every, double* s, double* E, double* h_or_null,
                   double* force_norm_out)
{
    const int64_t N = (int64_t)nx * ny * nz;
    const int64_t M = 3 * N;
    double* h = (double*)malloc((size_t)K * M * sizeof(double));
    double* ss = (double*)malloc((size_t)K * M * sizeof(double));
    double* al = (double*)malloc((size_t)K * sizeof(double));
    double* wt = (double*)malloc((size_t)K * sizeof(double));
    int32_t* jj = (int32_t*)malloc((size_t)K * sizeof(int32_t));
    int it = 0;
    double fn = -1.0;
    if (every < 1) every = 1;
    for (;;) {
        if (tol > 0.0 && it % every == 0) {
            for (int kk = 0; kk < K; ++kk)
                oracle_field(nx, ny, nz, J, d, k, D, s + kk * M, h + kk * M);
            fn = oracle_force_norm(K, N, s, h, NULL);
            if (fn < tol) break;
        }
        if (it >= max_iter) break;
        for (int kk = 0; kk < K; ++kk)
            oracle_field(nx, ny, nz, J, d, k, D, s + kk * M, h + kk * M);
        oracle_step(N, K, s, h, tau, ss);
        oracle_reparam(K, N, ss, s, al, jj, wt);
        ++it;
    }
    for (int kk = 0; kk < K; ++kk) {
        oracle_field(nx, ny, nz, J, d, k, D, s + kk * M, h + kk * M);
        E[kk] = oracle_energy_from_field(N, s + kk * M, h + kk * M);
    }
    if (h_or_null) memcpy(h_or_null, h, (size_t)K * M * sizeof(double));
    if (force_norm_out) *force_norm_out = oracle_force_norm(K, N, s, h, NULL);
    free(h); free(ss); free(al); free(wt); free(jj);
    return it;
}

/* ------------------------------------------------------------------------
 * Step 1 with the paper's integrator (Sec. III): every image is evolved
 * over an interval T of the damping-only dynamics (second term of eq. (9);
 * the Appendix identifies it with the potential force) by an explicit
 * embedded Runge-Kutta method with adaptive step size, here Dormand and
 * Prince's 5(4) pair (J. Comput. Appl. Math. 6 (1980) 19), local
 * extrapolation (the 5th-order solution is kept), first stage of a step =
 * last stage of the accepted step before.  The prefactor gamma alpha /
 * (1 + alpha^2) is absorbed into the time unit, as for the explicit step.
 *
 *   ds/dt = f(s) = -s x (s x h(s)) = (s.s) h - (s.h) s   (per spin)
 *
 * Error control (Hairer, Norsett, Wanner, Solving ODEs I, II.4), per image:
 *   err = sqrt(mean over the 3N components of (e_c / sc_c)^2),
 *   e = y5 - y4, sc_c = atol + rtol max(|y_c|, |y5_c|);
 *   accepted iff err <= 1;  h_new = h * clamp(0.9 err^(-1/5), 0.2, 5)
 *   (at most 1 after a rejection), h the step just attempted;
 *   a step is shortened to end exactly at T.
 * The stage states are not normalised; after the interval every spin is
 * renormalised (the exact flow keeps |s| = 1).
 * ---------------------------------------------------------------------- */
static const double DP_A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
/* 5th-order weights (= last row of A, weight 0 on the last stage) and the
 * embedded 4th-order weights */
static const double DP_B[7] = {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84, 0};
static const double DP_BS[7] = {5179.0 / 57600, 0, 7571.0 / 16695, 393.0 / 640,
                                -92097.0 / 339200, 187.0 / 2100, 1.0 / 40};
static const double DP_C[7] = {0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1, 1};

/* Tableau for the pins: a[49] row-major (7 x 7, zero above the diagonal),
 * b[7], bs[7], c[7]. */
void oracle_dopri_tableau(double* a, double* b, double* bs, double* c)
{
    for (int i = 0; i < 7; ++i) {
        for (int j = 0; j < 7; ++j) a[i * 7 + j] = (j < 6) ? DP_A[i][j] : 0.0;
        b[i] = DP_B[i];
        bs[i] = DP_BS[i];
        c[i] = DP_C[i];
    }
}

/* Right-hand side of eq. (9) in reduced time (unit mu0|S| / (gamma J)):
 *   ds/dt = -cp (s x h) - cd s x (s x h) = -cp (s x h) + cd ((s.s) h - (s.h) s)
 * with cp = 1/(1+alpha^2), cd = alpha/(1+alpha^2) for the full LLG equation,
 * and cp = 0, cd = 1 for the damping term alone (step 1 of the string
 * method, whose prefactor is absorbed into the time unit).  One image (SoA
 * [3][N]); h receives the field of y. */
void oracle_llg_rhs(int nx, int ny, int nz, double J, double d, double k, double D, double cp, double cd,
                    const double* y, double* f, double* h)
{
    const int64_t N = (int64_t)nx * ny * nz;
    oracle_field(nx, ny, nz, J, d, k, D, y, h);
    for (int64_t i = 0; i < N; ++i) {
        const double v[3] = {y[i], y[N + i], y[2 * N + i]};
        const double w[3] = {h[i], h[N + i], h[2 * N + i]};
        const double ss = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        const double sh = v[0] * w[0] + v[1] * w[1] + v[2] * w[2];
        const double x[3] = {v[1] * w[2] - v[2] * w[1], v[2] * w[0] - v[0] * w[2], v[0] * w[1] - v[1] * w[0]};
        for (int c = 0; c < 3; ++c) f[c * N + i] = cd * (ss * w[c] - sh * v[c]) - cp * x[c];
    }
}

/* the damping term alone (step 1 of the string method) */
void oracle_rk_rhs(int nx, int ny, int nz, double J, double d, double k, double D,
                   const double* y, double* f, double* h)
{
    oracle_llg_rhs(nx, ny, nz, J, d, k, D, 0.0, 1.0, y, f, h);
}

/* One attempted step of size hs from y.  kk[0..6]: stage slopes, kk[0] =
 * f(y) on entry; on return kk[6] = f(y5).  y5 receives the 5th-order
 * solution; returns the scaled error norm. */
static double dopri_attempt(int nx, int ny, int nz, double J, double d, double k, double D,
                            double cp, double cd, const double* y, double hs, double* kk[7], double* y5,
                            double* hscr, double rtol, double atol)
{
    const int64_t M = 3 * (int64_t)nx * ny * nz;
    for (int i = 1; i < 7; ++i) {
        for (int64_t m = 0; m < M; ++m) {
            double acc = 0.0;
            for (int j = 0; j < i; ++j) acc += DP_A[i][j] * kk[j][m];
            y5[m] = y[m] + hs * acc;
        }
        oracle_llg_rhs(nx, ny, nz, J, d, k, D, cp, cd, y5, kk[i], hscr);
    }
    /* y5 now holds the last stage's input, which is the 5th-order solution */
    double sq = 0.0;
    for (int64_t m = 0; m < M; ++m) {
        double e = 0.0;
        for (int j = 0; j < 7; ++j) e += (DP_B[j] - DP_BS[j]) * kk[j][m];
        e *= hs;
        const double sc = atol + rtol * fmax(fabs(y[m]), fabs(y5[m]));
        sq += (e / sc) * (e / sc);
    }
    return sqrt(sq / (double)M);
}

/* Fixed-size Dormand-Prince steps (no control) for the order pins: n steps
 * of size hs from y (in place), no renormalisation.  Returns the error
 * estimate norm of the last step (rtol = 0, atol = 1: the RMS of e). */
double oracle_dopri_fixed(int nx, int ny, int nz, double J, double d, double k, double D,
                          double* y, double hs, int n)
{
    const int64_t M = 3 * (int64_t)nx * ny * nz;
    double* kk[7];
    for (int i = 0; i < 7; ++i) kk[i] = (double*)malloc((size_t)M * sizeof(double));
    double* y5 = (double*)malloc((size_t)M * sizeof(double));
    double* hscr = (double*)malloc((size_t)M * sizeof(double));
    double err = 0.0;
    for (int st = 0; st < n; ++st) {
        oracle_rk_rhs(nx, ny, nz, J, d, k, D, y, kk[0], hscr);
        err = dopri_attempt(nx, ny, nz, J, d, k, D, 0.0, 1.0, y, hs, kk, y5, hscr, 0.0, 1.0);
        memcpy(y, y5, (size_t)M * sizeof(double));
    }
    for (int i = 0; i < 7; ++i) free(kk[i]);
    free(y5);
    free(hscr);
    return err;
}

/* Evolve one image y (in place) over T with step control; *dtp is the
 * proposed step size (in: start, out: proposal for the next interval).
 * n_acc, n_rej accumulate the accepted and rejected steps.  Returns 0, or
 * -1 if max_steps attempts did not reach T. */
int oracle_llg_interval(int nx, int ny, int nz, double J, double d, double k, double D, double cp,
                        double cd, double* y, double T, double rtol, double atol, double* dtp,
                        int64_t* n_acc, int64_t* n_rej, int max_steps)
{
    const int64_t N = (int64_t)nx * ny * nz, M = 3 * N;
    double* kk[7];
    for (int i = 0; i < 7; ++i) kk[i] = (double*)malloc((size_t)M * sizeof(double));
    double* y5 = (double*)malloc((size_t)M * sizeof(double));
    double* hscr = (double*)malloc((size_t)M * sizeof(double));
    oracle_llg_rhs(nx, ny, nz, J, d, k, D, cp, cd, y, kk[0], hscr);
    double t = 0.0;
    int done = 0, steps = 0, rc = 0;
    while (!done) {
        if (steps++ >= max_steps) { rc = -1; break; }
        const int capped = (*dtp >= T - t);
        const double hs = capped ? T - t : *dtp;
        const double err = dopri_attempt(nx, ny, nz, J, d, k, D, cp, cd, y, hs, kk, y5, hscr, rtol, atol);
        double fac = 0.9 * pow(fmax(err, 1e-10), -0.2);
        fac = fmin(5.0, fmax(0.2, fac));
        if (err <= 1.0) {
            memcpy(y, y5, (size_t)M * sizeof(double));
            double* tmp = kk[0];
            kk[0] = kk[6];
            kk[6] = tmp;
            if (capped) done = 1;
            else t += hs;
            ++*n_acc;
        } else {
            fac = fmin(fac, 1.0);
            ++*n_rej;
        }
        *dtp = hs * fac;
    }
    for (int64_t i = 0; i < N; ++i) {
        const double nrm = sqrt(y[i] * y[i] + y[N + i] * y[N + i] + y[2 * N + i] * y[2 * N + i]);
        for (int c = 0; c < 3; ++c) y[c * N + i] /= nrm;
    }
    for (int i = 0; i < 7; ++i) free(kk[i]);
    free(y5);
    free(hscr);
    return rc;
}

/* step 1 of the string method: the damping term alone */
int oracle_rk_interval(int nx, int ny, int nz, double J, double d, double k, double D,
                       double* y, double T, double rtol, double atol, double* dtp,
                       int64_t* n_acc, int64_t* n_rej, int max_steps)
{
    return oracle_llg_interval(nx, ny, nz, J, d, k, D, 0.0, 1.0, y, T, rtol, atol, dtp, n_acc, n_rej,
                               max_steps);
}

/* The string iteration of oracle_iterate with step 1 done by
 * oracle_rk_interval over T for every image (dtp[K]: per-image step
 * proposals, in/out; stats[2K]: accepted, rejected steps per image,
 * accumulated).  Returns the iterations done, or -1 on a failed interval. */
int oracle_iterate_rk(int nx, int ny, int nz, double J, double d, double k, double D, int K,
                      int max_iter, double T, double rtol, double atol, double tol, int every,
                      double* s, double* E, double* h_or_null, double* force_norm_out,
                      double* dtp, int64_t* stats)
{
    const int64_t N = (int64_t)nx * ny * nz;
    const int64_t M = 3 * N;
    double* h = (double*)malloc((size_t)K * M * sizeof(double));
    double* ss = (double*)malloc((size_t)K * M * sizeof(double));
    double* al = (double*)malloc((size_t)K * sizeof(double));
    double* wt = (double*)malloc((size_t)K * sizeof(double));
    int32_t* jj = (int32_t*)malloc((size_t)K * sizeof(int32_t));
    int it = 0;
    if (every < 1) every = 1;
    for (;;) {
        if (tol > 0.0 && it % every == 0) {
            for (int kk = 0; kk < K; ++kk)
                oracle_field(nx, ny, nz, J, d, k, D, s + kk * M, h + kk * M);
            if (oracle_force_norm(K, N, s, h, NULL) < tol) break;
        }
        if (it >= max_iter) break;
        memcpy(ss, s, (size_t)K * M * sizeof(double));
        for (int kk = 0; kk < K; ++kk) {
            if (oracle_rk_interval(nx, ny, nz, J, d, k, D, ss + kk * M, T, rtol, atol, &dtp[kk],
                                   &stats[2 * kk], &stats[2 * kk + 1], 1000000) != 0) {
                it = -1;
                goto out;
            }
        }
        oracle_reparam(K, N, ss, s, al, jj, wt);
        ++it;
    }
    for (int kk = 0; kk < K; ++kk) {
        oracle_field(nx, ny, nz, J, d, k, D, s + kk * M, h + kk * M);
        E[kk] = oracle_energy_from_field(N, s + kk * M, h + kk * M);
    }
    if (h_or_null) memcpy(h_or_null, h, (size_t)K * M * sizeof(double));
    if (force_norm_out) *force_norm_out = oracle_force_norm(K, N, s, h, NULL);
out:
    free(h); free(ss); free(al); free(wt); free(jj);
    return it;
}

/* ------------------------------------------------------------------------
 * Variants of step 2 (Sec. III).  The paper interpolates piecewise linearly
 * and omits the climbing-image refinement of the saddle it mentions; both
 * options are provided:
 *  - interpolation by a natural cubic spline in alpha through the images,
 *    per site and spin component (second derivatives from the tridiagonal
 *    system that makes the first derivative continuous, zero at both ends;
 *    Numerical Recipes 3.3), then renormalisation;
 *  - a climbing image: the image k* of highest energy (smallest index on
 *    ties), if interior, is stepped with F - 2 (F.t) t, F = h - (s.h) s its
 *    perpendicular force and t its tangent (per-spin projection of
 *    phi_{k*+1} - phi_{k*-1}, normalised over the image), and is kept fixed
 *    by the reparametrisation, which spaces images 0..k* and k*..K-1 to
 *    equal arc length within their own segment.
 * ---------------------------------------------------------------------- */

/* Natural cubic spline through (x_k, f_k), k < K, x strictly increasing,
 * evaluated at t[0..nt-1] (t in [x_0, x_{K-1}]).  Returns 1, or 0 when it
 * fell back to linear interpolation (K == 2 or an interval of zero width). */
int oracle_spline_eval(int K, const double* x, const double* f, int nt, const double* t, double* out)
{
    int ok = (K > 2);
    for (int j = 0; j + 1 < K; ++j)
        if (!(x[j + 1] - x[j] > 0.0)) ok = 0;
    double* M = (double*)calloc((size_t)K, sizeof(double));
    if (ok) {
        double* cp = (double*)calloc((size_t)K, sizeof(double));
        double* dp = (double*)calloc((size_t)K, sizeof(double));
        for (int i = 1; i <= K - 2; ++i) {
            const double hl = x[i] - x[i - 1], hr = x[i + 1] - x[i];
            const double a = hl / 6.0, b = (hl + hr) / 3.0, c = hr / 6.0;
            const double r = (f[i + 1] - f[i]) / hr - (f[i] - f[i - 1]) / hl;
            const double den = b - (i > 1 ? a * cp[i - 1] : 0.0);
            cp[i] = c / den;
            dp[i] = (r - (i > 1 ? a * dp[i - 1] : 0.0)) / den;
        }
        M[K - 2] = dp[K - 2];
        for (int i = K - 3; i >= 1; --i) M[i] = dp[i] - cp[i] * M[i + 1];
        free(cp);
        free(dp);
    }
    for (int q = 0; q < nt; ++q) {
        int j = 0;
        for (int jj = 0; jj <= K - 2; ++jj)
            if (x[jj] <= t[q]) j = jj;
        const double h = x[j + 1] - x[j];
        if (!(h > 0.0)) {
            out[q] = f[j];
            continue;
        }
        const double A = (x[j + 1] - t[q]) / h, B = 1.0 - A;
        out[q] = A * f[j] + B * f[j + 1];
        if (ok) out[q] += ((A * A * A - A) * M[j] + (B * B * B - B) * M[j + 1]) * h * h / 6.0;
    }
    free(M);
    return ok;
}

/* Climbing-image step of one image s (neighbours s_prev, s_next, field h)
 * with step tau: out = normalise(s + tau (F - 2 (F.t) t)). */
void oracle_climb_step(int64_t N, const double* s_prev, const double* s, const double* s_next,
                       const double* h, double tau, double* out)
{
    const int64_t M = 3 * N;
    double* tt = (double*)malloc((size_t)M * sizeof(double));
    double* F = (double*)malloc((size_t)M * sizeof(double));
    double* buf = (double*)malloc((size_t)N * sizeof(double));
    for (int64_t i = 0; i < N; ++i) {
        double v[3] = {s[i], s[N + i], s[2 * N + i]};
        double f[3] = {h[i], h[N + i], h[2 * N + i]};
        double dl[3];
        for (int c = 0; c < 3; ++c) dl[c] = s_next[c * N + i] - s_prev[c * N + i];
        const double sh = v[0] * f[0] + v[1] * f[1] + v[2] * f[2];
        const double sd = v[0] * dl[0] + v[1] * dl[1] + v[2] * dl[2];
        for (int c = 0; c < 3; ++c) {
            F[c * N + i] = f[c] - sh * v[c];
            tt[c * N + i] = dl[c] - sd * v[c];
        }
    }
    for (int64_t i = 0; i < N; ++i) buf[i] = tt[i] * tt[i] + tt[N + i] * tt[N + i] + tt[2 * N + i] * tt[2 * N + i];
    const double tn2 = psum(buf, N);
    for (int64_t i = 0; i < N; ++i) buf[i] = F[i] * tt[i] + F[N + i] * tt[N + i] + F[2 * N + i] * tt[2 * N + i];
    const double ft = psum(buf, N);
    const double cc = (tn2 > 0.0) ? ft / tn2 : 0.0;  /* (F.t) t = cc t~ */
    for (int64_t i = 0; i < N; ++i) {
        double w[3];
        for (int c = 0; c < 3; ++c) w[c] = s[c * N + i] + tau * (F[c * N + i] - 2.0 * cc * tt[c * N + i]);
        const double nrm = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        for (int c = 0; c < 3; ++c) out[c * N + i] = w[c] / nrm;
    }
    free(tt); free(F); free(buf);
}

/* Step 2 with the options: spline (0 linear, 1 natural cubic spline) and
 * kci (climbing image index, or -1).  Same outputs as oracle_reparam (for
 * the spline, jidx/wts are the intervals and linear weights used for the
 * renormalisation guard).  Returns 1 if applied, 0 if the total arc length
 * was zero (string copied). */
int oracle_reparam_opts(int K, int64_t N, const double* s_star, double* s_out, double* alpha_star,
                        int32_t* jidx, double* wts, int spline, int kci)
{
    const int64_t M = 3 * N;
    double* seg = (double*)malloc((size_t)K * sizeof(double));
    double* sq = (double*)malloc((size_t)M * sizeof(double));
    seg[0] = 0.0;
    for (int kk = 1; kk < K; ++kk) {
        const double* a = s_star + (int64_t)kk * M;
        const double* b = s_star + (int64_t)(kk - 1) * M;
        for (int64_t q = 0; q < M; ++q) sq[q] = (a[q] - b[q]) * (a[q] - b[q]);
        seg[kk] = sqrt(psum(sq, M));
    }
    double* S = (double*)malloc((size_t)K * sizeof(double));
    S[0] = 0.0;
    for (int kk = 1; kk < K; ++kk) S[kk] = S[kk - 1] + seg[kk];
    const double L = S[K - 1];
    free(seg);
    free(sq);
    if (!(L > 0.0)) {
        for (int kk = 0; kk < K; ++kk) { alpha_star[kk] = 0.0; jidx[kk] = kk; wts[kk] = 0.0; }
        memcpy(s_out, s_star, (size_t)K * M * sizeof(double));
        free(S);
        return 0;
    }
    for (int kk = 0; kk < K; ++kk) alpha_star[kk] = S[kk] / L;
    free(S);
    const int ci = (kci > 0 && kci < K - 1);
    double* tk = (double*)malloc((size_t)K * sizeof(double));
    for (int kk = 0; kk < K; ++kk) {
        if (!ci) tk[kk] = (double)kk / (double)(K - 1);
        else if (kk <= kci) tk[kk] = alpha_star[kci] * (double)kk / (double)kci;
        else tk[kk] = alpha_star[kci] + (1.0 - alpha_star[kci]) * (double)(kk - kci) / (double)(K - 1 - kci);
    }
    for (int kk = 0; kk < K; ++kk) {
        int j = 0;
        for (int jj = 0; jj <= K - 2; ++jj)
            if (alpha_star[jj] <= tk[kk]) j = jj;
        const double width = alpha_star[j + 1] - alpha_star[j];
        jidx[kk] = j;
        wts[kk] = (width > 0.0) ? (tk[kk] - alpha_star[j]) / width : 0.0;
    }
    /* endpoints and the climbing image are copied */
    for (int kk = 0; kk < K; ++kk) {
        if (kk == 0 || kk == K - 1 || (ci && kk == kci)) {
            jidx[kk] = kk;
            wts[kk] = 0.0;
            memcpy(s_out + (int64_t)kk * M, s_star + (int64_t)kk * M, (size_t)M * sizeof(double));
        }
    }
    #pragma omp parallel
    {
        double* fv = (double*)malloc((size_t)K * sizeof(double));
        double* ov = (double*)malloc((size_t)K * sizeof(double));
        /* interpolated (unnormalised) spin of every target image at site i,
         * sized by K (no limit on the number of images) */
        double (*v)[3] = (double (*)[3])malloc((size_t)K * sizeof(*v));
        #pragma omp for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            for (int c = 0; c < 3; ++c) {
                if (spline) {
                    for (int kk = 0; kk < K; ++kk) fv[kk] = s_star[(int64_t)kk * M + c * N + i];
                    oracle_spline_eval(K, alpha_star, fv, K, tk, ov);
                    for (int kk = 0; kk < K; ++kk) v[kk][c] = ov[kk];
                } else {
                    /* interior targets only: the endpoints are copied, and
                     * the last one's interval index is K-1 (no image K) */
                    for (int kk = 1; kk < K - 1; ++kk) {
                        const double w = wts[kk];
                        v[kk][c] = (1.0 - w) * s_star[(int64_t)jidx[kk] * M + c * N + i] +
                                   w * s_star[(int64_t)(jidx[kk] + 1) * M + c * N + i];
                    }
                }
            }
            for (int kk = 1; kk < K - 1; ++kk) {
                if (ci && kk == kci) continue;
                double* o = s_out + (int64_t)kk * M;
                const double nrm = sqrt(v[kk][0] * v[kk][0] + v[kk][1] * v[kk][1] + v[kk][2] * v[kk][2]);
                if (nrm < 1e-12) {
                    const double* src = s_star + (int64_t)(wts[kk] < 0.5 ? jidx[kk] : jidx[kk] + 1) * M;
                    for (int c = 0; c < 3; ++c) o[c * N + i] = src[c * N + i];
                } else {
                    for (int c = 0; c < 3; ++c) o[c * N + i] = v[kk][c] / nrm;
                }
            }
        }
        free(fv);
        free(ov);
        free(v);
    }
    free(tk);
    return 1;
}

/* oracle_iterate with the step-2 options (spline, climbing image). */
int oracle_iterate_opts(int nx, int ny, int nz, double J, double d, double k, double D, int K, int max_iter,
                        double tau, double tol, int every, int spline, int climb, double* s, double* E,
                        double* h_or_null, double* force_norm_out)
{
    const int64_t N = (int64_t)nx * ny * nz;
    const int64_t M = 3 * N;
    double* h = (double*)malloc((size_t)K * M * sizeof(double));
    double* ss = (double*)malloc((size_t)K * M * sizeof(double));
    double* al = (double*)malloc((size_t)K * sizeof(double));
    double* wt = (double*)malloc((size_t)K * sizeof(double));
    double* Ek = (double*)malloc((size_t)K * sizeof(double));
    int32_t* jj = (int32_t*)malloc((size_t)K * sizeof(int32_t));
    int it = 0;
    if (every < 1) every = 1;
    for (;;) {
        if (tol > 0.0 && it % every == 0) {
            for (int kk = 0; kk < K; ++kk)
                oracle_field(nx, ny, nz, J, d, k, D, s + kk * M, h + kk * M);
            if (oracle_force_norm(K, N, s, h, NULL) < tol) break;
        }
        if (it >= max_iter) break;
        for (int kk = 0; kk < K; ++kk) {
            oracle_field(nx, ny, nz, J, d, k, D, s + kk * M, h + kk * M);
            Ek[kk] = oracle_energy_from_field(N, s + kk * M, h + kk * M);
        }
        oracle_step(N, K, s, h, tau, ss);
        int kci = -1;
        if (climb) {
            int km = 0;
            for (int kk = 1; kk < K; ++kk)
                if (Ek[kk] > Ek[km]) km = kk;
            if (km > 0 && km < K - 1) {
                kci = km;
                oracle_climb_step(N, s + (km - 1) * M, s + km * M, s + (km + 1) * M, h + km * M, tau,
                                  ss + km * M);
            }
        }
        oracle_reparam_opts(K, N, ss, s, al, jj, wt, spline, kci);
        ++it;
    }
    for (int kk = 0; kk < K; ++kk) {
        oracle_field(nx, ny, nz, J, d, k, D, s + kk * M, h + kk * M);
        E[kk] = oracle_energy_from_field(N, s + kk * M, h + kk * M);
    }
    if (h_or_null) memcpy(h_or_null, h, (size_t)K * M * sizeof(double));
    if (force_norm_out) *force_norm_out = oracle_force_norm(K, N, s, h, NULL);
    free(h); free(ss); free(al); free(wt); free(Ek); free(jj);
    return it;
}
