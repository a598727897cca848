/* Drives every entry point of the oracle (oracle/oracle.c) on small inputs
 * so that an AddressSanitizer + UndefinedBehaviorSanitizer build reports any
 * out-of-bounds access, use of freed memory or undefined operation.  Test
 * infrastructure: compiled and run by tests/test_sanitize.py.  Prints OK
 * when every result is finite. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_version(void);
void oracle_energy_terms(int nx, int ny, int nz, const double* s, double* T);
double oracle_energy(int nx, int ny, int nz, double J, double d, double k, double D, const double* s);
void oracle_field(int nx, int ny, int nz, double J, double d, double k, double D, const double* s, double* h);
void oracle_field_at(int nx, int ny, int nz, double J, double d, double k, double D, const double* s,
                     const int64_t* sites, int64_t nsites, double* hout);
double oracle_energy_from_field(int64_t N, const double* s, const double* h);
void oracle_step(int64_t N, int K, const double* s, const double* h, double tau, double* s_star);
int oracle_reparam(int K, int64_t N, const double* s_star, double* s_out, double* alpha_star, int32_t* jidx,
                   double* wts);
double oracle_force_norm(int K, int64_t N, const double* s, const double* h, double* t_or_null);
int oracle_iterate(int nx, int ny, int nz, double J, double d, double k, double D, int K, int max_iter,
                   double tau, double tol, int every, double* s, double* E, double* h_or_null, double* fn);
void oracle_dopri_tableau(double* a, double* b, double* bs, double* c);
int oracle_llg_interval(int nx, int ny, int nz, double J, double d, double k, double D, double cp, double cd,
                        double* y, double T, double rtol, double atol, double* dtp, int64_t* n_acc,
                        int64_t* n_rej, int max_steps);
int oracle_iterate_rk(int nx, int ny, int nz, double J, double d, double k, double D, int K, int max_iter,
                      double T, double rtol, double atol, double tol, int every, double* s, double* E,
                      double* h_or_null, double* fn, double* dtp, int64_t* stats);
int oracle_spline_eval(int K, const double* x, const double* f, int nt, const double* t, double* out);
void oracle_climb_step(int64_t N, const double* s_prev, const double* s, const double* s_next, const double* h,
                       double tau, double* out);
int oracle_reparam_opts(int K, int64_t N, const double* s_star, double* s_out, double* alpha_star,
                        int32_t* jidx, double* wts, int spline, int kci);
int oracle_iterate_opts(int nx, int ny, int nz, double J, double d, double k, double D, int K, int max_iter,
                        double tau, double tol, int every, int spline, int climb, double* s, double* E,
                        double* h_or_null, double* fn);

static int bad = 0;
static void check(const char* what, const double* a, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) { printf("non-finite %s[%lld]\n", what, (long long)i); bad = 1; return; }
}

/* K images of unit spins on an nx*ny*nz lattice, rotating from -z to +z */
static double* string_of(int nx, int ny, int nz, int K)
{
    const int64_t N = (int64_t)nx * ny * nz;
    double* s = (double*)malloc((size_t)K * 3 * N * sizeof(double));
    for (int k = 0; k < K; ++k)
        for (int64_t i = 0; i < N; ++i) {
            const double th = 3.14159265358979 * (1.0 - (double)k / (K - 1)) + 0.01 * (double)(i % 7);
            const double ph = 0.3 * (double)i;
            s[(k * 3 + 0) * N + i] = sin(th) * cos(ph);
            s[(k * 3 + 1) * N + i] = sin(th) * sin(ph);
            s[(k * 3 + 2) * N + i] = cos(th);
        }
    return s;
}

int main(void)
{
    const int nx = 5, ny = 3, nz = 2, K = 5;
    const int64_t N = (int64_t)nx * ny * nz, M = 3 * N;
    double* s = string_of(nx, ny, nz, K);
    double* h = (double*)malloc((size_t)K * M * sizeof(double));
    double* ss = (double*)malloc((size_t)K * M * sizeof(double));
    double* out = (double*)malloc((size_t)K * M * sizeof(double));
    double T[4], E[K], al[K], w[K], fn = 0;
    int32_t j[K];
    printf("oracle version %d\n", oracle_version());
    oracle_energy_terms(nx, ny, nz, s, T);
    check("terms", T, 4);
    double e = oracle_energy(nx, ny, nz, 1.0, 0.3, 0.1, 0.02, s);
    check("energy", &e, 1);
    for (int k = 0; k < K; ++k) oracle_field(nx, ny, nz, 1.0, 0.3, 0.1, 0.02, s + k * M, h + k * M);
    check("field", h, K * M);
    int64_t sites[3] = {0, N / 2, N - 1};
    double hs[9];
    oracle_field_at(nx, ny, nz, 1.0, 0.3, 0.1, 0.02, s, sites, 3, hs);
    check("field_at", hs, 9);
    e = oracle_energy_from_field(N, s, h);
    check("energy_from_field", &e, 1);
    oracle_step(N, K, s, h, 0.1, ss);
    check("step", ss, K * M);
    oracle_reparam(K, N, ss, out, al, j, w);
    check("reparam", out, K * M);
    double* t = (double*)malloc((size_t)K * M * sizeof(double));
    fn = oracle_force_norm(K, N, s, h, t);
    check("force", &fn, 1);
    for (int spline = 0; spline < 2; ++spline)
        for (int kci = -1; kci < K; kci += 2) {
            oracle_reparam_opts(K, N, ss, out, al, j, w, spline, kci);
            check("reparam_opts", out, K * M);
        }
    double x[6] = {0, 0.1, 0.3, 0.35, 0.8, 1.0}, f[6] = {1, 2, 0, -1, 3, 2}, tq[4] = {0, 0.2, 0.9, 1.0}, o[4];
    oracle_spline_eval(6, x, f, 4, tq, o);
    check("spline", o, 4);
    oracle_climb_step(N, s, s + M, s + 2 * M, h + M, 0.1, out);
    check("climb", out, M);
    double a[49], b[7], bs[7], c[7];
    oracle_dopri_tableau(a, b, bs, c);
    double* s2 = string_of(nx, ny, nz, K);
    oracle_iterate(nx, ny, nz, 1.0, 0.3, 0.1, 0.02, K, 3, 0.1, 1e-9, 1, s2, E, h, &fn);
    check("iterate", s2, K * M);
    double* s3 = string_of(nx, ny, nz, K);
    oracle_iterate_opts(nx, ny, nz, 1.0, 0.3, 0.1, 0.02, K, 3, 0.1, 1e-9, 1, 1, 1, s3, E, h, &fn);
    check("iterate_opts", s3, K * M);
    double* s4 = string_of(nx, ny, nz, K);
    double dtp[K];
    int64_t st[2 * K];
    for (int k = 0; k < K; ++k) dtp[k] = 0.05;
    for (int k = 0; k < 2 * K; ++k) st[k] = 0;
    oracle_iterate_rk(nx, ny, nz, 1.0, 0.3, 0.1, 0.02, K, 2, 0.3, 1e-6, 1e-6, 0.0, 1, s4, E, h, &fn, dtp, st);
    check("iterate_rk", s4, K * M);
    double dt1 = 0.05;
    int64_t na = 0, nr = 0;
    oracle_llg_interval(nx, ny, nz, 1.0, 0.3, 0.1, 0.02, 0.5, 0.5, s4, 0.4, 1e-6, 1e-6, &dt1, &na, &nr, 100000);
    check("llg", s4, M);
    /* more images than the GPU path accepts: buffers sized by K */
    const int Kb = 1500;
    double* sb = string_of(1, 1, 1, Kb);
    double* ob = (double*)malloc((size_t)Kb * 3 * sizeof(double));
    double* alb = (double*)malloc((size_t)Kb * sizeof(double));
    double* wb = (double*)malloc((size_t)Kb * sizeof(double));
    int32_t* jb = (int32_t*)malloc((size_t)Kb * sizeof(int32_t));
    oracle_reparam_opts(Kb, 1, sb, ob, alb, jb, wb, 1, Kb / 3);
    check("reparam_opts_K1500", ob, Kb * 3);
    free(s); free(h); free(ss); free(out); free(t); free(s2); free(s3); free(s4);
    free(sb); free(ob); free(alb); free(wb); free(jb);
    if (bad) return 1;
    printf("OK\n");
    return 0;
}
