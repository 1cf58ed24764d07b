/*
 * Address- and undefined-behaviour-sanitizer run of the FP64 oracle
 * (test infrastructure): built together with isis_oracle.c under
 * -fsanitize=address,undefined by tests/test_sanitizers.py, it calls every
 * entry point of the oracle on small grids (each model's solve, the level
 * operators, both restrictions, the force, the masked patch operators and
 * their solve) and checks that the results are finite.  Any out-of-bounds
 * access, leak or undefined operation aborts the run.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int model;
    double a, lambda0, a_ssb, n, fR0_abs, omega_m, omega_l, kappa, m2, beta, cham_alpha, cham_mu,
        cham_n;
    int paper_u;
} orc_model;
typedef struct {
    int nu_pre, nu_post, nu_coarse, max_cycles, restrict_fw, prolong_w;
} orc_cfg;
typedef struct {
    int cycles;
    double r_ref, r0, rel_hist[256], wall_s;
    long long guard_hits;
} orc_stats;

int orc_solve(const orc_model*, const orc_cfg*, int, double, const double*, double*, int, double,
              orc_stats*);
void orc_defect(const orc_model*, int, double, const double*, const double*, const double*,
                double*);
void orc_newton_diag(const orc_model*, int, double, const double*, const double*, double*);
void orc_halfsweep(const orc_model*, int, double, double*, const double*, const double*, int);
void orc_restrict(int, const double*, double*);
void orc_restrict_fw(int, const double*, double*);
void orc_prolong_correct(int, double*, const double*, const double*);
void orc_prolong_correct_w(int, double*, const double*, const double*);
void orc_cold_start(const orc_model*, long, const double*, double*);
double orc_rms(int, const double*);
void orc_force(const orc_model*, int, double, const double*, const double*, double*, double*,
               double*);
void orc_masked_defect(const orc_model*, int, double, const double*, const double*,
                       const double*, const double*, const double*, const double*, double*);
void orc_masked_halfsweep(const orc_model*, int, double, double*, const double*, const double*,
                          const double*, const double*, const double*, int);
int orc_patch_solve(const orc_model*, int, double, double*, const double*, const double*,
                    const double*, int, int, double, double*);

static int fails = 0;
static void check_finite(const char* what, const double* v, long count)
{
    for (long q = 0; q < count; ++q)
        if (!isfinite(v[q])) {
            printf("FAIL %s: non-finite value at %ld\n", what, q);
            ++fails;
            return;
        }
}

static double* field(long count, unsigned seed, double lo, double hi)
{
    double* v = (double*)malloc(sizeof(double) * (size_t)count);
    unsigned s = seed;
    for (long q = 0; q < count; ++q) {
        s = s * 1664525u + 1013904223u;
        v[q] = lo + (hi - lo) * (double)(s >> 8) / 16777216.0;
    }
    return v;
}

int main(void)
{
    const int n = 16;
    const long n3 = (long)n * n * n;
    const double box = 16.0, h = box / n;
    orc_model models[4];
    memset(models, 0, sizeof(models));
    models[0] = (orc_model){0, 1.0, 1.0, 0.5, 1.0, 1e-5, 0.27, 0.73, 1.0, 0.0, 1.0, 1.0, 1.0, 1.0, 0};
    models[1] = (orc_model){1, 1.0, 1.0, 0.5, 1.0, 1e-5, 0.27, 0.73, 1.0, 0.0, 1.0, 1.0, 1.0, 1.0, 0};
    models[2] = (orc_model){2, 1.0, 1.0, 0.5, 1.0, 1e-5, 0.27, 0.73, 1.3, 0.4, 1.0, 1.0, 1.0, 1.0, 0};
    models[3] = (orc_model){3, 1.0, 1.0, 0.5, 1.0, 1e-5, 0.27, 0.73, 1.0, 0.0, 1.0, 2.0, 3.0, 1.0, 0};
    double* eta = field(n3, 7, 0.2, 3.0);
    double* phi = (double*)malloc(sizeof(double) * (size_t)n3);
    double* out = (double*)malloc(sizeof(double) * (size_t)n3);
    double* fx = (double*)malloc(sizeof(double) * (size_t)n3);
    double* fy = (double*)malloc(sizeof(double) * (size_t)n3);
    double* fz = (double*)malloc(sizeof(double) * (size_t)n3);
    double* coarse = (double*)malloc(sizeof(double) * (size_t)(n3 / 8));
    double* coarse2 = (double*)malloc(sizeof(double) * (size_t)(n3 / 8));
    for (int mi = 0; mi < 4; ++mi) {
        for (int opt = 0; opt < 6; ++opt) {
            const int fw = opt % 3, pw = opt / 3;  /* pw: only the flux-form models use it */
            orc_cfg cfg = {2, 2, 32, 40, fw, pw};
            orc_stats st;
            int rc = orc_solve(&models[mi], &cfg, n, box, eta, phi, 0, 1e-9, &st);
            if (rc != 0) {
                printf("FAIL solve model %d fw %d pw %d: status %d\n", mi, fw, pw, rc);
                ++fails;
            }
            check_finite("solve", phi, n3);
        }
        orc_defect(&models[mi], n, h, phi, eta, NULL, out);
        check_finite("defect", out, n3);
        orc_newton_diag(&models[mi], n, h, phi, eta, out);
        check_finite("newton_diag", out, n3);
        orc_halfsweep(&models[mi], n, h, phi, eta, out, 1);
        check_finite("halfsweep", phi, n3);
        orc_cold_start(&models[mi], n3, eta, out);
        check_finite("cold_start", out, n3);
        if (mi != 3) {
            orc_force(&models[mi], n, h, phi, eta, fx, fy, fz);
            check_finite("force", fx, n3);
        }
    }
    orc_restrict(n, eta, coarse);
    orc_restrict_fw(n, eta, coarse2);
    orc_prolong_correct(n, phi, coarse, coarse2);
    orc_prolong_correct_w(n, phi, coarse, coarse2);
    check_finite("transfers", phi, n3);
    if (!(orc_rms(n, phi) > 0.0)) ++fails;
    /* masked patch operators: inside 4..11, fractional masks outside */
    double* mask = field(n3, 11, -1.0, 0.0);
    double* u_int = field(n3, 12, 0.4, 0.9);
    double* u_pre = field(n3, 13, 0.4, 0.9);
    for (long i = 0; i < n; ++i)
        for (long j = 0; j < n; ++j)
            for (long k = 0; k < n; ++k)
                if (i >= 4 && i < 12 && j >= 4 && j < 12 && k >= 4 && k < 12)
                    mask[(i * n + j) * n + k] = 1.0;
    for (int mi = 0; mi < 4; ++mi) {
        double* p = field(n3, 20 + mi, 0.4, 0.9);
        orc_masked_defect(&models[mi], n, h, p, eta, NULL, mask, u_int, u_pre, out);
        check_finite("masked_defect", out, n3);
        orc_masked_halfsweep(&models[mi], n, h, p, eta, NULL, mask, u_int, u_pre, 0);
        check_finite("masked_halfsweep", p, n3);
        double rms = 0.0;
        int sw = orc_patch_solve(&models[mi], n, h, p, eta, mask, u_int, 4, 400, 1e-9, &rms);
        if (sw < 0 || !isfinite(rms)) {
            printf("FAIL patch_solve model %d\n", mi);
            ++fails;
        }
        free(p);
    }
    free(mask);
    free(u_int);
    free(u_pre);
    free(eta);
    free(phi);
    free(out);
    free(fx);
    free(fy);
    free(fz);
    free(coarse);
    free(coarse2);
    printf("sanitized oracle run: %d failures\n", fails);
    return fails ? 1 : 0;
}
