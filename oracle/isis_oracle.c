/*
 * FP64 CPU oracle for the nonlinear FAS multigrid solve of the quasi-static
 * scalar-field equation of Llinares, Mota & Winther (ISIS, arXiv:1307.6748).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * Everything is double precision, written as plain loops in the order in
 * which the paper states the algorithm:
 *   - 7-point Laplacian, Sec. 3.1 (eq. disc_lap);
 *   - FAS: L(phi, rho) = Sigma, Sigma = 0 on the finest grid and
 *     Sigma = -R[eps(phi,rho)] + eps(R phi, R rho) on coarser grids,
 *     eps = L - Sigma, Sigma built only on the way fine -> coarse (Sec. 3.2);
 *   - Newton-Gauss-Seidel update phi <- phi - (L - Sigma) / (dL/dphi)
 *     with dSigma/dphi = 0 (Sec. 3.2);
 *   - canonical Jacobian dL/dphi = -6/h^2 - dS/dphi (Sec. 3.3);
 *   - non-canonical flux form with arithmetic face averages of b(u) and
 *     its Jacobian (Sec. 3.4, eqs. disc_non_canonical and dbeq);
 *   - symmetron source (Sec. 4.1, dimensionless equation
 *     symmetron_dimensionles);
 *   - Hu-Sawicki f(R) in the non-canonical variable with b(u) = e^u
 *     (Sec. 4.2), solved in the shifted variable u = ln(f_R / f_R0);
 *   - V-cycle over all levels (Sec. 3.1, last paragraph).
 *
 * Readings of points the paper leaves open (the same readings are listed in
 * the design notes and used by the GPU path):
 *   R1  eps(R phi, R rho) is the coarse operator applied to the restricted
 *       fields with no coarse Sigma; R[eps] restricts the fine defect L - Sigma.
 *   R2  R is the mean of the 8 children; P is cell-centred trilinear
 *       interpolation (weights 27, 9, 3, 1 over 64) with periodic wrap.
 *       Option (orc_cfg.restrict_fw): the defect is restricted by full
 *       weighting, the adjoint of P over 8 (weights 1, 3, 3, 1 over 8 per
 *       axis on the 4 fine cells 2I-1 .. 2I+2); phi and rho keep the mean.
 *       Option (orc_cfg.restrict_fw = 2): full weighting in the first two
 *       V-cycles of a solve, the mean after them.
 *       Option (orc_cfg.prolong_w, flux-form models): P weighted by the
 *       coefficient b = e^u of the restricted field, see
 *       orc_prolong_correct_w.
 *   R3  The non-canonical operator carries the 1/h^2 that its Jacobian has.
 *   R4  The db/du term of the Jacobian carries the factor 1/2 that follows
 *       from differentiating the arithmetic face average.
 *   R5  f(R) is solved in u = ln(f_R/f_R0) = u_paper - ln(a^2 |f_R0|).
 *   R6  Lengths in comoving Mpc/h, c = 1, H0 = 1/2997.92458 h/Mpc.
 *   R7  Gauss-Seidel order is red-black: colour (i+j+k) mod 2, colour 0 first.
 *   R8  The coarsest grid (4^3) gets a fixed number of red-black sweeps.
 *   R9  Stop test: RMS of L_0(phi) relative to r_ref, the RMS of L_0 at the
 *       pointwise homogeneous root (the cold start), whatever the guess.  If
 *       r_ref <= 1e-14 (6/h^2) RMS(cold start) the cold start is an exact
 *       root up to rounding and the tolerance is absolute.
 *   R10 Symmetron Newton denominator is safeguarded as -6/h^2 - |dS/dphi|.
 *   R11 LINEAR with m2 = 0 is singular; its mean is removed after each cycle.
 *   R12 Forces on the grid use second-order central differences, periodic.
 *   R13 The chameleon (Sec. 6: lap phi = beta rho / M_pl - M^{4+n} / phi^{1+n}),
 *       with the free source written in code units as
 *       lap phi = alpha eta - mu phi^{-(1+n)}, is solved for psi = ln phi, the
 *       field redefinition of Sec. 4.2: lap e^psi = div(e^psi grad psi), so
 *       the non-canonical discretisation of Sec. 3.4 applies with b = e^psi,
 *       and S = alpha eta - mu e^{-(1+n) psi}.  phi = e^psi > 0 throughout.
 *   R14 f(R) in the paper's own variable (Sec. 4.2, f_R = -a^-2 e^u) uses
 *       the right-hand side exactly as the paper prints it.
 *   R15 A chameleon Gauss-Seidel step is bounded to |d psi| <= 2.  Where psi
 *       sits far above its local root, dS/dpsi is exponentially small and a
 *       full Newton step overshoots until e^{-(1+n) psi} overflows.  The bound
 *       changes the iteration only, not its fixed point.
 *
 * Built with -O2 -ffp-contract=off (no fused multiply-add, no fast-math).
 * OpenMP parallelises loops whose iterations are independent (one colour of
 * a red-black sweep, pointwise operators); reductions are taken over fixed
 * x-slabs and summed in slab order, so results do not depend on the thread
 * count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define ORC_SYMMETRON 0
#define ORC_FR_HS 1
#define ORC_LINEAR 2
#define ORC_CHAMELEON 3

/* Bound on one chameleon Gauss-Seidel step in psi (reading R15). */
#define ORC_CHAM_MAX_STEP 2.0

#define ORC_OK 0
#define ORC_INVALID (-1)
#define ORC_NOT_CONVERGED (-2)
#define ORC_DIVERGED (-3)

#define ORC_MAX_HIST 256

/* H0 in h/Mpc with c = 1 (reading R6). */
static const double ORC_H0 = 1.0 / 2997.92458;

typedef struct {
    int model;      /* ORC_SYMMETRON, ORC_FR_HS or ORC_LINEAR               */
    double a;       /* expansion factor                                      */
    double lambda0; /* symmetron vacuum range, Mpc/h                         */
    double a_ssb;   /* symmetron symmetry-breaking expansion factor          */
    double n;       /* Hu-Sawicki exponent                                   */
    double fR0_abs; /* |f_R0|                                                */
    double omega_m; /* matter density parameter                              */
    double omega_l; /* cosmological-constant density parameter               */
    double kappa;   /* LINEAR: S = m2 phi + kappa (eta - 1)                  */
    double m2;
    double beta;    /* symmetron coupling (enters the fifth force only)      */
    double cham_alpha; /* CHAMELEON: S = alpha eta - mu phi^{-(1+n)}          */
    double cham_mu;
    double cham_n;     /* exponent n (> -1)                                   */
    int paper_u;       /* FR_HS: field in the paper's u = ln(a^2 |f_R|)       */
} orc_model;

typedef struct {
    int nu_pre, nu_post, nu_coarse, max_cycles;
    int restrict_fw; /* 1: full-weighting restriction of the defect (reading R2);
                        2: full weighting in the first two V-cycles of the solve,
                        the mean of the children after them                      */
    int prolong_w;   /* 1: coefficient-weighted prolongation (reading R2; f(R),
                        chameleon: b = e^u of coarse_hat)                          */
} orc_cfg;

typedef struct {
    int cycles;
    double r_ref;                  /* RMS of L_0 at the cold start          */
    double r0;                     /* RMS of L_0 at the initial field       */
    double rel_hist[ORC_MAX_HIST]; /* rel. residual before cycle 1, after each cycle */
    double wall_s;
    long long guard_hits;          /* symmetron updates with the safeguarded
                                      denominator (reading R10), all levels      */
} orc_stats;

/* Running count of symmetron Gauss-Seidel updates at which dS/dchi < 0, i.e.
 * where the safeguarded denominator of reading R10 differs from the Jacobian.
 * Reset and reported by orc_solve; readable with orc_guard_hits(). */
static long long g_guard_hits = 0;

long long orc_guard_hits(int reset)
{
    long long v = g_guard_hits;
    if (reset) g_guard_hits = 0;
    return v;
}

/* ------------------------------------------------------------------ */
/* Pointwise source S(phi, eta) and its derivative dS/dphi.            */
/* ------------------------------------------------------------------ */

/* Symmetron, Sec. 4.1: laplacian chi = a^2/(2 lambda0^2) [ (a_ssb/a)^3 eta chi - chi + chi^3 ]. */
static void src_symmetron(const orc_model* m, double chi, double eta, double* S, double* dS)
{
    double K = m->a * m->a / (2.0 * m->lambda0 * m->lambda0);
    double r = m->a_ssb / m->a;
    double A = r * r * r;
    *S = K * (A * eta * chi - chi + chi * chi * chi);
    *dS = K * (A * eta - 1.0 + 3.0 * chi * chi);
}

/* Hu-Sawicki f(R), Sec. 4.2, right-hand side of the non-canonical equation
 * rewritten for u = ln(f_R/f_R0) (reading R5): dividing the paper's equation
 * by a^2 |f_R0| gives
 *   div(e^u grad u) = Q [ eta + cL a^3 - a^3 (1 + cL) e^{-u/(n+1)} ],
 *   Q = Omega_m H0^2 / (a |f_R0|),  cL = 4 Omega_L / Omega_m. */
static void src_fr(const orc_model* m, double u, double eta, double* S, double* dS)
{
    double Q = m->omega_m * ORC_H0 * ORC_H0 / (m->a * m->fR0_abs);
    double cL = 4.0 * m->omega_l / m->omega_m;
    double a3 = m->a * m->a * m->a;
    double e = exp(-u / (m->n + 1.0));
    *S = Q * (eta + cL * a3 - a3 * (1.0 + cL) * e);
    *dS = Q * a3 * (1.0 + cL) * e / (m->n + 1.0);
}

/* Hu-Sawicki f(R) in the paper's own variable u, f_R = -a^-2 e^u (reading
 * R14): the right-hand side of the non-canonical equation of Sec. 4.2 term
 * by term,
 *   Omega_m a H0^2 (eta - 1)
 *   - Omega_m a^4 H0^2 (1 + 4 Omega_L/Omega_m) (|f_R0| a^2)^{1/(n+1)} e^{-u/(n+1)}
 *   + Omega_m a H0^2 (1 + 4 a^3 Omega_L/Omega_m). */
static void src_fr_paper(const orc_model* m, double u, double eta, double* S, double* dS)
{
    double a = m->a, H2 = ORC_H0 * ORC_H0, om = m->omega_m;
    double g = 1.0 + 4.0 * m->omega_l / om;
    double c = pow(m->fR0_abs * a * a, 1.0 / (m->n + 1.0));
    double e = exp(-u / (m->n + 1.0));
    *S = om * a * H2 * (eta - 1.0) - om * a * a * a * a * H2 * g * c * e +
         om * a * H2 * (1.0 + 4.0 * a * a * a * m->omega_l / om);
    *dS = om * a * a * a * a * H2 * g * c * e / (m->n + 1.0);
}

/* Chameleon (reading R13) in psi = ln phi: S = alpha eta - mu e^{-(1+n) psi}. */
static void src_cham(const orc_model* m, double psi, double eta, double* S, double* dS)
{
    double e = exp(-(1.0 + m->cham_n) * psi);
    *S = m->cham_alpha * eta - m->cham_mu * e;
    *dS = (1.0 + m->cham_n) * m->cham_mu * e;
}

/* LINEAR test model (the Poisson problem of Sec. 3.1 plus a mass term). */
static void src_linear(const orc_model* m, double phi, double eta, double* S, double* dS)
{
    *S = m->m2 * phi + m->kappa * (eta - 1.0);
    *dS = m->m2;
}

void orc_source(const orc_model* m, double phi, double eta, double* S, double* dS)
{
    if (m->model == ORC_SYMMETRON)
        src_symmetron(m, phi, eta, S, dS);
    else if (m->model == ORC_FR_HS && m->paper_u)
        src_fr_paper(m, phi, eta, S, dS);
    else if (m->model == ORC_FR_HS)
        src_fr(m, phi, eta, S, dS);
    else if (m->model == ORC_CHAMELEON)
        src_cham(m, phi, eta, S, dS);
    else
        src_linear(m, phi, eta, S, dS);
}

/* ------------------------------------------------------------------ */
/* Operator L at one cell and the Newton denominator.                  */
/* ------------------------------------------------------------------ */

static inline long cidx(long n, long i, long j, long k)
{
    return (i * n + j) * n + k;
}
static inline long wrap(long i, long n)
{
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

/* Returns L(phi)_c (no Sigma).  If D is non-NULL it receives the Newton
 * denominator used by the smoother. */
static double op_cell(const orc_model* m, long n, double h, const double* phi, const double* eta,
                      long i, long j, long k, double* D)
{
    long c = cidx(n, i, j, k);
    double nb[6];
    nb[0] = phi[cidx(n, wrap(i - 1, n), j, k)];
    nb[1] = phi[cidx(n, wrap(i + 1, n), j, k)];
    nb[2] = phi[cidx(n, i, wrap(j - 1, n), k)];
    nb[3] = phi[cidx(n, i, wrap(j + 1, n), k)];
    nb[4] = phi[cidx(n, i, j, wrap(k - 1, n))];
    nb[5] = phi[cidx(n, i, j, wrap(k + 1, n))];
    double p = phi[c];
    double ih2 = 1.0 / (h * h);
    double S, dS;
    orc_source(m, p, eta[c], &S, &dS);

    if (m->model == ORC_FR_HS || m->model == ORC_CHAMELEON) {
        /* Sec. 3.4: sum over faces of b_f (u_nb - u), b_f = (b(u) + b(u_nb))/2,
         * b = e^u; Jacobian: sum over faces of [ (db/du)/2 (u_nb - u) - b_f ]
         * (readings R3, R4), minus dS/du. */
        double bc = exp(p);
        double flux = 0.0, dflux = 0.0;
        for (int f = 0; f < 6; ++f) {
            double bf = 0.5 * (bc + exp(nb[f]));
            flux += bf * (nb[f] - p);
            dflux += 0.5 * bc * (nb[f] - p) - bf;
        }
        if (D) *D = dflux * ih2 - dS;
        return flux * ih2 - S;
    }

    /* Canonical: eq. disc_lap and dL/dphi = -6/h^2 - dS/dphi (Sec. 3.3). */
    double sum = nb[0] + nb[1] + nb[2] + nb[3] + nb[4] + nb[5];
    double lap = (sum - 6.0 * p) * ih2;
    if (D) {
        if (m->model == ORC_SYMMETRON)
            *D = -6.0 * ih2 - fabs(dS); /* reading R10 */
        else
            *D = -6.0 * ih2 - dS;
    }
    return lap - S;
}

/* out = L(phi) - Sigma on an n^3 level with spacing h (Sigma may be NULL = 0). */
void orc_defect(const orc_model* m, int n, double h, const double* phi, const double* eta,
                const double* sigma, double* out)
{
    long nn = n;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < nn; ++i)
        for (long j = 0; j < nn; ++j)
            for (long k = 0; k < nn; ++k) {
                long c = cidx(nn, i, j, k);
                double L = op_cell(m, nn, h, phi, eta, i, j, k, NULL);
                out[c] = L - (sigma ? sigma[c] : 0.0);
            }
}

/* The Newton denominator the smoother divides by, for every cell. */
void orc_newton_diag(const orc_model* m, int n, double h, const double* phi, const double* eta,
                     double* out)
{
    long nn = n;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < nn; ++i)
        for (long j = 0; j < nn; ++j)
            for (long k = 0; k < nn; ++k) {
                double D;
                op_cell(m, nn, h, phi, eta, i, j, k, &D);
                out[cidx(nn, i, j, k)] = D;
            }
}

/* One colour of a red-black Newton-Gauss-Seidel sweep (Sec. 3.2):
 * phi_c <- phi_c - (L(phi)_c - Sigma_c) / D_c for every cell with
 * (i+j+k) mod 2 == colour.  Cells of one colour have no neighbour of the
 * same colour, so the order inside a colour does not matter. */
void orc_halfsweep(const orc_model* m, int n, double h, double* phi, const double* eta,
                   const double* sigma, int colour)
{
    long nn = n;
    long long hits = 0;
#pragma omp parallel for schedule(static) reduction(+ : hits)
    for (long i = 0; i < nn; ++i)
        for (long j = 0; j < nn; ++j)
            for (long k = (i + j + colour) & 1; k < nn; k += 2) {
                long c = cidx(nn, i, j, k);
                double D;
                double L = op_cell(m, nn, h, phi, eta, i, j, k, &D);
                if (m->model == ORC_SYMMETRON) {
                    double S, dS;
                    orc_source(m, phi[c], eta[c], &S, &dS);
                    if (dS < 0.0) ++hits;
                }
                double eps = L - (sigma ? sigma[c] : 0.0);
                double step = eps / D;
                if (m->model == ORC_CHAMELEON) /* reading R15 */
                    step = fmax(-ORC_CHAM_MAX_STEP, fmin(ORC_CHAM_MAX_STEP, step));
                phi[c] = phi[c] - step;
            }
    g_guard_hits += hits;
}

void orc_sweep(const orc_model* m, int n, double h, double* phi, const double* eta,
               const double* sigma)
{
    orc_halfsweep(m, n, h, phi, eta, sigma, 0);
    orc_halfsweep(m, n, h, phi, eta, sigma, 1);
}

/* ------------------------------------------------------------------ */
/* Transfer operators (reading R2).                                    */
/* ------------------------------------------------------------------ */

/* coarse = mean of the 8 children; n_fine even. */
void orc_restrict(int n_fine, const double* fine, double* coarse)
{
    long nf = n_fine, nc = n_fine / 2;
#pragma omp parallel for schedule(static)
    for (long I = 0; I < nc; ++I)
        for (long J = 0; J < nc; ++J)
            for (long K = 0; K < nc; ++K) {
                double s = 0.0;
                for (int di = 0; di < 2; ++di)
                    for (int dj = 0; dj < 2; ++dj)
                        for (int dk = 0; dk < 2; ++dk)
                            s += fine[cidx(nf, 2 * I + di, 2 * J + dj, 2 * K + dk)];
                coarse[cidx(nc, I, J, K)] = s / 8.0;
            }
}

/* Full weighting (reading R2, option): coarse = P^T fine / 8.  Along each
 * axis coarse cell I collects fine cells 2I-1, 2I, 2I+1, 2I+2 (periodic) with
 * weights 1/8, 3/8, 3/8, 1/8 -- the transposed 1D weights of the trilinear
 * prolongation below (1/4, 3/4, 3/4, 1/4) over 2 -- and the 3D weight is the
 * product of the three. */
void orc_restrict_fw(int n_fine, const double* fine, double* coarse)
{
    long nf = n_fine, nc = n_fine / 2;
    const double w[4] = {0.125, 0.375, 0.375, 0.125};
#pragma omp parallel for schedule(static)
    for (long I = 0; I < nc; ++I)
        for (long J = 0; J < nc; ++J)
            for (long K = 0; K < nc; ++K) {
                double s = 0.0;
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < 4; ++b)
                        for (int c = 0; c < 4; ++c)
                            s += w[a] * w[b] * w[c] *
                                 fine[cidx(nf, wrap(2 * I - 1 + a, nf), wrap(2 * J - 1 + b, nf),
                                           wrap(2 * K - 1 + c, nf))];
                coarse[cidx(nc, I, J, K)] = s;
            }
}

/* fine += P(coarse - coarse_hat): cell-centred trilinear interpolation.
 * For fine index i the parent is I = i/2 and the second coarse cell along
 * that axis is I + s with s = +1 for odd i and -1 for even i; the 1D weights
 * are 3/4 (parent) and 1/4 (other). */
void orc_prolong_correct(int n_fine, double* fine, const double* coarse, const double* coarse_hat)
{
    long nf = n_fine, nc = n_fine / 2;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < nf; ++i)
        for (long j = 0; j < nf; ++j)
            for (long k = 0; k < nf; ++k) {
                long I[2], J[2], K[2];
                I[0] = i / 2;
                I[1] = wrap(I[0] + ((i & 1) ? 1 : -1), nc);
                J[0] = j / 2;
                J[1] = wrap(J[0] + ((j & 1) ? 1 : -1), nc);
                K[0] = k / 2;
                K[1] = wrap(K[0] + ((k & 1) ? 1 : -1), nc);
                const double w[2] = {0.75, 0.25};
                double s = 0.0;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b)
                        for (int c = 0; c < 2; ++c) {
                            long q = cidx(nc, I[a], J[b], K[c]);
                            s += w[a] * w[b] * w[c] * (coarse[q] - coarse_hat[q]);
                        }
                fine[cidx(nf, i, j, k)] += s;
            }
}

/* fine += P_b(coarse - coarse_hat): the same stencil with weights taken from
 * the flux coefficient b = e^{coarse_hat} of the flux-form operators (Sec.
 * 3.4), an option of reading R2.  Along each axis the correction is taken to
 * vary linearly in the "resistance" integral of 1/b, with b constant over
 * each coarse cell: the fine centre lies a quarter coarse spacing from its
 * parent P (coefficient b_P) and, towards the other coarse centre N, a further
 * quarter in P and a half in N (coefficient b_N), so its weight on N is
 * (1/(4 b_P)) / (1/(2 b_P) + 1/(2 b_N)) = b_N / (2 (b_P + b_N)), and 1 minus
 * that on P; this keeps the flux b de/dx continuous across the face between
 * P and N.  The three axes' weights come from P and its neighbour along each
 * axis and multiply as in the trilinear stencil.  With b uniform the weights
 * are 3/4 and 1/4: the trilinear prolongation.  The weight is evaluated as
 * 1 / (2 (1 + e^{u_P - u_N})), which needs only the difference of the two
 * values and tends to 0 or 1/2 instead of overflowing. */
void orc_prolong_correct_w(int n_fine, double* fine, const double* coarse, const double* coarse_hat)
{
    long nf = n_fine, nc = n_fine / 2;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < nf; ++i)
        for (long j = 0; j < nf; ++j)
            for (long k = 0; k < nf; ++k) {
                long I[2], J[2], K[2];
                I[0] = i / 2;
                I[1] = wrap(I[0] + ((i & 1) ? 1 : -1), nc);
                J[0] = j / 2;
                J[1] = wrap(J[0] + ((j & 1) ? 1 : -1), nc);
                K[0] = k / 2;
                K[1] = wrap(K[0] + ((k & 1) ? 1 : -1), nc);
                const double up = coarse_hat[cidx(nc, I[0], J[0], K[0])];
                const double un[3] = {coarse_hat[cidx(nc, I[1], J[0], K[0])],
                                      coarse_hat[cidx(nc, I[0], J[1], K[0])],
                                      coarse_hat[cidx(nc, I[0], J[0], K[1])]};
                double w[3][2];
                for (int ax = 0; ax < 3; ++ax) {
                    w[ax][1] = 1.0 / (2.0 * (1.0 + exp(up - un[ax])));
                    w[ax][0] = 1.0 - w[ax][1];
                }
                double s = 0.0;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b)
                        for (int c = 0; c < 2; ++c) {
                            long q = cidx(nc, I[a], J[b], K[c]);
                            s += w[0][a] * w[1][b] * w[2][c] * (coarse[q] - coarse_hat[q]);
                        }
                fine[cidx(nf, i, j, k)] += s;
            }
}

/* ------------------------------------------------------------------ */
/* Cold start and norms.                                               */
/* ------------------------------------------------------------------ */

/* Pointwise homogeneous root, the field for which S(phi, eta) = 0 in every
 * cell (reading R9): symmetron chi = sqrt(max(0, 1 - (a_ssb/a)^3 eta));
 * f(R) u = -(n+1) ln[(eta a^-3 + cL)/(1 + cL)], plus ln(a^2 |f_R0|) in the
 * paper's variable; chameleon psi = ln(mu / (alpha eta)) / (1+n) (eta > 0);
 * LINEAR phi = 0. */
void orc_cold_start(const orc_model* m, long ncell, const double* eta, double* phi)
{
#pragma omp parallel for schedule(static)
    for (long c = 0; c < ncell; ++c) {
        if (m->model == ORC_SYMMETRON) {
            double r = m->a_ssb / m->a;
            double v = 1.0 - r * r * r * eta[c];
            phi[c] = v > 0.0 ? sqrt(v) : 0.0;
        } else if (m->model == ORC_FR_HS) {
            double cL = 4.0 * m->omega_l / m->omega_m;
            double a3 = m->a * m->a * m->a;
            phi[c] = -(m->n + 1.0) * log((eta[c] / a3 + cL) / (1.0 + cL));
            if (m->paper_u) phi[c] += log(m->a * m->a * m->fR0_abs);
        } else if (m->model == ORC_CHAMELEON) {
            phi[c] = log(m->cham_mu / (m->cham_alpha * eta[c])) / (1.0 + m->cham_n);
        } else {
            phi[c] = 0.0;
        }
    }
}

/* Sum of squares over x-slabs, combined in slab order (deterministic). */
static double sumsq(long n, const double* r)
{
    long plane = n * n;
    double* part = (double*)malloc(sizeof(double) * (size_t)n);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        double s = 0.0;
        for (long q = 0; q < plane; ++q) s += r[i * plane + q] * r[i * plane + q];
        part[i] = s;
    }
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += part[i];
    free(part);
    return s;
}

double orc_rms(int n, const double* r)
{
    long nn = n;
    return sqrt(sumsq(nn, r) / (double)(nn * nn * nn));
}

static double mean_of(long n, const double* r)
{
    long plane = n * n;
    double* part = (double*)malloc(sizeof(double) * (size_t)n);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        double s = 0.0;
        for (long q = 0; q < plane; ++q) s += r[i * plane + q];
        part[i] = s;
    }
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += part[i];
    free(part);
    return s / (double)(n * n * n);
}

/* ------------------------------------------------------------------ */
/* FAS V-cycle (Sec. 3.1 and 3.2).                                     */
/* ------------------------------------------------------------------ */

typedef struct {
    int n;
    double h;
    double* phi;    /* current approximation                       */
    double* phihat; /* restricted approximation (coarse levels)    */
    double* sigma;  /* FAS source (NULL on level 0: Sigma_0 = 0)    */
    double* eta;    /* restricted density                          */
    double* work;   /* defect, then its restriction                */
} orc_level;

static void vcycle(const orc_model* m, const orc_cfg* cfg, orc_level* lv, int l, int nlev)
{
    orc_level* f = &lv[l];
    if (l == nlev - 1) {
        for (int s = 0; s < cfg->nu_coarse; ++s) orc_sweep(m, f->n, f->h, f->phi, f->eta, f->sigma);
        return;
    }
    orc_level* c = &lv[l + 1];
    for (int s = 0; s < cfg->nu_pre; ++s) orc_sweep(m, f->n, f->h, f->phi, f->eta, f->sigma);

    /* eps_l = L_l(phi_l) - Sigma_l */
    orc_defect(m, f->n, f->h, f->phi, f->eta, f->sigma, f->work);
    /* full approximation: phi_{l+1} = R phi_l, stored also as phihat_{l+1} */
    orc_restrict(f->n, f->phi, c->phi);
    long nc3 = (long)c->n * c->n * c->n;
    memcpy(c->phihat, c->phi, sizeof(double) * (size_t)nc3);
    /* Sigma_{l+1} = L_{l+1}(R phi, R eta) - R eps_l (reading R1); R of the
     * defect: mean of the children, or full weighting (reading R2) */
    if (cfg->restrict_fw)
        orc_restrict_fw(f->n, f->work, c->work);
    else
        orc_restrict(f->n, f->work, c->work);
    orc_defect(m, c->n, c->h, c->phi, c->eta, NULL, c->sigma);
    for (long q = 0; q < nc3; ++q) c->sigma[q] -= c->work[q];

    vcycle(m, cfg, lv, l + 1, nlev);

    /* phi_l += P(phi_{l+1} - phihat_{l+1}) */
    if (cfg->prolong_w && (m->model == ORC_FR_HS || m->model == ORC_CHAMELEON))
        orc_prolong_correct_w(f->n, f->phi, c->phi, c->phihat);
    else
        orc_prolong_correct(f->n, f->phi, c->phi, c->phihat);
    for (int s = 0; s < cfg->nu_post; ++s) orc_sweep(m, f->n, f->h, f->phi, f->eta, f->sigma);
}

static int valid_model(const orc_model* m)
{
    if (!(m->a > 0.0) || !isfinite(m->a)) return 0;
    if (m->model == ORC_SYMMETRON) return m->lambda0 > 0.0 && m->a_ssb > 0.0;
    if (m->model == ORC_FR_HS)
        return m->n > 0.0 && m->fR0_abs > 0.0 && m->omega_m > 0.0 && m->omega_l >= 0.0;
    if (m->model == ORC_LINEAR) return isfinite(m->kappa) && m->m2 >= 0.0;
    if (m->model == ORC_CHAMELEON)
        return m->cham_alpha > 0.0 && isfinite(m->cham_alpha) && m->cham_mu > 0.0 &&
               isfinite(m->cham_mu) && m->cham_n > -1.0 && isfinite(m->cham_n);
    return 0;
}

int orc_num_levels(int n)
{
    int L = 1;
    while (n > 4) {
        if (n & 1) return -1;
        n /= 2;
        ++L;
    }
    return n == 4 ? L : -1;
}

/* Full solve: eta (n^3, read-only) -> phi (n^3).  If use_guess is 0 the
 * iteration starts from the cold start.  Stops when
 * rms(L_0(phi)) <= tol * r_ref (reading R9), or after max_cycles cycles. */
int orc_solve(const orc_model* m, const orc_cfg* cfg, int n, double box, const double* eta,
              double* phi, int use_guess, double tol, orc_stats* st)
{
    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    int nlev = orc_num_levels(n);
    if (nlev < 2 || !valid_model(m) || !(box > 0.0) || !(tol >= 0.0) || cfg->max_cycles < 0 ||
        cfg->max_cycles >= ORC_MAX_HIST)
        return ORC_INVALID;
    long n3 = (long)n * n * n;
    orc_level lv[32];
    memset(lv, 0, sizeof(lv));
    for (int l = 0; l < nlev; ++l) {
        lv[l].n = n >> l;
        lv[l].h = (box / n) * (double)(1 << l);
        long c3 = (long)lv[l].n * lv[l].n * lv[l].n;
        lv[l].work = (double*)malloc(sizeof(double) * (size_t)c3);
        if (l == 0) {
            lv[l].phi = phi;
            lv[l].eta = (double*)eta;
            lv[l].sigma = NULL;
            lv[l].phihat = NULL;
        } else {
            lv[l].phi = (double*)malloc(sizeof(double) * (size_t)c3);
            lv[l].phihat = (double*)malloc(sizeof(double) * (size_t)c3);
            lv[l].sigma = (double*)malloc(sizeof(double) * (size_t)c3);
            lv[l].eta = (double*)malloc(sizeof(double) * (size_t)c3);
            orc_restrict(lv[l - 1].n, lv[l - 1].eta, lv[l].eta);
        }
    }

    /* r_ref from the cold start, independent of the guess. */
    double* cold = (double*)malloc(sizeof(double) * (size_t)n3);
    orc_cold_start(m, n3, eta, cold);
    orc_defect(m, n, lv[0].h, cold, eta, NULL, lv[0].work);
    double r_ref = orc_rms(n, lv[0].work);
    /* r_ref at the rounding level of the Laplacian of the cold start means
     * the cold start is an exact root (uniform density): the tolerance is
     * then absolute (reading R9). */
    double cold_scale = 1e-14 * 6.0 / (lv[0].h * lv[0].h) * orc_rms(n, cold);
    if (!use_guess) memcpy(phi, cold, sizeof(double) * (size_t)n3);
    free(cold);
    g_guard_hits = 0;
    double r_norm = r_ref > cold_scale ? r_ref : 1.0;
    int singular = (m->model == ORC_LINEAR && m->m2 == 0.0);
    if (singular) {
        double mu = mean_of(n, phi);
        for (long q = 0; q < n3; ++q) phi[q] -= mu;
    }

    orc_defect(m, n, lv[0].h, phi, eta, NULL, lv[0].work);
    double r0 = orc_rms(n, lv[0].work);
    int status = ORC_NOT_CONVERGED;
    int cyc = 0;
    if (st) {
        st->r_ref = r_ref;
        st->r0 = r0;
        st->rel_hist[0] = r0 / r_norm;
    }
    if (!isfinite(r0)) status = ORC_DIVERGED;
    else if (r0 <= tol * r_norm) status = ORC_OK;
    while (status == ORC_NOT_CONVERGED && cyc < cfg->max_cycles) {
        orc_cfg cc = *cfg; /* restrict_fw 2: full weighting in cycles 1 and 2 only */
        if (cfg->restrict_fw == 2) cc.restrict_fw = cyc < 2;
        vcycle(m, &cc, lv, 0, nlev);
        ++cyc;
        if (singular) {
            double mu = mean_of(n, phi);
            for (long q = 0; q < n3; ++q) phi[q] -= mu;
        }
        orc_defect(m, n, lv[0].h, phi, eta, NULL, lv[0].work);
        double r = orc_rms(n, lv[0].work);
        if (st) st->rel_hist[cyc] = r / r_norm;
        if (!isfinite(r) || r > 1e3 * r0) status = ORC_DIVERGED;
        else if (r <= tol * r_norm) status = ORC_OK;
    }
    clock_gettime(CLOCK_MONOTONIC, &t1);
    if (st) {
        st->cycles = cyc;
        st->guard_hits = g_guard_hits;
        st->wall_s = (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
    }

    for (int l = 0; l < nlev; ++l) {
        free(lv[l].work);
        if (l > 0) {
            free(lv[l].phi);
            free(lv[l].phihat);
            free(lv[l].sigma);
            free(lv[l].eta);
        }
    }
    return status;
}

/* Exactly k V-cycles from the given field (no stop test); the relative
 * residual after each cycle goes to rel (k+1 entries, entry 0 = before). */
int orc_vcycles(const orc_model* m, const orc_cfg* cfg, int n, double box, const double* eta,
                double* phi, int k, double* rel)
{
    orc_cfg c2 = *cfg;
    c2.max_cycles = k;
    orc_stats st;
    memset(&st, 0, sizeof(st));
    int s = orc_solve(m, &c2, n, box, eta, phi, 1, 0.0, &st);
    if (s == ORC_INVALID) return s;
    for (int q = 0; q <= st.cycles; ++q) rel[q] = st.rel_hist[q];
    return st.cycles;
}

/* ------------------------------------------------------------------ */
/* Force on the grid (the step after the solve in the paper's pipeline) */
/* ------------------------------------------------------------------ */

/* Second-order central difference of f along axis `ax` at cell (i,j,k),
 * periodic (reading R12: the paper does not state the gradient stencil). */
static double cdiff(long n, double h, const double* f, long i, long j, long k, int ax)
{
    long ip = i, im = i, jp = j, jm = j, kp = k, km = k;
    if (ax == 0) { ip = wrap(i + 1, n); im = wrap(i - 1, n); }
    if (ax == 1) { jp = wrap(j + 1, n); jm = wrap(j - 1, n); }
    if (ax == 2) { kp = wrap(k + 1, n); km = wrap(k - 1, n); }
    return (f[cidx(n, ip, jp, kp)] - f[cidx(n, im, jm, km)]) / (2.0 * h);
}

/* Acceleration d^2x/dtau^2 in super-comoving variables at every cell:
 *   - grad(potential)                        (if potential != NULL; the
 *                                              caller's potential is a^2 Phi)
 *   minus the scalar-field term of the geodesic equation:
 *   symmetron, Sec. 4.1 (eq. symmetron_geodesics_tilde_chi), chi~ = a chi:
 *       6 Omega_m H0^2 (beta lambda0)^2 / a_ssb^3 * chi~ grad chi~
 *   Hu-Sawicki f(R), Sec. 4.2 (geodesic equation), with the paper's variable
 *   e^{u_paper} = a^2 |f_R0| e^u (reading R5), grad u_paper = grad u:
 *       (1/2) a^2 |f_R0| e^u grad u
 *   LINEAR: no scalar-field term.
 * fx, fy, fz: n^3 each, component along x, y, z. */
void orc_force(const orc_model* m, int n, double h, const double* field, const double* potential,
               double* fx, double* fy, double* fz)
{
    const long N = n;
    double* out[3] = {fx, fy, fz};
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i)
        for (long j = 0; j < N; ++j)
            for (long k = 0; k < N; ++k) {
                const long c = cidx(N, i, j, k);
                for (int ax = 0; ax < 3; ++ax) {
                    double acc = 0.0;
                    if (potential) acc -= cdiff(N, h, potential, i, j, k, ax);
                    if (m->model == ORC_SYMMETRON) {
                        const double chit = m->a * field[c];
                        const double gchit = m->a * cdiff(N, h, field, i, j, k, ax);
                        const double bl = m->beta * m->lambda0;
                        const double coef = 6.0 * m->omega_m * ORC_H0 * ORC_H0 * bl * bl /
                                            (m->a_ssb * m->a_ssb * m->a_ssb);
                        acc -= coef * chit * gchit;
                    } else if (m->model == ORC_FR_HS) {
                        /* e^u of the paper's variable (Sec. 4.2 geodesic equation) */
                        const double eup = m->paper_u ? exp(field[c])
                                                      : m->a * m->a * m->fR0_abs * exp(field[c]);
                        acc -= 0.5 * eup * cdiff(N, h, field, i, j, k, ax);
                    }
                    out[ax][c] = acc;
                }
            }
}

/* ------------------------------------------------------------------ */
/* Refinement boundaries with masks (Sec. 3.3.1, 3.4.1).               */
/* ------------------------------------------------------------------ */
/* A refinement patch is an n^3 grid at spacing h whose cells carry a mask
 * m: m > 0 for cells whose centre lies inside the refinement (they are
 * relaxed with the discretisation above), m <= 0 for cells outside it
 * (m = -1: the cell does not exist on this level; -1 < m <= 0: it exists,
 * its centre outside the boundary, on coarser levels where the mask is
 * restricted).  The boundary lies where the linear interpolation of the mask
 * between two cell centres crosses zero.  Indices wrap periodically; a patch
 * keeps a layer of m = -1 cells around its inside, so the wrap never joins
 * inside cells.
 *
 * At an inside cell c with a masked neighbour f (m_f <= 0) the neighbour's
 * value is replaced by the ghost value of eq. ueq,
 *     u_G = u_f^Int + (m_f / m_c) (u_c - u_c^Pre),
 * u_f^Int = u_f^Pre if -1 < m_f <= 0, else the value interpolated from the
 * coarse grid (given in u_int); u^Pre is the field at the time the boundary
 * values were set (given in u_pre).  This is the linear extrapolation through
 * u_c and the boundary value u_# of eq. bpsi.  For the non-canonical operator
 * the face coefficient uses b(u_G) (the consistent choice of Sec. 3.4.1).
 * Since u_G depends on u_c, the Newton denominator gains
 *     canonical:     (m_f/m_c) / h^2                       (d L/d u_f = 1/h^2),
 *     non-canonical: (m_f/m_c) [b_f + b'(u_G) (u_G - u_c)/2] / h^2
 * per masked face (the two extra terms printed in Sec. 3.4.1).  Cells with
 * m <= 0 are not relaxed and have no residual. */

static int orc_inside(double mk) { return mk > 0.0; }

/* L(phi)_c at an inside cell with ghost values for masked neighbours; D gets
 * the Newton denominator with the extra ghost terms. */
static double op_cell_masked(const orc_model* m, long n, double h, const double* phi,
                             const double* eta, const double* mask, const double* u_int,
                             const double* u_pre, long i, long j, long k, double* D)
{
    const long c = cidx(n, i, j, k);
    const long nbi[6] = {cidx(n, wrap(i - 1, n), j, k), cidx(n, wrap(i + 1, n), j, k),
                         cidx(n, i, wrap(j - 1, n), k), cidx(n, i, wrap(j + 1, n), k),
                         cidx(n, i, j, wrap(k - 1, n)), cidx(n, i, j, wrap(k + 1, n))};
    const double p = phi[c];
    const double mc = mask[c];
    double v[6], r[6]; /* neighbour values (ghost where masked), d v / d u_c */
    for (int f = 0; f < 6; ++f) {
        const long q = nbi[f];
        if (orc_inside(mask[q])) {
            v[f] = phi[q];
            r[f] = 0.0;
        } else {
            const double uint_f = mask[q] > -1.0 ? u_pre[q] : u_int[q]; /* eq. bpsi */
            r[f] = mask[q] / mc;
            v[f] = uint_f + r[f] * (p - u_pre[c]); /* eq. ueq */
        }
    }
    const double ih2 = 1.0 / (h * h);
    double S, dS;
    orc_source(m, p, eta[c], &S, &dS);
    if (m->model == ORC_FR_HS || m->model == ORC_CHAMELEON) {
        const double bc = exp(p);
        double flux = 0.0, dflux = 0.0;
        for (int f = 0; f < 6; ++f) {
            const double bg = exp(v[f]);
            const double bf = 0.5 * (bc + bg);
            flux += bf * (v[f] - p);
            dflux += 0.5 * bc * (v[f] - p) - bf;
            dflux += r[f] * (bf + 0.5 * bg * (v[f] - p)); /* ghost terms, Sec. 3.4.1 */
        }
        if (D) *D = dflux * ih2 - dS;
        return flux * ih2 - S;
    }
    double sum = v[0] + v[1] + v[2] + v[3] + v[4] + v[5];
    double lap = (sum - 6.0 * p) * ih2;
    if (D) {
        double g = 0.0;
        for (int f = 0; f < 6; ++f) g += r[f];
        if (m->model == ORC_SYMMETRON)
            *D = -6.0 * ih2 - fabs(dS) + g * ih2; /* reading R10 */
        else
            *D = -6.0 * ih2 - dS + g * ih2;
    }
    return lap - S;
}

/* out = L(phi) - Sigma at inside cells (Sigma may be NULL), 0 elsewhere. */
void orc_masked_defect(const orc_model* m, int n, double h, const double* phi, const double* eta,
                       const double* sigma, const double* mask, const double* u_int,
                       const double* u_pre, double* out)
{
    long nn = n;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < nn; ++i)
        for (long j = 0; j < nn; ++j)
            for (long k = 0; k < nn; ++k) {
                long c = cidx(nn, i, j, k);
                if (!orc_inside(mask[c])) {
                    out[c] = 0.0;
                    continue;
                }
                double L = op_cell_masked(m, nn, h, phi, eta, mask, u_int, u_pre, i, j, k, NULL);
                out[c] = L - (sigma ? sigma[c] : 0.0);
            }
}

/* The Newton denominator at inside cells (0 elsewhere). */
void orc_masked_newton_diag(const orc_model* m, int n, double h, const double* phi,
                            const double* eta, const double* mask, const double* u_int,
                            const double* u_pre, double* out)
{
    long nn = n;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < nn; ++i)
        for (long j = 0; j < nn; ++j)
            for (long k = 0; k < nn; ++k) {
                long c = cidx(nn, i, j, k);
                double D = 0.0;
                if (orc_inside(mask[c]))
                    op_cell_masked(m, nn, h, phi, eta, mask, u_int, u_pre, i, j, k, &D);
                out[c] = D;
            }
}

/* One colour of the red-black Newton-Gauss-Seidel sweep over the inside
 * cells (Sec. 3.2 with the ghost values above); masked cells keep their
 * values. */
void orc_masked_halfsweep(const orc_model* m, int n, double h, double* phi, const double* eta,
                          const double* sigma, const double* mask, const double* u_int,
                          const double* u_pre, int colour)
{
    long nn = n;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < nn; ++i)
        for (long j = 0; j < nn; ++j)
            for (long k = (i + j + colour) & 1; k < nn; k += 2) {
                long c = cidx(nn, i, j, k);
                if (!orc_inside(mask[c])) continue;
                double D;
                double L = op_cell_masked(m, nn, h, phi, eta, mask, u_int, u_pre, i, j, k, &D);
                double eps = L - (sigma ? sigma[c] : 0.0);
                double step = eps / D;
                if (m->model == ORC_CHAMELEON) /* reading R15 */
                    step = fmax(-ORC_CHAM_MAX_STEP, fmin(ORC_CHAM_MAX_STEP, step));
                phi[c] = phi[c] - step;
            }
}

/* RMS of the masked defect over the inside cells. */
static double masked_rms(const orc_model* m, int n, double h, const double* phi,
                         const double* eta, const double* mask, const double* u_int,
                         const double* u_pre, double* work)
{
    orc_masked_defect(m, n, h, phi, eta, NULL, mask, u_int, u_pre, work);
    long n3 = (long)n * n * n, inside = 0;
    for (long q = 0; q < n3; ++q) inside += orc_inside(mask[q]);
    return inside ? sqrt(sumsq(n, work) / (double)inside) : 0.0;
}

/* Relaxation solve of a refinement patch: blocks of `block` red-black sweeps,
 * each block starting with u_pre = phi (the boundary values are set again,
 * Sec. 3.4.1), until the RMS defect over the inside cells is <= tol (absolute)
 * or max_sweeps sweeps are done.  Returns the sweeps made (negative on bad
 * arguments); *rms receives the final RMS defect. */
int orc_patch_solve(const orc_model* m, int n, double h, double* phi, const double* eta,
                    const double* mask, const double* u_int, int block, int max_sweeps,
                    double tol, double* rms)
{
    if (n < 2 || (n & 1) || block < 1 || max_sweeps < 0 || !valid_model(m)) return -1;
    long n3 = (long)n * n * n;
    double* pre = (double*)malloc(sizeof(double) * (size_t)n3);
    double* work = (double*)malloc(sizeof(double) * (size_t)n3);
    memcpy(pre, phi, sizeof(double) * (size_t)n3);
    double r = masked_rms(m, n, h, phi, eta, mask, u_int, pre, work);
    int sweeps = 0;
    while (r > tol && sweeps < max_sweeps) {
        memcpy(pre, phi, sizeof(double) * (size_t)n3);
        for (int b = 0; b < block && sweeps < max_sweeps; ++b, ++sweeps) {
            orc_masked_halfsweep(m, n, h, phi, eta, NULL, mask, u_int, pre, 0);
            orc_masked_halfsweep(m, n, h, phi, eta, NULL, mask, u_int, pre, 1);
        }
        /* the residual with the boundary values of the final field */
        memcpy(pre, phi, sizeof(double) * (size_t)n3);
        r = masked_rms(m, n, h, phi, eta, mask, u_int, pre, work);
    }
    if (rms) *rms = r;
    free(pre);
    free(work);
    return sweeps;
}
