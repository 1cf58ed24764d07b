/*
 * isis_mg — nonlinear FAS multigrid for the quasi-static scalar-field
 * equation of the symmetron and Hu-Sawicki f(R) models on one GPU
 * (MI355X, gfx950).
 *
 * The problem (Llinares, Mota & Winther 2013, "ISIS", Sec. 2 and 3.2): given
 * the density eta (in units of the mean) on a periodic N^3 cell-centred grid
 * and the expansion factor a, find phi with L(phi, eta) = 0, where
 *   canonical (Sec. 3.3):      L = lap_h(phi) - S(phi, eta)
 *   non-canonical (Sec. 3.4):  L = (1/h^2) sum_faces b_f (u_nb - u) - S(u, eta),
 *                              b_f = (b(u) + b(u_nb)) / 2,  b(u) = e^u
 * with the model sources
 *   ISIS_SYMMETRON (Sec. 4.1, dimensionless symmetron equation):
 *       S = a^2/(2 lambda0^2) [ (a_ssb/a)^3 eta chi - chi + chi^3 ]
 *   ISIS_FR_HS (Sec. 4.2, non-canonical f(R) equation, solved for
 *       u = ln(f_R/f_R0), i.e. the paper's u shifted by ln(a^2 |f_R0|)):
 *       S = Q [ eta + cL a^3 - a^3 (1 + cL) exp(-u/(n+1)) ],
 *       Q = Omega_m H0^2 / (a |f_R0|), cL = 4 Omega_L / Omega_m,
 *       H0 = 1/2997.92458 h/Mpc (lengths in comoving Mpc/h, c = 1)
 *   ISIS_LINEAR (the Poisson problem of Sec. 3.1 with a mass term):
 *       S = m2 phi + kappa (eta - 1)
 * The solve is FAS multigrid (Sec. 3.2): red-black Newton-Gauss-Seidel
 * smoothing, 8-child mean restriction, cell-centred trilinear prolongation,
 * V(nu_pre, nu_post) cycles down to a 4^3 grid.
 *
 * Conventions for every entry point:
 *  - Arrays are C-order [x][y][z] (z fastest), index (i*N + j)*N + k, cell
 *    centres at (i + 1/2) h, periodic in all three directions.
 *  - Array pointers are DEVICE pointers on the current HIP device, owned by
 *    the caller; the library never frees them and never calls hipMalloc.
 *    Scratch memory is the caller-provided workspace (see
 *    isis_mg_workspace_size).  Array pointers must be 16-byte aligned (the
 *    kernels move neighbouring cells as pairs); the workspace 256-byte
 *    aligned.  A misaligned pointer is rejected with ISIS_ERR_INVALID_ARG.
 *  - All work is enqueued on the given stream (a hipStream_t passed as
 *    void*; NULL is the null stream).  isis_op_* calls return once the work
 *    is enqueued; isis_mg_solve / isis_mg_residual synchronise the stream.
 *  - Return value: ISIS_OK (0) or a negative isis_status.  On error nothing
 *    is guaranteed about output arrays except where stated.
 */
#ifndef ISIS_MG_H
#define ISIS_MG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ISIS_MG_ABI_VERSION 5
#define ISIS_MG_MAX_HIST 128

typedef enum {
    ISIS_OK = 0,
    ISIS_ERR_INVALID_ARG = -1,  /* bad size, parameter, pointer or alignment        */
    ISIS_ERR_NOT_CONVERGED = -2,/* max_cycles reached; field holds the last iterate */
    ISIS_ERR_DIVERGED = -3,     /* residual non-finite or > 1e3 x initial           */
    ISIS_ERR_HIP = -4,          /* a HIP runtime call failed (see last_error)       */
    ISIS_ERR_UNSUPPORTED = -5   /* option not available for this model / size       */
} isis_status;

/* ISIS_CHAMELEON: the chameleon equation of Sec. 6,
 * lap phi = beta rho / M_pl - M^{4+n} / phi^{1+n}, with the source in code
 * units as lap phi = cham_alpha eta - cham_mu phi^{-(1+n)} (n = cham_n).  Its
 * field is psi = ln phi (phi = e^psi > 0), the field redefinition Sec. 4.2
 * uses for f(R): lap e^psi = div(e^psi grad psi) is discretised in the
 * non-canonical form of Sec. 3.4 with b = e^psi, and
 * S(psi) = cham_alpha eta - cham_mu e^{-(1+n) psi}.  Needs eta > 0. */
typedef enum { ISIS_SYMMETRON = 0, ISIS_FR_HS = 1, ISIS_LINEAR = 2, ISIS_CHAMELEON = 3 } isis_model;

typedef enum {
    ISIS_FP64 = 0,  /* every step in double precision                               */
    ISIS_MIXED = 1  /* FP32 smoothing and coarse-grid work, FP64 fine-level defect
                       and FP64 refinement cycles (see isis_mg_solve)                */
} isis_precision;

typedef struct {
    int model;        /* isis_model                                              */
    double lambda0;   /* symmetron: vacuum range, Mpc/h (> 0)                      */
    double a_ssb;     /* symmetron: symmetry-breaking expansion factor (> 0)       */
    double beta;      /* symmetron coupling: enters only the fifth force, unused   */
    double n;         /* f(R): Hu-Sawicki exponent (> 0)                           */
    double fR0_abs;   /* f(R): |f_R0| (> 0)                                        */
    double omega_m;   /* f(R): Omega_m (> 0)                                       */
    double omega_l;   /* f(R): Omega_Lambda (>= 0)                                 */
    double kappa;     /* LINEAR: source coefficient                                */
    double m2;        /* LINEAR: mass term (>= 0; 0 = singular Poisson, needs a
                         zero-mean source; the mean of phi is then removed)        */
    double cham_alpha;/* CHAMELEON: density coefficient (> 0)                      */
    double cham_mu;   /* CHAMELEON: potential coefficient (> 0)                    */
    double cham_n;    /* CHAMELEON: exponent n (> -1)                              */
    int paper_u;      /* f(R): 0 = field u = ln(f_R/f_R0); 1 = the paper's own
                         variable u = ln(a^2 |f_R|) (Sec. 4.2, f_R = -a^-2 e^u),
                         with the equation as the paper writes it (its residual is
                         a^2 |f_R0| times the other form's).  Other models: 0.    */
} isis_model_params;

typedef struct {
    int N;             /* grid cells per side: power of two, >= 8                 */
    double box;        /* box side, comoving Mpc/h (> 0)                           */
    int nu_pre;        /* pre-smoothing sweeps per level (>= 0; default 2)          */
    int nu_post;       /* post-smoothing sweeps per level (>= 0), or -1: per model,
                          1 for ISIS_SYMMETRON and ISIS_CHAMELEON, 2 otherwise
                          (the faster choice measured on lognormal + halo
                          densities at 256^3 and 512^3)                         */
    int nu_coarse;     /* red-black sweeps on the 4^3 grid (>= 1; default 32)       */
    int max_cycles;    /* V-cycle limit (1 .. ISIS_MG_MAX_HIST-1; default 50)       */
    int precision;     /* isis_precision                                           */
    double fp32_floor; /* ISIS_MIXED: relative residual at which the FP32 phase
                          hands over to FP64 cycles (see isis_mg_solve); 0 (the
                          default): once one more cycle at the last factor is
                          expected to reach tol; else in [1e-12, 1]             */
    int temporal_block;/* 0: one HBM pass per red or black half-sweep;
                          1: one pass per full red-black sweep (fused);
                          2: two full sweeps per pass (temporal blocking);
                          -1: chosen per model at each solve: 2 for the canonical
                          models (symmetron, linear), whose sweeps are bound by
                          HBM; 1 for the non-canonical ones (f(R), chameleon),
                          whose sweeps are bound by arithmetic and latency      */
    void* stream;      /* hipStream_t                                              */
    void* workspace;   /* device scratch, >= isis_mg_workspace_size bytes          */
    size_t workspace_bytes;
    double guess_accept;/* use_guess = 2 keeps the caller's field when its RMS
                          residual is <= guess_accept * r_ref; 0 (the default):
                          the relative residual after the first V-cycle of the
                          handle's last converged cold-started solve of the same
                          model, or 1e-2 before there is one; else in (0, 1]    */
    int restriction;   /* restriction of the defect in the FAS descent (Sec. 3.1
                          leaves R open): 0 = mean of the 8 children; 1 = full
                          weighting, the adjoint of the trilinear prolongation
                          over 8 (weights 1, 3, 3, 1 over 8 per axis; phi and
                          eta keep the mean); -1 = per model at each solve:
                          for f(R) full weighting in the first two V-cycles
                          and the mean after them (full weighting throughout
                          with the trilinear prolongation), the mean for the
                          others.  The converged field does not depend on it,
                          the V-cycles' convergence factors do               */
    int judge_skip;    /* 0: the FP64 fine defect (the judge of the stop test) is
                          evaluated after every V-cycle; 1: after a judged cycle,
                          the cycles that the mean factor per cycle since the
                          previous judged one predicts to stay above tol (at
                          most 4 in a row: FP64 cycles all but the last before
                          the predicted end, FP32 cycles all but the last two)
                          run without it, and in mixed precision an
                          FP32 cycle predicted to end above max(3e-5, 1e3 tol)
                          relative is judged by the FP32 problem's own defect
                          (FP32 density and arithmetic; its rel_hist entry is
                          then within 1% of the FP64 one; not for
                          f(R) in the paper's variable).  The stop test is
                          unchanged (the last cycle is always judged in FP64);
                          unjudged cycles have rel_hist = NaN                   */
    int prolongation;  /* prolongation of the coarse-grid correction (Sec. 3.1
                          leaves P open): 0 = cell-centred trilinear; 1 =
                          weighted by the flux coefficient b = e^u of the
                          flux-form operators (Sec. 3.4; f(R) and the
                          chameleon only, else the solve returns
                          ISIS_ERR_UNSUPPORTED; see
                          isis_op_prolong_correct_w); -1 = per model at each
                          solve: weighted for f(R), trilinear for the others.
                          The converged field does not depend on it          */
} isis_mg_desc;

typedef struct {
    int cycles;          /* V-cycles run (FP32 + FP64 in mixed mode)              */
    int cycles_fp32;     /* of which FP32 cycles (mixed mode)                     */
    double r_ref;        /* RMS of L_0 at the pointwise homogeneous root          */
    double r0;           /* RMS of L_0 at the initial field                       */
    double rel_res;      /* final RMS(L_0(phi)) / r_ref; absolute RMS when r_ref <=
                            1e-14 (6/h^2) RMS(cold start), i.e. when the cold
                            start is an exact root (uniform density)             */
    double rel_hist[ISIS_MG_MAX_HIST]; /* [0] initial, [k] after cycle k (NaN if
                                            not judged, see desc.judge_skip)     */
    double ms_total;     /* wall time of the solve call, milliseconds             */
    double cell_updates; /* Newton-GS cell updates performed, all levels          */
    int used_guess;      /* 1 if the caller's field was used as initial guess     */
    /* Finest-level smoother timing, filled when profiling is on
     * (isis_mg_set_profiling): HIP events on the solver's stream around the
     * sweep launches of the finest level.  Index 0: FP64 sweeps, index 1: FP32
     * sweeps (mixed mode). */
    double fine_sweep_ms[2];      /* summed kernel time of those launches        */
    int fine_sweep_launches[2];   /* number of kernel launches                    */
    double fine_sweep_updates[2]; /* cell updates they performed                  */
    double fine_sweep_bytes[2];   /* their compulsory HBM bytes: per pass over the
                                     grid, read phi + eta and write phi (8+8+8 B
                                     per cell in FP64, 4+4+4 in FP32); a pass is
                                     one sweep, or temporal_block sweeps when
                                     blocked                                      */
    int temporal_block;           /* the temporal block the solve used (0..2)     */
    double rho_hist[ISIS_MG_MAX_HIST]; /* convergence factors: [k] = rel_hist[k] /
                                     rel_hist[k-1] for 1 <= k <= cycles; [0] = 0;
                                     with desc.judge_skip, NaN for unjudged cycles
                                     and the mean factor per cycle since the
                                     previous judged cycle for judged ones         */
    long long safeguard_hits;     /* ISIS_SYMMETRON: Newton-Gauss-Seidel updates
                                     (every level, both precisions) at which
                                     dS/dchi < 0, so that the safeguarded
                                     denominator -6/h^2 - |dS/dchi| replaced the
                                     Jacobian -6/h^2 - dS/dchi (Sec. 3.3); each
                                     cell update counts once; 0 for other models */
    double ms_smooth;             /* profiling on: summed kernel time of the
                                     smoothing steps on the finest level and on
                                     every level of side >= 256 (the smaller
                                     levels are not timed), milliseconds          */
    int restriction;              /* the restriction of the defect the solve used
                                     (0 mean, 1 full weighting, 2 full weighting
                                     in the first two cycles, the mean after)     */
    int judged_cycles;            /* V-cycles after which the judge ran (FP64,
                                     or FP32: judged_fp32)                         */
    /* Finest-level first post-smoothing pass with the prolongation
     * phi += P(phi_c - phihat_c) fused in (fused sweep kernels with a
     * single-sweep first pass, i.e. temporal block 1; profiling on): [0] FP64,
     * [1] FP32.  These launches are not in fine_sweep_*. */
    double fine_prol_ms[2];       /* summed kernel time                           */
    int fine_prol_launches[2];    /* number of kernel launches                    */
    double fine_prol_bytes[2];    /* compulsory HBM bytes: a pass's (as in
                                     fine_sweep_bytes) plus the two coarse fields,
                                     2 x (n/2)^3 values                           */
    int nu_pre, nu_post;          /* the smoothing sweeps per level the solve used */
    int prolongation;             /* the prolongation the solve used (0 trilinear,
                                     1 coefficient-weighted)                       */
    int judged_fp32;              /* of judged_cycles, those judged by the FP32
                                     problem's own defect (desc.judge_skip)        */
} isis_mg_stats;

typedef struct isis_mg isis_mg_t;

/* Bytes of device workspace needed for desc (N, precision, temporal_block are
 * used); 0 if desc is invalid. */
size_t isis_mg_workspace_size(const isis_mg_desc* desc);

/* Create a solver handle for one grid size.  desc is copied; the workspace
 * must stay valid until isis_mg_destroy.  The handle is bound to the HIP
 * device current at creation.  On error *out is NULL. */
int isis_mg_create(const isis_mg_desc* desc, isis_mg_t** out);

/* FAS V-cycles until RMS(L_0(phi)) <= tol * r_ref (Sec. 3.2; the norm and
 * r_ref are defined in isis_mg_stats).
 *  density: device, N^3 doubles, eta > 0, read-only.
 *  field:   device, N^3 doubles.  In: initial guess if use_guess != 0, else
 *           ignored (the pointwise homogeneous root is used).  Out: solution.
 *  use_guess: 0 cold start; 1 the caller's field; 2 the caller's field if
 *           it cannot cost a V-cycle over the cold start: its RMS residual is
 *           at most desc.guess_accept * r_ref (see isis_mg_desc), else the cold
 *           start (stats->used_guess tells which).
 *  tol > 0.  stats may be NULL.
 * Symmetron: the positive branch is the one reached from the cold start.
 * ISIS_MIXED: FP32 V-cycles (FP32 fields, FP32 smoothing and coarse-grid
 * work; the f(R) source in FP64), each followed by the FP64 defect of the
 * FP32 iterate on the finest level (skipped when the initial field's relative
 * residual is already <= 1e-6, near the FP32 round-off floor), while that
 * residual falls by at least
 * 0.6x per cycle, no cycle at a relative residual <= 1e-6 has a factor
 * above both 0.2 and 3x the previous one's (the FP32 round-off floor coming
 * into view: ~2e-7 relative for the symmetron, below 1e-8 for f(R) on the
 * 512^3 halo workload) and, by
 * default, one more cycle at the last factor rho is not expected to reach tol
 * (residual * rho > 0.7 tol; with desc.fp32_floor set: the residual is above
 * that level); then FP64 V-cycles from the promoted iterate to tol, by default
 * a single one.  The FP64 defect decides convergence in both phases.  If the
 * FP32 cycles fail (residual non-finite or above 1e3 x the initial one) or
 * end no better than the initial field, the FP64 cycles start from the
 * initial field instead.
 * Returns ISIS_OK, ISIS_ERR_NOT_CONVERGED (field = last iterate) or
 * ISIS_ERR_DIVERGED (field = last iterate, may be non-finite). */
int isis_mg_solve(isis_mg_t* h, const double* density, double* field,
                  const isis_model_params* params, double a, double tol, int use_guess,
                  isis_mg_stats* stats);

/* Defect of the finest level, Sec. 3.2: res = L(field, density) (no Sigma).
 * out_res: device N^3 doubles or NULL.  out_rms: host double, receives
 * sqrt(mean(res^2)); may be NULL. */
int isis_mg_residual(isis_mg_t* h, const double* density, const double* field,
                     const isis_model_params* params, double a, double* out_res,
                     double* out_rms);

/* isis_mg_residual without a handle or workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same kernels, with the norm's partial
 * sums in a static device array of 8208 doubles (64.1 KiB) that each device
 * holds until the process ends.  It allocates nothing.
 *  N: power of two in [8, 4096] (ISIS_ERR_INVALID_ARG beyond), box > 0.
 *  density, field: device N^3 doubles; out_res: device N^3 doubles or NULL.
 *  out_rms: host double or NULL; when set, the call synchronises the stream.
 * All calls on one device share the array: calls that overlap (other
 * streams, other threads, or a second call before the first one's kernels
 * have finished when out_rms is NULL) race and give wrong norms.  Nothing in
 * the array needs clearing between calls. */
int isis_mg_residual_noalloc(const isis_model_params* params, double a, int N, double box,
                             const double* density, const double* field, double* out_res,
                             double* out_rms, void* stream);

void isis_mg_destroy(isis_mg_t* h);

/* Turn the finest-level sweep timing of isis_mg_stats on (1) or off (0).  On
 * adds two hipEventRecord calls per smoothing step of the finest level. */
int isis_mg_set_profiling(isis_mg_t* h, int enable);

/* Message of the last error on this handle ("" if none); h may be NULL for
 * errors of isis_mg_create and isis_op_* (thread-local). */
const char* isis_mg_last_error(const isis_mg_t* h);

/* ------------------------------------------------------------------------
 * Level operators: the individual steps of the V-cycle on caller buffers,
 * n^3 grid with spacing h (n even, >= 4 unless stated).  They launch the same
 * kernels the solver uses.  phi, eta, sigma, ... are device pointers.
 * ---------------------------------------------------------------------- */

/* One colour of a red-black Newton-Gauss-Seidel sweep (Sec. 3.2):
 * phi_c <- phi_c - (L(phi)_c - sigma_c) / D_c for (i+j+k) % 2 == colour,
 * D_c = dL_c/dphi_c (Sec. 3.3; eq. dbeq of Sec. 3.4 with the exact 1/2 on
 * db/du), symmetron safeguarded as -6/h^2 - |dS/dphi|.  sigma may be NULL. */
int isis_op_halfsweep(const isis_model_params* p, double a, int n, double h, double* phi,
                      const double* eta, const double* sigma, int colour, void* stream);

/* The coarse-grid correction phi += P(coarse - coarse_hat) (cell-centred
 * trilinear prolongation, as isis_op_prolong_correct; coarse and coarse_hat of
 * side n/2) followed by `count` sweeps as isis_op_sweeps, the way the solver
 * makes its post-smoothing step: where the sweeps run on the fused kernels
 * (temporal_block >= 1, n a power of two >= 64) and the first pass is a
 * single sweep (temporal_block 1, or count 1) the correction is applied
 * inside that pass to the values it loads, never written on its own; else by
 * its own kernel first.  n even >= 4; tmp: device n^3 doubles of
 * scratch; sigma may be NULL; the result is in phi. */
int isis_op_prolong_sweeps(const isis_model_params* p, double a, int n, double h, double* phi,
                           double* tmp, const double* eta, const double* sigma,
                           const double* coarse, const double* coarse_hat, int count,
                           int temporal_block, void* stream);

/* `count` full red-black sweeps with the solver's production kernels
 * (temporal_block as in isis_mg_desc).  tmp: device n^3 doubles of scratch.
 * The result is in phi; identical to 2*count isis_op_halfsweep calls up to
 * floating-point contraction. */
int isis_op_sweeps(const isis_model_params* p, double a, int n, double h, double* phi,
                   double* tmp, const double* eta, const double* sigma, int count,
                   int temporal_block, void* stream);

/* out = L(phi, eta) - sigma (sigma may be NULL = 0). */
int isis_op_defect(const isis_model_params* p, double a, int n, double h, const double* phi,
                   const double* eta, const double* sigma, double* out, void* stream);

/* coarse = mean of the 8 children of each coarse cell (n_fine even >= 2). */
int isis_op_restrict(int n_fine, const double* fine, double* coarse, void* stream);

/* One FAS descent step (Sec. 3.2), fine level of n_fine^3 cells and spacing
 * h_fine to the coarse level (n_fine/2)^3, spacing 2 h_fine:
 *   phi_c = phihat_c = R phi_f,
 *   sigma_c = L_c(phi_c, eta_c) - R'[L_f(phi_f, eta_f) - sigma_f],
 * R the mean of the 8 children; R' = R, or full weighting (see
 * isis_op_restrict_fw) when fine_scratch (device n_fine^3 doubles, receives
 * the fine defect) is not NULL.  sigma_f may be NULL (finest level).  rr_c:
 * coarse scratch; on the paths that restrict the defect before forming
 * sigma_c it receives R' of the fine defect, while the LDS-tiled descent
 * (n_fine a power of two >= 64, with R' = R) forms sigma_c in the same pass
 * and leaves rr_c untouched. */
int isis_op_fas_descend(const isis_model_params* p, double a, int n_fine, double h_fine,
                        const double* phi_f, const double* eta_f, const double* sigma_f,
                        const double* eta_c, double* phi_c, double* phihat_c, double* sigma_c,
                        double* rr_c, double* fine_scratch, void* stream);

/* coarse = full-weighting restriction of fine, the adjoint of the trilinear
 * prolongation over 8: along each axis coarse cell I takes fine cells 2I-1,
 * 2I, 2I+1, 2I+2 (periodic) with weights 1/8, 3/8, 3/8, 1/8, and the 3D
 * weight is their product (n_fine even >= 2; Sec. 3.1 leaves R open). */
int isis_op_restrict_fw(int n_fine, const double* fine, double* coarse, void* stream);

/* fine += P(coarse - coarse_hat), cell-centred trilinear interpolation with
 * weights 27, 9, 3, 1 over 64 and periodic wrap (n_fine even >= 4). */
int isis_op_prolong_correct(int n_fine, double* fine, const double* coarse,
                            const double* coarse_hat, void* stream);

/* fine += P_b(coarse - coarse_hat): the same stencil with the weights taken
 * from the flux coefficient b = e^{coarse_hat} of the flux-form operators
 * (Sec. 3.4; coarse_hat in u, or in any variable that differs from u by a
 * constant, as the paper's f(R) variable does).  Along each axis the weight
 * of the other coarse cell N of a fine cell whose parent is P is
 * 1 / (2 (1 + b_P / b_N)), 1/4 when b_P = b_N, and the parent takes 1 minus
 * it: with b constant over each coarse cell and the correction linear in
 * between, the flux b de/dx stays continuous across the face between P and N.
 * n_fine even >= 4. */
int isis_op_prolong_correct_w(int n_fine, double* fine, const double* coarse,
                              const double* coarse_hat, void* stream);

/* nu_c red-black sweeps on the coarsest (n = 4) grid in one workgroup. */
int isis_op_coarse_solve(const isis_model_params* p, double a, double h, double* phi,
                         const double* eta, const double* sigma, int nu_c, void* stream);

/* ------------------------------------------------------------------------
 * Learned warm start (a project addition, not part of the paper's method):
 * a 3D U-Net predicts the correction phi* - phi_cold from (log eta, a,
 * phi_cold); isis_mg_solve with use_guess = 2 then starts from the
 * prediction unless its residual is not below the cold start's.
 *
 * Network: 4 levels, channels 16/32/64/64, periodic 3x3x3 convolutions with
 * ReLU, 2x2x2 average pooling, nearest upsampling, skip concatenation
 * [upsampled, skip], 1x1x1 head (16 -> 1):
 *   16->16, 16->16 | pool 16->32, 32->32 | pool 32->64, 64->64 |
 *   pool 64->64, 64->64 | up+cat 128->64, 64->64 | up+cat 96->32, 32->32 |
 *   up+cat 48->16, 16->16 | head.
 * Inputs (16 channels, bf16): log(eta)/2, a, phi_cold, then zeros.
 * Parameters: one flat FP32 vector; per convolution W[t][cout][cin] then
 * b[cout], t = (di+1)*9 + (dj+1)*3 + (dk+1) for the input at
 * (i+di, j+dj, k+dk); then the head w[16], b.  Activations and gradients are
 * stored as bfloat16 (round to nearest even), products accumulate in FP32 on
 * the matrix cores.  Tensors of the conv entry points are channels-last
 * [x][y][z][c], bf16 as raw uint16 bits.
 * ---------------------------------------------------------------------- */

size_t isis_unet_param_count(void);

/* Device workspace bytes for an n^3 grid (n a power of two, 16 <= n <= 2048);
 * training = 1 adds the gradient buffers.  0 if n is invalid. */
size_t isis_unet_workspace_size(int n, int training);

/* guess[v] = phi_cold[v] + net(log eta, a, phi_cold)[v] (FP64 out; guess may
 * be NULL), out[v] = the network output (FP32; may be NULL).  eta, phi_cold:
 * device n^3 doubles. */
int isis_unet_predict(const float* params, const double* eta, const double* phi_cold, double a,
                      int n, double* guess, float* out, void* workspace, size_t workspace_bytes,
                      void* stream);

/* One training step on one sample: forward, loss = mean((out - (phi_target -
 * phi_cold))^2), backward, Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias
 * corrected with the 1-based step).  params, adam_m, adam_v: device FP32
 * vectors of isis_unet_param_count() entries, updated in place.  loss_out
 * (host, may be NULL) receives the loss before the update (synchronises the
 * stream); grad_out (device, may be NULL) the gradient. */
int isis_unet_train_step(float* params, float* adam_m, float* adam_v, int step, float lr,
                         const double* eta, const double* phi_cold, const double* phi_target,
                         double a, int n, void* workspace, size_t workspace_bytes,
                         float* loss_out, float* grad_out, void* stream);

/* The training step in its three parts (the same kernels; isis_unet_train_step
 * is forward + backward + Adam).  They share a training-size workspace
 * (isis_unet_workspace_size(n, 1)), which carries the activations from
 * isis_unet_forward to isis_unet_backward; calls on one workspace must not
 * overlap.
 *
 * isis_unet_forward: the network on (log eta, a, phi_cold), every activation
 * kept in the workspace (bf16), the head output (FP32) also in out (device n^3
 * floats, may be NULL). */
int isis_unet_forward(const float* params, const double* eta, const double* phi_cold, double a,
                      int n, float* out, void* workspace, size_t workspace_bytes, void* stream);

/* isis_unet_backward: after isis_unet_forward on the same workspace, the
 * gradient of loss = mean((out - (phi_target - phi_cold))^2) with respect to
 * params (ReLU, pooling, upsampling, concatenation and the 14 convolutions:
 * data gradients by the adjoint convolution, weight gradients by fixed-order
 * sums, so the result is deterministic).  grad: device FP32 vector of
 * isis_unet_param_count() entries (may be NULL: the gradient then stays in the
 * workspace for isis_unet_train_step).  loss_out (host, may be NULL) receives
 * the loss (synchronises the stream). */
int isis_unet_backward(const float* params, const double* phi_cold, const double* phi_target,
                       int n, void* workspace, size_t workspace_bytes, float* grad,
                       float* loss_out, void* stream);

/* isis_unet_adam_step: one Adam update of count parameters in place (beta1
 * 0.9, beta2 0.999, eps 1e-8, bias correction with the 1-based step):
 * m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 * All four arrays are device FP32. */
int isis_unet_adam_step(float* params, const float* grad, float* adam_m, float* adam_v,
                        long count, int step, float lr, void* stream);

/* A tensor of a training-size workspace after isis_unet_forward (for
 * inspection): *ptr = its device address, *voxels and *channels its shape
 * (channels-last bf16, except id 21).  id 0..13: output of convolution id
 * (after bias and ReLU); 14: the input; 15, 16, 17: the pooled inputs of
 * levels 1, 2, 3; 18, 19, 20: the concatenations [upsampled, skip] read by
 * convolutions 8, 10, 12; 21: the head output (FP32). */
int isis_unet_tensor(void* workspace, int n, int id, void** ptr, long* voxels, int* channels);

/* Message of the last error of the isis_unet_* / isis_conv3_* calls
 * (thread-local). */
const char* isis_unet_last_error(void);

/* y[v][co] = sum_t sum_ci x[v + d_t][ci] w[t][co][ci] + bias[co], ReLU if
 * relu != 0; periodic n^3 grid (n a power of two >= 2).  (cin, cout) must be
 * one of the network's shapes or their transposes.  y (bf16) and/or yf
 * (FP32) receive the result; bias may be NULL.  With weights prepared by
 * isis_conv3_flip_weights and the channel counts swapped, this is the data
 * gradient of a convolution. */
int isis_conv3_fwd(const uint16_t* x, int n, int cin, const uint16_t* w, const float* bias,
                   int cout, int relu, uint16_t* y, float* yf, void* stream);

/* wt[t][ci][co] = bf16(w[26 - t][co][ci]): the weights of the adjoint
 * (data-gradient) convolution. */
int isis_conv3_flip_weights(const float* w, int cin, int cout, uint16_t* wt, void* stream);

size_t isis_conv3_bwd_weight_workspace(int n, int cin, int cout);

/* dw[t][co][ci] = sum_v dy[v][co] x[v + d_t][ci] (FP32), db[co] = sum_v
 * dy[v][co] (may be NULL); deterministic (fixed-order partial sums). */
int isis_conv3_bwd_weight(const uint16_t* x, int n, int cin, const uint16_t* dy, int cout,
                          float* dw, float* db, void* workspace, size_t workspace_bytes,
                          void* stream);

/* ------------------------------------------------------------------------
 * Refinement boundaries with masks (Sec. 3.3.1 canonical, Sec. 3.4.1
 * non-canonical): the operator on a refinement patch, an n^3 grid of spacing
 * h (indices periodic; n even >= 2) whose cells carry a mask.  Cells with
 * mask > 0 lie inside the refinement and are relaxed; cells with mask <= 0
 * lie outside (mask = -1: the cell does not exist on this level and u_int
 * holds its value interpolated from the coarser grid; -1 < mask <= 0: the
 * cell exists with its centre outside the boundary and its u_pre value is
 * used).  The boundary is where the linear interpolation of the mask between
 * two centres crosses zero.  An inside cell c with a masked neighbour f uses
 * the ghost value u_G = u_int_f + (mask_f / mask_c)(phi_c - u_pre_c) (eqs.
 * bpsi, intpsi, ueq; u_int_f replaced by u_pre_f when mask_f > -1), u_pre
 * being the field when the boundary values were set; the non-canonical face
 * coefficient is b(u_G), and the Newton denominator gains the ghosts'
 * dependence on phi_c.  A patch needs a layer of mask = -1 cells around its
 * inside so that the wrap never joins inside cells.  All arrays are device
 * n^3 doubles (sigma may be NULL). */

/* out = L(phi) - sigma at inside cells, 0 at the others. */
int isis_op_masked_defect(const isis_model_params* p, double a, int n, double h,
                          const double* phi, const double* eta, const double* sigma,
                          const double* mask, const double* u_int, const double* u_pre,
                          double* out, void* stream);

/* One colour ((i+j+k) % 2 == colour) of the red-black Newton-Gauss-Seidel
 * sweep over the inside cells; cells with mask <= 0 keep their values. */
int isis_op_masked_halfsweep(const isis_model_params* p, double a, int n, double h, double* phi,
                             const double* eta, const double* sigma, const double* mask,
                             const double* u_int, const double* u_pre, int colour, void* stream);

/* Bytes of workspace isis_patch_solve needs for an n^3 patch (0 if n is
 * invalid). */
size_t isis_patch_workspace_size(int n);

/* Relaxation solve of a refinement patch: blocks of `block` red-black
 * sweeps, the boundary values (u_pre) set from phi before each block, until
 * the RMS defect over the inside cells (boundary values from the final
 * field) is <= tol (absolute) or max_sweeps sweeps are done.  phi: in the
 * initial field (its outside values are not changed), out the solution.
 * workspace: device, 256-byte aligned, >= isis_patch_workspace_size(n).
 * *sweeps_out, *rms_out (host, may be NULL): sweeps made, final RMS.
 * Returns ISIS_OK, ISIS_ERR_NOT_CONVERGED or ISIS_ERR_DIVERGED; synchronises
 * the stream once per block. */
int isis_patch_solve(const isis_model_params* p, double a, int n, double h, double* phi,
                     const double* eta, const double* mask, const double* u_int, int block,
                     int max_sweeps, double tol, void* workspace, size_t workspace_bytes,
                     int* sweeps_out, double* rms_out, void* stream);

/* Acceleration on the grid, the step after the solve in the paper's
 * pipeline: f = -grad(potential) - F, F the scalar-field term of the model's
 * geodesic equation in super-comoving variables:
 *   ISIS_SYMMETRON (Sec. 4.1, eq. symmetron_geodesics_tilde_chi):
 *       F = 6 Omega_m H0^2 (beta lambda0)^2 / a_ssb^3 chi~ grad chi~, chi~ = a field;
 *   ISIS_FR_HS (Sec. 4.2, geodesic equation): F = (1/2) e^{u_paper} grad u_paper
 *       = (1/2) a^2 |f_R0| e^u grad u, u = field = ln(f_R/f_R0);
 *   ISIS_LINEAR: F = 0 (field unused, may be NULL).
 * Gradients are second-order periodic central differences (the paper does not
 * state the stencil).  field, potential: device n^3 doubles (potential may be
 * NULL; for the Newtonian force pass a^2 Phi with Phi from an ISIS_LINEAR
 * solve of the Poisson equation of Sec. 3.1, kappa = 1.5 Omega_m H0^2 / a,
 * m2 = 0); fx, fy, fz: device n^3 doubles, written.  n even >= 2, h = box/n.
 * ISIS_ERR_INVALID_ARG on bad sizes, parameters (the symmetron also needs
 * Omega_m > 0 and a finite beta) or pointers. */
int isis_force(const isis_model_params* p, double a, int n, double h, const double* field,
               const double* potential, double* fx, double* fy, double* fz, void* stream);

/* Pointwise homogeneous root (cold start): symmetron sqrt(max(0, 1 -
 * (a_ssb/a)^3 eta)); f(R) -(n+1) ln[(eta/a^3 + cL)/(1 + cL)]; LINEAR 0. */
int isis_op_cold_start(const isis_model_params* p, double a, long ncell, const double* eta,
                       double* phi, void* stream);

#ifdef __cplusplus
}
#endif
#endif
