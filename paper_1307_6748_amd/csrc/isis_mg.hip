// Host driver and C ABI of the FAS multigrid scalar-field solver.
//
// The V-cycle (Sec. 3.1 and 3.2 of Llinares, Mota & Winther 2013) runs level
// by level on the caller's stream:
//   smooth nu_pre, descend (defect + restriction + FAS source), recurse,
//   prolongate + correct, smooth nu_post; nu_coarse sweeps on the 4^3 grid.
// The only device->host traffic is one scalar per V-cycle (the residual
// norm of the stop test).  Device memory is the caller's workspace.
#include <hip/hip_runtime.h>

#include <initializer_list>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "../../include/isis_mg.h"
#include "amr.hpp"
#include "bottom.hpp"
#include "force.hpp"
#include "full_weighting.hpp"
#include "fused_sweep.hpp"
#include "kernels.hpp"
#include "pair_kernels.hpp"

using namespace isis;

namespace {

constexpr double kH0 = 1.0 / 2997.92458;  // h/Mpc with c = 1
constexpr int kMaxLevels = 16;
constexpr int kMaxGrid = 16384;
thread_local char g_err[512];

void fmt_err(char* buf, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, 512, fmt, ap);
    va_end(ap);
}

int grid_for(long work)
{
    long b = (work + kBlock - 1) / kBlock;
    return (int)std::max(1L, std::min(b, (long)kMaxGrid));
}

bool is_pow2_ge(int n, int lo)
{
    return n >= lo && (n & (n - 1)) == 0;
}

int num_levels(int N)
{
    int L = 1;
    while (N > 4) {
        N >>= 1;
        ++L;
    }
    return L;
}

// Post-smoothing sweeps when desc.nu_post = -1: one for the symmetron and the
// chameleon, two otherwise (measured in mixed precision on lognormal + halo
// densities at 256^3 and 512^3: the symmetron 9-17 % faster with V(2,1) at
// one more cycle or none, the chameleon 6-22 %; f(R) 7 % slower at 512^3, the
// linear model 3 cycles more at 256^3).
int default_nu_post(int model)
{
    return (model == ISIS_SYMMETRON || model == ISIS_CHAMELEON) ? 1 : 2;
}

// Level at which the V-cycle hands over to the one-workgroup bottom kernel:
// the first level below the finest with side <= kBottomMaxN, if at least two
// levels (it and the 4^3 grid) remain; else -1.
int bottom_level(int N, int nlev)
{
    for (int l = 1; l < nlev; ++l)
        if ((N >> l) <= kBottomMaxN)
            return (nlev - l >= 2 && (N >> l) == (4 << (nlev - 1 - l))) ? l : -1;
    return -1;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

bool valid_params(const isis_model_params* p, double a, char* err)
{
    if (!p) {
        fmt_err(err, "model params is NULL");
        return false;
    }
    if (!finite_pos(a)) {
        fmt_err(err, "expansion factor a must be finite and > 0 (got %g)", a);
        return false;
    }
    switch (p->model) {
    case ISIS_SYMMETRON:
        if (!finite_pos(p->lambda0) || !finite_pos(p->a_ssb)) {
            fmt_err(err, "symmetron needs lambda0 > 0 and a_ssb > 0");
            return false;
        }
        break;
    case ISIS_FR_HS:
        if (!finite_pos(p->n) || !finite_pos(p->fR0_abs) || !finite_pos(p->omega_m) ||
            !std::isfinite(p->omega_l) || p->omega_l < 0.0) {
            fmt_err(err, "f(R) needs n > 0, |fR0| > 0, Omega_m > 0, Omega_L >= 0");
            return false;
        }
        break;
    case ISIS_LINEAR:
        if (!std::isfinite(p->kappa) || !std::isfinite(p->m2) || p->m2 < 0.0) {
            fmt_err(err, "linear model needs finite kappa and m2 >= 0");
            return false;
        }
        break;
    case ISIS_CHAMELEON:
        if (!finite_pos(p->cham_alpha) || !finite_pos(p->cham_mu) || !std::isfinite(p->cham_n) ||
            !(p->cham_n > -1.0)) {
            fmt_err(err, "chameleon needs alpha > 0, mu > 0 and n > -1");
            return false;
        }
        break;
    default:
        fmt_err(err, "unknown model %d", p->model);
        return false;
    }
    if (!(p->paper_u == 0 || (p->paper_u == 1 && p->model == ISIS_FR_HS))) {
        fmt_err(err, "paper_u must be 0, or 1 for the f(R) model");
        return false;
    }
    return true;
}

// hits: device counter of safeguard activations (NULL: not counted).
template <class T>
Symmetron<T> make_symmetron(const isis_model_params& p, double a,
                            unsigned long long* hits = nullptr)
{
    double K = a * a / (2.0 * p.lambda0 * p.lambda0);
    double r = p.a_ssb / a;
    double A = r * r * r;
    return Symmetron<T>{(T)K, (T)A, hits};
}

// Hu-Sawicki f(R), Sec. 4.2.  In u = ln(f_R/f_R0):
//   S = Q [eta + cL a^3 - a^3 (1 + cL) e^{-u/(n+1)}],  Q = Omega_m H0^2/(a |f_R0|).
// In the paper's u_p = u + c, c = ln(a^2 |f_R0|), the paper's equation is the
// same one times e^c: Q -> Omega_m H0^2 a, c1 -> c1 e^{c/(n+1)}, and the cold
// start and the stiff threshold on e^{-u_p/(n+1)} shift accordingly.
template <class T>
FofR<T> make_fofr(const isis_model_params& p, double a)
{
    FofR<T> m;
    double cL = 4.0 * p.omega_l / p.omega_m;
    double a3 = a * a * a;
    m.Q = p.omega_m * kH0 * kH0 / (a * p.fR0_abs);
    m.cLa3 = cL * a3;
    m.c1 = a3 * (1.0 + cL);
    m.inv_np1 = 1.0 / (p.n + 1.0);
    m.a3 = a3;
    m.cL = cL;
    m.inv_a3 = 1.0 / a3;
    m.inv_1pcl = 1.0 / (1.0 + cL);
    m.np1 = p.n + 1.0;
    m.ushift = 0.0;
    m.stiff_e = kFofRStiff;
    m.max_step = (T)0;  // unused: no step bound for f(R)
    if (p.paper_u) {
        const double c = std::log(a * a * p.fR0_abs);
        m.Q = p.omega_m * kH0 * kH0 * a;
        m.c1 *= std::exp(c * m.inv_np1);
        m.ushift = c;
        m.stiff_e = (float)(kFofRStiff * std::exp(-c * m.inv_np1));
    }
    m.qc1n = m.Q * m.c1 * m.inv_np1;
    m.n_is_one = p.n == 1.0 ? 1 : 0;
    return m;
}

// Chameleon (Sec. 6) in psi = ln phi: the same non-canonical operator with
// S = alpha eta - mu e^{-(1+n) psi}, i.e. Q = alpha, cL = 0, c1 = mu/alpha,
// 1/(n_f+1) = 1+n.  Cold start psi = ln(mu/(alpha eta))/(1+n), which is the
// f(R) form -np1 ln((eta/a3 + cL)/(1 + cL)) with a3 = c1, cL = 0,
// np1 = 1/(1+n).  Stiff where the potential term exceeds 100 alpha.
// Gauss-Seidel steps are bounded to |d psi| <= 2: where psi sits far above
// its local root the source's derivative is tiny and a full Newton step would
// overshoot by orders of magnitude (e^{-(1+n) psi} then overflows).
constexpr double kChameleonMaxStep = 2.0;
template <class T>
FofR<T, true> make_chameleon(const isis_model_params& p)
{
    FofR<T, true> m;
    m.Q = p.cham_alpha;
    m.cLa3 = 0.0;
    m.c1 = p.cham_mu / p.cham_alpha;
    m.inv_np1 = 1.0 + p.cham_n;
    m.a3 = m.c1;
    m.cL = 0.0;
    m.inv_a3 = 1.0 / m.a3;
    m.inv_1pcl = 1.0;
    m.np1 = 1.0 / m.inv_np1;
    m.ushift = 0.0;
    m.stiff_e = (float)(100.0 / m.c1);
    m.max_step = (T)(kChameleonMaxStep * FofR<T, true>::kVar);  // in the stored variable
    m.qc1n = m.Q * m.c1 * m.inv_np1;
    m.n_is_one = m.inv_np1 == 0.5 ? 1 : 0;
    return m;
}

template <class T>
Linear<T> make_linear(const isis_model_params& p)
{
    return Linear<T>{(T)p.kappa, (T)p.m2};
}

// Calls f(model) with the device model of p (precision T).
template <class T, class F>
int with_model(const isis_model_params& p, double a, F&& f)
{
    switch (p.model) {
    case ISIS_SYMMETRON:
        return f(make_symmetron<T>(p, a));
    case ISIS_FR_HS:
        return f(make_fofr<T>(p, a));
    case ISIS_CHAMELEON:
        return f(make_chameleon<T>(p));
    default:
        return f(make_linear<T>(p));
    }
}

int hip_fail(char* err, hipError_t e, const char* what)
{
    fmt_err(err, "%s: %s", what, hipGetErrorString(e));
    return ISIS_ERR_HIP;
}

#define HIP_TRY(err, call)                                           \
    do {                                                             \
        hipError_t e_ = (call);                                      \
        if (e_ != hipSuccess) return hip_fail((err), e_, #call);     \
    } while (0)

#define LAUNCH_CHECK(err, what)                                      \
    do {                                                             \
        hipError_t e_ = hipGetLastError();                           \
        if (e_ != hipSuccess) return hip_fail((err), e_, (what));    \
    } while (0)

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// ---------------------------------------------------------------------------
// Level launches (shared by the solver and the isis_op_* entry points).
// ---------------------------------------------------------------------------

template <class T, class M>
int launch_halfsweep(const M& m, int n, double h, T* phi, const T* eta, const T* sigma,
                     int colour, hipStream_t s, char* err)
{
    T ih2 = (T)(1.0 / (h * h));
    hipLaunchKernelGGL((k_halfsweep<T, M>), dim3(grid_for((long)n * n * n / 2)), dim3(kBlock), 0,
                       s, m, n, ih2, phi, eta, sigma, colour);
    LAUNCH_CHECK(err, "k_halfsweep");
    return ISIS_OK;
}

// count full sweeps of *phi.  The fused kernels work out of place between
// *phi and *tmp (n^3 each) and may leave the two pointers swapped: on return
// *phi is the buffer that holds the result.
// Levels smaller than this (per side) use the per-colour kernels inside the
// solver: there the streaming pipeline of the fused kernel has too few
// workgroups to hide its per-plane latency.
constexpr int kFusedSolverMinN = 256;

template <class T, int PW = 0>
int launch_prolong(int nf, T* fine, const T* coarse, const T* coarse_hat, hipStream_t s,
                   char* err);

// The prolongation weights (k_prolong_correct) of the coefficient-weighted
// option for model M in precision T: 2 for the single-precision flux-form
// models (their field carried as w = u / ln 2), 1 for the double-precision
// ones, 0 (trilinear) for the canonical models, which have no coefficient.
template <class T, class M>
constexpr int weighted_code()
{
    if constexpr (StageOp<T, M>::kStaged)
        return M::kW ? 2 : 1;
    else
        return 0;
}

template <class T, class M>
bool fused_level(int n, int tb, int min_fused_n = kFusedSolverMinN)
{
    return tb >= 1 && n >= min_fused_n && fused_supported<T, M>(n);
}

// Whether a smoothing step of `count` sweeps takes the prolongation inside
// its first fused pass (fused level, single-sweep first pass).
template <class T, class M>
bool prolong_fused(int n, int count, int tb, int min_fused_n = kFusedSolverMinN)
{
    return count > 0 && fused_level<T, M>(n, tb, min_fused_n) && fused_first_pass(count, tb) == 1;
}

// With cphi (and cphat, side n/2): phi += P(cphi - cphat) first, inside the
// first fused pass where prolong_fused(), else by its own kernel; pw: with
// the coefficient-weighted prolongation (always its own kernel).
template <class T, class M>
int launch_sweeps(const M& m, int n, double h, T** phi, T** tmp, const T* eta, const T* sigma,
                  int count, int tb, hipStream_t s, char* err, int min_fused_n = kFusedSolverMinN,
                  const T* cphi = nullptr, const T* cphat = nullptr, bool pw = false,
                  const float* in32 = nullptr, double in_scale = 1.0, double in_offset = 0.0)
{
    constexpr int PWc = weighted_code<T, M>();
    if (in32) {  // the field in single precision (fused double levels only)
        if (!(count > 0 && fused_level<T, M>(n, tb, min_fused_n) && !cphi)) {
            snprintf(err, 512, "launch_sweeps: a single-precision input needs fused sweeps");
            return ISIS_ERR_INVALID_ARG;
        }
        return launch_fused_sweeps<T, M>(m, n, h, phi, tmp, eta, sigma, count, tb, s, err,
                                         nullptr, nullptr, in32, in_scale, in_offset);
    }
    if (cphi && pw && PWc != 0) {
        int r = launch_prolong<T, PWc>(n, *phi, cphi, cphat, s, err);
        if (r) return r;
        cphi = cphat = nullptr;
    }
    if (cphi && prolong_fused<T, M>(n, count, tb, min_fused_n))
        return launch_fused_sweeps<T, M>(m, n, h, phi, tmp, eta, sigma, count, tb, s, err, cphi,
                                         cphat);
    if (count > 0 && fused_level<T, M>(n, tb, min_fused_n)) {
        if (cphi) {
            int r = launch_prolong<T>(n, *phi, cphi, cphat, s, err);
            if (r) return r;
        }
        return launch_fused_sweeps<T, M>(m, n, h, phi, tmp, eta, sigma, count, tb, s, err);
    }
    if (cphi) {
        int r = launch_prolong<T>(n, *phi, cphi, cphat, s, err);
        if (r) return r;
    }
    for (int q = 0; q < count; ++q) {
        int r = launch_halfsweep<T, M>(m, n, h, *phi, eta, sigma, 0, s, err);
        if (r) return r;
        r = launch_halfsweep<T, M>(m, n, h, *phi, eta, sigma, 1, s, err);
        if (r) return r;
    }
    return ISIS_OK;
}

// FW: the fine defect to dfine (restricted afterwards); else the 8-child
// mean of the defect, and with it the coarse source sigma_c in the same pass.
// XC coarse planes per workgroup: 16 at 512^3 and above (a shorter x halo per
// plane: f(R) 3.7% faster in single, 4.9% in double precision, the symmetron
// unchanged), 8 at 256^3, and 4 or 2 on the small levels (more workgroups;
// see launch_defect_fw).
template <class T, class M, bool SIG, bool FW, int XC>
int launch_restrict_tiled_xc(const M& m, int nf, T ih2f, const T* phi_f, const T* eta_f,
                             const T* sigma_f, T* phi_c, T* phihat_c, T* rr_c, T* dfine, T ih2c,
                             const T* eta_c, T* sigma_c, hipStream_t s, char* err)
{
    constexpr bool SIGC = !FW;
    using G = RestrictTile<XC, SIGC>;
    auto kern = k_defect_restrict_tiled<T, M, SIG, FW, SIGC, XC>;
    constexpr int lds = restrict_tiled_lds_bytes<T, M, SIGC>();
    static std::atomic<unsigned> lds_done{0};  // per instantiation: devices set up
    HIP_TRY(err, ensure_dynamic_lds((const void*)kern, lds, lds_done));
    const int blocks = (nf / G::TZ) * (nf / G::TY) * ((nf / 2) / G::XC);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(kBlock), lds, s, m, nf, ih2f, phi_f, eta_f,
                       sigma_f, phi_c, phihat_c, rr_c, dfine, ih2c, eta_c, sigma_c);
    LAUNCH_CHECK(err, "k_defect_restrict_tiled");
    return ISIS_OK;
}

template <class T, class M, bool SIG, bool FW>
int launch_restrict_tiled(const M& m, int nf, T ih2f, const T* phi_f, const T* eta_f,
                          const T* sigma_f, T* phi_c, T* phihat_c, T* rr_c, T* dfine, T ih2c,
                          const T* eta_c, T* sigma_c, hipStream_t s, char* err)
{
    if (nf >= 512)
        return launch_restrict_tiled_xc<T, M, SIG, FW, 16>(m, nf, ih2f, phi_f, eta_f, sigma_f, phi_c,
                                                           phihat_c, rr_c, dfine, ih2c, eta_c,
                                                           sigma_c, s, err);
    if (nf >= 256)
        return launch_restrict_tiled_xc<T, M, SIG, FW, 8>(m, nf, ih2f, phi_f, eta_f, sigma_f, phi_c,
                                                          phihat_c, rr_c, dfine, ih2c, eta_c,
                                                          sigma_c, s, err);
    if (nf == 128)
        return launch_restrict_tiled_xc<T, M, SIG, FW, 4>(m, nf, ih2f, phi_f, eta_f, sigma_f, phi_c,
                                                          phihat_c, rr_c, dfine, ih2c, eta_c,
                                                          sigma_c, s, err);
    return launch_restrict_tiled_xc<T, M, SIG, FW, 2>(m, nf, ih2f, phi_f, eta_f, sigma_f, phi_c,
                                                      phihat_c, rr_c, dfine, ih2c, eta_c, sigma_c,
                                                      s, err);
}

// FAS descent with the full-weighting restriction in one pass (single
// precision, tiled levels).  XC coarse planes per workgroup: 16 at 512^3 and
// above, 8 at 256^3 (enough workgroups to fill the device), and 4 or 2 below,
// where the few tiles of a level would otherwise leave most of the device
// idle while each workgroup steps through its planes.
template <class T, class M, bool SIG, int XC>
int launch_defect_fw_tiled(const M& m, int nf, T ih2f, const T* phi_f, const T* eta_f,
                           const T* sigma_f, T* phi_c, T* phihat_c, T ih2c, const T* eta_c,
                           T* sigma_c, hipStream_t s, char* err)
{
    using G = DefectFwTile<XC>;
    auto kern = k_defect_restrict_fw_tiled<T, M, SIG, XC>;
    constexpr int lds = defect_fw_lds_bytes<T, M, XC>();
    static std::atomic<unsigned> lds_done{0};  // per instantiation: devices set up
    HIP_TRY(err, ensure_dynamic_lds((const void*)kern, lds, lds_done));
    const int blocks = (nf / G::TZ) * (nf / G::TY) * ((nf / 2) / XC);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(kBlock), lds, s, m, nf, ih2f, phi_f, eta_f,
                       sigma_f, phi_c, phihat_c, ih2c, eta_c, sigma_c);
    LAUNCH_CHECK(err, "k_defect_restrict_fw_tiled");
    return ISIS_OK;
}

template <class T, class M, int XC>
int launch_defect_fw_xc(const M& m, int nf, T ih2f, const T* phi_f, const T* eta_f,
                        const T* sigma_f, T* phi_c, T* phihat_c, T ih2c, const T* eta_c,
                        T* sigma_c, hipStream_t s, char* err)
{
    return sigma_f ? launch_defect_fw_tiled<T, M, true, XC>(m, nf, ih2f, phi_f, eta_f, sigma_f,
                                                            phi_c, phihat_c, ih2c, eta_c, sigma_c,
                                                            s, err)
                   : launch_defect_fw_tiled<T, M, false, XC>(m, nf, ih2f, phi_f, eta_f, sigma_f,
                                                             phi_c, phihat_c, ih2c, eta_c,
                                                             sigma_c, s, err);
}

// nf: a power of two >= 64
template <class T, class M>
int launch_defect_fw(const M& m, int nf, T ih2f, const T* phi_f, const T* eta_f,
                     const T* sigma_f, T* phi_c, T* phihat_c, T ih2c, const T* eta_c, T* sigma_c,
                     hipStream_t s, char* err)
{
    if (nf >= 512)
        return launch_defect_fw_xc<T, M, 16>(m, nf, ih2f, phi_f, eta_f, sigma_f, phi_c, phihat_c,
                                             ih2c, eta_c, sigma_c, s, err);
    if (nf == 256)
        return launch_defect_fw_xc<T, M, 8>(m, nf, ih2f, phi_f, eta_f, sigma_f, phi_c, phihat_c,
                                            ih2c, eta_c, sigma_c, s, err);
    if (nf == 128)
        return launch_defect_fw_xc<T, M, 4>(m, nf, ih2f, phi_f, eta_f, sigma_f, phi_c, phihat_c,
                                            ih2c, eta_c, sigma_c, s, err);
    return launch_defect_fw_xc<T, M, 2>(m, nf, ih2f, phi_f, eta_f, sigma_f, phi_c, phihat_c, ih2c,
                                        eta_c, sigma_c, s, err);
}

// coarse = full-weighting restriction of an nf^3 fine field (nf even >= 4).
template <class T>
int launch_restrict_fw(int nf, const T* fine, T* coarse, hipStream_t s, char* err)
{
    const int nc = nf / 2;
    using FG = FwTileF;
    if ((nc & (nc - 1)) == 0 && nc % FG::TK == 0 && nc % FG::TJ == 0 && nc % FG::XC == 0)
        hipLaunchKernelGGL((k_restrict_fw_tiled<T>), dim3((nc / FG::TK) * (nc / FG::TJ) * (nc / FG::XC)),
                           dim3(kBlock), 0, s, nf, fine, coarse);
    else
        hipLaunchKernelGGL((k_restrict_fw<T>), dim3(grid_for((long)nc * nc * nc)), dim3(kBlock), 0,
                           s, nf, fine, coarse);
    LAUNCH_CHECK(err, "k_restrict_fw");
    return ISIS_OK;
}

// The FAS descent.  dfine: NULL for the 8-child mean of the defect; else full
// weighting, in one pass on single-precision tiled levels, elsewhere through
// dfine, an nf^3 scratch field that receives the fine defect, which is then
// restricted.  On tiled levels with the mean, and with full weighting in one
// pass, the descent kernel also computes the coarse source sigma_c; the other
// paths restrict the defect to rr_c and finish with k_fas_sigma.
template <class T, class M>
int launch_descend(const M& m, int nf, double hf, const T* phi_f, const T* eta_f,
                   const T* sigma_f, const T* eta_c, T* phi_c, T* phihat_c, T* sigma_c, T* rr_c,
                   hipStream_t s, char* err, T* dfine = nullptr)
{
    int nc = nf / 2;
    long c3 = (long)nc * nc * nc;
    T ih2f = (T)(1.0 / (hf * hf));
    double hc = 2.0 * hf;
    T ih2c = (T)(1.0 / (hc * hc));
    using RG = RestrictTile<8, false>;  // the tile (every chunk length divides nc here)
    const bool tiled =
        (nf & (nf - 1)) == 0 && nf % RG::TZ == 0 && nf % RG::TY == 0 && nc % RG::XC == 0;
    if constexpr (sizeof(T) == 4) {
        if (dfine && tiled)  // single pass; dfine is not needed
            return launch_defect_fw<T, M>(m, nf, ih2f, phi_f, eta_f, sigma_f, phi_c, phihat_c,
                                          ih2c, eta_c, sigma_c, s, err);
    }
    if (tiled && !dfine)
        return sigma_f ? launch_restrict_tiled<T, M, true, false>(m, nf, ih2f, phi_f, eta_f,
                                                                  sigma_f, phi_c, phihat_c, rr_c,
                                                                  nullptr, ih2c, eta_c, sigma_c,
                                                                  s, err)
                       : launch_restrict_tiled<T, M, false, false>(m, nf, ih2f, phi_f, eta_f,
                                                                   sigma_f, phi_c, phihat_c, rr_c,
                                                                   nullptr, ih2c, eta_c, sigma_c,
                                                                   s, err);
    if (tiled) {
        const int r =
            sigma_f ? launch_restrict_tiled<T, M, true, true>(m, nf, ih2f, phi_f, eta_f, sigma_f,
                                                              phi_c, phihat_c, rr_c, dfine, ih2c,
                                                              eta_c, sigma_c, s, err)
                    : launch_restrict_tiled<T, M, false, true>(m, nf, ih2f, phi_f, eta_f, sigma_f,
                                                               phi_c, phihat_c, rr_c, dfine, ih2c,
                                                               eta_c, sigma_c, s, err);
        if (r) return r;
    } else if (nf >= 4) {
        hipLaunchKernelGGL((k_defect_restrict_pairs<T, M>), dim3(grid_for(c3)), dim3(kBlock), 0, s,
                           m, nf, ih2f, phi_f, eta_f, sigma_f, phi_c, phihat_c, rr_c, dfine);
    } else {
        if (dfine) {
            fmt_err(err, "full-weighting descent needs a fine side >= 4");
            return ISIS_ERR_INVALID_ARG;
        }
        hipLaunchKernelGGL((k_defect_restrict<T, M>), dim3(grid_for(c3)), dim3(kBlock), 0, s, m,
                           nf, ih2f, phi_f, eta_f, sigma_f, phi_c, phihat_c, rr_c);
    }
    LAUNCH_CHECK(err, "k_defect_restrict");
    if (dfine) {
        int r = launch_restrict_fw<T>(nf, dfine, rr_c, s, err);
        if (r) return r;
    }
    hipLaunchKernelGGL((k_fas_sigma<T, M>), dim3(grid_for(c3)), dim3(kBlock), 0, s, m, nc, ih2c,
                       phi_c, eta_c, rr_c, sigma_c);
    LAUNCH_CHECK(err, "k_fas_sigma");
    return ISIS_OK;
}

template <class T, int PW>
int launch_prolong(int nf, T* fine, const T* coarse, const T* coarse_hat, hipStream_t s,
                   char* err)
{
    long f3 = (long)nf * nf * nf;
    using PG = ProlongTileF;
    const int nc = nf / 2;
    if ((nc & (nc - 1)) == 0 && nc % PG::TK == 0 && nc % PG::TJ == 0 && nc % PG::XC == 0)
        hipLaunchKernelGGL((k_prolong_tiled<T, PW>),
                           dim3((nc / PG::TK) * (nc / PG::TJ) * (nc / PG::XC)), dim3(kBlock), 0, s,
                           nf, fine, coarse, coarse_hat);
    else if (nf >= 4)
        hipLaunchKernelGGL((k_prolong_pairs<T, PW>), dim3(grid_for(f3 / 8)), dim3(kBlock), 0, s,
                           nf, fine, coarse, coarse_hat);
    else
        hipLaunchKernelGGL((k_prolong_correct<T, PW>), dim3(grid_for(f3)), dim3(kBlock), 0, s, nf,
                           fine, coarse, coarse_hat);
    LAUNCH_CHECK(err, "k_prolong_correct");
    return ISIS_OK;
}

template <class T>
int launch_restrict(int nf, const T* fine, T* coarse, hipStream_t s, char* err,
                    float* fine32 = nullptr)
{
    long c3 = (long)(nf / 2) * (nf / 2) * (nf / 2);
    hipLaunchKernelGGL((k_restrict<T>), dim3(grid_for(c3)), dim3(kBlock), 0, s, nf, fine, coarse,
                       fine32);
    LAUNCH_CHECK(err, "k_restrict");
    return ISIS_OK;
}

template <class T, class M>
int launch_coarse(const M& m, double h, T* phi, const T* eta, const T* sigma, int nu_c,
                  hipStream_t s, char* err)
{
    T ih2 = (T)(1.0 / (h * h));
    hipLaunchKernelGGL((k_coarse_solve<T, M>), dim3(1), dim3(64), 0, s, m, ih2, phi, eta, sigma,
                       nu_c);
    LAUNCH_CHECK(err, "k_coarse_solve");
    return ISIS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Solver handle.
// ---------------------------------------------------------------------------

template <class T>
struct LevP {
    int n;
    double h;
    T *phi, *phihat, *sigma, *eta, *rr, *tmp;
};

struct isis_mg {
    isis_mg_desc d;
    int nlev;
    int lb;  // bottom_level(), -1: none
    int nu_post;  // post-smoothing sweeps of the current solve (desc.nu_post, or per model)
    int device;
    hipStream_t s;
    LevP<double> L64[kMaxLevels];
    LevP<float> L32[kMaxLevels];
    double* partial;  // 2 * kReduceBlocks
    double* scal;     // 16: [0] reduction result, [8] safeguard counter (64-bit)
    double* host;     // pinned, 16
    double* tmp0;     // finest-level scratch field (workspace)
    char err[512];
    // smoothing timing (profiling on): one event pair per smoothing step of
    // any level, created on the first isis_mg_set_profiling(h, 1)
    static constexpr int kMaxTimed = 2048;
    int tb;  // temporal block of the current solve (desc.temporal_block resolved)
    int fw;  // full-weighting restriction of the defect in the current cycle
    int fw_after;  // ... after the first fw_first cycles of a solve (with them: full weighting)
    int fw_first;
    int pw;  // coefficient-weighted prolongation (desc.prolongation resolved)
    // FP32 iterate handed over to the FP64 cycles, consumed by their first
    // finest-level smoothing pass (value * in32_scale + in32_offset)
    const float* in32 = nullptr;
    double in32_scale = 1.0, in32_offset = 0.0;
    int profile;
    int ntimed;
    int events_ready;
    hipEvent_t ev0[kMaxTimed], ev1[kMaxTimed];
    int tlaunch[kMaxTimed], tprec[kMaxTimed], tlevel[kMaxTimed];  // tprec: 0 FP64, 1 FP32
    int tprol[kMaxTimed];  // 1: a pass with the prolongation fused in
    double tupd[kMaxTimed], tbytes[kMaxTimed];
    // use_guess = 2: relative residual after the first V-cycle of the last
    // cold-started solve of each model on this handle (0: none yet)
    double cold_first[4];
    unsigned long long* hits() const { return reinterpret_cast<unsigned long long*>(scal + 8); }
};

namespace {

// Lays out the workspace; with h == NULL only measures it.
size_t carve(const isis_mg_desc& d, char* base, isis_mg* h)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        off = (off + 255) & ~(size_t)255;
        char* p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    const int nlev = num_levels(d.N);
    for (int l = 0; l < nlev; ++l) {
        const long n = d.N >> l;
        const size_t n3 = (size_t)n * n * n;
        LevP<double> a{};
        a.n = (int)n;
        a.h = (d.box / d.N) * (double)(1 << l);
        a.tmp = (double*)take(n3 * 8);
        if (l > 0) {
            a.phi = (double*)take(n3 * 8);
            a.phihat = (double*)take(n3 * 8);
            a.sigma = (double*)take(n3 * 8);
            a.eta = (double*)take(n3 * 8);
            a.rr = (double*)take(n3 * 8);
        }
        LevP<float> b{};
        b.n = a.n;
        b.h = a.h;
        if (d.precision == ISIS_MIXED) {
            b.phi = (float*)take(n3 * 4);
            b.eta = (float*)take(n3 * 4);
            b.tmp = (float*)take(n3 * 4);
            if (l > 0) {
                b.phihat = (float*)take(n3 * 4);
                b.sigma = (float*)take(n3 * 4);
                b.rr = (float*)take(n3 * 4);
            }
        }
        if (h) {
            h->L64[l] = a;
            h->L32[l] = b;
            if (l == 0) h->tmp0 = a.tmp;
        }
    }
    double* partial = (double*)take(sizeof(double) * 2 * kReduceBlocks);  // two sums at once
    double* scal = (double*)take(sizeof(double) * 16);
    if (h) {
        h->partial = partial;
        h->scal = scal;
    }
    return off + 256;
}

bool valid_desc(const isis_mg_desc* d, char* err)
{
    if (!d) {
        fmt_err(err, "desc is NULL");
        return false;
    }
    if (!is_pow2_ge(d->N, 8) || d->N > 4096) {
        fmt_err(err, "N must be a power of two in [8, 4096] (got %d)", d->N);
        return false;
    }
    if (!finite_pos(d->box)) {
        fmt_err(err, "box must be finite and > 0");
        return false;
    }
    if (d->nu_pre < 0 || d->nu_post < -1 || d->nu_coarse < 1 || d->max_cycles < 1 ||
        d->max_cycles >= ISIS_MG_MAX_HIST || (d->nu_post >= 0 && d->nu_pre + d->nu_post < 1)) {
        fmt_err(err, "need nu_pre >= 0, nu_post >= 0 or -1 (sum >= 1), nu_coarse >= 1, "
                     "1 <= max_cycles < %d", ISIS_MG_MAX_HIST);
        return false;
    }
    if (d->precision != ISIS_FP64 && d->precision != ISIS_MIXED) {
        fmt_err(err, "unknown precision %d", d->precision);
        return false;
    }
    if (d->temporal_block < -1 || d->temporal_block > 2) {
        fmt_err(err, "temporal_block must be -1 (per model), 0, 1 or 2");
        return false;
    }
    if (!(d->fp32_floor == 0.0 || (d->fp32_floor >= 1e-12 && d->fp32_floor <= 1.0))) {
        fmt_err(err, "fp32_floor must be 0 (default) or in [1e-12, 1]");
        return false;
    }
    if (!(d->guess_accept == 0.0 || (d->guess_accept > 0.0 && d->guess_accept <= 1.0))) {
        fmt_err(err, "guess_accept must be 0 (automatic) or in (0, 1]");
        return false;
    }
    if (d->judge_skip != 0 && d->judge_skip != 1) {
        fmt_err(err, "judge_skip must be 0 or 1");
        return false;
    }
    if (d->restriction < -1 || d->restriction > 1) {
        fmt_err(err, "restriction must be -1 (per model), 0 (mean) or 1 (full weighting)");
        return false;
    }
    if (d->prolongation < -1 || d->prolongation > 1) {
        fmt_err(err, "prolongation must be -1 (per model), 0 (trilinear) or 1 (coefficient-weighted)");
        return false;
    }
    return true;
}

// The FP64 defect L(phi) of an n^3 level with spacing h (into res unless
// NULL) and the sum of its squares: per-block partial sums in
// partial[0 .. kReduceBlocks), their fixed-order total in *total (device).
template <class TF, class M>
int launch_defect_norm(const M& m, int n, double h, const TF* phi, const double* eta,
                       double* res, double* partial, double* total, hipStream_t s, char* err,
                       double uscale = 1.0, double uoffset = 0.0)
{
    const long n3 = (long)n * n * n;
    int g = std::min(kReduceBlocks, grid_for(n3 / 2));
    using NG = NormTileF;
    const bool tiled = (n & (n - 1)) == 0 && n % NG::TZ == 0 && n % NG::TY == 0 && n % NG::XC == 0;
    if (tiled) {
        const long tiles = (long)(n / NG::TZ) * (n / NG::TY) * (n / NG::XC);
        g = (int)std::min<long>(kReduceBlocks, tiles);
        hipLaunchKernelGGL((k_defect_norm_tiled<TF, M>), dim3(g), dim3(kBlock), 0, s, m, n,
                           1.0 / (h * h), uscale, uoffset, phi, eta, res, partial);
    }
    if (!tiled)
        hipLaunchKernelGGL((k_defect_norm_pairs<TF, M>), dim3(g), dim3(kBlock), 0, s, m, n,
                           1.0 / (h * h), uscale, uoffset, phi, eta, res, partial);
    LAUNCH_CHECK(err, "k_defect_norm");
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, s, partial, g, total);
    LAUNCH_CHECK(err, "k_reduce");
    return ISIS_OK;
}

// sqrt(mean(L_0(phi)^2)) of the finest level, in double; res may be NULL.
template <class TF, class M>
int fine_rms(isis_mg* H, const M& m, const TF* phi, const double* eta, double* res, double* out,
             double uscale = 1.0, double uoffset = 0.0)
{
    const int n = H->d.N;
    const long n3 = (long)n * n * n;
    int r = launch_defect_norm<TF, M>(m, n, H->L64[0].h, phi, eta, res, H->partial, H->scal, H->s,
                                      H->err, uscale, uoffset);
    if (r) return r;
    HIP_TRY(H->err, hipMemcpyAsync(H->host, H->scal, sizeof(double), hipMemcpyDeviceToHost, H->s));
    HIP_TRY(H->err, hipStreamSynchronize(H->s));
    *out = std::sqrt(H->host[0] / (double)n3);
    return ISIS_OK;
}

// The same norm of the FP32 problem's own defect (FP32 field, FP32 density,
// float arithmetic, double sums): the light judge of the judge schedule.
// Only for the tiled sizes (norm_tiled).
inline bool norm_tiled(int n)
{
    using NG = NormTileF;
    return (n & (n - 1)) == 0 && n % NG::TZ == 0 && n % NG::TY == 0 && n % NG::XC == 0;
}

template <class M>
int fine_rms_fp32(isis_mg* H, const M& m, const float* phi, const float* eta, double* out)
{
    using NG = NormTileF;
    const int n = H->d.N;
    const long n3 = (long)n * n * n;
    const double h = H->L64[0].h;
    const long tiles = (long)(n / NG::TZ) * (n / NG::TY) * (n / NG::XC);
    const int g = (int)std::min<long>(kReduceBlocks, tiles);
    hipLaunchKernelGGL((k_defect_norm_tiled<float, M, float>), dim3(g), dim3(kBlock), 0, H->s, m,
                       n, 1.0 / (h * h), 1.0, 0.0, phi, eta, nullptr, H->partial);
    LAUNCH_CHECK(H->err, "k_defect_norm_tiled");
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, H->s, H->partial, g, H->scal);
    LAUNCH_CHECK(H->err, "k_reduce");
    HIP_TRY(H->err, hipMemcpyAsync(H->host, H->scal, sizeof(double), hipMemcpyDeviceToHost, H->s));
    HIP_TRY(H->err, hipStreamSynchronize(H->s));
    *out = std::sqrt(H->host[0] / (double)n3);
    return ISIS_OK;
}

template <class T>
int sub_mean(isis_mg* H, T* f, long n3)
{
    int g = std::min(kReduceBlocks, grid_for(n3));
    hipLaunchKernelGGL((k_sum<T>), dim3(g), dim3(kBlock), 0, H->s, n3, f, H->partial);
    LAUNCH_CHECK(H->err, "k_sum");
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, H->s, H->partial, g, H->scal);
    LAUNCH_CHECK(H->err, "k_reduce");
    hipLaunchKernelGGL((k_sub_mean<T>), dim3(grid_for(n3)), dim3(kBlock), 0, H->s, n3, f, H->scal);
    LAUNCH_CHECK(H->err, "k_sub_mean");
    return ISIS_OK;
}

// Levels whose smoothing steps are timed with profiling on: an event pair
// holds the stream for a few microseconds, about the length of a whole
// smoothing step on the small levels, so those are left untimed.
constexpr int kTimedMinN = 256;

// `count` sweeps of level l (cphi: with the prolongation fused into the first
// pass); with profiling on, on levels of side >= kTimedMinN, bracketed by HIP
// events on the solver stream.
template <class T, class M>
int timed_block(isis_mg* H, const M& m, LevP<T>& f, int l, int count, const T* cphi,
                const T* cphat)
{
    const int tb = H->tb;
    const bool timed = H->profile && count > 0 && (f.n >= kTimedMinN || l == 0) &&
                       H->ntimed < isis_mg::kMaxTimed;
    const int q = H->ntimed;
    if (timed) HIP_TRY(H->err, hipEventRecord(H->ev0[q], H->s));
    // the FP32 iterate handed over to the FP64 cycles (solve_impl), read by
    // the first pass of their first smoothing step in place of the field
    const float* in32 = nullptr;
    if constexpr (sizeof(T) == 8) {
        if (l == 0 && count > 0 && H->in32) {
            in32 = H->in32;
            H->in32 = nullptr;
        }
    }
    int r = launch_sweeps<T, M>(m, f.n, f.h, &f.phi, &f.tmp, f.eta, f.sigma, count, tb, H->s,
                                H->err, kFusedSolverMinN, cphi, cphat, false, in32,
                                H->in32_scale, H->in32_offset);
    if (r) return r;
    if (timed) {
        HIP_TRY(H->err, hipEventRecord(H->ev1[q], H->s));
        const double n3 = (double)f.n * f.n * f.n;
        const int tblk = std::max(1, tb);
        const bool fused = fused_level<T, M>(f.n, tb);
        const int passes = fused ? (count + tblk - 1) / tblk : count;
        H->tlaunch[q] = fused ? fused_launches(count, tb) : 2 * count;
        H->tupd[q] = n3 * count;
        // compulsory bytes: per pass read phi, eta, write phi; the fused
        // prolongation adds the two coarse fields
        H->tbytes[q] = (double)passes * n3 * 3.0 * sizeof(T) + (cphi ? 2.0 * n3 / 8 * sizeof(T) : 0.0) -
                       (in32 ? n3 * (sizeof(T) - sizeof(float)) : 0.0);
        H->tprec[q] = sizeof(T) == 4 ? 1 : 0;
        H->tlevel[q] = l;
        H->tprol[q] = cphi ? 1 : 0;
        H->ntimed = q + 1;
    }
    return ISIS_OK;
}

// Smoothing step of level l.  cphi, cphat (the coarse level's field and its
// restriction, after the coarse-grid correction): phi += P(cphi - cphat)
// first; where prolong_fused() inside the first pass, which is then timed on
// its own, elsewhere by the prolongation kernel before the (timed) sweeps.
template <class T, class M>
int timed_sweeps(isis_mg* H, const M& m, LevP<T>& f, int l, int count, const T* cphi = nullptr,
                 const T* cphat = nullptr)
{
    constexpr int PWc = weighted_code<T, M>();
    if (cphi && H->pw && PWc != 0) {
        int r = launch_prolong<T, PWc>(f.n, f.phi, cphi, cphat, H->s, H->err);
        if (r) return r;
        return timed_block<T, M>(H, m, f, l, count, nullptr, nullptr);
    }
    if (cphi && prolong_fused<T, M>(f.n, count, H->tb)) {
        int r = timed_block<T, M>(H, m, f, l, 1, cphi, cphat);  // the first, single-sweep pass
        if (r) return r;
        return timed_block<T, M>(H, m, f, l, count - 1, nullptr, nullptr);
    }
    if (cphi) {
        int r = launch_prolong<T>(f.n, f.phi, cphi, cphat, H->s, H->err);
        if (r) return r;
    }
    return timed_block<T, M>(H, m, f, l, count, nullptr, nullptr);
}

// Levels l .. nlev-1 of the V-cycle in one launch of k_bottom_cycle.
template <class T, class M>
int launch_bottom(isis_mg* H, const M& m, LevP<T>* L, int l, double* updates)
{
    const isis_mg_desc& d = H->d;
    BottomArgs<T> a{};
    a.nlev = H->nlev - l;
    a.nu_pre = d.nu_pre;
    a.nu_post = H->nu_post;
    a.nu_coarse = d.nu_coarse;
    a.phi0 = L[l].phi;
    a.sigma0 = L[l].sigma;
    for (int q = 0; q < a.nlev; ++q) {
        const LevP<T>& v = L[l + q];
        a.eta[q] = v.eta;
        a.ih2[q] = (T)(1.0 / (v.h * v.h));
        const double n3 = (double)v.n * v.n * v.n;
        *updates += (q + 1 < a.nlev ? d.nu_pre + H->nu_post : d.nu_coarse) * n3;
    }
    constexpr int PWc = weighted_code<T, M>();
    const bool pw = H->pw && PWc != 0;
    auto kern = H->fw ? (pw ? k_bottom_cycle<T, M, true, PWc> : k_bottom_cycle<T, M, true, 0>)
                      : (pw ? k_bottom_cycle<T, M, false, PWc> : k_bottom_cycle<T, M, false, 0>);
    static std::atomic<unsigned> lds_done[4];  // per instantiation: devices set up
    HIP_TRY(H->err, ensure_dynamic_lds((const void*)kern,
                                       bottom_lds_elems(kBottomMaxLevels) * (int)sizeof(T),
                                       lds_done[(H->fw ? 1 : 0) + (pw ? 2 : 0)]));
    hipLaunchKernelGGL(kern, dim3(1), dim3(bottom_threads<T>()),
                       bottom_lds_elems(a.nlev) * (int)sizeof(T), H->s, m, a);
    LAUNCH_CHECK(H->err, "k_bottom_cycle");
    return ISIS_OK;
}

template <class T, class M>
int vcycle(isis_mg* H, const M& m, LevP<T>* L, int l, double* updates)
{
    const isis_mg_desc& d = H->d;
    LevP<T>& f = L[l];
    const double n3 = (double)f.n * f.n * f.n;
    int r;
    if (l == H->lb) return launch_bottom<T, M>(H, m, L, l, updates);
    if (l == H->nlev - 1) {
        *updates += (double)d.nu_coarse * n3;
        return launch_coarse<T, M>(m, f.h, f.phi, f.eta, f.sigma, d.nu_coarse, H->s, H->err);
    }
    LevP<T>& c = L[l + 1];
    if ((r = timed_sweeps<T, M>(H, m, f, l, d.nu_pre))) return r;
    *updates += d.nu_pre * n3;
    // full weighting: the fine defect goes through the level's scratch field,
    // free between the smoothing steps
    if ((r = launch_descend<T, M>(m, f.n, f.h, f.phi, f.eta, f.sigma, c.eta, c.phi, c.phihat,
                                  c.sigma, c.rr, H->s, H->err, H->fw ? f.tmp : nullptr)))
        return r;
    if ((r = vcycle<T, M>(H, m, L, l + 1, updates))) return r;
    // the correction phi += P(phi_c - phihat_c), then post-smoothing
    if ((r = timed_sweeps<T, M>(H, m, f, l, H->nu_post, c.phi, c.phihat))) return r;
    *updates += H->nu_post * n3;
    return ISIS_OK;
}

// Relative residual above which a jump of the FP32 cycles' factor is not taken
// for their round-off floor: FP32 floors sit within ~20 eps_32 of the scale
// of the equation's terms (symmetron ~2e-7 relative, f(R) below 1e-8).
constexpr double kFloorJumpMax = 1e-6;

// Judge schedule (desc.judge_skip): after a judged cycle whose residual rc
// fell at the mean factor rho per cycle since the previous judged one, the
// number of cycles until rc rho^m <= target is m; the next `ahead` cycles
// then run without the judge, ahead = min(m - margin, 4) >= 0.  FP64 cycles
// (margin 1) resume the judge at the cycle predicted to reach the target: the
// factors of these solves rise towards their asymptotic value, so the
// prediction errs on the early side, and a residual still above the target
// is judged again after the next cycle.  FP32 cycles (margin 2) resume one
// cycle earlier: their factor collapses at the FP32 round-off floor, which
// the prediction cannot see and which lies above the hand-over level for
// some problems (the Poisson equation of the Newtonian potential: ~4e-6
// relative), so a later judge would let cycles run on at the floor.
inline int judge_ahead(bool lazy, int cyc, double rc, double rho, double target, int margin)
{
    if (!lazy || cyc < 2 || !(rho > 0.0) || !(rho < 0.6) || !(rc > target)) return 0;
    const double m = std::ceil(std::log(target / rc) / std::log(rho));
    return (int)std::max(0.0, std::min(m - margin, 4.0));
}

// Judge schedule, FP32 cycles: a cycle whose residual is predicted to stay
// above max(kLightJudgeMin, 1e3 tol) (relative) is judged by the FP32
// problem's own defect (fine_rms_fp32), whose rounding (about the FP32
// cycles' round-off floor: 2e-7 relative for the symmetron, 4e-6 for the
// Poisson equation of the Newtonian potential) adds to the residual in
// quadrature, under 1% of it; a light result below that level is taken again
// by the FP64 judge, so the stop test and the predictive hand-over to FP64 see
// the FP64 defect.
constexpr double kLightJudgeMin = 3e-5;

// The solve for one model; M64/M32 are its double and float device models.
// In mixed precision the FP32 field is (field - shift32) * M32::kVar: f(R) in
// the paper's variable runs its FP32 cycles in ln(f_R/f_R0) (shift32 =
// ln(a^2 |f_R0|)), whose small magnitude keeps FP32 rounding small.
template <class M64, class M32>
int solve_impl(isis_mg* H, const M64& m64, const M32& m32, const isis_model_params& p,
               const double* density, double* field, double tol, int use_guess,
               isis_mg_stats* st, double shift32 = 0.0)
{
    const isis_mg_desc& d = H->d;
    const int N = d.N;
    const long n3 = (long)N * N * N;
    const bool singular = (p.model == ISIS_LINEAR && p.m2 == 0.0);
    const bool mixed = (d.precision == ISIS_MIXED);
    int r;
    H->ntimed = 0;
    H->in32 = nullptr;
    HIP_TRY(H->err, hipMemsetAsync(H->hits(), 0, sizeof(unsigned long long), H->s));
    H->L64[0].phi = field;
    H->L64[0].tmp = H->tmp0;
    H->L64[0].eta = const_cast<double*>(density);
    H->L64[0].sigma = nullptr;
    // r_ref from the cold start, whatever the initial guess.  Without a
    // guess the cold start is built in the field itself (in mixed precision
    // together with the FP32 copy the first cycle starts from); its sum of
    // squares serves the exact-root test below.  The density hierarchy: in
    // mixed precision each restriction also writes the FP32 copy of its fine
    // level (the coarsest is converted below).
    double* cold = use_guess ? H->L64[0].tmp : field;
    const bool cold32 = mixed && !use_guess && !singular;
    const double h0 = H->L64[0].h;
    double cold_rms, r_ref;
    using NG = NormTileF;
    // From the cold start in mixed precision the FP32 copy is the field the
    // cycles start from; the FP64 field is needed only if the FP32 phase
    // does not run or does not promote its iterate, and is then written
    // there (cold_pending).
    bool cold_pending = false;
    if ((N & (N - 1)) == 0 && N % NG::TZ == 0 && N % NG::TY == 0 && N % NG::XC == 0) {
        cold_pending = cold32;
        // one pass over the FP64 density: cold start, its copies, the
        // density's FP32 copy and first restriction, and both sums
        const long tiles = (long)(N / NG::TZ) * (N / NG::TY) * (N / NG::XC);
        const int g = (int)std::min<long>(kReduceBlocks, tiles);
        hipLaunchKernelGGL((k_setup_tiled<M64>), dim3(g), dim3(kBlock), 0, H->s, m64, N,
                           1.0 / (h0 * h0), density, cold_pending ? nullptr : cold,
                           cold32 ? H->L32[0].phi : nullptr,
                           M32::kVar, -shift32 * M32::kVar, mixed ? H->L32[0].eta : nullptr,
                           H->L64[1].eta, H->partial, H->partial + kReduceBlocks);
        LAUNCH_CHECK(H->err, "k_setup_tiled");
        for (int l = 2; l < H->nlev; ++l)
            if ((r = launch_restrict<double>(H->L64[l - 1].n, H->L64[l - 1].eta, H->L64[l].eta,
                                             H->s, H->err, mixed ? H->L32[l - 1].eta : nullptr)))
                return r;
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, H->s, H->partial, g, H->scal);
        LAUNCH_CHECK(H->err, "k_reduce");
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, H->s, H->partial + kReduceBlocks, g,
                           H->scal + 1);
        LAUNCH_CHECK(H->err, "k_reduce");
        HIP_TRY(H->err, hipMemcpyAsync(H->host, H->scal, 2 * sizeof(double),
                                       hipMemcpyDeviceToHost, H->s));
        HIP_TRY(H->err, hipStreamSynchronize(H->s));
        r_ref = std::sqrt(H->host[0] / (double)n3);
        cold_rms = std::sqrt(H->host[1] / (double)n3);
    } else {
        for (int l = 1; l < H->nlev; ++l)
            if ((r = launch_restrict<double>(H->L64[l - 1].n, H->L64[l - 1].eta, H->L64[l].eta,
                                             H->s, H->err, mixed ? H->L32[l - 1].eta : nullptr)))
                return r;
        const int g = std::min(kReduceBlocks, grid_for(n3));
        hipLaunchKernelGGL((k_cold_start_sumsq<M64>), dim3(g), dim3(kBlock), 0, H->s, m64, n3,
                           density, cold, cold32 ? H->L32[0].phi : nullptr, M32::kVar,
                           -shift32 * M32::kVar, H->partial);
        LAUNCH_CHECK(H->err, "k_cold_start_sumsq");
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, H->s, H->partial, g, H->scal);
        LAUNCH_CHECK(H->err, "k_reduce");
        HIP_TRY(H->err,
                hipMemcpyAsync(H->host, H->scal, sizeof(double), hipMemcpyDeviceToHost, H->s));
        HIP_TRY(H->err, hipStreamSynchronize(H->s));
        cold_rms = std::sqrt(H->host[0] / (double)n3);
        if ((r = fine_rms<double, M64>(H, m64, cold, density, nullptr, &r_ref))) return r;
    }
    // A cold-start residual at the rounding level of its Laplacian means the
    // cold start is an exact root (uniform density): absolute tolerance.
    if (!std::isfinite(r_ref)) {
        fmt_err(H->err, "density gives a non-finite cold-start residual (NaN/Inf or invalid "
                        "values in eta)");
        return ISIS_ERR_INVALID_ARG;
    }
    const double cold_scale = 1e-14 * 6.0 / (h0 * h0) * cold_rms;
    if (singular && (r = sub_mean<double>(H, field, n3))) return r;
    const double rnorm = r_ref > cold_scale ? r_ref : 1.0;
    LevP<double>& F = H->L64[0];  // F.phi: the current finest field (may move to tmp0)
    double r0 = r_ref;            // the field is the cold start (zero-mean for LINEAR m2 = 0)
    if (use_guess && (r = fine_rms<double, M64>(H, m64, field, density, nullptr, &r0))) return r;
    // use_guess = 2: keep the guess only if it is at least as close to the
    // root as one cold-started V-cycle gets (so that it cannot cost a cycle):
    // RMS residual <= accept * r_ref, accept = desc.guess_accept, else the
    // first-cycle factor of this handle's last cold solve of the model, else
    // 1e-2 (the first cold cycle reduces the residual by ~100x or more on the
    // lognormal + halo densities).
    const double accept = d.guess_accept > 0.0 ? d.guess_accept
                          : H->cold_first[p.model] > 0.0 ? H->cold_first[p.model] : 1e-2;
    if (use_guess == 2 && !(r0 <= accept * r_ref)) {
        // the supplied guess cannot save a cycle over the cold start: use the latter
        HIP_TRY(H->err, hipMemcpyAsync(field, cold, sizeof(double) * n3,
                                       hipMemcpyDeviceToDevice, H->s));
        if (singular && (r = sub_mean<double>(H, field, n3))) return r;
        if ((r = fine_rms<double, M64>(H, m64, field, density, nullptr, &r0))) return r;
        use_guess = 0;
    }
    if (st) {
        st->r_ref = r_ref;
        st->r0 = r0;
        st->rel_hist[0] = r0 / rnorm;
        st->used_guess = use_guess ? 1 : 0;
    }
    double updates = 0.0, rcur = r0;
    double first_rel = 0.0;  // relative residual after the first cycle
    int cyc = 0, cyc32 = 0;
    int status = ISIS_ERR_NOT_CONVERGED;
    if (!std::isfinite(r0)) status = ISIS_ERR_DIVERGED;
    else if (r0 <= tol * rnorm) status = ISIS_OK;

    const bool lazy = d.judge_skip != 0;
    int blind = 0, judged = 0, cprev = 0;  // judge schedule; cprev: last judged cycle
    int judged_fp32 = 0;                   // of which by the light (FP32) judge
    // Mixed precision, phase 1: FP32 V-cycles on the FP32 copy of the
    // problem, monitored by the FP64 defect of the FP32 iterate.  Skipped when
    // the initial field is already near the FP32 round-off floor, where FP32
    // cycles cannot lower the residual.
    if (mixed && status == ISIS_ERR_NOT_CONVERGED && r0 > kFloorJumpMax * rnorm) {
        {  // the coarsest density (the finer ones came with the restrictions)
            const int l = H->nlev - 1;
            long c3 = (long)H->L32[l].n * H->L32[l].n * H->L32[l].n;
            hipLaunchKernelGGL((k_convert<float, double>), dim3(grid_for(c3)), dim3(kBlock), 0,
                               H->s, c3, H->L64[l].eta, H->L32[l].eta, 1.0, 0.0);
            LAUNCH_CHECK(H->err, "k_convert");
        }
        // the FP32 models may carry a scaled variable (f(R): u / ln 2); from
        // the cold start the copy was written by k_cold_start_sumsq
        if (!cold32) {
            hipLaunchKernelGGL((k_convert<float, double>), dim3(grid_for(n3)), dim3(kBlock), 0,
                               H->s, n3, field, H->L32[0].phi, M32::kVar, -shift32 * M32::kVar);
            LAUNCH_CHECK(H->err, "k_convert");
        }
        H->L32[0].sigma = nullptr;
        // The last cycle runs in FP64, so the answer carries FP64-cycle error
        // (an FP32-only solve meeting the same tol is ~10% less accurate in phi
        // for f(R)).  Default hand-over: as soon as one more cycle at the last
        // factor is expected to reach tol (with a 0.7 margin), so that a single
        // FP64 cycle finishes the solve; with desc.fp32_floor set, at that
        // level instead.  An earlier stall of the FP32 cycles at their
        // round-off floor also hands over.
        const bool predict = !(d.fp32_floor > 0.0);
        const double fp32_floor = predict ? 0.0 : d.fp32_floor;
        double rprev = r0, rho_prev = 1.0;
        bool fp32_failed = false;
        // Light judges (judge schedule): the FP32 problem's defect is the
        // FP64 one's only where both solve in the same variable.
        const bool light_ok = lazy && shift32 == 0.0 && norm_tiled(N);
        const double light_min = std::max(kLightJudgeMin, 1e3 * tol) * rnorm;
        const double first_factor =
            H->cold_first[p.model] > 0.0 ? H->cold_first[p.model] : 1e-2;
        while (cyc < d.max_cycles) {
            H->fw = cyc < H->fw_first ? 1 : H->fw_after;
            if ((r = vcycle<float, M32>(H, m32, H->L32, 0, &updates))) return r;
            if (singular && (r = sub_mean<float>(H, H->L32[0].phi, n3))) return r;
            ++cyc;
            ++cyc32;
            if (blind > 0 && cyc < d.max_cycles) {  // not judged (desc.judge_skip)
                --blind;
                if (st) st->rel_hist[cyc] = std::nan("");
                continue;
            }
            blind = 0;
            ++judged;
            double rc = 0.0;
            // predicted residual: the last judged one at the mean factor per
            // cycle since (before the first judged cycle, the model's
            // first-cycle factor)
            const double rho_est = judged == 1 ? first_factor : rho_prev;
            bool light = light_ok && rprev * std::pow(rho_est, cyc - cprev) >= light_min;
            if (light) {
                if ((r = fine_rms_fp32<M32>(H, m32, H->L32[0].phi, H->L32[0].eta, &rc))) return r;
                light = rc >= light_min;  // else (or NaN) the FP64 judge decides
            }
            if (light) ++judged_fp32;
            else if ((r = fine_rms<float, M64>(H, m64, H->L32[0].phi, density, nullptr, &rc,
                                               M32::kVarInv, shift32)))
                return r;
            if (st) st->rel_hist[cyc] = rc / rnorm;
            if (cyc == 1) first_rel = rc / rnorm;
            rcur = rc;
            if (!std::isfinite(rc) || rc > 1e3 * r0) {
                // the FP32 cycles failed: the FP64 cycles start over from the
                // FP64 field, which the FP32 phase has not touched
                fp32_failed = true;
                break;
            }
            if (rc <= tol * rnorm) {
                status = ISIS_OK;
                break;
            }
            // Refine in FP64 once the FP32 cycles reach their round-off floor:
            // a cycle reduces the residual by less than 0.6x, or, near FP32
            // round-off (kFloorJumpMax), its factor jumps to more than 3x the
            // previous cycle's (and above 0.2) as the floor comes into view;
            // or once one more cycle is expected to finish (default), or at
            // the caller's hand-over level.  Far above round-off a rising
            // factor is the cycle's own asymptotic rate settling in (f(R)
            // with three sweeps per side: 0.06 then 0.23 at 3e-5).  rho is
            // the mean factor per cycle since the previous judged cycle.
            const int gap = cyc - cprev;
            const double rho = gap == 1 ? rc / rprev : std::pow(rc / rprev, 1.0 / gap);
            const bool jump = rho > 0.2 && rho > 3.0 * rho_prev && rc <= kFloorJumpMax * rnorm;
            if (rho > 0.6 || jump ||
                (predict ? rc * rho <= 0.7 * tol * rnorm : rc <= fp32_floor * rnorm))
                break;
            // a factor more than twice the previous judged one (that of a
            // cycle after the first, which starts from the cold start) may be
            // the floor coming into view: judge the next cycle too
            const bool rising = cprev >= 2 && rho > 2.0 * rho_prev;
            rho_prev = rho;
            rprev = rc;
            cprev = cyc;
            // the FP32 phase hands over one cycle early: aim one cycle short
            blind = rising ? 0
                           : judge_ahead(lazy, cyc, rc, rho, tol * rnorm / std::max(rho, 1e-300), 2);
        }
        // Promote the FP32 iterate unless it is no better than the field the
        // phase started from (then the FP64 cycles continue from that field).
        // When FP64 cycles follow and their first finest-level smoothing pass
        // is a fused one, that pass reads the FP32 iterate itself (timed_block)
        // instead of a converted copy.
        if (!fp32_failed && rcur < r0) {
            const bool fp64_next = status != ISIS_OK && cyc < d.max_cycles;
            if (fp64_next && d.nu_pre > 0 && H->lb != 0 && H->nlev > 1 &&
                fused_level<double, M64>(N, H->tb)) {
                H->in32 = H->L32[0].phi;
                H->in32_scale = M32::kVarInv;
                H->in32_offset = shift32;
            } else {
                hipLaunchKernelGGL((k_convert<double, float>), dim3(grid_for(n3)), dim3(kBlock),
                                   0, H->s, n3, H->L32[0].phi, F.phi, M32::kVarInv, shift32);
                LAUNCH_CHECK(H->err, "k_convert");
            }
            cold_pending = false;
        } else {
            status = ISIS_ERR_NOT_CONVERGED;
            rcur = r0;
        }
    }
    if (cold_pending) {  // the FP64 field is the cold start after all
        hipLaunchKernelGGL((k_cold_start<double, M64>), dim3(grid_for(n3)), dim3(kBlock), 0, H->s,
                           m64, n3, density, field);
        LAUNCH_CHECK(H->err, "k_cold_start");
    }

    // FP64 V-cycles (the whole solve in ISIS_FP64; the refinement phase in
    // ISIS_MIXED).
    // residual at the last judged cycle, clast (the FP32 phase ends with a
    // judged cycle, or restarts from the initial field's r0)
    double rlast = rcur;
    int clast = cyc;
    double rho_last = 0.0;  // factor at the last judged FP64 cycle after the first cycle
    blind = 0;
    while (status == ISIS_ERR_NOT_CONVERGED && cyc < d.max_cycles) {
        H->fw = cyc < H->fw_first ? 1 : H->fw_after;
        if ((r = vcycle<double, M64>(H, m64, H->L64, 0, &updates))) return r;
        if (singular && (r = sub_mean<double>(H, F.phi, n3))) return r;
        ++cyc;
        if (blind > 0 && cyc < d.max_cycles) {  // not judged (desc.judge_skip)
            --blind;
            if (st) st->rel_hist[cyc] = std::nan("");
            continue;
        }
        blind = 0;
        ++judged;
        double rc;
        if ((r = fine_rms<double, M64>(H, m64, F.phi, density, nullptr, &rc))) return r;
        if (st) st->rel_hist[cyc] = rc / rnorm;
        if (cyc == 1) first_rel = rc / rnorm;
        rcur = rc;
        if (!std::isfinite(rc) || rc > 1e3 * r0) status = ISIS_ERR_DIVERGED;
        else if (rc <= tol * rnorm) status = ISIS_OK;
        else {
            const int gap = cyc - clast;
            const double rho = std::pow(rc / rlast, 1.0 / std::max(gap, 1));
            // erratic or rising factors (more than twice the last): no skipping
            const bool rising = rho_last > 0.0 && rho > 2.0 * rho_last;
            blind = rising ? 0 : judge_ahead(lazy, cyc, rc, rho, tol * rnorm, 1);
            if (cyc >= 2) rho_last = rho;
        }
        rlast = rc;
        clast = cyc;
    }
    if (F.phi != field) {  // an odd number of fused passes left the result in tmp0
        HIP_TRY(H->err, hipMemcpyAsync(field, F.phi, sizeof(double) * n3,
                                       hipMemcpyDeviceToDevice, H->s));
        F.tmp = F.phi;
        F.phi = field;
    }
    unsigned long long* hits_host = reinterpret_cast<unsigned long long*>(H->host + 8);
    HIP_TRY(H->err, hipMemcpyAsync(hits_host, H->hits(), sizeof(unsigned long long),
                                   hipMemcpyDeviceToHost, H->s));
    HIP_TRY(H->err, hipStreamSynchronize(H->s));
    if (st && H->profile) {
        for (int q = 0; q < H->ntimed; ++q) {
            float e = 0.f;
            HIP_TRY(H->err, hipEventElapsedTime(&e, H->ev0[q], H->ev1[q]));
            st->ms_smooth += e;
            if (H->tlevel[q] != 0) continue;
            const int k = H->tprec[q];
            if (H->tprol[q]) {
                st->fine_prol_ms[k] += e;
                st->fine_prol_launches[k] += H->tlaunch[q];
                st->fine_prol_bytes[k] += H->tbytes[q];
                continue;
            }
            st->fine_sweep_ms[k] += e;
            st->fine_sweep_launches[k] += H->tlaunch[q];
            st->fine_sweep_updates[k] += H->tupd[q];
            st->fine_sweep_bytes[k] += H->tbytes[q];
        }
    }
    if (!use_guess && status == ISIS_OK && first_rel > 0.0 && first_rel < 1.0)
        H->cold_first[p.model] = first_rel;
    if (st) {
        st->cycles = cyc;
        st->cycles_fp32 = cyc32;
        st->rel_res = rcur / rnorm;
        st->cell_updates = updates;
        st->safeguard_hits = (long long)*hits_host;
        st->judged_cycles = judged;
        st->judged_fp32 = judged_fp32;
        // per-cycle factors; after cycles without the judge, the mean factor
        // per cycle since the previous judged one (NaN for the unjudged ones)
        int prev = 0;
        for (int k = 1; k <= cyc; ++k) {
            if (std::isnan(st->rel_hist[k])) {
                st->rho_hist[k] = std::nan("");
                continue;
            }
            const double a0 = st->rel_hist[prev];
            st->rho_hist[k] = a0 > 0.0 ? std::pow(st->rel_hist[k] / a0, 1.0 / (k - prev)) : 0.0;
            prev = k;
        }
    }
    if (status == ISIS_ERR_NOT_CONVERGED)
        fmt_err(H->err, "not converged after %d cycles (rel. residual %.3e)", cyc, rcur / rnorm);
    if (status == ISIS_ERR_DIVERGED)
        fmt_err(H->err, "diverged after %d cycles (residual %.3e, initial %.3e)", cyc, rcur, r0);
    return status;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI.
// ---------------------------------------------------------------------------

namespace {

template <ScalarForce SF, bool POT>
int launch_force_t(int n, double h, double c, const double* field, const double* pot, double* fx,
                   double* fy, double* fz, hipStream_t s, char* err)
{
    using FG = ForceTileF;
    const double inv2h = 0.5 / h;
    if ((n & (n - 1)) == 0 && n % FG::TZ == 0 && n % FG::TY == 0 && n % FG::XC == 0) {
        const long tiles = (long)(n / FG::TZ) * (n / FG::TY) * (n / FG::XC);
        const int g = (int)std::min<long>(8192, tiles);
        hipLaunchKernelGGL((k_force_tiled<SF, POT>), dim3(g), dim3(kBlock), 0, s, n, inv2h, c,
                           field, pot, fx, fy, fz);
    } else {
        hipLaunchKernelGGL((k_force_cells<SF, POT>), dim3(grid_for((long)n * n * n)),
                           dim3(kBlock), 0, s, n, inv2h, c, field, pot, fx, fy, fz);
    }
    LAUNCH_CHECK(err, "k_force");
    return ISIS_OK;
}

template <ScalarForce SF>
int launch_force(int n, double h, double c, const double* field, const double* pot, double* fx,
                 double* fy, double* fz, hipStream_t s, char* err)
{
    return pot ? launch_force_t<SF, true>(n, h, c, field, pot, fx, fy, fz, s, err)
               : launch_force_t<SF, false>(n, h, c, field, pot, fx, fy, fz, s, err);
}

// Scratch of isis_mg_residual_noalloc: the defect norm's per-block partial
// sums and their total, in a static device array (every device the library
// runs on holds its own copy until the process ends).  Host code never passes
// the array's name to a kernel or copy: it uses the device's address of it,
// looked up once per device with hipGetSymbolAddress.
constexpr int kStaticScratch = kReduceBlocks + 16;  // doubles: 64 KiB + 128 B
static __device__ __align__(256) double scratch[kStaticScratch];
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices];

// The current device's address of `scratch`.
int static_scratch(double** out, char* err)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(err, e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) {
        fmt_err(err, "device %d: the static scratch supports devices 0..%d", dev, kMaxDevices - 1);
        return ISIS_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(err, e, "hipGetSymbolAddress(scratch)");
        if (!p) {
            fmt_err(err, "hipGetSymbolAddress(scratch) returned NULL");
            return ISIS_ERR_HIP;
        }
        g_scratch_dev[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_dev[dev];
    return ISIS_OK;
}

}  // namespace

extern "C" {

size_t isis_mg_workspace_size(const isis_mg_desc* desc)
{
    char err[512];
    if (!valid_desc(desc, err)) return 0;
    return carve(*desc, nullptr, nullptr);
}

int isis_mg_create(const isis_mg_desc* desc, isis_mg_t** out)
{
    if (!out) {
        fmt_err(g_err, "out is NULL");
        return ISIS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    if (!valid_desc(desc, g_err)) return ISIS_ERR_INVALID_ARG;
    size_t need = carve(*desc, nullptr, nullptr);
    if (!desc->workspace || desc->workspace_bytes < need || !aligned(desc->workspace, 256)) {
        fmt_err(g_err, "workspace must be 256-byte aligned and >= %zu bytes", need);
        return ISIS_ERR_INVALID_ARG;
    }
    isis_mg* H = new (std::nothrow) isis_mg();
    if (!H) {
        fmt_err(g_err, "out of host memory");
        return ISIS_ERR_HIP;
    }
    H->d = *desc;
    H->nlev = num_levels(desc->N);
    H->lb = bottom_level(desc->N, H->nlev);
    H->s = (hipStream_t)desc->stream;
    H->err[0] = 0;
    if (hipGetDevice(&H->device) != hipSuccess ||
        hipHostMalloc((void**)&H->host, 16 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        fmt_err(g_err, "HIP device or pinned host buffer unavailable");
        delete H;
        return ISIS_ERR_HIP;
    }
    carve(*desc, (char*)desc->workspace, H);
    *out = H;
    return ISIS_OK;
}

int isis_mg_set_profiling(isis_mg_t* h, int enable)
{
    if (!h) {
        fmt_err(g_err, "handle is NULL");
        return ISIS_ERR_INVALID_ARG;
    }
    if (enable && !h->events_ready) {
        if (hipSetDevice(h->device) != hipSuccess)
            return hip_fail(h->err, hipGetLastError(), "hipSetDevice");
        for (int q = 0; q < isis_mg::kMaxTimed; ++q) {
            if (!h->ev0[q]) HIP_TRY(h->err, hipEventCreate(&h->ev0[q]));
            if (!h->ev1[q]) HIP_TRY(h->err, hipEventCreate(&h->ev1[q]));
        }
        h->events_ready = 1;
    }
    h->profile = enable ? 1 : 0;
    return ISIS_OK;
}

void isis_mg_destroy(isis_mg_t* h)
{
    if (!h) return;
    for (int q = 0; q < isis_mg::kMaxTimed; ++q) {
        if (h->ev0[q]) (void)hipEventDestroy(h->ev0[q]);
        if (h->ev1[q]) (void)hipEventDestroy(h->ev1[q]);
    }
    if (h->host) (void)hipHostFree(h->host);
    delete h;
}

const char* isis_mg_last_error(const isis_mg_t* h)
{
    return h ? h->err : g_err;
}

int isis_mg_solve(isis_mg_t* H, const double* density, double* field,
                  const isis_model_params* params, double a, double tol, int use_guess,
                  isis_mg_stats* stats)
{
    if (!H) {
        fmt_err(g_err, "handle is NULL");
        return ISIS_ERR_INVALID_ARG;
    }
    H->err[0] = 0;
    auto t0 = std::chrono::steady_clock::now();
    if (!density || !field || !aligned(density, 16) || !aligned(field, 16)) {
        fmt_err(H->err, "density and field must be non-NULL, 16-byte aligned device pointers");
        return ISIS_ERR_INVALID_ARG;
    }
    if (!valid_params(params, a, H->err)) return ISIS_ERR_INVALID_ARG;
    if (!(tol > 0.0) || !std::isfinite(tol)) {
        fmt_err(H->err, "tol must be finite and > 0");
        return ISIS_ERR_INVALID_ARG;
    }
    if (hipSetDevice(H->device) != hipSuccess) return hip_fail(H->err, hipGetLastError(), "hipSetDevice");
    if (stats) memset(stats, 0, sizeof(*stats));
    // Per-model temporal block (desc.temporal_block = -1): two sweeps per HBM
    // pass for the canonical models, whose fused sweeps are HBM-bound; one for
    // f(R) and the chameleon, whose two-sweep kernels are arithmetic- and
    // register-bound (measured at 512^3: symmetron -8 %, f(R) +32 %).
    H->tb = H->d.temporal_block >= 0 ? H->d.temporal_block
            : (params->model == ISIS_FR_HS || params->model == ISIS_CHAMELEON) ? 1 : 2;
    if (stats) stats->temporal_block = H->tb;
    // Per-model prolongation (desc.prolongation = -1): weighted by the flux
    // coefficient e^u for f(R), trilinear for the others (the chameleon: no
    // change).  Per-model restriction of the defect (desc.restriction = -1):
    // for f(R) with the weighted prolongation, full weighting in the first
    // two V-cycles of the solve and the 8-child mean after them; full
    // weighting throughout with the trilinear one; the mean for the other
    // models (for the canonical models and the chameleon full weighting took
    // one to two cycles more).  Measured on f(R) solves to 1e-8 over
    // |f_R0| = 1e-4 .. 1e-6, a = 0.5 .. 1, n = 1, 2 and three densities: the
    // mean from the first cycle diverged twice at 512^3 (its first or second
    // cycle), full weighting throughout converged everywhere in 7-9 cycles,
    // two full-weighting cycles and then the mean everywhere in 6-7 (8 -> 7
    // on the 512^3 halo workload; 11 with the trilinear prolongation, which
    // also diverged once).
    const bool flux_form = params->model == ISIS_FR_HS || params->model == ISIS_CHAMELEON;
    H->pw = H->d.prolongation >= 0 ? H->d.prolongation : (params->model == ISIS_FR_HS ? 1 : 0);
    if (H->pw && !flux_form) {
        fmt_err(H->err, "the coefficient-weighted prolongation needs a flux-form model "
                        "(f(R) or the chameleon)");
        return ISIS_ERR_UNSUPPORTED;
    }
    H->fw_first = 0;
    if (H->d.restriction >= 0)
        H->fw_after = H->d.restriction;
    else if (params->model == ISIS_FR_HS && H->pw) {
        H->fw_after = 0;
        H->fw_first = 2;
    } else {
        H->fw_after = params->model == ISIS_FR_HS ? 1 : 0;
    }
    H->fw = H->fw_first > 0 ? 1 : H->fw_after;
    H->nu_post = H->d.nu_post >= 0 ? H->d.nu_post : default_nu_post(params->model);
    if (stats) {
        stats->restriction = H->fw_first > 0 ? 2 : H->fw_after;
        stats->prolongation = H->pw;
        stats->nu_pre = H->d.nu_pre;
        stats->nu_post = H->nu_post;
    }
    int r;
    switch (params->model) {
    case ISIS_SYMMETRON:
        r = solve_impl(H, make_symmetron<double>(*params, a, H->hits()),
                       make_symmetron<float>(*params, a, H->hits()), *params, density, field, tol,
                       use_guess, stats);
        break;
    case ISIS_FR_HS: {
        isis_model_params q = *params;  // FP32 cycles in ln(f_R/f_R0) (see solve_impl)
        q.paper_u = 0;
        const double shift32 = params->paper_u ? std::log(a * a * params->fR0_abs) : 0.0;
        r = solve_impl(H, make_fofr<double>(*params, a), make_fofr<float>(q, a), *params, density,
                       field, tol, use_guess, stats, shift32);
        break;
    }
    case ISIS_CHAMELEON:
        r = solve_impl(H, make_chameleon<double>(*params), make_chameleon<float>(*params),
                       *params, density, field, tol, use_guess, stats);
        break;
    default:
        r = solve_impl(H, make_linear<double>(*params), make_linear<float>(*params), *params,
                       density, field, tol, use_guess, stats);
        break;
    }
    H->in32 = nullptr;  // a solve that ended early may not have consumed it
    if (stats) {
        auto t1 = std::chrono::steady_clock::now();
        stats->ms_total = std::chrono::duration<double, std::milli>(t1 - t0).count();
    }
    return r;
}

int isis_mg_residual(isis_mg_t* H, const double* density, const double* field,
                     const isis_model_params* params, double a, double* out_res, double* out_rms)
{
    if (!H) {
        fmt_err(g_err, "handle is NULL");
        return ISIS_ERR_INVALID_ARG;
    }
    H->err[0] = 0;
    if (!density || !field || !aligned(density, 16) || !aligned(field, 16) ||
        (out_res && !aligned(out_res, 16))) {
        fmt_err(H->err, "density, field (and out_res) must be 16-byte aligned device pointers");
        return ISIS_ERR_INVALID_ARG;
    }
    if (!valid_params(params, a, H->err)) return ISIS_ERR_INVALID_ARG;
    if (hipSetDevice(H->device) != hipSuccess) return hip_fail(H->err, hipGetLastError(), "hipSetDevice");
    double rms = 0.0;
    int r = with_model<double>(*params, a, [&](auto m) {
        return fine_rms<double, decltype(m)>(H, m, field, density, out_res, &rms);
    });
    if (r) return r;
    if (out_rms) *out_rms = rms;
    return ISIS_OK;
}

int isis_mg_residual_noalloc(const isis_model_params* params, double a, int N, double box,
                             const double* density, const double* field, double* out_res,
                             double* out_rms, void* stream)
{
    g_err[0] = 0;
    if (!valid_params(params, a, g_err)) return ISIS_ERR_INVALID_ARG;
    if (!is_pow2_ge(N, 8) || N > 4096) {
        fmt_err(g_err, "residual_noalloc: N must be a power of two in [8, 4096] (got %d)", N);
        return ISIS_ERR_INVALID_ARG;
    }
    if (!finite_pos(box)) {
        fmt_err(g_err, "residual_noalloc: box must be finite and > 0");
        return ISIS_ERR_INVALID_ARG;
    }
    if (!density || !field || !aligned(density, 16) || !aligned(field, 16) ||
        (out_res && !aligned(out_res, 16))) {
        fmt_err(g_err, "residual_noalloc: density, field (and out_res) must be 16-byte aligned "
                       "device pointers");
        return ISIS_ERR_INVALID_ARG;
    }
    double* sc = nullptr;
    int r = static_scratch(&sc, g_err);
    if (r) return r;
    hipStream_t s = (hipStream_t)stream;
    const double h = box / N;
    r = with_model<double>(*params, a, [&](auto m) {
        return launch_defect_norm<double, decltype(m)>(m, N, h, field, density, out_res, sc,
                                                       sc + kReduceBlocks, s, g_err);
    });
    if (r) return r;
    if (out_rms) {
        double total = 0.0;
        HIP_TRY(g_err, hipMemcpyAsync(&total, sc + kReduceBlocks, sizeof(double),
                                      hipMemcpyDeviceToHost, s));
        HIP_TRY(g_err, hipStreamSynchronize(s));
        *out_rms = std::sqrt(total / ((double)N * N * N));
    }
    return ISIS_OK;
}

static bool op_grid_ok(int n, int lo)
{
    return n >= lo && n % 2 == 0 && n <= 4096;
}

// Every array argument (NULL allowed where optional) 16-byte aligned.
static bool ptrs_aligned(std::initializer_list<const void*> ps)
{
    for (const void* q : ps)
        if (q && !aligned(q, 16)) {
            fmt_err(g_err, "array pointers must be 16-byte aligned");
            return false;
        }
    return true;
}

int isis_op_halfsweep(const isis_model_params* p, double a, int n, double h, double* phi,
                      const double* eta, const double* sigma, int colour, void* stream)
{
    if (!valid_params(p, a, g_err)) return ISIS_ERR_INVALID_ARG;
    if (!op_grid_ok(n, 2) || !finite_pos(h) || !phi || !eta || (colour != 0 && colour != 1)) {
        fmt_err(g_err, "halfsweep: need even n >= 2, h > 0, phi/eta non-NULL, colour 0 or 1");
        return ISIS_ERR_INVALID_ARG;
    }
    if (!ptrs_aligned({phi, eta, sigma})) return ISIS_ERR_INVALID_ARG;
    return with_model<double>(*p, a, [&](auto m) {
        return launch_halfsweep<double, decltype(m)>(m, n, h, phi, eta, sigma, colour,
                                                     (hipStream_t)stream, g_err);
    });
}

int isis_op_sweeps(const isis_model_params* p, double a, int n, double h, double* phi,
                   double* tmp, const double* eta, const double* sigma, int count,
                   int temporal_block, void* stream)
{
    if (!valid_params(p, a, g_err)) return ISIS_ERR_INVALID_ARG;
    if (!op_grid_ok(n, 2) || !finite_pos(h) || !phi || !tmp || !eta || count < 0 ||
        temporal_block < 0 || temporal_block > 2) {
        fmt_err(g_err, "sweeps: need even n >= 2, h > 0, phi/tmp/eta non-NULL, count >= 0, "
                       "temporal_block in 0..2");
        return ISIS_ERR_INVALID_ARG;
    }
    if (!ptrs_aligned({phi, tmp, eta, sigma})) return ISIS_ERR_INVALID_ARG;
    return with_model<double>(*p, a, [&](auto m) {
        double* cur = phi;
        double* other = tmp;
        int r = launch_sweeps<double, decltype(m)>(m, n, h, &cur, &other, eta, sigma, count,
                                                   temporal_block, (hipStream_t)stream, g_err,
                                                   kFusedMinN);
        if (r) return r;
        if (cur != phi)
            HIP_TRY(g_err, hipMemcpyAsync(phi, cur, sizeof(double) * (size_t)n * n * n,
                                          hipMemcpyDeviceToDevice, (hipStream_t)stream));
        return (int)ISIS_OK;
    });
}

int isis_op_prolong_sweeps(const isis_model_params* p, double a, int n, double h, double* phi,
                           double* tmp, const double* eta, const double* sigma,
                           const double* coarse, const double* coarse_hat, int count,
                           int temporal_block, void* stream)
{
    if (!valid_params(p, a, g_err)) return ISIS_ERR_INVALID_ARG;
    if (!op_grid_ok(n, 4) || !finite_pos(h) || !phi || !tmp || !eta || !coarse ||
        !coarse_hat || count < 0 || temporal_block < 0 || temporal_block > 2) {
        fmt_err(g_err, "prolong_sweeps: need even n >= 4, h > 0, phi/tmp/eta/coarse/coarse_hat "
                       "non-NULL, count >= 0, temporal_block in 0..2");
        return ISIS_ERR_INVALID_ARG;
    }
    if (!ptrs_aligned({phi, tmp, eta, sigma, coarse, coarse_hat})) return ISIS_ERR_INVALID_ARG;
    return with_model<double>(*p, a, [&](auto m) {
        double* cur = phi;
        double* other = tmp;
        int r = launch_sweeps<double, decltype(m)>(m, n, h, &cur, &other, eta, sigma, count,
                                                   temporal_block, (hipStream_t)stream, g_err,
                                                   kFusedMinN, coarse, coarse_hat);
        if (r) return r;
        if (cur != phi)
            HIP_TRY(g_err, hipMemcpyAsync(phi, cur, sizeof(double) * (size_t)n * n * n,
                                          hipMemcpyDeviceToDevice, (hipStream_t)stream));
        return (int)ISIS_OK;
    });
}

int isis_op_defect(const isis_model_params* p, double a, int n, double h, const double* phi,
                   const double* eta, const double* sigma, double* out, void* stream)
{
    if (!valid_params(p, a, g_err)) return ISIS_ERR_INVALID_ARG;
    if (!op_grid_ok(n, 2) || !finite_pos(h) || !phi || !eta || !out) {
        fmt_err(g_err, "defect: need even n >= 2, h > 0, phi/eta/out non-NULL");
        return ISIS_ERR_INVALID_ARG;
    }
    if (!ptrs_aligned({phi, eta, sigma, out})) return ISIS_ERR_INVALID_ARG;
    return with_model<double>(*p, a, [&](auto m) {
        using M = decltype(m);
        hipLaunchKernelGGL((k_defect<double, M>), dim3(grid_for((long)n * n * n)), dim3(kBlock),
                           0, (hipStream_t)stream, m, n, 1.0 / (h * h), phi, eta, sigma, out);
        LAUNCH_CHECK(g_err, "k_defect");
        return (int)ISIS_OK;
    });
}

int isis_op_restrict(int n_fine, const double* fine, double* coarse, void* stream)
{
    if (!op_grid_ok(n_fine, 2) || !fine || !coarse) {
        fmt_err(g_err, "restrict: need even n_fine >= 2 and non-NULL arrays");
        return ISIS_ERR_INVALID_ARG;
    }
    if (!ptrs_aligned({fine, coarse})) return ISIS_ERR_INVALID_ARG;
    return launch_restrict<double>(n_fine, fine, coarse, (hipStream_t)stream, g_err);
}

int isis_op_fas_descend(const isis_model_params* p, double a, int n_fine, double h_fine,
                        const double* phi_f, const double* eta_f, const double* sigma_f,
                        const double* eta_c, double* phi_c, double* phihat_c, double* sigma_c,
                        double* rr_c, double* fine_scratch, void* stream)
{
    if (!valid_params(p, a, g_err)) return ISIS_ERR_INVALID_ARG;
    if (!op_grid_ok(n_fine, 4) || !finite_pos(h_fine) || !phi_f || !eta_f || !eta_c || !phi_c ||
        !phihat_c || !sigma_c || !rr_c) {
        fmt_err(g_err, "fas_descend: need even n_fine >= 4, h > 0, non-NULL arrays");
        return ISIS_ERR_INVALID_ARG;
    }
    if (!ptrs_aligned({phi_f, eta_f, sigma_f, eta_c, phi_c, phihat_c, sigma_c, rr_c, fine_scratch}))
        return ISIS_ERR_INVALID_ARG;
    return with_model<double>(*p, a, [&](auto m) {
        return launch_descend<double, decltype(m)>(m, n_fine, h_fine, phi_f, eta_f, sigma_f,
                                                   eta_c, phi_c, phihat_c, sigma_c, rr_c,
                                                   (hipStream_t)stream, g_err, fine_scratch);
    });
}

static bool masked_args_ok(int n, double h, std::initializer_list<const void*> need)
{
    if (!op_grid_ok(n, 2) || !finite_pos(h)) {
        fmt_err(g_err, "masked operators: need even n >= 2 and h > 0");
        return false;
    }
    for (const void* q : need)
        if (!q) {
            fmt_err(g_err, "masked operators: NULL array");
            return false;
        }
    return true;
}

int isis_op_masked_defect(const isis_model_params* p, double a, int n, double h,
                          const double* phi, const double* eta, const double* sigma,
                          const double* mask, const double* u_int, const double* u_pre,
                          double* out, void* stream)
{
    if (!valid_params(p, a, g_err)) return ISIS_ERR_INVALID_ARG;
    if (!masked_args_ok(n, h, {phi, eta, mask, u_int, u_pre, out})) return ISIS_ERR_INVALID_ARG;
    if (!ptrs_aligned({phi, eta, sigma, mask, u_int, u_pre, out})) return ISIS_ERR_INVALID_ARG;
    return with_model<double>(*p, a, [&](auto m) {
        hipLaunchKernelGGL((k_masked_defect<decltype(m)>), dim3(grid_for((long)n * n * n)),
                           dim3(kBlock), 0, (hipStream_t)stream, m, n, 1.0 / (h * h), phi, eta,
                           sigma, mask, u_int, u_pre, out, nullptr);
        LAUNCH_CHECK(g_err, "k_masked_defect");
        return (int)ISIS_OK;
    });
}

int isis_op_masked_halfsweep(const isis_model_params* p, double a, int n, double h, double* phi,
                             const double* eta, const double* sigma, const double* mask,
                             const double* u_int, const double* u_pre, int colour, void* stream)
{
    if (!valid_params(p, a, g_err)) return ISIS_ERR_INVALID_ARG;
    if (!masked_args_ok(n, h, {phi, eta, mask, u_int, u_pre}) || (colour != 0 && colour != 1)) {
        if (colour != 0 && colour != 1) fmt_err(g_err, "masked halfsweep: colour must be 0 or 1");
        return ISIS_ERR_INVALID_ARG;
    }
    if (!ptrs_aligned({phi, eta, sigma, mask, u_int, u_pre})) return ISIS_ERR_INVALID_ARG;
    return with_model<double>(*p, a, [&](auto m) {
        hipLaunchKernelGGL((k_masked_halfsweep<decltype(m)>),
                           dim3(grid_for((long)n * n * n / 2)), dim3(kBlock), 0,
                           (hipStream_t)stream, m, n, 1.0 / (h * h), phi, eta, sigma, mask, u_int,
                           u_pre, colour);
        LAUNCH_CHECK(g_err, "k_masked_halfsweep");
        return (int)ISIS_OK;
    });
}

size_t isis_patch_workspace_size(int n)
{
    if (!op_grid_ok(n, 2)) return 0;
    return (size_t)n * n * n * sizeof(double) + (2 * kReduceBlocks + 16) * sizeof(double) + 256;
}

int isis_patch_solve(const isis_model_params* p, double a, int n, double h, double* phi,
                     const double* eta, const double* mask, const double* u_int, int block,
                     int max_sweeps, double tol, void* workspace, size_t workspace_bytes,
                     int* sweeps_out, double* rms_out, void* stream)
{
    if (!valid_params(p, a, g_err)) return ISIS_ERR_INVALID_ARG;
    if (!masked_args_ok(n, h, {phi, eta, mask, u_int, workspace})) return ISIS_ERR_INVALID_ARG;
    if (block < 1 || max_sweeps < 0 || !(tol >= 0.0) || !std::isfinite(tol)) {
        fmt_err(g_err, "patch_solve: need block >= 1, max_sweeps >= 0, finite tol >= 0");
        return ISIS_ERR_INVALID_ARG;
    }
    if (!ptrs_aligned({phi, eta, mask, u_int}) || !aligned(workspace, 256) ||
        workspace_bytes < isis_patch_workspace_size(n)) {
        fmt_err(g_err, "patch_solve: aligned arrays and a 256-byte aligned workspace of >= %zu "
                       "bytes needed", isis_patch_workspace_size(n));
        return ISIS_ERR_INVALID_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    const long n3 = (long)n * n * n;
    double* pre = static_cast<double*>(workspace);
    double* partial = pre + n3 + 32;  // per-block sums, then their totals
    double* scal = partial + 2 * kReduceBlocks;
    const double ih2 = 1.0 / (h * h);
    return with_model<double>(*p, a, [&](auto m) {
        using M = decltype(m);
        const int g = std::min(kReduceBlocks, grid_for(n3));
        // RMS of the defect over the inside cells, boundary values from phi
        auto rms = [&](double* out) -> int {
            HIP_TRY(g_err, hipMemcpyAsync(pre, phi, sizeof(double) * n3, hipMemcpyDeviceToDevice, s));
            hipLaunchKernelGGL((k_masked_defect<M>), dim3(g), dim3(kBlock), 0, s, m, n, ih2, phi,
                               eta, nullptr, mask, u_int, pre, nullptr, partial);
            LAUNCH_CHECK(g_err, "k_masked_defect");
            hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, s, partial, g, scal);
            hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, s, partial + g, g, scal + 1);
            LAUNCH_CHECK(g_err, "k_reduce");
            double host[2];
            HIP_TRY(g_err, hipMemcpyAsync(host, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
            HIP_TRY(g_err, hipStreamSynchronize(s));
            *out = host[1] > 0.0 ? std::sqrt(host[0] / host[1]) : 0.0;
            return (int)ISIS_OK;
        };
        double r = 0.0;
        int rc = rms(&r);
        if (rc) return rc;
        int sweeps = 0;
        while (r > tol && sweeps < max_sweeps) {
            // the boundary values are set from the field before each block
            HIP_TRY(g_err, hipMemcpyAsync(pre, phi, sizeof(double) * n3, hipMemcpyDeviceToDevice, s));
            for (int b = 0; b < block && sweeps < max_sweeps; ++b, ++sweeps) {
                for (int colour = 0; colour < 2; ++colour) {
                    hipLaunchKernelGGL((k_masked_halfsweep<M>), dim3(grid_for(n3 / 2)),
                                       dim3(kBlock), 0, s, m, n, ih2, phi, eta, nullptr, mask,
                                       u_int, pre, colour);
                    LAUNCH_CHECK(g_err, "k_masked_halfsweep");
                }
            }
            if ((rc = rms(&r))) return rc;
            if (!std::isfinite(r)) {
                fmt_err(g_err, "patch_solve: non-finite defect after %d sweeps", sweeps);
                if (sweeps_out) *sweeps_out = sweeps;
                if (rms_out) *rms_out = r;
                return (int)ISIS_ERR_DIVERGED;
            }
        }
        if (sweeps_out) *sweeps_out = sweeps;
        if (rms_out) *rms_out = r;
        return r <= tol ? (int)ISIS_OK : (int)ISIS_ERR_NOT_CONVERGED;
    });
}

int isis_op_restrict_fw(int n_fine, const double* fine, double* coarse, void* stream)
{
    if (!op_grid_ok(n_fine, 2) || !fine || !coarse) {
        fmt_err(g_err, "restrict_fw: need even n_fine >= 2 and non-NULL arrays");
        return ISIS_ERR_INVALID_ARG;
    }
    if (!ptrs_aligned({fine, coarse})) return ISIS_ERR_INVALID_ARG;
    return launch_restrict_fw<double>(n_fine, fine, coarse, (hipStream_t)stream, g_err);
}

int isis_op_prolong_correct(int n_fine, double* fine, const double* coarse,
                            const double* coarse_hat, void* stream)
{
    if (!op_grid_ok(n_fine, 4) || !fine || !coarse || !coarse_hat) {
        fmt_err(g_err, "prolong_correct: need even n_fine >= 4 and non-NULL arrays");
        return ISIS_ERR_INVALID_ARG;
    }
    if (!ptrs_aligned({fine, coarse, coarse_hat})) return ISIS_ERR_INVALID_ARG;
    return launch_prolong<double>(n_fine, fine, coarse, coarse_hat, (hipStream_t)stream, g_err);
}

int isis_op_prolong_correct_w(int n_fine, double* fine, const double* coarse,
                              const double* coarse_hat, void* stream)
{
    if (!op_grid_ok(n_fine, 4) || !fine || !coarse || !coarse_hat) {
        fmt_err(g_err, "prolong_correct_w: need even n_fine >= 4 and non-NULL arrays");
        return ISIS_ERR_INVALID_ARG;
    }
    if (!ptrs_aligned({fine, coarse, coarse_hat})) return ISIS_ERR_INVALID_ARG;
    return launch_prolong<double, 1>(n_fine, fine, coarse, coarse_hat, (hipStream_t)stream,
                                     g_err);
}

int isis_op_coarse_solve(const isis_model_params* p, double a, double h, double* phi,
                         const double* eta, const double* sigma, int nu_c, void* stream)
{
    if (!valid_params(p, a, g_err)) return ISIS_ERR_INVALID_ARG;
    if (!finite_pos(h) || !phi || !eta || nu_c < 0) {
        fmt_err(g_err, "coarse_solve: need h > 0, phi/eta non-NULL, nu_c >= 0");
        return ISIS_ERR_INVALID_ARG;
    }
    if (!ptrs_aligned({phi, eta, sigma})) return ISIS_ERR_INVALID_ARG;
    return with_model<double>(*p, a, [&](auto m) {
        return launch_coarse<double, decltype(m)>(m, h, phi, eta, sigma, nu_c,
                                                  (hipStream_t)stream, g_err);
    });
}

int isis_force(const isis_model_params* p, double a, int n, double h, const double* field,
               const double* potential, double* fx, double* fy, double* fz, void* stream)
{
    if (!valid_params(p, a, g_err)) return ISIS_ERR_INVALID_ARG;
    if (p->model == ISIS_CHAMELEON) {
        fmt_err(g_err, "force: not provided for the chameleon model");
        return ISIS_ERR_UNSUPPORTED;
    }
    const bool scalar = p->model != ISIS_LINEAR;
    if (!op_grid_ok(n, 2) || !finite_pos(h) || !fx || !fy || !fz || (scalar && !field)) {
        fmt_err(g_err, "force: need even n >= 2, h > 0, fx/fy/fz non-NULL and the field for "
                       "a scalar-field model");
        return ISIS_ERR_INVALID_ARG;
    }
    if (p->model == ISIS_SYMMETRON && (!finite_pos(p->omega_m) || !std::isfinite(p->beta))) {
        fmt_err(g_err, "symmetron force needs Omega_m > 0 and a finite beta");
        return ISIS_ERR_INVALID_ARG;
    }
    if (!ptrs_aligned({field, potential, fx, fy, fz})) return ISIS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (p->model == ISIS_SYMMETRON) {
        const double bla = p->beta * p->lambda0 * a;
        const double c = 6.0 * p->omega_m * kH0 * kH0 * bla * bla /
                         (p->a_ssb * p->a_ssb * p->a_ssb);
        return launch_force<ScalarForce::kChiGradChi>(n, h, c, field, potential, fx, fy, fz, s,
                                                      g_err);
    }
    if (p->model == ISIS_FR_HS) {
        // 1/2 e^{u_p} grad u_p with u_p = u + ln(a^2 |f_R0|)
        const double c = p->paper_u ? 0.5 : 0.5 * a * a * p->fR0_abs;
        return launch_force<ScalarForce::kExpGrad>(n, h, c, field, potential, fx, fy, fz, s,
                                                   g_err);
    }
    return launch_force<ScalarForce::kNone>(n, h, 0.0, field, potential, fx, fy, fz, s, g_err);
}

int isis_op_cold_start(const isis_model_params* p, double a, long ncell, const double* eta,
                       double* phi, void* stream)
{
    if (!valid_params(p, a, g_err)) return ISIS_ERR_INVALID_ARG;
    if (ncell < 0 || (ncell > 0 && (!eta || !phi))) {
        fmt_err(g_err, "cold_start: need ncell >= 0 and non-NULL arrays");
        return ISIS_ERR_INVALID_ARG;
    }
    if (!ptrs_aligned({eta, phi})) return ISIS_ERR_INVALID_ARG;
    if (ncell == 0) return ISIS_OK;
    return with_model<double>(*p, a, [&](auto m) {
        using M = decltype(m);
        hipLaunchKernelGGL((k_cold_start<double, M>), dim3(grid_for(ncell)), dim3(kBlock), 0,
                           (hipStream_t)stream, m, ncell, eta, phi);
        LAUNCH_CHECK(g_err, "k_cold_start");
        return (int)ISIS_OK;
    });
}

}  // extern "C"
