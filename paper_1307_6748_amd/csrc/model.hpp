// Pointwise physics of the scalar-field equation, evaluated on the GPU.
//
// Each model type provides
//   op(p, nb, eta, ih2, L, D): the discrete operator L(phi)_c of one cell and
//       the Newton denominator D_c = dL_c/dphi_c used by the Gauss-Seidel
//       update (Sec. 3.2), from the cell value p, its six neighbours nb
//       (order x-, x+, y-, y+, z-, z+), the density and 1/h^2;
//   cold(eta): the pointwise homogeneous root (the cold start).
// T is the storage/arithmetic type (double, or float for the FP32 phase of
// the mixed-precision solve).
#pragma once
#include <hip/hip_runtime.h>

namespace isis {

// 7-point Laplacian (Sec. 3.1) summed as neighbour differences: each
// difference of nearby values is exact (Sterbenz), so a smooth field loses no
// digits to the cancellation of sum(nb) against 6 phi -- in FP32 this lowers
// the round-off floor of the mixed-precision cycles.
template <class T>
__device__ __forceinline__ T lap7(T p, const T nb[6], T ih2)
{
    return (((nb[0] - p) + (nb[1] - p)) + ((nb[2] - p) + (nb[3] - p)) +
            ((nb[4] - p) + (nb[5] - p))) * ih2;
}

// Symmetron, Sec. 4.1 (dimensionless equation):
//   lap chi = K [ (A eta - 1) chi + chi^3 ],  K = a^2/(2 lambda0^2),
//   A = (a_ssb/a)^3.
// Canonical Jacobian -6/h^2 - dS/dchi (Sec. 3.3).  Where dS/dchi < 0 the
// Newton step would point away from the positive branch on coarse grids
// (K h^2 >> 6), so the denominator is safeguarded as -6/h^2 - |dS/dchi|;
// this changes only the iteration, not the root.
//
// kGuard: the smoothing kernels count the Gauss-Seidel updates at which the
// safeguard is active (dS/dchi < 0) into *hits when hits is not NULL.
template <class T>
struct Symmetron {
    static constexpr double kVar = 1.0, kVarInv = 1.0;  // stored value = phi
    static constexpr bool kGuard = true;
    T K, A;
    unsigned long long* hits;  // safeguard activations (device counter), or NULL
    __device__ __forceinline__ T limit(T step) const { return step; }
    __device__ __forceinline__ T dsource(T p, T eta) const
    {
        return K * (A * eta - T(1) + T(3) * p * p);
    }
    __device__ __forceinline__ void op(T p, const T nb[6], T eta, T ih2, T& L, T& D) const
    {
        T lap = lap7(p, nb, ih2);
        T S = K * (A * eta * p - p + p * p * p);
        T dS = dsource(p, eta);
        L = lap - S;
        D = -T(6) * ih2 - fabs(dS);
    }
    // Refinement boundaries (Sec. 3.3.1): the Newton denominator's term from a
    // ghost neighbour v = u^Int + r (p - u^Pre), dL/dv * dv/dp = r / h^2.
    __device__ __forceinline__ T ghost_dD(T, T, T r, T ih2) const { return r * ih2; }
    // 1 if the safeguard replaced dS/dchi by |dS/dchi| at this cell
    __device__ __forceinline__ unsigned guarded(T p, T eta) const
    {
        return dsource(p, eta) < T(0) ? 1u : 0u;
    }
    __device__ __forceinline__ T cold(T eta) const
    {
        T v = T(1) - A * eta;
        return v > T(0) ? sqrt(v) : T(0);
    }
};

// Hu-Sawicki f(R), Sec. 4.2, non-canonical form with b(u) = e^u, written for
// u = ln(f_R/f_R0):
//   (1/h^2) sum_f b_f (u_nb - u) = Q [ eta + cLa3 - c1 e^{-u/(n+1)} ],
//   b_f = (e^u + e^{u_nb})/2,  Q = Omega_m H0^2/(a |f_R0|),
//   cLa3 = cL a^3, c1 = a^3 (1 + cL), cL = 4 Omega_L/Omega_m.
// Jacobian (Sec. 3.4, eq. dbeq, with the exact factor 1/2 on db/du):
//   (1/h^2) sum_f [ e^u (u_nb - u)/2 - b_f ] - dS/du.
constexpr double kLn2 = 0.6931471805599453;    // ln 2
constexpr double kLog2e = 1.4426950408889634;  // 1 / ln 2

// 2^(x c) in single precision from the hardware base-2 exponential: the
// rounding error of t = fl(x c) is recovered exactly by an FMA, and
// 2^(x c) = 2^t (1 + err ln 2) to first order (no overflow handling: the
// fields here stay far from it).
__device__ __forceinline__ float exp2_scaled(float x, float c)
{
    const float t = x * c;
    const float err = fmaf(x, c, -t);
    const float r = __builtin_amdgcn_exp2f(t);
    return fmaf(r, err * float(kLn2), r);
}

// e^x in double precision by the table-driven method of P. T. P. Tang (ACM
// TOMS 15 (1989) 144): x = (64 k + j) ln2/64 + r with |r| <= ln2/128, so
// e^x = 2^k 2^(j/64) e^r, and e^r - 1 is its Taylor series through r^5 (the
// first omitted term is below 4e-17).  ln2/64 is split in two so that r is
// exact to ~1e-18.  tab[j] = 2^(j/64), j < 64 (exp_table_fill).  Outside
// |x| <= 708 (never met by these fields) the result saturates branch-free:
// +inf above, 0 below (e^x < 3.3e-308 there), NaN stays NaN.
constexpr int kExpTable = 64;
__device__ __forceinline__ double exp_tab(double x, const double* tab)
{
    constexpr double kInvStep = 92.33248261689366;         // 64 / ln 2
    constexpr double kStepHi = 0x1.62e42fefa39efp-7;       // ln2/64 rounded
    constexpr double kStepLo = 0x1.abc9e3b39803fp-62;      // ln2/64 - kStepHi
    constexpr double kMax = 708.0;
    const double xc = fmin(fmax(x, -kMax), kMax);
    const double nd = rint(xc * kInvStep);
    const int ni = (int)nd;
    double r = fma(-nd, kStepHi, xc);
    r = fma(-nd, kStepLo, r);
    double q = fma(r, 1.0 / 120.0, 1.0 / 24.0);
    q = fma(r, q, 1.0 / 6.0);
    q = fma(r, q, 0.5);
    q = fma(r, q, 1.0);
    const double t = tab[ni & (kExpTable - 1)];
    const double y = ldexp(fma(t, r * q, t), ni >> 6);  // ni >> 6 = floor(ni / 64)
    return fabs(x) <= kMax ? y : (x > 0.0 ? __builtin_inf() : (x < 0.0 ? 0.0 : x));
}

// Fill tab[0..63] with 2^(j/64) (all threads of the block take part; the
// caller synchronises before use).
__device__ __forceinline__ void exp_table_fill(double* tab)
{
    for (int j = threadIdx.x; j < kExpTable; j += blockDim.x) tab[j] = exp2(j * (1.0 / kExpTable));
}

// 1/d for the Newton-Gauss-Seidel step: the hardware reciprocal (FP32), or
// the hardware estimate refined by two Newton iterations (FP64).  Only the iteration uses it;
// its fixed point L = Sigma does not depend on how 1/D is rounded.
template <class T>
__device__ __forceinline__ T recip(T d)
{
    if constexpr (sizeof(T) == 4) {
        return __builtin_amdgcn_rcpf(d);  // within 1 ulp
    } else {
        double r = __builtin_amdgcn_rcp(d);
        r = fma(r, fma(-d, r, 1.0), r);
        return fma(r, fma(-d, r, 1.0), r);
    }
}

// Stiff regime of the source: where the field is screened, e^{-u/(n+1)} is
// large and eta cancels against c1 e^{-u/(n+1)} (both ~1e4 in halo cores), and
// dS/du dominates the Newton denominator.  There the FP32 operator still
// evaluates the source in FP64; elsewhere in FP32.
constexpr float kFofRStiff = 8.0f;  // e^{-u/(n+1)} above which the source is stiff

//
// In single precision the field is carried as w = u / ln 2 (kVar converts):
// then e^u = 2^w is one hardware exponential, exact to its own rounding,
// with no rounding of a scaled argument to correct.  The operator below
// evaluates the same residual L(u) from w, and the Newton denominator is
// dL/dw = ln2 dL/du.
//
// LIM: Gauss-Seidel steps are bounded by max_step (a compile-time choice, so
// that models without the bound carry no extra instruction).
template <class T, bool LIM = false>
struct FofR {
    static constexpr bool kW = sizeof(T) == 4;    // carried as w = u / ln 2
    static constexpr double kVar = kW ? kLog2e : 1.0;     // stored value = u * kVar
    static constexpr double kVarInv = kW ? kLn2 : 1.0;    // u = stored value * kVarInv
    static constexpr bool kGuard = false;  // no safeguard: D < 0 always
    __device__ __forceinline__ unsigned guarded(T, T) const { return 0u; }
    double Q, cLa3, c1, inv_np1;
    double a3, cL, np1;  // for the cold start
    double inv_a3, inv_1pcl;  // 1/a^3 and 1/(1 + cL): the cold start without divisions
    double ushift;       // added to the cold start (variable offset)
    double qc1n;         // Q c1 / (n+1): dS/du = qc1n e^{-u/(n+1)}
    float stiff_e;       // e^{-u/(n+1)} above which the FP32 source is evaluated in FP64
    T max_step;          // LIM: bound on one Gauss-Seidel step of the stored value
    // The Gauss-Seidel step, bounded by max_step when LIM: changes only the
    // iteration (where L = Sigma the step is zero), not its fixed point.
    __device__ __forceinline__ T limit(T step) const
    {
        if constexpr (LIM)
            return fmin(fmax(step, -max_step), max_step);
        else
            return step;
    }
    int n_is_one;        // n = 1: e^{-u/2} = 1/sqrt(e^u)
    // e^u from the stored value (2^w in single precision)
    __device__ __forceinline__ static T expv(T p)
    {
        if constexpr (kW)
            return __builtin_amdgcn_exp2f(p);
        else
            return exp(p);
    }
    // S(u) and dS/du at one cell, given the stored value p and e^u (ep)
    __device__ __forceinline__ void source(T p, T ep, T eta, T& S, T& dS) const
    {
        if constexpr (kW) {
            // (e^u >= 1e-30 for any field these solves meet; the bound only
            // keeps the reciprocal square root finite)
            const float e = n_is_one ? __builtin_amdgcn_rsqf(fmaxf(ep, 1e-30f))
                                     : exp2_scaled(-p, float(inv_np1));
            if (e <= stiff_e) {
                // Q eta + Q cLa3 - Q c1 e: no cancellation to speak of here
                S = fmaf(float(Q), eta, fmaf(-float(Q * c1), e, float(Q * cLa3)));
                dS = float(qc1n) * e;
                return;
            }
            const double ed = exp2(-(double)p * inv_np1);
            S = (T)(Q * ((double)eta + cLa3 - c1 * ed));
            dS = (T)(qc1n * ed);
        } else {
            const T e = n_is_one ? rsqrt(ep) : exp(-p * inv_np1);
            S = Q * (eta + cLa3 - c1 * e);
            dS = qc1n * e;
        }
    }
    // L and D from the cell value p, its e^p (ep) and the neighbours' values
    // and exponentials: the exponentials may be computed once per cell and
    // shared by all stencils that use them.
    // With d_f = u_f - u: sum_f b_f d_f = (e^u sum d_f + sum e^{u_f} d_f)/2 and
    // sum_f [e^u d_f/2 - b_f] = (e^u sum d_f - 6 e^u - sum e^{u_f})/2.
    __device__ __forceinline__ void op_staged(T p, const T nb[6], T ep, const T enb[6], T eta,
                                              T ih2, T& L, T& D) const
    {
        T sd = nb[0] - p;
        T sed = enb[0] * sd, se = enb[0];
#pragma unroll
        for (int f = 1; f < 6; ++f) {
            const T d = nb[f] - p;
            sd += d;
            sed += enb[f] * d;
            se += enb[f];
        }
        const T esd = ep * sd;
        const T hih2 = T(0.5) * ih2;  // the 1/2 of b_f, exactly
        T S, dS;
        source(p, ep, eta, S, dS);
        if constexpr (kW) {
            // differences are in w: u_f - u = ln2 (w_f - w)
            constexpr float l2 = float(kLn2);
            L = (esd + sed) * (hih2 * l2) - S;
            D = l2 * ((l2 * esd - T(6) * ep - se) * hih2 - dS);
        } else {
            L = (esd + sed) * hih2 - S;
            D = (esd - T(6) * ep - se) * hih2 - dS;
        }
    }
    // Refinement boundaries (Sec. 3.4.1): the Newton denominator's terms from
    // a ghost neighbour v = u^Int + r (p - u^Pre) whose face coefficient is
    // b(v): r [b_f + b'(v) (v - p) / 2] / h^2 (double precision only).
    __device__ __forceinline__ T ghost_dD(T p, T v, T r, T ih2) const
    {
        static_assert(!kW, "masked operators run in double precision");
        const T ev = exp(v);
        return r * ih2 * (T(0.5) * (exp(p) + ev) + T(0.5) * ev * (v - p));
    }
    __device__ __forceinline__ void op(T p, const T nb[6], T eta, T ih2, T& L, T& D) const
    {
        T enb[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) enb[f] = expv(nb[f]);
        op_staged(p, nb, expv(p), enb, eta, ih2, L, D);
    }
    __device__ __forceinline__ T cold(T eta) const
    {
        // u = -(n+1) ln[(eta/a^3 + cL)/(1 + cL)]
        return (T)((-np1 * log(fma((double)eta, inv_a3, cL) * inv_1pcl) + ushift) * kVar);
    }
};

// Linear test problem (the Poisson equation of Sec. 3.1 plus a mass term):
//   lap phi = m2 phi + kappa (eta - 1),  Jacobian -6/h^2 - m2.
template <class T>
struct Linear {
    static constexpr double kVar = 1.0, kVarInv = 1.0;  // stored value = phi
    static constexpr bool kGuard = false;
    T kappa, m2;
    __device__ __forceinline__ unsigned guarded(T, T) const { return 0u; }
    __device__ __forceinline__ T limit(T step) const { return step; }
    __device__ __forceinline__ void op(T p, const T nb[6], T eta, T ih2, T& L, T& D) const
    {
        T lap = lap7(p, nb, ih2);
        T S = m2 * p + kappa * (eta - T(1));
        L = lap - S;
        D = -T(6) * ih2 - m2;
    }
    __device__ __forceinline__ T ghost_dD(T, T, T r, T ih2) const { return r * ih2; }
    __device__ __forceinline__ T cold(T) const { return T(0); }
};

// Per-model form of the operator for kernels that share per-cell work between
// neighbouring stencils.  Staged models (f(R)) take a per-cell quantity
// computed once, stage(phi) = e^phi, next to each value; others ignore it.
// Kernels that stage in double precision hold the exp_tab table in LDS
// (kTable) and pass it to stage().
template <class T, class M>
struct StageOp {
    static constexpr bool kStaged = false, kTable = false;
    __device__ __forceinline__ static T stage(T) { return T(0); }
    __device__ __forceinline__ static T stage(T, const double*) { return T(0); }
    __device__ __forceinline__ static void eval(const M& m, T p, const T nb[6], T, const T*,
                                                T eta, T ih2, T& L, T& D)
    {
        m.op(p, nb, eta, ih2, L, D);
    }
};

template <class T, bool LIM>
struct StageOp<T, FofR<T, LIM>> {
    static constexpr bool kStaged = true, kTable = sizeof(T) == 8;
    __device__ __forceinline__ static T stage(T x) { return FofR<T, LIM>::expv(x); }
    __device__ __forceinline__ static T stage(T x, const double* tab)
    {
        if constexpr (sizeof(T) == 8)
            return exp_tab(x, tab);
        else
            return FofR<T, LIM>::expv(x);
    }
    __device__ __forceinline__ static void eval(const FofR<T, LIM>& m, T p, const T nb[6], T ep,
                                                const T enb[6], T eta, T ih2, T& L, T& D)
    {
        m.op_staged(p, nb, ep, enb, eta, ih2, L, D);
    }
};

}  // namespace isis
