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

// Symmetron, Sec. 4.1 (dimensionless equation):
//   lap chi = K [ (A eta - 1) chi + chi^3 ],  K = a^2/(2 lambda0^2),
//   A = (a_ssb/a)^3.
// Canonical Jacobian -6/h^2 - dS/dchi (Sec. 3.3).  Where dS/dchi < 0 the
// Newton step would point away from the positive branch on coarse grids
// (K h^2 >> 6), so the denominator is safeguarded as -6/h^2 - |dS/dchi|;
// this changes only the iteration, not the root.
template <class T>
struct Symmetron {
    T K, A;
    __device__ __forceinline__ void op(T p, const T nb[6], T eta, T ih2, T& L, T& D) const
    {
        T sum = nb[0] + nb[1] + nb[2] + nb[3] + nb[4] + nb[5];
        T lap = (sum - T(6) * p) * ih2;
        T S = K * (A * eta * p - p + p * p * p);
        T dS = K * (A * eta - T(1) + T(3) * p * p);
        L = lap - S;
        D = -T(6) * ih2 - fabs(dS);
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
// The source is always evaluated in double precision: in dense haloes eta and
// c1 e^{-u/(n+1)} are both ~1e4 and cancel.
template <class T>
struct FofR {
    double Q, cLa3, c1, inv_np1;
    double a3, cL, np1;  // for the cold start
    __device__ __forceinline__ void op(T p, const T nb[6], T eta, T ih2, T& L, T& D) const
    {
        T bc = exp(p);
        T flux = T(0), dflux = T(0);
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            T bf = T(0.5) * (bc + exp(nb[f]));
            flux += bf * (nb[f] - p);
            dflux += T(0.5) * bc * (nb[f] - p) - bf;
        }
        double pd = (double)p;
        double e = exp(-pd * inv_np1);
        double S = Q * ((double)eta + cLa3 - c1 * e);
        double dS = Q * c1 * e * inv_np1;
        L = flux * ih2 - (T)S;
        D = dflux * ih2 - (T)dS;
    }
    __device__ __forceinline__ T cold(T eta) const
    {
        // u = -(n+1) ln[(eta/a^3 + cL)/(1 + cL)]
        return (T)(-np1 * log(((double)eta / a3 + cL) / (1.0 + cL)));
    }
};

// Linear test problem (the Poisson equation of Sec. 3.1 plus a mass term):
//   lap phi = m2 phi + kappa (eta - 1),  Jacobian -6/h^2 - m2.
template <class T>
struct Linear {
    T kappa, m2;
    __device__ __forceinline__ void op(T p, const T nb[6], T eta, T ih2, T& L, T& D) const
    {
        T sum = nb[0] + nb[1] + nb[2] + nb[3] + nb[4] + nb[5];
        T lap = (sum - T(6) * p) * ih2;
        T S = m2 * p + kappa * (eta - T(1));
        L = lap - S;
        D = -T(6) * ih2 - m2;
    }
    __device__ __forceinline__ T cold(T) const { return T(0); }
};

}  // namespace isis
