// Acceleration on the grid from the solved field (the step after the solve
// in the paper's pipeline): f = -grad(potential) - F, where F is the
// scalar-field term of the model's geodesic equation in super-comoving
// variables,
//   symmetron (Sec. 4.1, eq. symmetron_geodesics_tilde_chi), chi~ = a chi:
//       F = 6 Omega_m H0^2 (beta lambda0)^2 / a_ssb^3 * chi~ grad chi~
//         = c * chi grad chi,                  c = 6 Omega_m H0^2 (beta lambda0 a)^2 / a_ssb^3
//   Hu-Sawicki f(R) (Sec. 4.2), e^{u_paper} = a^2 |f_R0| e^u:
//       F = (1/2) e^{u_paper} grad u_paper = c * e^u grad u,   c = a^2 |f_R0| / 2
//   linear test model: F = 0,
// with second-order periodic central differences.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace isis {

enum class ScalarForce { kNone = 0, kChiGradChi = 1, kExpGrad = 2 };

template <ScalarForce SF>
__device__ __forceinline__ double scalar_factor(double c, double v)
{
    if constexpr (SF == ScalarForce::kChiGradChi) return c * v;
    else if constexpr (SF == ScalarForce::kExpGrad) return c * exp(v);
    else return 0.0;
}

// One output z-pair per thread; field and potential stream through rings of
// three planes (TY x TZ tile plus a one-cell halo, z-halo widened to keep
// pairs aligned) in LDS; tiles are visited grid-stride with an XCD-aware
// order.  n must be a power of two and a multiple of TZ, TY and XC.
template <int TY_, int TZ_, int XC_>
struct ForceTile {
    static constexpr int TY = TY_, TZ = TZ_, XC = XC_, NT = kBlock;
    static constexpr int EY = TY + 2, EZ = TZ + 4, NP = EZ / 2;
    static constexpr int PAIRS = EY * NP, LPT = (PAIRS + NT - 1) / NT, PLANE = EY * EZ;
    static_assert(TY * TZ == 2 * NT, "one z-pair of cells per thread");
};
using ForceTileF = ForceTile<8, 64, 32>;

template <ScalarForce SF, bool POT>
__global__ __launch_bounds__(kBlock) void k_force_tiled(int n, double inv2h, double c,
                                                        const double* __restrict__ field,
                                                        const double* __restrict__ pot,
                                                        double* __restrict__ fx,
                                                        double* __restrict__ fy,
                                                        double* __restrict__ fz)
{
    using G = ForceTileF;
    using VD = typename Vec2<double>::type;
    constexpr bool FLD = SF != ScalarForce::kNone;
    __shared__ __align__(16) double rf[FLD ? 3 : 1][FLD ? G::PLANE : 2];
    __shared__ __align__(16) double rp[POT ? 3 : 1][POT ? G::PLANE : 2];
    const int tid = threadIdx.x;
    const int msk = n - 1;
    const size_t n2 = (size_t)n * n;
    const int ntz = n / G::TZ, nty = n / G::TY, ntx = n / G::XC;
    const int ntiles = ntz * nty * ntx;
    const int nb = gridDim.x;
    const bool remap = (nb & 7) == 0 && (ntiles & 7) == 0;
    const int xcd = blockIdx.x & 7, lb = blockIdx.x >> 3, per = ntiles >> 3;
    const int rr = tid / (G::TZ / 2), cp = tid - rr * (G::TZ / 2);
    for (int it = 0;; ++it) {
        int t;
        if (remap) {
            const int loc = lb + it * (nb >> 3);
            if (loc >= per) break;
            t = xcd * per + loc;
        } else {
            t = blockIdx.x + it * nb;
            if (t >= ntiles) break;
        }
        const int zt = t % ntz, yt = (t / ntz) % nty, xt = t / (ntz * nty);
        const int x0 = xt * G::XC, y0 = yt * G::TY, z0 = zt * G::TZ;
        unsigned poff[G::LPT];
#pragma unroll
        for (int q = 0; q < G::LPT; ++q) {
            const int k = min(tid + q * G::NT, G::PAIRS - 1);
            const int r = k / G::NP, c2 = k - r * G::NP;
            poff[q] = (unsigned)(((y0 - 1 + r) & msk) * n + ((z0 - 2 + 2 * c2) & msk));
        }
        const unsigned ooff = (unsigned)((y0 + rr) * n + z0 + 2 * cp);
        VD lf[G::LPT], lp[G::LPT];
        auto load = [&](int x) __attribute__((always_inline)) {
            const size_t xo = (size_t)(x & msk) * n2;
#pragma unroll
            for (int q = 0; q < G::LPT; ++q) {
                if constexpr (FLD) lf[q] = *reinterpret_cast<const VD*>(field + xo + poff[q]);
                if constexpr (POT) lp[q] = *reinterpret_cast<const VD*>(pot + xo + poff[q]);
            }
        };
        auto deposit = [&](int x) __attribute__((always_inline)) {
            const int sl = (x - x0 + 3) % 3;
#pragma unroll
            for (int q = 0; q < G::LPT; ++q) {
                const int k = tid + q * G::NT;
                if ((q + 1) * G::NT <= G::PAIRS || k < G::PAIRS) {
                    if constexpr (FLD) *reinterpret_cast<VD*>(&rf[sl][2 * k]) = lf[q];
                    if constexpr (POT) *reinterpret_cast<VD*>(&rp[sl][2 * k]) = lp[q];
                }
            }
        };
        load(x0 - 1);
        deposit(x0 - 1);
        load(x0);
        deposit(x0);
        load(x0 + 1);
        __syncthreads();
        for (int x = x0; x < x0 + G::XC; ++x) {
            deposit(x + 1);
            load(min(x + 2, x0 + G::XC));  // clamped: branch-free
            __syncthreads();
            const int sp = (x - 1 - x0 + 3) % 3, sc = (x - x0 + 3) % 3, sn = (x + 1 - x0 + 3) % 3;
            const int o = (rr + 1) * G::EZ + 2 + 2 * cp;
            // central differences of a ring at this thread's pair
            auto grad = [&](const double (*ring)[G::PLANE], VD& gx, VD& gy, VD& gz, VD& cen)
                            __attribute__((always_inline)) {
                const VD c = *reinterpret_cast<const VD*>(&ring[sc][o]);
                const VD xm = *reinterpret_cast<const VD*>(&ring[sp][o]);
                const VD xp = *reinterpret_cast<const VD*>(&ring[sn][o]);
                const VD ym = *reinterpret_cast<const VD*>(&ring[sc][o - G::EZ]);
                const VD yp = *reinterpret_cast<const VD*>(&ring[sc][o + G::EZ]);
                const double zm = ring[sc][o - 1], zp = ring[sc][o + 2];
                gx = (xp - xm) * inv2h;
                gy = (yp - ym) * inv2h;
                gz = VD{(c[1] - zm) * inv2h, (zp - c[0]) * inv2h};
                cen = c;
            };
            VD ax = VD{0.0, 0.0}, ay = ax, az = ax;
            if constexpr (POT) {
                VD gx, gy, gz, cen;
                grad(reinterpret_cast<const double (*)[G::PLANE]>(&rp[0][0]), gx, gy, gz, cen);
                ax -= gx;
                ay -= gy;
                az -= gz;
            }
            if constexpr (FLD) {
                VD gx, gy, gz, cen;
                grad(reinterpret_cast<const double (*)[G::PLANE]>(&rf[0][0]), gx, gy, gz, cen);
                const VD s = VD{scalar_factor<SF>(c, cen[0]), scalar_factor<SF>(c, cen[1])};
                ax -= s * gx;
                ay -= s * gy;
                az -= s * gz;
            }
            const size_t g = (size_t)(x & msk) * n2 + ooff;
            *reinterpret_cast<VD*>(fx + g) = ax;
            *reinterpret_cast<VD*>(fy + g) = ay;
            *reinterpret_cast<VD*>(fz + g) = az;
            __syncthreads();  // plane x-1's slot is refilled next
        }
    }
}

// Any even n: one thread per cell, neighbours through the caches.
template <ScalarForce SF, bool POT>
__global__ __launch_bounds__(kBlock) void k_force_cells(int n, double inv2h, double c,
                                                        const double* __restrict__ field,
                                                        const double* __restrict__ pot,
                                                        double* __restrict__ fx,
                                                        double* __restrict__ fy,
                                                        double* __restrict__ fz)
{
    constexpr bool FLD = SF != ScalarForce::kNone;
    const long total = (long)n * n * n;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (long)gridDim.x * blockDim.x) {
        const int k = (int)(q % n);
        const long r = q / n;
        const int j = (int)(r % n), i = (int)(r / n);
        const long nb[6] = {cell(n, wrap_dec(i, n), j, k), cell(n, wrap_inc(i, n), j, k),
                            cell(n, i, wrap_dec(j, n), k), cell(n, i, wrap_inc(j, n), k),
                            cell(n, i, j, wrap_dec(k, n)), cell(n, i, j, wrap_inc(k, n))};
        double a3[3] = {0.0, 0.0, 0.0};
        for (int d = 0; d < 3; ++d) {
            if constexpr (POT) a3[d] -= (pot[nb[2 * d + 1]] - pot[nb[2 * d]]) * inv2h;
            if constexpr (FLD)
                a3[d] -= scalar_factor<SF>(c, field[q]) *
                         ((field[nb[2 * d + 1]] - field[nb[2 * d]]) * inv2h);
        }
        fx[q] = a3[0];
        fy[q] = a3[1];
        fz[q] = a3[2];
    }
}

}  // namespace isis
