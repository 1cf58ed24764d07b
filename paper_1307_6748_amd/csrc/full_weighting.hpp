// Full-weighting restriction of the fine defect (an option of the FAS
// descent): coarse = P^T fine / 8, P the cell-centred trilinear
// prolongation.  Along each axis coarse cell I collects fine cells 2I-1, 2I,
// 2I+1, 2I+2 (periodic) with weights 1/8, 3/8, 3/8, 1/8; the 3D weight is the
// product of the three.  The fine defect comes from the descent kernel, which
// writes it to a fine scratch field when this restriction is selected.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace isis {

// One thread per coarse cell, the 64 fine values read directly (small levels).
template <class T>
__global__ __launch_bounds__(kBlock) void k_restrict_fw(int nf, const T* __restrict__ fine,
                                                        T* __restrict__ coarse)
{
    const int nc = nf >> 1;
    const long total = (long)nc * nc * nc;
    const T w[4] = {T(0.125), T(0.375), T(0.375), T(0.125)};
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (long)gridDim.x * blockDim.x) {
        const int K = (int)(q % nc);
        const long r = q / nc;
        const int J = (int)(r % nc), I = (int)(r / nc);
        T sx = T(0);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int i = (2 * I - 1 + a + nf) % nf;
            T sy = T(0);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int j = (2 * J - 1 + b + nf) % nf;
                const T* row = fine + ((long)i * nf + j) * nf;
                T sz = T(0);
#pragma unroll
                for (int c = 0; c < 4; ++c) sz += w[c] * row[(2 * K - 1 + c + nf) % nf];
                sy += w[b] * sz;
            }
            sx += w[a] * sy;
        }
        coarse[q] = sx;
    }
}

// LDS-staged version: each workgroup owns a TJ x TK tile of coarse (y, z)
// cells, one per thread, and streams along coarse x over XC planes.  Per step
// it stages fine planes 2I+1 and 2I+2 (tile plus a one-cell halo) and filters
// each along z and y into a coarse-resolution partial Q_p; the x filter
// combines Q_{2I-1} .. Q_{2I+2}, the first two kept in registers from the
// previous step.  Each fine value is read from HBM about 1.1 times.
template <int TJ_, int TK_, int XC_>
struct FwTile {
    static constexpr int TJ = TJ_, TK = TK_, XC = XC_, NT = kBlock;
    static constexpr int ER = 2 * TJ + 2;       // fine rows 2J0-1 .. 2J0+2TJ
    static constexpr int EC = 2 * TK + 4;       // fine columns 2K0-2 .. 2K0+2TK+1 (pairs)
    static constexpr int NPR = EC / 2;          // pairs per row
    static constexpr int PAIRS = ER * NPR;
    static constexpr int LPT = (PAIRS + NT - 1) / NT;
    static constexpr int PLANE = ER * EC;
    static_assert(TJ * TK == NT, "one coarse cell per thread");
};
using FwTileF = FwTile<8, 32, 8>;

template <class T>
__global__ __launch_bounds__(kBlock) void k_restrict_fw_tiled(int nf, const T* __restrict__ fine,
                                                              T* __restrict__ coarse)
{
    using G = FwTileF;
    using V = typename Vec2<T>::type;
    __shared__ __align__(16) T pl[2][G::PLANE];
    const int nc = nf >> 1, msk = nf - 1;
    const size_t nf2 = (size_t)nf * nf;
    const int tid = threadIdx.x;
    const int ntk = nc / G::TK, ntj = nc / G::TJ;
    int b = blockIdx.x;
    const int nb = gridDim.x;
    if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);  // contiguous tiles per XCD
    const int kt = b % ntk, jt = (b / ntk) % ntj, it = b / (ntk * ntj);
    const int J0 = jt * G::TJ, K0 = kt * G::TK, I0 = it * G::XC;
    const int jj = tid / G::TK, kk = tid - jj * G::TK;

    unsigned poff[G::LPT];
    int doff[G::LPT];
#pragma unroll
    for (int q = 0; q < G::LPT; ++q) {
        const int e = min(tid + q * G::NT, G::PAIRS - 1);
        const int r = e / G::NPR, c2 = e - r * G::NPR;
        poff[q] = (unsigned)(((2 * J0 - 1 + r) & msk) * nf + ((2 * K0 - 2 + 2 * c2) & msk));
        doff[q] = r * G::EC + 2 * c2;
    }
    V ra[G::LPT], rb[G::LPT];
    auto load2 = [&](int x) __attribute__((always_inline)) {  // fine planes x, x + 1
        const T* pa = fine + (size_t)(x & msk) * nf2;
        const T* pb = fine + (size_t)((x + 1) & msk) * nf2;
#pragma unroll
        for (int q = 0; q < G::LPT; ++q) {
            ra[q] = *reinterpret_cast<const V*>(pa + poff[q]);
            rb[q] = *reinterpret_cast<const V*>(pb + poff[q]);
        }
    };
    auto deposit2 = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < G::LPT; ++q) {
            if ((q + 1) * G::NT <= G::PAIRS || tid + q * G::NT < G::PAIRS) {
                *reinterpret_cast<V*>(&pl[0][doff[q]]) = ra[q];
                *reinterpret_cast<V*>(&pl[1][doff[q]]) = rb[q];
            }
        }
    };
    const T w[4] = {T(0.125), T(0.375), T(0.375), T(0.125)};
    // y and z filter of staged plane s at this thread's coarse cell: rows
    // 2jj-1 .. 2jj+2 and columns 2kk-1 .. 2kk+2 of the tile (staged row 2jj + b,
    // staged column 2kk + 1 + c)
    auto filt = [&](int s) __attribute__((always_inline)) {
        const T* p = pl[s];
        T sy = T(0);
#pragma unroll
        for (int bq = 0; bq < 4; ++bq) {
            const T* row = p + (2 * jj + bq) * G::EC + 2 * kk + 1;
            T sz = T(0);
#pragma unroll
            for (int c = 0; c < 4; ++c) sz += w[c] * row[c];
            sy += w[bq] * sz;
        }
        return sy;
    };
    // prologue: Q of fine planes 2I0-1, 2I0
    load2(2 * I0 - 1);
    deposit2();
    __syncthreads();
    T qa = filt(0), qb = filt(1);
    load2(2 * I0 + 1);
    for (int I = I0; I < I0 + G::XC; ++I) {
        __syncthreads();  // planes of the previous step consumed
        deposit2();       // fine planes 2I+1, 2I+2
        __syncthreads();
        if (I + 1 < I0 + G::XC) load2(2 * I + 3);
        const T qc = filt(0), qd = filt(1);
        const T v = w[0] * qa + w[1] * qb + w[2] * qc + w[3] * qd;
        coarse[((size_t)I * nc + J0 + jj) * nc + K0 + kk] = v;
        qa = qc;
        qb = qd;
    }
}

}  // namespace isis
