// Full-weighting restriction of the fine defect (an option of the FAS
// descent): coarse = P^T fine / 8, P the cell-centred trilinear
// prolongation.  Along each axis coarse cell I collects fine cells 2I-1, 2I,
// 2I+1, 2I+2 (periodic) with weights 1/8, 3/8, 3/8, 1/8; the 3D weight is the
// product of the three.  k_defect_restrict_fw_tiled computes the fine defect
// and restricts it in one pass; elsewhere the descent kernel writes the fine
// defect to a scratch field and k_restrict_fw(_tiled) restricts that.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "pair_kernels.hpp"

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

// FAS descent with the full-weighting restriction of the defect in one pass
// (single precision): each workgroup owns a 16 x 64 tile of fine (y, z) cells
// -- 8 x 32 coarse cells, one per thread -- and streams along x over XC
// coarse planes.  Coarse plane I needs the defect of fine planes 2I-1 ..
// 2I+2 on the tile plus a one-cell ring, so the defect is evaluated there
// (the tile's 2 x 2 children of each thread as z-pairs, the 164 ring cells
// one per thread), two new fine planes per step, into an LDS buffer; each is
// filtered along z and y to the coarse partial Q_x, and the x filter combines
// Q_{2I-1} .. Q_{2I+2}, the first two kept in registers from the previous
// step (the combination and the per-plane filter are those of
// k_restrict_fw_tiled).  phi_c = phihat_c = the mean of the 8 children, as in
// k_defect_restrict_tiled.  The phi ring holds fine planes 2I .. 2I+3 with a
// two-cell halo (rows y0-2 .. y0+17, columns z0-2 .. z0+65), with e^phi beside
// them for staged models.  The coarse FAS source sigma_c = L_c(phi_c) - R'(d)
// is completed in the same step, as k_fas_sigma computes it: the ring also
// holds the children of the coarse cell's four y-z neighbours and of its
// successor in x, whose means are summed again there (the predecessor's is
// kept from the previous step); the restricted defect is not stored.
template <int XC_>
struct DefectFwTile {
    static constexpr int TY = 16, TZ = 64, XC = XC_, NT = kBlock;
    static constexpr int EY = TY + 4;          // phi rows y0-2 .. y0+17
    static constexpr int EZ = TZ + 4;          // phi columns z0-2 .. z0+65
    static constexpr int NP = EZ / 2;
    static constexpr int PAIRS = EY * NP;
    static constexpr int LPT = (PAIRS + NT - 1) / NT;
    static constexpr int PLANE = EY * EZ;
    static constexpr int RY = TY + 2, RZ = TZ + 2;   // defect region: rows y0-1 .., columns z0-1 ..
    static constexpr int DS = TZ + 4;                // defect buffer row stride (region column c at c + 1)
    static constexpr int DPLANE = RY * DS;
    static constexpr int RING = 2 * RZ + 2 * (RY - 2);  // cells of the region outside the tile
    static_assert((TY / 2) * (TZ / 2) == NT, "one coarse cell per thread");
    static_assert(RING <= NT, "one ring cell per thread");
};

template <class T, class M, int XC>
constexpr int defect_fw_lds_bytes()
{
    using G = DefectFwTile<XC>;
    return (4 * G::PLANE * (StageOp<T, M>::kStaged ? 2 : 1) + 2 * G::DPLANE) * (int)sizeof(T);
}

// At least three waves per SIMD (at most 168 VGPRs), as many workgroups as
// the LDS allows: the f(R) form then keeps two values in scratch, only in the
// double-precision branch of the stiff source.
template <class T, class M, bool SIG, int XC>
__global__ __launch_bounds__(kBlock, 3) void k_defect_restrict_fw_tiled(
    M m, int nf, T ih2, const T* __restrict__ phi, const T* __restrict__ eta,
    const T* __restrict__ sigma, T* __restrict__ phi_c, T* __restrict__ phihat_c, T ih2c,
    const T* __restrict__ eta_c, T* __restrict__ sigma_c)
{
    using G = DefectFwTile<XC>;
    using V = typename Vec2<T>::type;
    using SO = StageOp<T, M>;
    constexpr bool STAGED = SO::kStaged;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* ring = reinterpret_cast<T*>(smem_raw);              // 4 fine planes of phi
    T* xring = ring + 4 * G::PLANE;                        // 4 planes of e^phi (staged)
    T* dbuf = ring + 4 * G::PLANE * (STAGED ? 2 : 1);      // defect of 2 fine planes
    __shared__ double exptab[SO::kTable ? kExpTable : 1];
    if constexpr (SO::kTable) {
        exp_table_fill(exptab);
        __syncthreads();
    }
    const int nc = nf >> 1;
    const int msk = nf - 1;
    const size_t nf2 = (size_t)nf * nf;
    const int tid = threadIdx.x;
    const int ntz = nf / G::TZ, nty = nf / G::TY;
    int b = blockIdx.x;
    const int nb = gridDim.x;
    if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);  // contiguous tiles per XCD
    const int zt = b % ntz, yt = (b / ntz) % nty, it = b / (ntz * nty);
    const int y0 = yt * G::TY, z0 = zt * G::TZ, I0 = it * G::XC;
    const int jj = tid / (G::TZ / 2), kk = tid - jj * (G::TZ / 2);  // coarse cell in the tile

    unsigned poff[G::LPT];
    int doff[G::LPT];
#pragma unroll
    for (int q = 0; q < G::LPT; ++q) {
        const int e = min(tid + q * G::NT, G::PAIRS - 1);
        const int r = e / G::NP, c2 = e - r * G::NP;
        poff[q] = (unsigned)(((y0 - 2 + r) & msk) * nf + ((z0 - 2 + 2 * c2) & msk));
        doff[q] = r * G::EZ + 2 * c2;
    }
    // this thread's 8 children: fine rows 2jj, 2jj+1 of the tile, columns 2kk, 2kk+1
    const unsigned coff0 = (unsigned)((y0 + 2 * jj) * nf + z0 + 2 * kk);
    const unsigned coff1 = coff0 + (unsigned)nf;
    const int o00 = (2 * jj + 2) * G::EZ + 2 * kk + 2;   // ring offset of child (2jj, 2kk)
    const int b00 = (2 * jj + 1) * G::DS + 2 * kk + 2;   // defect buffer offset of that child
    // this thread's ring cell (region row hr, column hc), if tid < RING; the
    // others compute a clamped copy and store nothing
    const bool hown = tid < G::RING;
    int hr, hc;
    {
        const int e = min(tid, G::RING - 1);
        if (e < G::RZ) {
            hr = 0;
            hc = e;
        } else if (e < 2 * G::RZ) {
            hr = G::RY - 1;
            hc = e - G::RZ;
        } else {
            const int e2 = e - 2 * G::RZ;
            hr = 1 + (e2 >> 1);
            hc = (e2 & 1) ? G::RZ - 1 : 0;
        }
    }
    const int hro = (hr + 1) * G::EZ + hc + 1;  // ring offset
    const int hbo = hr * G::DS + hc + 1;        // defect buffer offset
    const unsigned hgo = (unsigned)(((y0 - 1 + hr) & msk) * nf + ((z0 - 1 + hc) & msk));

    V ra[G::LPT], rb[G::LPT];
    auto load2 = [&](int x) __attribute__((always_inline)) {  // fine planes x, x+1
        const T* pa = phi + (size_t)(x & msk) * nf2;
        const T* pb = phi + (size_t)((x + 1) & msk) * nf2;
#pragma unroll
        for (int q = 0; q < G::LPT; ++q) {
            ra[q] = *reinterpret_cast<const V*>(pa + poff[q]);
            rb[q] = *reinterpret_cast<const V*>(pb + poff[q]);
        }
    };
    auto deposit1 = [&](int x, const V (&regs)[G::LPT]) __attribute__((always_inline)) {
        T* d = ring + (x & 3) * G::PLANE;
        T* e = xring + (x & 3) * G::PLANE;
#pragma unroll
        for (int q = 0; q < G::LPT; ++q) {
            if ((q + 1) * G::NT <= G::PAIRS || tid + q * G::NT < G::PAIRS) {
                *reinterpret_cast<V*>(d + doff[q]) = regs[q];
                if constexpr (STAGED)
                    *reinterpret_cast<V*>(e + doff[q]) =
                        V{SO::stage(regs[q].x, exptab), SO::stage(regs[q].y, exptab)};
            }
        }
    };
    // densities (and sources) of the defect cells of fine planes x, x+1
    V e2[2][2], s2[2][2];
    T eh[2], sh[2];
    auto load_cells = [&](int x) __attribute__((always_inline)) {
#pragma unroll
        for (int di = 0; di < 2; ++di) {
            const size_t xo = (size_t)((x + di) & msk) * nf2;
            e2[di][0] = *reinterpret_cast<const V*>(eta + xo + coff0);
            e2[di][1] = *reinterpret_cast<const V*>(eta + xo + coff1);
            eh[di] = eta[xo + hgo];
            if constexpr (SIG) {
                s2[di][0] = *reinterpret_cast<const V*>(sigma + xo + coff0);
                s2[di][1] = *reinterpret_cast<const V*>(sigma + xo + coff1);
                sh[di] = sigma[xo + hgo];
            } else {
                s2[di][0] = s2[di][1] = V{T(0), T(0)};
                sh[di] = T(0);
            }
        }
    };
    // defect L - sigma of fine planes x, x+1 on the region, into dbuf[0], dbuf[1]
    auto defects = [&](int x) __attribute__((always_inline)) {
#pragma unroll
        for (int di = 0; di < 2; ++di) {
            const int xx = x + di;
            const T* cu = ring + (xx & 3) * G::PLANE;
            const T* pv = ring + ((xx - 1) & 3) * G::PLANE;
            const T* nx = ring + ((xx + 1) & 3) * G::PLANE;
            const T* ecu = xring + (xx & 3) * G::PLANE;
            const T* epv = xring + ((xx - 1) & 3) * G::PLANE;
            const T* enx = xring + ((xx + 1) & 3) * G::PLANE;
            T* db = dbuf + di * G::DPLANE;
#pragma unroll
            for (int dj = 0; dj < 2; ++dj) {
                const int o = o00 + dj * G::EZ;
                V rv;
                const V c = *reinterpret_cast<const V*>(cu + o);
                const V xm = *reinterpret_cast<const V*>(pv + o);
                const V xp = *reinterpret_cast<const V*>(nx + o);
                const V ym = *reinterpret_cast<const V*>(cu + o - G::EZ);
                const V yp = *reinterpret_cast<const V*>(cu + o + G::EZ);
                const T zm = cu[o - 1], zp = cu[o + 2];
                V ec, exm, exq, eym, eyp;
                T ezm = T(0), ezp = T(0);
                if constexpr (STAGED) {
                    ec = *reinterpret_cast<const V*>(ecu + o);
                    exm = *reinterpret_cast<const V*>(epv + o);
                    exq = *reinterpret_cast<const V*>(enx + o);
                    eym = *reinterpret_cast<const V*>(ecu + o - G::EZ);
                    eyp = *reinterpret_cast<const V*>(ecu + o + G::EZ);
                    ezm = ecu[o - 1];
                    ezp = ecu[o + 2];
                }
#pragma unroll
                for (int dk = 0; dk < 2; ++dk) {
                    T nbv[6];
                    nbv[0] = xm[dk];
                    nbv[1] = xp[dk];
                    nbv[2] = ym[dk];
                    nbv[3] = yp[dk];
                    nbv[4] = dk ? c[0] : zm;
                    nbv[5] = dk ? zp : c[1];
                    T L, D;
                    if constexpr (STAGED) {
                        T enb[6];
                        enb[0] = exm[dk];
                        enb[1] = exq[dk];
                        enb[2] = eym[dk];
                        enb[3] = eyp[dk];
                        enb[4] = dk ? ec[0] : ezm;
                        enb[5] = dk ? ezp : ec[1];
                        SO::eval(m, c[dk], nbv, ec[dk], enb, e2[di][dj][dk], ih2, L, D);
                    } else {
                        m.op(c[dk], nbv, e2[di][dj][dk], ih2, L, D);
                    }
                    rv[dk] = L - s2[di][dj][dk];
                }
                *reinterpret_cast<V*>(db + b00 + dj * G::DS) = rv;
            }
            // the ring cell
            {
                const int o = hro;
                T nbv[6];
                nbv[0] = pv[o];
                nbv[1] = nx[o];
                nbv[2] = cu[o - G::EZ];
                nbv[3] = cu[o + G::EZ];
                nbv[4] = cu[o - 1];
                nbv[5] = cu[o + 1];
                T L, D;
                if constexpr (STAGED) {
                    T enb[6];
                    enb[0] = epv[o];
                    enb[1] = enx[o];
                    enb[2] = ecu[o - G::EZ];
                    enb[3] = ecu[o + G::EZ];
                    enb[4] = ecu[o - 1];
                    enb[5] = ecu[o + 1];
                    SO::eval(m, cu[o], nbv, ecu[o], enb, eh[di], ih2, L, D);
                } else {
                    m.op(cu[o], nbv, eh[di], ih2, L, D);
                }
                if (hown) db[hbo] = L - sh[di];
            }
        }
    };
    // the mean of the 8 children of the coarse cell whose child (0, 0) sits at
    // ring offset o, coarse plane X (fine planes 2X, 2X+1 in the ring), in the
    // order of k_defect_restrict_tiled
    auto ring_mean = [&](int X, int o) __attribute__((always_inline)) {
        T sp = T(0);
#pragma unroll
        for (int di = 0; di < 2; ++di) {
            const T* cu = ring + ((2 * X + di) & 3) * G::PLANE;
#pragma unroll
            for (int dj = 0; dj < 2; ++dj) {
                const V c = *reinterpret_cast<const V*>(cu + o + dj * G::EZ);
                sp += c[0];
                sp += c[1];
            }
        }
        return sp / T(8);
    };
    const T w[4] = {T(0.125), T(0.375), T(0.375), T(0.125)};
    // y and z filter of buffered plane s at this thread's coarse cell: region
    // rows 2jj .. 2jj+3 and columns 2kk .. 2kk+3 (fine rows 2jj-1 .. 2jj+2 and
    // columns 2kk-1 .. 2kk+2 of the tile)
    auto filt = [&](int sl) __attribute__((always_inline)) {
        const T* p = dbuf + sl * G::DPLANE;
        T sy = T(0);
#pragma unroll
        for (int bq = 0; bq < 4; ++bq) {
            const T* row = p + (2 * jj + bq) * G::DS + 2 * kk + 1;
            T sz = T(0);
#pragma unroll
            for (int c = 0; c < 4; ++c) sz += w[c] * row[c];
            sy += w[bq] * sz;
        }
        return sy;
    };
    // prologue: phi planes 2I0-2 .. 2I0+1 in LDS, defect and Q of 2I0-1, 2I0,
    // and the means of coarse planes I0-1 and I0
    load2(2 * I0 - 2);
    deposit1(2 * I0 - 2, ra);
    deposit1(2 * I0 - 1, rb);
    load2(2 * I0);
    deposit1(2 * I0, ra);
    deposit1(2 * I0 + 1, rb);
    load_cells(2 * I0 - 1);
    load2(2 * I0 + 2);
    __syncthreads();
    defects(2 * I0 - 1);
    T pm = ring_mean(I0 - 1, o00), pc = ring_mean(I0, o00);
    __syncthreads();
    T qa = filt(0), qb = filt(1);
    for (int I = I0; I < I0 + G::XC; ++I) {
        __syncthreads();  // ring slots of planes 2I-2, 2I-1 and the buffer are free
        deposit1(2 * I + 2, ra);
        deposit1(2 * I + 3, rb);
        load_cells(2 * I + 1);
        const size_t q = ((size_t)I * nc + (y0 / 2 + jj)) * nc + z0 / 2 + kk;
        const T ec = eta_c[q];
        load2(min(2 * I + 4, 2 * (I0 + G::XC)));  // clamped: branch-free
        __syncthreads();
        defects(2 * I + 1);
        __syncthreads();
        const T qc = filt(0), qd = filt(1);
        // the coarse plane I's neighbours of this thread's cell (fine planes
        // 2I, 2I+1: means of the neighbouring cells' children; 2I+2, 2I+3:
        // the mean of plane I+1), all in the ring until the next step
        T nbv[6];
        nbv[0] = pm;
        nbv[1] = ring_mean(I + 1, o00);
        nbv[2] = ring_mean(I, o00 - 2 * G::EZ);
        nbv[3] = ring_mean(I, o00 + 2 * G::EZ);
        nbv[4] = ring_mean(I, o00 - 2);
        nbv[5] = ring_mean(I, o00 + 2);
        phi_c[q] = pc;
        phihat_c[q] = pc;
        // sigma_c = L_c(phi_c) - R'(defect), as k_fas_sigma computes it
        // (carrying e^phi_c of the x-neighbours from step to step instead of
        // recomputing them measured slower: the extra registers spill)
        T L, D;
        m.op(pc, nbv, ec, ih2c, L, D);
        sigma_c[q] = L - (w[0] * qa + w[1] * qb + w[2] * qc + w[3] * qd);
        qa = qc;
        qb = qd;
        pm = pc;
        pc = nbv[1];
    }
}

}  // namespace isis
