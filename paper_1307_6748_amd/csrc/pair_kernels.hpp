// Level kernels that move data in z-pairs: each thread owns either one
// coarse cell and its 8 children (restriction side, prolongation) or two
// z-neighbouring fine cells (defect norm), and loads the fine field as
// 16-byte (FP64) / 8-byte (FP32) pairs.  They compute exactly what the
// per-cell kernels in kernels.hpp compute, in the same summation order, with
// about a third of the load instructions.  Fine sides must be even and >= 4.
#pragma once
#include <type_traits>
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace isis {

// FAS descent, first half (see k_defect_restrict): one thread per coarse
// cell.  The 32 fine values its 8 stencils touch are loaded once (as pairs
// along z); for f(R) their e^phi are computed once as well (32 instead of 56
// exponentials per coarse cell).  With dfine (full-weighting restriction of
// the defect) the fine defect L - sigma is written there instead of its
// 8-child mean into rr_c.
template <class T, class M>
__global__ __launch_bounds__(kBlock) void k_defect_restrict_pairs(
    M m, int nf, T ih2, const T* __restrict__ phi, const T* __restrict__ eta,
    const T* __restrict__ sigma, T* __restrict__ phi_c, T* __restrict__ phihat_c,
    T* __restrict__ rr_c, T* __restrict__ dfine = nullptr)
{
    using V = typename Vec2<T>::type;
    using SO = StageOp<T, M>;
    const int nc = nf >> 1;
    const long total = (long)nc * nc * nc;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (long)gridDim.x * blockDim.x) {
        const int K = (int)(q % nc);
        const long r = q / nc;
        const int J = (int)(r % nc), I = (int)(r / nc);
        const int k0 = 2 * K, km = wrap_dec(k0, nf), kp = wrap_inc(k0 + 1, nf);
        // fine rows: x index 2I-1 .. 2I+2, y index 2J-1 .. 2J+2 (periodic)
        int xi[4], yj[4];
        xi[0] = wrap_dec(2 * I, nf);
        xi[1] = 2 * I;
        xi[2] = 2 * I + 1;
        xi[3] = wrap_inc(2 * I + 1, nf);
        yj[0] = wrap_dec(2 * J, nf);
        yj[1] = 2 * J;
        yj[2] = 2 * J + 1;
        yj[3] = wrap_inc(2 * J + 1, nf);
        auto row = [&](int a, int b) { return ((long)xi[a] * nf + yj[b]) * nf; };
        // the 8 children: cp[di][dj] = cells (2I+di, 2J+dj, 2K..2K+1); their
        // z-neighbours outside the pair: cm (2K-1) and cq (2K+2)
        V cp[2][2];
        T cm[2][2], cq[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const long o = row(a + 1, b + 1);
                cp[a][b] = *reinterpret_cast<const V*>(phi + o + k0);
                cm[a][b] = phi[o + km];
                cq[a][b] = phi[o + kp];
            }
        // x-neighbours outside the block: xs[0][dj] at 2I-1, xs[1][dj] at 2I+2;
        // y-neighbours: ys[0][di] at 2J-1, ys[1][di] at 2J+2
        V xs[2][2], ys[2][2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            xs[0][t] = *reinterpret_cast<const V*>(phi + row(0, t + 1) + k0);
            xs[1][t] = *reinterpret_cast<const V*>(phi + row(3, t + 1) + k0);
            ys[0][t] = *reinterpret_cast<const V*>(phi + row(t + 1, 0) + k0);
            ys[1][t] = *reinterpret_cast<const V*>(phi + row(t + 1, 3) + k0);
        }
        V cpE[2][2], xsE[2][2], ysE[2][2];
        T cmE[2][2], cqE[2][2];
        if constexpr (SO::kStaged) {
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    cpE[a][b] = V{SO::stage(cp[a][b].x), SO::stage(cp[a][b].y)};
                    xsE[a][b] = V{SO::stage(xs[a][b].x), SO::stage(xs[a][b].y)};
                    ysE[a][b] = V{SO::stage(ys[a][b].x), SO::stage(ys[a][b].y)};
                    cmE[a][b] = SO::stage(cm[a][b]);
                    cqE[a][b] = SO::stage(cq[a][b]);
                }
        }
        T sr = T(0), sp = T(0);
#pragma unroll
        for (int di = 0; di < 2; ++di)
#pragma unroll
            for (int dj = 0; dj < 2; ++dj) {
                const long o = row(di + 1, dj + 1) + k0;
                const V e2 = *reinterpret_cast<const V*>(eta + o);
                V s2 = V{T(0), T(0)};
                if (sigma) s2 = *reinterpret_cast<const V*>(sigma + o);
                V rv;
#pragma unroll
                for (int dk = 0; dk < 2; ++dk) {
                    // neighbour order x-, x+, y-, y+, z-, z+
                    T nb[6];
                    nb[0] = di ? cp[0][dj][dk] : xs[0][dj][dk];
                    nb[1] = di ? xs[1][dj][dk] : cp[1][dj][dk];
                    nb[2] = dj ? cp[di][0][dk] : ys[0][di][dk];
                    nb[3] = dj ? ys[1][di][dk] : cp[di][1][dk];
                    nb[4] = dk ? cp[di][dj][0] : cm[di][dj];
                    nb[5] = dk ? cq[di][dj] : cp[di][dj][1];
                    const T p = cp[di][dj][dk];
                    T L, D;
                    if constexpr (SO::kStaged) {
                        T enb[6];
                        enb[0] = di ? cpE[0][dj][dk] : xsE[0][dj][dk];
                        enb[1] = di ? xsE[1][dj][dk] : cpE[1][dj][dk];
                        enb[2] = dj ? cpE[di][0][dk] : ysE[0][di][dk];
                        enb[3] = dj ? ysE[1][di][dk] : cpE[di][1][dk];
                        enb[4] = dk ? cpE[di][dj][0] : cmE[di][dj];
                        enb[5] = dk ? cqE[di][dj] : cpE[di][dj][1];
                        SO::eval(m, p, nb, cpE[di][dj][dk], enb, e2[dk], ih2, L, D);
                    } else {
                        m.op(p, nb, e2[dk], ih2, L, D);
                    }
                    rv[dk] = L - (sigma ? s2[dk] : T(0));
                    sr += rv[dk];
                    sp += p;
                }
                if (dfine) *reinterpret_cast<V*>(dfine + o) = rv;
            }
        const T pc = sp / T(8);
        phi_c[q] = pc;
        phihat_c[q] = pc;
        if (!dfine) rr_c[q] = sr / T(8);
    }
}

// fine += P(coarse - coarse_hat) (see k_prolong_correct; PW its weights):
// one thread per coarse cell updates its 8 children, in the same order of
// terms per child.
template <class T, int PW = 0>
__global__ __launch_bounds__(kBlock) void k_prolong_pairs(int nf, T* __restrict__ fine,
                                                          const T* __restrict__ coarse,
                                                          const T* __restrict__ coarse_hat)
{
    using V = typename Vec2<T>::type;
    const int nc = nf >> 1;
    const long total = (long)nc * nc * nc;
    const T w[2] = {T(0.75), T(0.25)};
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (long)gridDim.x * blockDim.x) {
        const int K = (int)(q % nc);
        const long r = q / nc;
        const int J = (int)(r % nc), I = (int)(r / nc);
        // coarse index offsets -1, 0, +1 per axis (periodic)
        const int Ix[3] = {wrap_dec(I, nc), I, wrap_inc(I, nc)};
        const int Jy[3] = {wrap_dec(J, nc), J, wrap_inc(J, nc)};
        const int Kz[3] = {wrap_dec(K, nc), K, wrap_inc(K, nc)};
        T d[3][3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const long cq = ((long)Ix[a] * nc + Jy[b]) * nc + Kz[c];
                    d[a][b][c] = coarse[cq] - coarse_hat[cq];
                }
        // weight of the other cell per axis and side (index 0: -1, 1: +1)
        T wo[3][2] = {{w[1], w[1]}, {w[1], w[1]}, {w[1], w[1]}};
        if constexpr (PW != 0) {
            const T hp = coarse_hat[((long)I * nc + J) * nc + K];
#pragma unroll
            for (int sd = 0; sd < 2; ++sd) {
                wo[0][sd] = prolong_weight<PW>(hp, coarse_hat[((long)Ix[2 * sd] * nc + J) * nc + K]);
                wo[1][sd] = prolong_weight<PW>(hp, coarse_hat[((long)I * nc + Jy[2 * sd]) * nc + K]);
                wo[2][sd] = prolong_weight<PW>(hp, coarse_hat[((long)I * nc + J) * nc + Kz[2 * sd]]);
            }
        }
#pragma unroll
        for (int di = 0; di < 2; ++di)
#pragma unroll
            for (int dj = 0; dj < 2; ++dj) {
                const long o = ((long)(2 * I + di) * nf + (2 * J + dj)) * nf + 2 * K;
                V f = *reinterpret_cast<const V*>(fine + o);
#pragma unroll
                for (int dk = 0; dk < 2; ++dk) {
                    // parent index 1; the other coarse cell is 2 for odd, 0 for even
                    const int ai[2] = {1, di ? 2 : 0};
                    const int bj[2] = {1, dj ? 2 : 0};
                    const int ck[2] = {1, dk ? 2 : 0};
                    const T wx[2] = {PW ? T(1) - wo[0][di] : w[0], PW ? wo[0][di] : w[1]};
                    const T wy[2] = {PW ? T(1) - wo[1][dj] : w[0], PW ? wo[1][dj] : w[1]};
                    const T wz[2] = {PW ? T(1) - wo[2][dk] : w[0], PW ? wo[2][dk] : w[1]};
                    T s = T(0);
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int b = 0; b < 2; ++b)
#pragma unroll
                            for (int c = 0; c < 2; ++c)
                                s += wx[a] * wy[b] * wz[c] * d[ai[a]][bj[b]][ck[c]];
                    f[dk] += s;
                }
                *reinterpret_cast<V*>(fine + o) = f;
            }
    }
}

// FAS descent (see k_defect_restrict), LDS-staged: each workgroup owns a
// 16 x 64 tile of fine (y, z) cells -- 8 x 32 coarse cells, one per thread --
// and streams along x over XC coarse planes.  Fine planes pass through a ring
// of four (2I-1 .. 2I+2 for coarse plane I; two new ones per step), with e^phi
// beside them for staged models, so each fine value is read from HBM about 1.2
// times and each exponential computed about 1.2 times per fine cell.  The 8
// children are summed in the order of k_defect_restrict.
//
// SIGC: the coarse FAS source sigma_c = L_c(phi_c) - rr_c is computed here
// too, one coarse plane behind, instead of by k_fas_sigma (same operator call
// on the same values, so the same result), and rr_c is not stored.  The mean
// of plane I is kept in LDS on the tile and a one-cell ring around it (two
// slots, planes I-1 and I), which needs fine rows y0-2 .. y0+17 in the ring;
// the x-neighbours come from registers.  The mean of plane I0-1 (first plane's
// x-neighbour) and of plane I0+XC (last plane's) are summed from HBM.
template <int XC_, bool SIGC_ = false>
struct RestrictTile {
    static constexpr int TY = 16, TZ = 64, XC = XC_, NT = kBlock;  // fine tile; XC coarse planes
    static constexpr int YH = SIGC_ ? 2 : 1;   // fine halo rows
    static constexpr int EY = TY + 2 * YH;     // fine rows y0-YH .. y0+15+YH
    static constexpr int EZ = TZ + 4;          // fine columns z0-2 .. z0+65 (pairs aligned)
    static constexpr int NP = EZ / 2;
    static constexpr int PAIRS = EY * NP;
    static constexpr int LPT = (PAIRS + NT - 1) / NT;
    static constexpr int PLANE = EY * EZ;
    // coarse plane (SIGC): rows -1 .. 8, columns -1 .. 32 of the coarse tile
    static constexpr int CY = TY / 2 + 2, CZ = TZ / 2 + 2, CPL = CY * CZ;
    static constexpr int CRING = 2 * CZ + 2 * (CY - 2);
    static_assert((TY / 2) * (TZ / 2) == NT, "one coarse cell per thread");
    static_assert(CRING <= NT, "one coarse ring cell per thread");
};
template <class T, class M, bool SIGC>
constexpr int restrict_tiled_lds_bytes()
{
    using G = RestrictTile<8, SIGC>;  // the same for every XC
    return (4 * G::PLANE * (StageOp<T, M>::kStaged ? 2 : 1) + (SIGC ? 2 * G::CPL : 0)) *
           (int)sizeof(T);
}

// FW: the fine defect L - sigma goes to dfine (full-weighting restriction of
// the defect follows in k_restrict_fw_tiled) instead of its mean to rr_c.
// SIGC (not with FW): sigma_c (coarse density eta_c, 1/h_c^2 = ih2c) instead
// of rr_c.  XC: coarse planes per workgroup.  Single-precision f(R) forms:
// at least three waves per SIMD (at most 168 VGPRs), as many workgroups as
// their LDS allows.
template <class T, class M>
constexpr int restrict_tiled_min_waves()
{
    return sizeof(T) == 4 && StageOp<T, M>::kStaged ? 3 : 1;
}
template <class T, class M, bool SIG, bool FW = false, bool SIGC = false, int XC = 8>
__global__ __launch_bounds__(kBlock, (restrict_tiled_min_waves<T, M>())) void k_defect_restrict_tiled(
    M m, int nf, T ih2, const T* __restrict__ phi, const T* __restrict__ eta,
    const T* __restrict__ sigma, T* __restrict__ phi_c, T* __restrict__ phihat_c,
    T* __restrict__ rr_c, T* __restrict__ dfine = nullptr, T ih2c = T(0),
    const T* __restrict__ eta_c = nullptr, T* __restrict__ sigma_c = nullptr)
{
    static_assert(!(FW && SIGC), "the full-weighting path restricts the defect afterwards");
    using G = RestrictTile<XC, SIGC>;
    using V = typename Vec2<T>::type;
    using SO = StageOp<T, M>;
    constexpr bool STAGED = SO::kStaged;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* ring = reinterpret_cast<T*>(smem_raw);  // 4 fine planes of phi
    T* xring = ring + 4 * G::PLANE;            // 4 planes of e^phi (staged models)
    T* cbuf = ring + 4 * G::PLANE * (STAGED ? 2 : 1);  // 2 coarse planes (SIGC)
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
        poff[q] = (unsigned)(((y0 - G::YH + r) & msk) * nf + ((z0 - 2 + 2 * c2) & msk));
        doff[q] = r * G::EZ + 2 * c2;
    }
    // this thread's 8 children: fine rows 2jj, 2jj+1 of the tile, columns 2kk, 2kk+1
    const unsigned coff0 = (unsigned)((y0 + 2 * jj) * nf + z0 + 2 * kk);  // row 2jj
    const unsigned coff1 = coff0 + (unsigned)nf;                          // row 2jj+1
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
    // SIGC: the mean of this thread's children of coarse plane X, from HBM
    auto hbm_mean = [&](int X) __attribute__((always_inline)) {
        T sp = T(0);
#pragma unroll
        for (int di = 0; di < 2; ++di) {
            const T* pl = phi + (size_t)((2 * X + di) & msk) * nf2;
#pragma unroll
            for (int dj = 0; dj < 2; ++dj) {
                const V c = *reinterpret_cast<const V*>(pl + (dj ? coff1 : coff0));
                sp += c[0];
                sp += c[1];
            }
        }
        return sp / T(8);
    };
    // SIGC: this thread's coarse ring cell (row cr, column cq of the coarse
    // tile, -1 .. 8 and -1 .. 32) if tid < CRING; the others take the last
    // ring cell and store the same value there (a store under a branch let
    // the compiler sink the defect arithmetic below it: more registers)
    int cr, cq;
    {
        const int e = min(tid, G::CRING - 1);
        if (e < G::CZ) {
            cr = -1;
            cq = e - 1;
        } else if (e < 2 * G::CZ) {
            cr = G::CY - 2;
            cq = e - G::CZ - 1;
        } else {
            const int e2 = e - 2 * G::CZ;
            cr = e2 >> 1;
            cq = (e2 & 1) ? G::CZ - 2 : -1;
        }
    }
    const int cro = (2 * cr + G::YH) * G::EZ + 2 + 2 * cq;  // fine ring offset of its child (0,0)
    const int crb = (cr + 1) * G::CZ + cq + 1;              // coarse plane offset
    const int cob = (jj + 1) * G::CZ + kk + 1;              // this thread's cell there
    T pm2 = T(0), pm1 = T(0), rm1 = T(0), em1 = T(0);       // planes I-2, I-1
    if constexpr (SIGC) pm1 = hbm_mean(I0 - 1);
    // prologue: fine planes 2I0-1, 2I0 in LDS, 2I0+1, 2I0+2 in registers
    load2(2 * I0 - 1);
    deposit1(2 * I0 - 1, ra);
    deposit1(2 * I0, rb);
    load2(2 * I0 + 1);
    const int o00 = (2 * jj + G::YH) * G::EZ + 2 + 2 * kk;  // LDS offset of child (row 2jj, col 2kk)
    // sigma_c of coarse plane X from the buffered plane X and its x-neighbours
    auto coarse_source = [&](int X, T pxm, T pc, T pxp, T ec, T rr)
        __attribute__((always_inline)) {
        const T* cb = cbuf + (X & 1) * G::CPL;
        T nbv[6];
        nbv[0] = pxm;
        nbv[1] = pxp;
        nbv[2] = cb[cob - G::CZ];
        nbv[3] = cb[cob + G::CZ];
        nbv[4] = cb[cob - 1];
        nbv[5] = cb[cob + 1];
        T L, D;
        m.op(pc, nbv, ec, ih2c, L, D);
        sigma_c[((size_t)(X & (nc - 1)) * nc + (y0 / 2 + jj)) * nc + z0 / 2 + kk] = L - rr;
    };
    // one coarse plane; SRC: also the source of plane I-1 (a compile-time
    // flag rather than a branch, for the same reason)
    auto step = [&](int I, auto src) __attribute__((always_inline)) {
        constexpr bool SRC = decltype(src)::value;
        deposit1(2 * I + 1, ra);
        deposit1(2 * I + 2, rb);
        // this step's densities (and sources), then the next two planes
        V e2[2][2], s2[2][2];
#pragma unroll
        for (int di = 0; di < 2; ++di) {
            const size_t xo = (size_t)((2 * I + di) & msk) * nf2;
            e2[di][0] = *reinterpret_cast<const V*>(eta + xo + coff0);
            e2[di][1] = *reinterpret_cast<const V*>(eta + xo + coff1);
            if constexpr (SIG) {
                s2[di][0] = *reinterpret_cast<const V*>(sigma + xo + coff0);
                s2[di][1] = *reinterpret_cast<const V*>(sigma + xo + coff1);
            } else {
                s2[di][0] = s2[di][1] = V{T(0), T(0)};
            }
        }
        T ec = T(0);
        if constexpr (SIGC) ec = eta_c[((size_t)I * nc + (y0 / 2 + jj)) * nc + z0 / 2 + kk];
        load2(min(2 * I + 3, 2 * (I0 + G::XC) - 1));  // clamped: branch-free
        __syncthreads();
        if constexpr (SIGC && SRC) {
            // plane I-1's source first: its operator's branches then cannot
            // draw the defects' arithmetic below them (more live registers)
            T pn = T(0);
#pragma unroll
            for (int di = 0; di < 2; ++di) {
                const T* cu = ring + ((2 * I + di) & 3) * G::PLANE;
#pragma unroll
                for (int dj = 0; dj < 2; ++dj) {
                    const V c = *reinterpret_cast<const V*>(cu + o00 + dj * G::EZ);
                    pn += c[0];
                    pn += c[1];
                }
            }
            coarse_source(I - 1, pm2, pm1, pn / T(8), em1, rm1);
        }
        T sr = T(0), sp = T(0);
#pragma unroll
        for (int di = 0; di < 2; ++di) {
            const int x = 2 * I + di;
            const T* cu = ring + (x & 3) * G::PLANE;
            const T* pv = ring + ((x - 1) & 3) * G::PLANE;
            const T* nx = ring + ((x + 1) & 3) * G::PLANE;
            const T* ecu = xring + (x & 3) * G::PLANE;
            const T* epv = xring + ((x - 1) & 3) * G::PLANE;
            const T* enx = xring + ((x + 1) & 3) * G::PLANE;
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
                V ec2, exm, exq, eym, eyp;
                T ezm = T(0), ezp = T(0);
                if constexpr (STAGED) {
                    ec2 = *reinterpret_cast<const V*>(ecu + o);
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
                        enb[4] = dk ? ec2[0] : ezm;
                        enb[5] = dk ? ezp : ec2[1];
                        SO::eval(m, c[dk], nbv, ec2[dk], enb, e2[di][dj][dk], ih2, L, D);
                    } else {
                        m.op(c[dk], nbv, e2[di][dj][dk], ih2, L, D);
                    }
                    rv[dk] = L - s2[di][dj][dk];
                    sr += rv[dk];
                    sp += c[dk];
                }
                if constexpr (FW)
                    *reinterpret_cast<V*>(dfine + (size_t)(x & msk) * nf2 +
                                          (dj ? coff1 : coff0)) = rv;
            }
        }
        const size_t q = ((size_t)I * nc + (y0 / 2 + jj)) * nc + z0 / 2 + kk;
        const T pc = sp / T(8);
        phi_c[q] = pc;
        phihat_c[q] = pc;
        if constexpr (!FW && !SIGC) rr_c[q] = sr / T(8);
        if constexpr (SIGC) {
            // plane I into its slot (free: plane I-2's source was computed
            // before the previous step's closing barrier), then plane I-1's source
            T* cb = cbuf + (I & 1) * G::CPL;
            cb[cob] = pc;
            T hp = T(0);
#pragma unroll
            for (int di = 0; di < 2; ++di) {
                const T* cu = ring + ((2 * I + di) & 3) * G::PLANE;
#pragma unroll
                for (int dj = 0; dj < 2; ++dj) {
                    const V c = *reinterpret_cast<const V*>(cu + cro + dj * G::EZ);
                    hp += c[0];
                    hp += c[1];
                }
            }
            cb[crb] = hp / T(8);
            pm2 = pm1;
            pm1 = pc;
            rm1 = sr / T(8);
            em1 = ec;
        }
        __syncthreads();  // the slots of planes 2I-1, 2I are refilled next
    };
    step(I0, std::false_type{});
    for (int I = I0 + 1; I < I0 + G::XC; ++I) step(I, std::true_type{});
    if constexpr (SIGC) coarse_source(I0 + G::XC - 1, pm2, pm1, hbm_mean(I0 + G::XC), em1, rm1);
}

// fine += P(coarse - coarse_hat), LDS-staged: each workgroup owns a TJ x TK
// tile of coarse (y, z) cells and streams along coarse x over XC planes.  The
// coarse differences pass through a ring of three planes (tile plus a
// one-cell halo) in LDS, so each is loaded about 1.6 times instead of 27;
// each thread then updates the 8 children of one coarse cell with 16-byte
// pair loads and stores.  Same terms, same order as k_prolong_correct.
template <int TJ_, int TK_, int XC_>
struct ProlongTile {
    static constexpr int TJ = TJ_, TK = TK_, XC = XC_, NT = kBlock;
    static constexpr int EJ = TJ + 2, EK = TK + 2;
    static constexpr int PLANE = EJ * EK;
    static constexpr int LPT = (PLANE + NT - 1) / NT;
    static_assert(TJ * TK == NT, "one coarse cell per thread");
};
using ProlongTileF = ProlongTile<4, 64, 8>;

// PW: the weights of k_prolong_correct; for PW != 0 each thread reads the
// restricted field of its coarse cell and of the cell's six neighbours.
template <class T, int PW = 0>
__global__ __launch_bounds__(kBlock) void k_prolong_tiled(int nf, T* __restrict__ fine,
                                                          const T* __restrict__ coarse,
                                                          const T* __restrict__ coarse_hat)
{
    using G = ProlongTileF;
    using V = typename Vec2<T>::type;
    __shared__ T ring[3][G::PLANE];
    const int nc = nf >> 1;
    const int cm = nc - 1;
    const int tid = threadIdx.x;
    const int ntk = nc / G::TK, ntj = nc / G::TJ;
    int b = blockIdx.x;
    const int nb = gridDim.x;
    if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);  // contiguous tiles per XCD
    const int kt = b % ntk, jt = (b / ntk) % ntj, it = b / (ntk * ntj);
    const int I0 = it * G::XC, J0 = jt * G::TJ, K0 = kt * G::TK;
    const T w[2] = {T(0.75), T(0.25)};
    T d[G::LPT];
    // coarse differences of plane I (tile + halo) into registers
    auto load = [&](int I) __attribute__((always_inline)) {
        const long xoff = (long)(I & cm) * nc;
#pragma unroll
        for (int q = 0; q < G::LPT; ++q) {
            const int e = min(tid + q * G::NT, G::PLANE - 1);
            const int r = e / G::EK, c = e - r * G::EK;
            const long g = (xoff + ((J0 - 1 + r) & cm)) * nc + ((K0 - 1 + c) & cm);
            d[q] = coarse[g] - coarse_hat[g];
        }
    };
    auto deposit = [&](int I) __attribute__((always_inline)) {
        T* dst = ring[(I - I0 + 3) % 3];
#pragma unroll
        for (int q = 0; q < G::LPT; ++q) {
            const int e = tid + q * G::NT;
            if (e < G::PLANE) dst[e] = d[q];
        }
    };
    const int jj = tid / G::TK, kk = tid - jj * G::TK;  // this thread's coarse (J, K)
    load(I0 - 1);
    deposit(I0 - 1);
    load(I0);
    deposit(I0);
    load(I0 + 1);
    for (int I = I0; I < I0 + G::XC; ++I) {
        deposit(I + 1);
        load(min(I + 2, I0 + G::XC));  // clamped: branch-free
        // weight of the other cell per axis and side (index 0: -1, 1: +1)
        T wo[3][2] = {{w[1], w[1]}, {w[1], w[1]}, {w[1], w[1]}};
        if constexpr (PW != 0) {
            const int J = J0 + jj, K = K0 + kk;
            auto hat = [&](int a, int b, int c) __attribute__((always_inline)) {
                return coarse_hat[((long)(a & cm) * nc + (b & cm)) * nc + (c & cm)];
            };
            const T hp = hat(I, J, K);
            wo[0][0] = prolong_weight<PW>(hp, hat(I - 1, J, K));
            wo[0][1] = prolong_weight<PW>(hp, hat(I + 1, J, K));
            wo[1][0] = prolong_weight<PW>(hp, hat(I, J - 1, K));
            wo[1][1] = prolong_weight<PW>(hp, hat(I, J + 1, K));
            wo[2][0] = prolong_weight<PW>(hp, hat(I, J, K - 1));
            wo[2][1] = prolong_weight<PW>(hp, hat(I, J, K + 1));
        }
        // this coarse cell's 8 children: 4 z-pairs
        V f[2][2];
#pragma unroll
        for (int di = 0; di < 2; ++di)
#pragma unroll
            for (int dj = 0; dj < 2; ++dj) {
                const long o = ((long)(2 * I + di) * nf + (2 * (J0 + jj) + dj)) * nf +
                               2 * (K0 + kk);
                f[di][dj] = *reinterpret_cast<const V*>(fine + o);
            }
        __syncthreads();
        const T* pl[3] = {ring[(I - 1 - I0 + 3) % 3], ring[(I - I0 + 3) % 3],
                          ring[(I + 1 - I0 + 3) % 3]};
#pragma unroll
        for (int di = 0; di < 2; ++di)
#pragma unroll
            for (int dj = 0; dj < 2; ++dj) {
#pragma unroll
                for (int dk = 0; dk < 2; ++dk) {
                    // parent at window index 1; the other neighbour at 2 (odd child) or 0
                    const int ai[2] = {1, di ? 2 : 0};
                    const int bj[2] = {1, dj ? 2 : 0};
                    const int ck[2] = {1, dk ? 2 : 0};
                    const T wx[2] = {PW ? T(1) - wo[0][di] : w[0], PW ? wo[0][di] : w[1]};
                    const T wy[2] = {PW ? T(1) - wo[1][dj] : w[0], PW ? wo[1][dj] : w[1]};
                    const T wz[2] = {PW ? T(1) - wo[2][dk] : w[0], PW ? wo[2][dk] : w[1]};
                    T s = T(0);
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
                            for (int c = 0; c < 2; ++c)
                                s += wx[a] * wy[bb] * wz[c] *
                                     pl[ai[a]][(jj + bj[bb]) * G::EK + kk + ck[c]];
                    f[di][dj][dk] += s;
                }
                const long o = ((long)(2 * I + di) * nf + (2 * (J0 + jj) + dj)) * nf +
                               2 * (K0 + kk);
                // streamed out: nothing reads it again before it leaves L2
                __builtin_nontemporal_store(f[di][dj], reinterpret_cast<V*>(fine + o));
            }
        __syncthreads();  // the slot of plane I-1 is refilled next
    }
}

// Finest-level defect in double precision and per-block partial sums of r^2
// (see k_defect_norm): one thread per z-pair of cells.
template <class TF, class M>
__global__ __launch_bounds__(kBlock) void k_defect_norm_pairs(M m, int n, double ih2, double uscale, double uoffset,
                                                              const TF* __restrict__ phi,
                                                              const double* __restrict__ eta,
                                                              double* __restrict__ res,
                                                              double* __restrict__ partial)
{
    using VF = typename Vec2<TF>::type;
    using VD = typename Vec2<double>::type;
    const int hn = n >> 1;
    const long total = (long)n * n * hn;
    double acc = 0.0;
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (long)gridDim.x * blockDim.x) {
        const int kk = (int)(t % hn);
        const long r = t / hn;
        const int j = (int)(r % n), i = (int)(r / n);
        const int k0 = 2 * kk;
        const long o = ((long)i * n + j) * n;
        const long oxm = ((long)wrap_dec(i, n) * n + j) * n, oxp = ((long)wrap_inc(i, n) * n + j) * n;
        const long oym = ((long)i * n + wrap_dec(j, n)) * n, oyp = ((long)i * n + wrap_inc(j, n)) * n;
        const VF c = *reinterpret_cast<const VF*>(phi + o + k0);
        const VF xm = *reinterpret_cast<const VF*>(phi + oxm + k0);
        const VF xp = *reinterpret_cast<const VF*>(phi + oxp + k0);
        const VF ym = *reinterpret_cast<const VF*>(phi + oym + k0);
        const VF yp = *reinterpret_cast<const VF*>(phi + oyp + k0);
        const double zm = fma((double)phi[o + wrap_dec(k0, n)], uscale, uoffset);
        const double zp = fma((double)phi[o + wrap_inc(k0 + 1, n)], uscale, uoffset);
        const VD e = *reinterpret_cast<const VD*>(eta + o + k0);
        double L2[2];
#pragma unroll
        for (int dk = 0; dk < 2; ++dk) {
            double nb[6];
            nb[0] = fma((double)xm[dk], uscale, uoffset);
            nb[1] = fma((double)xp[dk], uscale, uoffset);
            nb[2] = fma((double)ym[dk], uscale, uoffset);
            nb[3] = fma((double)yp[dk], uscale, uoffset);
            nb[4] = dk ? fma((double)c[0], uscale, uoffset) : zm;
            nb[5] = dk ? zp : fma((double)c[1], uscale, uoffset);
            double L, D;
            m.op(fma((double)c[dk], uscale, uoffset), nb, e[dk], ih2, L, D);
            L2[dk] = L;
            acc += L * L;
        }
        if (res) *reinterpret_cast<VD*>(res + o + k0) = VD{L2[0], L2[1]};
    }
    double s = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Finest-level defect and per-block partial sums of r^2, computed in the
// arithmetic type TA (double: the judge of the stop test; float: the FP32
// problem's own defect, with its FP32 density) and summed in double: each
// workgroup streams a TY x TZ tile of the y-z plane along x
// through a ring of three planes in LDS (phi and, for staged models such as
// f(R), e^phi), so every value is fetched from HBM about once and each
// exponential is computed once per loaded cell (about 1.3 per cell with the
// halo) instead of seven times per stencil.  Tiles are visited grid-stride;
// n must be a power of two and a multiple of TZ, TY and XC.
template <int TY_, int TZ_, int XC_>
struct NormTile {
    static constexpr int TY = TY_, TZ = TZ_, XC = XC_, NT = kBlock;
    static constexpr int EY = TY + 2;         // rows with the y halo
    static constexpr int EZ = TZ + 4;         // columns z0-2 .. z0+TZ+1 (pairs stay aligned)
    static constexpr int NP = EZ / 2;         // pairs per row
    static constexpr int PAIRS = EY * NP;     // pairs per plane
    static constexpr int LPT = (PAIRS + NT - 1) / NT;
    static constexpr int PLANE = EY * EZ;
    static_assert(TY * TZ == 2 * NT, "one z-pair of cells per thread");
};
using NormTileF = NormTile<8, 64, 32>;

template <class TF, class M, class TA = double>
__global__ __launch_bounds__(kBlock) void k_defect_norm_tiled(M m, int n, double ih2_, double uscale_,
                                                              double uoffset_,
                                                              const TF* __restrict__ phi,
                                                              const TA* __restrict__ eta,
                                                              double* __restrict__ res,
                                                              double* __restrict__ partial)
{
    using G = NormTileF;
    using SO = StageOp<TA, M>;
    using VF = typename Vec2<TF>::type;
    using VD = typename Vec2<double>::type;
    using VA = typename Vec2<TA>::type;
    constexpr bool STAGED = SO::kStaged;
    const TA ih2 = (TA)ih2_, uscale = (TA)uscale_, uoffset = (TA)uoffset_;
    __shared__ __align__(16) TA ring[3][G::PLANE];
    __shared__ __align__(16) TA xring[STAGED ? 3 : 1][STAGED ? G::PLANE : 2];
    __shared__ double exptab[SO::kTable ? kExpTable : 1];
    if constexpr (SO::kTable) {
        exp_table_fill(exptab);
        __syncthreads();
    }
    const int tid = threadIdx.x;
    const int msk = n - 1;
    const int ntz = n / G::TZ, nty = n / G::TY, ntx = n / G::XC;
    const int ntiles = ntz * nty * ntx;
    // Each XCD (block ids are dealt round-robin over 8) walks a contiguous
    // range of tiles, so the rows neighbouring tiles share stay in its L2.
    const int nb = gridDim.x;
    const bool remap = (nb & 7) == 0 && (ntiles & 7) == 0;
    const int xcd = blockIdx.x & 7, lb = blockIdx.x >> 3, per = ntiles >> 3;
    // this thread's output pair: row rr, columns 2cp, 2cp+1 of the tile
    const int rr = tid / (G::TZ / 2), cp = tid - rr * (G::TZ / 2);
    double acc = 0.0;
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
        const size_t n2 = (size_t)n * n;
        // in-plane element offsets of this thread's pair loads (clamped tail)
        unsigned poff[G::LPT];
#pragma unroll
        for (int q = 0; q < G::LPT; ++q) {
            const int k = min(tid + q * G::NT, G::PAIRS - 1);
            const int r = k / G::NP, c2 = k - r * G::NP;
            poff[q] = (unsigned)(((y0 - 1 + r) & msk) * n + ((z0 - 2 + 2 * c2) & msk));
        }
        const unsigned eoff = (unsigned)((y0 + rr) * n + z0 + 2 * cp);
        VF regs[G::LPT];
        auto load = [&](int x) __attribute__((always_inline)) {
            const TF* pl = phi + (size_t)(x & msk) * n2;
#pragma unroll
            for (int q = 0; q < G::LPT; ++q) regs[q] = *reinterpret_cast<const VF*>(pl + poff[q]);
        };
        auto deposit = [&](int x) __attribute__((always_inline)) {
            TA* d = ring[(x - x0 + 3) % 3];
#pragma unroll
            for (int q = 0; q < G::LPT; ++q) {
                const int k = tid + q * G::NT;
                if ((q + 1) * G::NT <= G::PAIRS || k < G::PAIRS) {
                    const TA a = fma((TA)regs[q].x, uscale, uoffset),
                             b = fma((TA)regs[q].y, uscale, uoffset);
                    *reinterpret_cast<VA*>(d + 2 * k) = VA{a, b};
                    if constexpr (STAGED) {
                        TA* e = xring[(x - x0 + 3) % 3];
                        *reinterpret_cast<VA*>(e + 2 * k) = VA{SO::stage(a, exptab), SO::stage(b, exptab)};
                    }
                }
            }
        };
        auto eta_at = [&](int x) __attribute__((always_inline)) {
            return (size_t)(x & msk) * n2 + eoff;
        };
        load(x0 - 1);
        deposit(x0 - 1);
        load(x0);
        deposit(x0);
        VA enext = *reinterpret_cast<const VA*>(eta + eta_at(x0));
        load(x0 + 1);
        __syncthreads();
        for (int x = x0; x < x0 + G::XC; ++x) {
            // Everything loaded last step is consumed now; this step's loads
            // (clamped to the chunk: branch-free, so the compiler's wait
            // counts stay exact) overlap the stencil work below.
            deposit(x + 1);
            const VA e2 = enext;
            const size_t g = eta_at(x);
            enext = *reinterpret_cast<const VA*>(eta + eta_at(min(x + 1, x0 + G::XC - 1)));
            load(min(x + 2, x0 + G::XC));
            __syncthreads();
            const TA* pv = ring[(x - 1 - x0 + 3) % 3];
            const TA* cu = ring[(x - x0 + 3) % 3];
            const TA* nx = ring[(x + 1 - x0 + 3) % 3];
            const int o = (rr + 1) * G::EZ + 2 + 2 * cp;
            const VA c = *reinterpret_cast<const VA*>(cu + o);
            const VA xm = *reinterpret_cast<const VA*>(pv + o);
            const VA xp = *reinterpret_cast<const VA*>(nx + o);
            const VA ym = *reinterpret_cast<const VA*>(cu + o - G::EZ);
            const VA yp = *reinterpret_cast<const VA*>(cu + o + G::EZ);
            const TA zm = cu[o - 1], zp = cu[o + 2];
            VA ec, exm, exp_, eym, eyp;
            TA ezm = TA(0), ezp = TA(0);
            if constexpr (STAGED) {
                const TA* epv = xring[(x - 1 - x0 + 3) % 3];
                const TA* ecu = xring[(x - x0 + 3) % 3];
                const TA* enx = xring[(x + 1 - x0 + 3) % 3];
                ec = *reinterpret_cast<const VA*>(ecu + o);
                exm = *reinterpret_cast<const VA*>(epv + o);
                exp_ = *reinterpret_cast<const VA*>(enx + o);
                eym = *reinterpret_cast<const VA*>(ecu + o - G::EZ);
                eyp = *reinterpret_cast<const VA*>(ecu + o + G::EZ);
                ezm = ecu[o - 1];
                ezp = ecu[o + 2];
            }
            double L2[2];
#pragma unroll
            for (int dk = 0; dk < 2; ++dk) {
                TA nbv[6];
                nbv[0] = xm[dk];
                nbv[1] = xp[dk];
                nbv[2] = ym[dk];
                nbv[3] = yp[dk];
                nbv[4] = dk ? c[0] : zm;
                nbv[5] = dk ? zp : c[1];
                TA L, D;
                if constexpr (STAGED) {
                    TA enb[6];
                    enb[0] = exm[dk];
                    enb[1] = exp_[dk];
                    enb[2] = eym[dk];
                    enb[3] = eyp[dk];
                    enb[4] = dk ? ec[0] : ezm;
                    enb[5] = dk ? ezp : ec[1];
                    SO::eval(m, c[dk], nbv, ec[dk], enb, e2[dk], ih2, L, D);
                } else {
                    m.op(c[dk], nbv, e2[dk], ih2, L, D);
                }
                L2[dk] = (double)L;
                acc += L2[dk] * L2[dk];
            }
            if (res) *reinterpret_cast<VD*>(res + g) = VD{L2[0], L2[1]};
            __syncthreads();  // plane x-1's slot is refilled next
        }
    }
    double s = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Solve setup in one pass over the FP64 density (tiles, ring and summation
// order of k_defect_norm_tiled): the cold start phi_c = cold(eta), computed
// for every loaded value and staged in the ring, gives the defect whose
// squares sum to r_ref^2 (partial); the same pass writes phi_c to `cold` (if
// not NULL), its
// FP32 copy (cold - shift) * kVar to cold32 (if not NULL), the FP32 copy of
// eta to eta32 (if not NULL) and the 8-child mean of eta to eta_c (the next
// level, children summed in the order of k_restrict: x, then y, then z), and
// sums cold^2 into partial2.  n a power of two, a multiple of the tile.
template <class M>
__global__ __launch_bounds__(kBlock) void k_setup_tiled(M m, int n, double ih2,
                                                        const double* __restrict__ eta,
                                                        double* __restrict__ cold,
                                                        float* __restrict__ cold32, double scale32,
                                                        double offset32, float* __restrict__ eta32,
                                                        double* __restrict__ eta_c,
                                                        double* __restrict__ partial,
                                                        double* __restrict__ partial2)
{
    using G = NormTileF;
    using SO = StageOp<double, M>;
    using VD = typename Vec2<double>::type;
    using VF = typename Vec2<float>::type;
    constexpr bool STAGED = SO::kStaged;
    static_assert(G::XC % 2 == 0 && G::TY % 2 == 0, "tiles cover whole coarse cells");
    __shared__ __align__(16) double ring[3][G::PLANE];
    __shared__ __align__(16) double xring[STAGED ? 3 : 1][STAGED ? G::PLANE : 2];
    __shared__ double exptab[SO::kTable ? kExpTable : 1];
    if constexpr (SO::kTable) {
        exp_table_fill(exptab);
        __syncthreads();
    }
    const int tid = threadIdx.x;
    const int msk = n - 1;
    const int nc = n >> 1;
    const int ntz = n / G::TZ, nty = n / G::TY, ntx = n / G::XC;
    const int ntiles = ntz * nty * ntx;
    const int nb = gridDim.x;
    const bool remap = (nb & 7) == 0 && (ntiles & 7) == 0;
    const int xcd = blockIdx.x & 7, lb = blockIdx.x >> 3, per = ntiles >> 3;
    // this thread's pair: row rr, columns 2cp, 2cp+1 of the tile; rows rr and
    // rr ^ 1 sit in the two halves of one wave (32 pairs per row)
    const int rr = tid / (G::TZ / 2), cp = tid - rr * (G::TZ / 2);
    double acc = 0.0, acc2 = 0.0;
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
        const size_t n2 = (size_t)n * n;
        unsigned poff[G::LPT];
#pragma unroll
        for (int q = 0; q < G::LPT; ++q) {
            const int k = min(tid + q * G::NT, G::PAIRS - 1);
            const int r = k / G::NP, c2 = k - r * G::NP;
            poff[q] = (unsigned)(((y0 - 1 + r) & msk) * n + ((z0 - 2 + 2 * c2) & msk));
        }
        const unsigned eoff = (unsigned)((y0 + rr) * n + z0 + 2 * cp);
        VD regs[G::LPT];
        auto load = [&](int x) __attribute__((always_inline)) {
            const double* pl = eta + (size_t)(x & msk) * n2;
#pragma unroll
            for (int q = 0; q < G::LPT; ++q) regs[q] = *reinterpret_cast<const VD*>(pl + poff[q]);
        };
        auto deposit = [&](int x) __attribute__((always_inline)) {
            double* d = ring[(x - x0 + 3) % 3];
#pragma unroll
            for (int q = 0; q < G::LPT; ++q) {
                const int k = tid + q * G::NT;
                if ((q + 1) * G::NT <= G::PAIRS || k < G::PAIRS) {
                    const double a = (double)m.cold(regs[q].x), b = (double)m.cold(regs[q].y);
                    *reinterpret_cast<VD*>(d + 2 * k) = VD{a, b};
                    if constexpr (STAGED) {
                        double* e = xring[(x - x0 + 3) % 3];
                        *reinterpret_cast<VD*>(e + 2 * k) = VD{SO::stage(a, exptab), SO::stage(b, exptab)};
                    }
                }
            }
        };
        auto eta_at = [&](int x) __attribute__((always_inline)) {
            return (size_t)(x & msk) * n2 + eoff;
        };
        load(x0 - 1);
        deposit(x0 - 1);
        load(x0);
        deposit(x0);
        VD enext = *reinterpret_cast<const VD*>(eta + eta_at(x0));
        load(x0 + 1);
        __syncthreads();
        double csum = 0.0;  // the coarse cell's children so far (even rows)
        for (int x = x0; x < x0 + G::XC; ++x) {
            deposit(x + 1);
            const VD e2 = enext;
            const size_t g = eta_at(x);
            enext = *reinterpret_cast<const VD*>(eta + eta_at(min(x + 1, x0 + G::XC - 1)));
            load(min(x + 2, x0 + G::XC));
            __syncthreads();
            const double* pv = ring[(x - 1 - x0 + 3) % 3];
            const double* cu = ring[(x - x0 + 3) % 3];
            const double* nx = ring[(x + 1 - x0 + 3) % 3];
            const int o = (rr + 1) * G::EZ + 2 + 2 * cp;
            const VD c = *reinterpret_cast<const VD*>(cu + o);
            const VD xm = *reinterpret_cast<const VD*>(pv + o);
            const VD xp = *reinterpret_cast<const VD*>(nx + o);
            const VD ym = *reinterpret_cast<const VD*>(cu + o - G::EZ);
            const VD yp = *reinterpret_cast<const VD*>(cu + o + G::EZ);
            const double zm = cu[o - 1], zp = cu[o + 2];
            VD ec, exm, exp_, eym, eyp;
            double ezm = 0.0, ezp = 0.0;
            if constexpr (STAGED) {
                const double* epv = xring[(x - 1 - x0 + 3) % 3];
                const double* ecu = xring[(x - x0 + 3) % 3];
                const double* enx = xring[(x + 1 - x0 + 3) % 3];
                ec = *reinterpret_cast<const VD*>(ecu + o);
                exm = *reinterpret_cast<const VD*>(epv + o);
                exp_ = *reinterpret_cast<const VD*>(enx + o);
                eym = *reinterpret_cast<const VD*>(ecu + o - G::EZ);
                eyp = *reinterpret_cast<const VD*>(ecu + o + G::EZ);
                ezm = ecu[o - 1];
                ezp = ecu[o + 2];
            }
#pragma unroll
            for (int dk = 0; dk < 2; ++dk) {
                double nbv[6];
                nbv[0] = xm[dk];
                nbv[1] = xp[dk];
                nbv[2] = ym[dk];
                nbv[3] = yp[dk];
                nbv[4] = dk ? c[0] : zm;
                nbv[5] = dk ? zp : c[1];
                double L, D;
                if constexpr (STAGED) {
                    double enb[6];
                    enb[0] = exm[dk];
                    enb[1] = exp_[dk];
                    enb[2] = eym[dk];
                    enb[3] = eyp[dk];
                    enb[4] = dk ? ec[0] : ezm;
                    enb[5] = dk ? ezp : ec[1];
                    SO::eval(m, c[dk], nbv, ec[dk], enb, e2[dk], ih2, L, D);
                } else {
                    m.op(c[dk], nbv, e2[dk], ih2, L, D);
                }
                acc += L * L;
                acc2 += c[dk] * c[dk];
            }
            if (cold) *reinterpret_cast<VD*>(cold + g) = c;
            if (cold32)
                *reinterpret_cast<VF*>(cold32 + g) =
                    VF{(float)(c[0] * scale32 + offset32), (float)(c[1] * scale32 + offset32)};
            if (eta32) *reinterpret_cast<VF*>(eta32 + g) = VF{(float)e2[0], (float)e2[1]};
            // the next level's density: children (x, row, z) in the order x, y, z
            const double p0 = __shfl_xor(e2[0], 32, 64), p1 = __shfl_xor(e2[1], 32, 64);
            if ((x & 1) == 0) csum = 0.0;
            csum += e2[0];
            csum += e2[1];
            csum += p0;
            csum += p1;
            if ((x & 1) && (rr & 1) == 0)
                eta_c[((size_t)(x >> 1) * nc + ((y0 + rr) >> 1)) * nc + (z0 >> 1) + cp] = csum / 8.0;
            __syncthreads();  // plane x-1's slot is refilled next
        }
    }
    double s = block_sum(acc);
    double s2 = block_sum(acc2);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = s;
        partial2[blockIdx.x] = s2;
    }
}

}  // namespace isis
