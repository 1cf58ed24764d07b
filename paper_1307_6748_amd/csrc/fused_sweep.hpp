// Fused red-black Newton-Gauss-Seidel sweeps: TB full sweeps (2*TB colour
// stages) per pass over HBM, out of place (in -> out).
//
// Each workgroup owns a TY x TZ tile of the y-z plane and streams along x over
// one of NXC chunks of about n / NXC planes (chunk ends even; the host picks
// NXC, see fused_chunks).  Planes of phi (with a y/z halo of H = 2*TB cells)
// pass through a ring of NR = 2*TB + 2 planes in LDS.  At step s the
// workgroup holds planes s-NR+1 .. s and applies, in this order,
//   stage 1 (red)   to plane s-1,
//   stage 2 (black) to plane s-2,
//   stage 3 (red)   to plane s-3,   (TB = 2)
//   stage 4 (black) to plane s-4,   (TB = 2)
// each stage on the part of its plane whose six neighbours are already at the
// previous stage (the valid region shrinks by one cell of halo per stage), and
// writes plane s-2*TB's interior.  This ordering reads every neighbour at
// exactly the stage the sequential red-black sweep would see, so the result
// equals 2*TB in-place half-sweeps up to rounding of contracted FMAs.  The
// input array is only read, so workgroups never race.
//
// Only phi (and, for f(R), its e^u) lives in LDS.  Each thread loads the
// density (and the FAS source on coarse levels) of exactly the cells it will
// update one step ahead, into registers.  Planes of phi are fetched two steps
// ahead into registers and stored to LDS after the stages of the step in
// between, so HBM latency overlaps two steps of compute.  For f(R) the flux
// coefficients e^u are computed once per loaded cell and refreshed only for
// updated cells (instead of seven exponentials per cell update).  Workgroup
// ids are remapped so that each XCD (ids are dealt round-robin over 8 XCDs)
// processes a contiguous, spatially adjacent range of tiles, whose shared
// halo rows then hit in that XCD's L2.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.hpp"

namespace isis {

template <class T, int TB_, int TY_, int TZ_, int NT_>
struct FusedGeom {
    static constexpr int TB = TB_, TY = TY_, TZ = TZ_, NT = NT_;
    static constexpr int H = 2 * TB;            // y/z halo of loaded planes
    static constexpr int EY = TY + 2 * H;       // loaded plane rows
    static constexpr int EZ = TZ + 2 * H;       // loaded plane columns (even)
    static constexpr int NP = EZ / 2;           // column pairs per row
    static constexpr int HZ = EZ / 2;           // LDS rows: HZ even columns, then HZ odd
    static constexpr int PLANE = EY * EZ;       // elements per plane
    static constexpr int NR = 2 * TB + 2;       // phi ring planes
    static constexpr int PAIRS = EY * NP;       // pair loads per plane
    static constexpr int LPT = (PAIRS + NT - 1) / NT;  // pair loads per thread
    // cells of one colour updated by stage k (1-based) and per thread
    // coarse planes for the prolongation fused into a pass (see PROL): the
    // parents and their neighbours of the loaded fine rows and columns
    static constexpr int CJ = EY / 2 + 2, CK = EZ / 2 + 2, CP = CJ * CK;
    static constexpr int CLPT = (CP + NT - 1) / NT;
    static constexpr int items(int k) { return (EY - 2 * k) * ((EZ - 2 * k) / 2); }
    static constexpr int ipt(int k) { return (items(k) + NT - 1) / NT; }
    static constexpr int MAXI = (items(1) + NT - 1) / NT;
};

// Work item `it` of a region of R rows of L items each (cells of one colour,
// or column pairs).  SPLIT: the first R * M items, M = L rounded down to a
// multiple of 32, take rows whole, M per row, so every 32-lane half of a wave
// covers 32 consecutive items of one row; the L - M items left over at the
// end of each row follow, row by row.  With the colour-split rows in LDS a
// half-wave then reads 32 consecutive words, which LDS serves without bank
// conflicts; in plain row-major order half-waves straddle two rows whose
// words share banks (33 or 34 items per row: about 1.5 conflict cycles per
// LDS access, 0.16 split).  The split order pays for f(R), whose stages read
// two LDS rings (its sweep 2 % faster, 4 % with the prolongation fused in);
// the symmetron's HBM-bound passes measured 1 % slower with it (the leftover
// items' density loads scatter over many rows), so they keep row-major order.
template <bool SPLIT>
__device__ __forceinline__ void row_split(int it, int R, int L, int& r, int& c)
{
    const int M = SPLIT ? L & ~31 : 0, E = L - M;
    if (SPLIT && it < R * M) {
        r = it / M;
        c = it - r * M;
    } else {
        const int j = it - R * M;
        r = j / E;
        c = M + (j - r * E);
    }
}

// Compile-time loop: f(std::integral_constant<int, i>) for i in [B, E).
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Shared-memory footprint of one workgroup, in bytes.
template <class T, class M, int TB, int TY, int TZ, bool PROL = false>
constexpr int fused_lds_bytes()
{
    using G = FusedGeom<T, TB, TY, TZ, 256>;
    int planes = G::NR * (StageOp<T, M>::kStaged ? 2 : 1);
    return (planes * G::PLANE + (PROL ? G::CP : 0)) * (int)sizeof(T);
}

// Element at byte offset `off` from `base` (32-bit offsets from a uniform
// base let loads use the scalar-base addressing mode).
template <class T>
__device__ __forceinline__ const T& at_bytes(const T* base, unsigned off)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
}
template <class T>
__device__ __forceinline__ T& at_bytes(T* base, unsigned off)
{
    return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off);
}

// PROL: the pass first adds the coarse-grid correction P(cphi - cphat) to
// every value of `in` it loads (cell-centred trilinear prolongation, Sec. 3.2;
// cphi, cphat of side n/2), so `in` holds the field before the correction and
// the corrected field is never written.  A fine plane x reads its parent
// plane x/2 and the neighbour on its side; the two current coarse planes of
// the tile's window live in registers (each thread the same elements), coarse
// plane s/2 + 1 replacing s/2 - 1 at each even step s, fetched two steps
// ahead.
// TI (not with PROL): the type of `in`; a float input of a double pass holds
// the field as stored in single precision, and each loaded value v enters as
// v * in_scale + in_offset (the FP32 iterate handed over to FP64 cycles).
template <class T, class M, int TB, int TY, int TZ, int NT, bool SIG, bool PROL = false,
          class TI = T>
__global__ __launch_bounds__(NT) void k_sweep_fused(M m, int n, int nxc, T ih2,
                                                    const TI* __restrict__ in, T* __restrict__ out,
                                                    const T* __restrict__ eta,
                                                    const T* __restrict__ sigma,
                                                    const T* __restrict__ cphi = nullptr,
                                                    const T* __restrict__ cphat = nullptr,
                                                    T in_scale = T(1), T in_offset = T(0))
{
    static_assert(std::is_same<TI, T>::value || (!PROL && sizeof(TI) < sizeof(T)),
                  "a converted input is wider, and not with the fused prolongation");
    using G = FusedGeom<T, TB, TY, TZ, NT>;
    using V = typename Vec2<T>::type;
    using VI = typename Vec2<TI>::type;
    constexpr bool CONV = !std::is_same<TI, T>::value;
    using SO = StageOp<T, M>;
    constexpr bool STAGED = SO::kStaged;
    constexpr int NK = 2 * TB;
    constexpr int SZ = (int)sizeof(T);
    // For TB = 1 the black stage's density (and source) of a plane is loaded
    // in the same step as the red stage's, two steps before use, so both
    // colours of a cache line are fetched together.
    constexpr bool LATE2 = (TB == 1);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* ring = reinterpret_cast<T*>(smem_raw);  // NR planes of phi
    T* xring = ring + G::NR * G::PLANE;        // NR planes of e^phi (f(R) only)
    __shared__ double exptab[SO::kTable ? kExpTable : 1];
    if constexpr (SO::kTable) {
        exp_table_fill(exptab);
        __syncthreads();
    }

    // XCD-aware tile order: ids are dealt round-robin to 8 XCDs; give each
    // XCD a contiguous range of tiles.
    const int nb = gridDim.x;
    int b = blockIdx.x;
    if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
    const int ntz = n / TZ, nty = n / TY;
    const int zt = b % ntz;
    const int yt = (b / ntz) % nty;
    const int xt = b / (ntz * nty);
    // chunk [x0, x1) with both ends even (n is even)
    const int x0 = (xt * n / nxc) & ~1, x1 = ((xt + 1) * n / nxc) & ~1;
    const int y0 = yt * TY, z0 = zt * TZ;
    // x0 and H are even, so sbeg is even: the unrolled steps below alternate
    // even and odd planes, which fixes every parity at compile time.
    const int sbeg = x0 - G::H, send = x1 - 1 + G::H;
    const int msk = n - 1;
    const size_t n2 = (size_t)n * n;
    const int tid = threadIdx.x;

    // Ring slot of plane s + d at step index J = (s - sbeg) mod NR: the loop
    // below is unrolled over NR steps, so every slot is a compile-time
    // constant and LDS addresses fold into the instructions' offsets.
    auto slotc = [](int J, int d) constexpr { return ((J + d) % G::NR + G::NR) % G::NR; };
    auto stage_valid = [&](int p, int k) __attribute__((always_inline)) { return p >= sbeg + k && p <= send - k; };
    // Plane row r, column c of a plane in LDS.  Rows are stored colour-split
    // (even columns, then odd columns): the cells one stage updates have one
    // column parity per row, so consecutive lanes of a row touch consecutive
    // words (and for f(R) row_split keeps each half-wave within one row).
    auto lds = [&](int r, int c) __attribute__((always_inline)) {
        return r * G::EZ + (c & 1) * G::HZ + (c >> 1);
    };

    // ---- Per-thread address tables (byte offsets; independent of the plane) ----
    // Pair loads of a plane (the tail clamped to a valid pair: branch-free
    // loads let the compiler count outstanding loads exactly).
    unsigned poff[G::LPT];
    int doff[G::LPT];  // LDS element offset of the pair's even column
#pragma unroll
    for (int q = 0; q < G::LPT; ++q) {
        const int it = min(tid + q * NT, G::PAIRS - 1);
        int r, cp;
        row_split<STAGED>(it, G::EY, G::NP, r, cp);
        poff[q] = (unsigned)((((y0 - G::H + r) & msk) * n + ((z0 - G::H + 2 * cp) & msk)) * SZ);
        doff[q] = r * G::EZ + cp;
    }
    // Cells updated by stage k (1-based), per item q, for plane parity pb:
    // global byte offset in the plane (items clamped: the load is always
    // valid) and LDS element offset.
    unsigned goff[NK][G::MAXI][2];
    int loff[NK][G::MAXI][2];
    int zoff[NK][G::MAXI][2];  // LDS offset of the z- neighbour; z+ is the next word
    // Safeguard counting (models with kGuard): bit (k-1, q, pb) is set when the
    // item's cell lies in this workgroup's own TY x TZ tile, so updates of the
    // halo, which neighbouring tiles also make, are counted once.
    static_assert(!M::kGuard || NK * G::MAXI * 2 <= 32, "ownership mask needs 32 bits");
    unsigned own = 0;
    static_for<0, NK>([&](auto kc) {
        constexpr int k = decltype(kc)::value + 1;
        constexpr int colour = (k - 1) & 1;  // stages 1, 3: red; 2, 4: black
        constexpr int pairs = (G::EZ - 2 * k) / 2;
        static_for<0, G::ipt(k)>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            const int it = min(tid + q * NT, G::items(k) - 1);
            int rr, cp;
            row_split<STAGED>(it, G::EY - 2 * k, pairs, rr, cp);
            const int r = k + rr;
#pragma unroll
            for (int pb = 0; pb < 2; ++pb) {
                const int par = (pb + y0 + z0 + k + colour + r) & 1;
                const int c = k + 2 * cp + par;
                goff[k - 1][q][pb] = (unsigned)((((y0 - G::H + r) & msk) * n +
                                                 ((z0 - G::H + c) & msk)) * SZ);
                loff[k - 1][q][pb] = lds(r, c);
                zoff[k - 1][q][pb] = lds(r, c - 1);  // lds(r, c + 1) == lds(r, c - 1) + 1
                if constexpr (M::kGuard) {
                    const bool mine = r >= G::H && r < G::H + TY && c >= G::H && c < G::H + TZ;
                    own |= (mine ? 1u : 0u) << (((k - 1) * G::MAXI + q) * 2 + pb);
                }
            }
        });
    });
    constexpr int OP = TZ / 2;                         // output pairs per row
    constexpr int WPT = (TY * OP + NT - 1) / NT;       // output pairs per thread
    unsigned woff[WPT];
    int wl[WPT];
#pragma unroll
    for (int j = 0; j < WPT; ++j) {
        const int it = min(tid + j * NT, TY * OP - 1);
        const int rr = it / OP, cp = it - rr * OP;
        woff[j] = (unsigned)(((y0 + rr) * n + z0 + 2 * cp) * SZ);
        wl[j] = lds(G::H + rr, G::H + 2 * cp);  // even column (H is even)
    }

    // PROL: each thread owns elements e = tid + q*NT of the coarse window (the
    // tile's parents plus a one-cell halo: rows from coarse row (y0 - H)/2 - 1,
    // columns from (z0 - H)/2 - 1) and keeps them, for the two coarse planes
    // the current fine plane reads, in registers (older, newer), with the next
    // plane in flight (cA - cB).  Per fine plane x it writes the window
    // interpolated along x (3/4 parent x/2, 1/4 its neighbour on x's side) to
    // LDS, from which each fine pair interpolates along y and z.
    const int nc = n >> 1, cmsk = nc - 1;
    const size_t nc2 = (size_t)nc * nc;
    unsigned cgoff[PROL ? G::CLPT : 1];
    T cA[PROL ? G::CLPT : 1], cB[PROL ? G::CLPT : 1];
    T cold_[PROL ? G::CLPT : 1] = {}, cnew[PROL ? G::CLPT : 1] = {};
    T* xbuf = ring + G::NR * G::PLANE * (STAGED ? 2 : 1);  // the x-interpolated window (PROL)
    if constexpr (PROL) {
        const int jb = ((y0 - G::H) >> 1) - 1, kb = ((z0 - G::H) >> 1) - 1;
#pragma unroll
        for (int q = 0; q < G::CLPT; ++q) {
            const int e = min(tid + q * NT, G::CP - 1);
            const int cr = e / G::CK, cc = e - cr * G::CK;
            cgoff[q] = (unsigned)((((jb + cr) & cmsk) * nc + ((kb + cc) & cmsk)) * SZ);
        }
    }
    auto load_coarse = [&](int cpl) __attribute__((always_inline)) {  // into cA, cB
        if constexpr (PROL) {
            const T* a0 = cphi + (size_t)(cpl & cmsk) * nc2;
            const T* b0 = cphat + (size_t)(cpl & cmsk) * nc2;
#pragma unroll
            for (int q = 0; q < G::CLPT; ++q) {
                cA[q] = at_bytes(a0, cgoff[q]);
                cB[q] = at_bytes(b0, cgoff[q]);
            }
        }
    };
    auto advance_coarse = [&]() __attribute__((always_inline)) {  // newer plane arrives
        if constexpr (PROL) {
#pragma unroll
            for (int q = 0; q < G::CLPT; ++q) {
                cold_[q] = cnew[q];
                cnew[q] = cA[q] - cB[q];
            }
        }
    };
    // x-interpolated window for fine plane x: x odd reads parents (older,
    // newer) = (x/2, x/2 + 1), x even (newer, older) = (x/2, x/2 - 1)
    auto write_xbuf = [&](auto oddc) __attribute__((always_inline)) {
        if constexpr (PROL) {
            constexpr bool ODD = decltype(oddc)::value;
#pragma unroll
            for (int q = 0; q < G::CLPT; ++q)
                if ((q + 1) * NT <= G::CP || tid + q * NT < G::CP)
                    xbuf[tid + q * NT] = ODD ? T(0.75) * cold_[q] + T(0.25) * cnew[q]
                                             : T(0.75) * cnew[q] + T(0.25) * cold_[q];
        }
    };
    // the correction of the loaded pairs: per pair (fine row r, columns 2cp,
    // 2cp+1 of the loaded plane), parent window row (r >> 1) + 1 (3/4) and its
    // neighbour on r's side (1/4); columns cp, cp+1, cp+2 hold K'-1, K', K'+1
    // of the pair's parent K' (cell 2K' takes 3/4 K' + 1/4 K'-1, cell 2K'+1
    // 3/4 K' + 1/4 K'+1)
    auto correct = [&](V (&regs)[G::LPT]) __attribute__((always_inline)) {
        if constexpr (PROL) {
            const T w0 = T(0.75), w1 = T(0.25);
#pragma unroll
            for (int q = 0; q < G::LPT; ++q) {
                const int r = doff[q] / G::EZ, cp = doff[q] - r * G::EZ;
                const int j0 = (r >> 1) + 1, j1 = j0 + ((r & 1) ? 1 : -1);
                const T* a0 = xbuf + j0 * G::CK + cp;
                const T* a1 = xbuf + j1 * G::CK + cp;
                T t[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) t[d] = w0 * a0[d] + w1 * a1[d];
                regs[q].x += w0 * t[1] + w1 * t[0];
                regs[q].y += w0 * t[1] + w1 * t[2];
            }
        }
    };

    unsigned hits = 0;  // safeguard activations on owned cells (kGuard models)
    VI pA[G::LPT], pB[G::LPT];
    T eA[NK][G::MAXI], eB[NK][G::MAXI];
    T sA[SIG ? NK : 1][SIG ? G::MAXI : 1], sB[SIG ? NK : 1][SIG ? G::MAXI : 1];

    auto load_plane = [&](int x, VI (&regs)[G::LPT]) __attribute__((always_inline)) {
        const TI* src = in + (size_t)(x & msk) * n2;
        constexpr unsigned shr = CONV ? (SZ == 8 ? 1 : 0) : 0;  // poff counts T-sized elements
#pragma unroll
        for (int q = 0; q < G::LPT; ++q)
            regs[q] = at_bytes(reinterpret_cast<const VI*>(src), poff[q] >> shr);
    };
    // Density (and FAS source) of stage k's cells on plane p (parity PB).
    auto fetch_stage = [&](auto kc, auto pbc, int p, T (&e)[NK][G::MAXI],
                           T (&sg)[SIG ? NK : 1][SIG ? G::MAXI : 1]) __attribute__((always_inline)) {
        constexpr int k = decltype(kc)::value;
        constexpr int PB = decltype(pbc)::value;
        const T* ep = eta + (size_t)(p & msk) * n2;
        const T* sp = SIG ? sigma + (size_t)(p & msk) * n2 : nullptr;
        static_for<0, G::ipt(k)>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            e[k - 1][q] = at_bytes(ep, goff[k - 1][q][PB]);
            if constexpr (SIG) sg[k - 1][q] = at_bytes(sp, goff[k - 1][q][PB]);
        });
    };

    auto deposit = [&](auto slc, VI (&regs)[G::LPT]) __attribute__((always_inline)) {
        constexpr int SL = decltype(slc)::value;
        if constexpr (PROL) correct(regs);
        T* dst = ring + SL * G::PLANE;
        T* xd = xring + SL * G::PLANE;
#pragma unroll
        for (int q = 0; q < G::LPT; ++q) {
            if ((q + 1) * NT <= G::PAIRS || tid + q * NT < G::PAIRS) {
                const int oe = doff[q];      // column 2cp (even half)
                const int oo = oe + G::HZ;   // column 2cp+1 (odd half)
                T a, b;
                if constexpr (CONV) {
                    a = fma((T)regs[q].x, in_scale, in_offset);
                    b = fma((T)regs[q].y, in_scale, in_offset);
                } else {
                    a = regs[q].x;
                    b = regs[q].y;
                }
                dst[oe] = a;
                dst[oo] = b;
                if constexpr (STAGED) {
                    xd[oe] = SO::stage(a, exptab);
                    xd[oo] = SO::stage(b, exptab);
                }
            }
        }
    };

    // Stages of step s (step index J = (s - sbeg) mod NR, fixed at compile
    // time; its parity is that of s since sbeg is even).
    auto stages = [&](auto jc, int s, const T (&e)[NK][G::MAXI],
                      const T (&sg)[SIG ? NK : 1][SIG ? G::MAXI : 1]) __attribute__((always_inline)) {
        constexpr int J = decltype(jc)::value;
        constexpr int S2 = J & 1;
        static_for<0, NK>([&](auto kc) {
            constexpr int k = decltype(kc)::value + 1;
            constexpr int PB = (S2 + k) & 1;  // parity of plane s - k
            constexpr int SC = slotc(J, -k), SP = slotc(J, -k - 1), SN = slotc(J, -k + 1);
            const int p = s - k;
            if (stage_valid(p, k)) {
                T* cur = ring + SC * G::PLANE;
                const T* prv = ring + SP * G::PLANE;
                const T* nxt = ring + SN * G::PLANE;
                T* xcur = xring + SC * G::PLANE;
                const T* xprv = xring + SP * G::PLANE;
                const T* xnxt = xring + SN * G::PLANE;
                static_for<0, G::ipt(k)>([&](auto qc) {
                    constexpr int q = decltype(qc)::value;
                    if ((q + 1) * NT <= G::items(k) || tid + q * NT < G::items(k)) {
                        const int o = loff[k - 1][q][PB];
                        T nb[6];
                        nb[0] = prv[o];
                        nb[1] = nxt[o];
                        nb[2] = cur[o - G::EZ];
                        nb[3] = cur[o + G::EZ];
                        const int ozm = zoff[k - 1][q][PB], ozp = ozm + 1;
                        nb[4] = cur[ozm];
                        nb[5] = cur[ozp];
                        const T pc = cur[o];
                        T L, D;
                        if constexpr (STAGED) {
                            T enb[6];
                            enb[0] = xprv[o];
                            enb[1] = xnxt[o];
                            enb[2] = xcur[o - G::EZ];
                            enb[3] = xcur[o + G::EZ];
                            enb[4] = xcur[ozm];
                            enb[5] = xcur[ozp];
                            SO::eval(m, pc, nb, xcur[o], enb, e[k - 1][q], ih2, L, D);
                        } else {
                            SO::eval(m, pc, nb, T(0), nullptr, e[k - 1][q], ih2, L, D);
                        }
                        if constexpr (M::kGuard) {
                            constexpr int bit = ((k - 1) * G::MAXI + q) * 2 + PB;
                            if ((own >> bit) & 1u)
                                hits += (p >= x0 && p < x1) ? m.guarded(pc, e[k - 1][q]) : 0u;
                        }
                        T eps = L;
                        if constexpr (SIG) eps -= sg[k - 1][q];
                        const T nv = pc - m.limit(eps * recip(D));
                        cur[o] = nv;
                        if constexpr (STAGED) {
                            if (k < NK) xcur[o] = SO::stage(nv, exptab);
                        }
                    }
                });
            }
            __syncthreads();
        });
    };

    auto write_out = [&](auto jc, int s) __attribute__((always_inline)) {
        constexpr int J = decltype(jc)::value;
        const int pw = s - NK;
        if (pw >= x0 && pw < x1) {
            const T* src = ring + slotc(J, -NK) * G::PLANE;
            T* dst = out + (size_t)(pw & msk) * n2;
#pragma unroll
            for (int j = 0; j < WPT; ++j) {
                if ((j + 1) * NT <= TY * OP || tid + j * NT < TY * OP) {
                    V v;
                    v.x = src[wl[j]];
                    v.y = src[wl[j] + G::HZ];
                    // streaming store: keeps L2 for the halo rows that
                    // neighbouring tiles still have to read
                    __builtin_nontemporal_store(v, &at_bytes(reinterpret_cast<V*>(dst), woff[j]));
                }
            }
        }
    };

    // One step: planes up to s are in LDS, plane s+1 is in `ready`; `spare`
    // (which held plane s) receives plane s+2.  ec/sc hold this step's cell
    // data, en/sn receive the next step's (with LATE2, the black stage's
    // entries of ec/sc are consumed here and refilled for step s+2).
    auto step = [&](auto jc, int s, VI (&spare)[G::LPT], VI (&ready)[G::LPT],
                    T (&ec)[NK][G::MAXI], T (&sc)[SIG ? NK : 1][SIG ? G::MAXI : 1],
                    T (&en)[NK][G::MAXI], T (&sn)[SIG ? NK : 1][SIG ? G::MAXI : 1]) __attribute__((always_inline)) {
        constexpr int J = decltype(jc)::value;
        constexpr int S2 = J & 1;
        if constexpr (PROL) {
            // even s: coarse plane s/2 + 1 arrives (s/2 becomes the older);
            // then the window for plane s + 1, read by this step's deposit
            // after the stage barriers (the previous deposit's reads ended at
            // the previous step's closing barrier)
            if constexpr (S2 == 0) {
                advance_coarse();
                load_coarse((s >> 1) + 2);
            }
            write_xbuf(std::integral_constant<bool, S2 == 0>{});
        }
        // (past the chunk end these load wrapped, unused planes: branch-free)
        load_plane(s + 2, spare);
        // next step's stage k works on plane s + 1 - k
        static_for<0, NK>([&](auto kc) {
            constexpr int k = decltype(kc)::value + 1;
            if constexpr (!(LATE2 && k == 2))
                fetch_stage(std::integral_constant<int, k>{},
                            std::integral_constant<int, (S2 + 1 + k) & 1>{}, s + 1 - k, en, sn);
        });
        stages(jc, s, ec, sc);  // ends with a barrier: the slot of plane s+1-NR is free
        if constexpr (LATE2)    // black stage of plane s, used at step s+2
            fetch_stage(std::integral_constant<int, 2>{}, std::integral_constant<int, S2>{}, s,
                        ec, sc);
        write_out(jc, s);
        if (s + 1 <= send) deposit(std::integral_constant<int, slotc(J, 1)>{}, ready);
        __syncthreads();
    };

    // Prologue: planes sbeg, sbeg+1 in flight; step sbeg's red-stage data;
    // the black-stage data of the first two steps belong to invalid stages.
#pragma unroll
    for (int k = 0; k < NK; ++k)
#pragma unroll
        for (int q = 0; q < G::MAXI; ++q) {
            eA[k][q] = T(1);
            eB[k][q] = T(1);
            if constexpr (SIG) {
                sA[k][q] = T(0);
                sB[k][q] = T(0);
            }
        }
    load_plane(sbeg, pA);
    load_plane(sbeg + 1, pB);
    if constexpr (PROL) {  // older sbeg/2 - 1, newer sbeg/2; sbeg/2 + 1 in flight
        load_coarse((sbeg >> 1) - 1);
        advance_coarse();
        load_coarse(sbeg >> 1);
        advance_coarse();
        load_coarse((sbeg >> 1) + 1);
        write_xbuf(std::integral_constant<bool, false>{});  // plane sbeg (even)
        __syncthreads();
    }
    deposit(std::integral_constant<int, 0>{}, pA);
    static_for<0, NK>([&](auto kc) {
        constexpr int k = decltype(kc)::value + 1;
        if constexpr (!(LATE2 && k == 2))
            fetch_stage(std::integral_constant<int, k>{}, std::integral_constant<int, k & 1>{},
                        sbeg - k, eA, sA);
    });
    __syncthreads();
    for (int s0 = sbeg; s0 <= send; s0 += G::NR) {
        static_for<0, G::NR>([&](auto jc) {
            constexpr int J = decltype(jc)::value;
            const int s = s0 + J;
            if (s <= send) {
                if constexpr ((J & 1) == 0)
                    step(jc, s, pA, pB, eA, sA, eB, sB);
                else
                    step(jc, s, pB, pA, eB, sB, eA, sA);
            }
        });
    }
    guard_flush(m, hits);
}

// ---------------------------------------------------------------------------
// Host side: configuration per (type, model), launch, and sweep sequencing.
// ---------------------------------------------------------------------------

// Tile height for a given (type, model, temporal block): the tallest of 16, 8
// that lets two workgroups share a CU's 160 KiB of LDS, else 8 (one
// workgroup per CU).
template <class T, class M, int TB>
struct FusedTile {
    static constexpr int TZ = 64, NT = 256;
    static constexpr int kHalf = 80 * 1024, kFull = 160 * 1024;
    static constexpr int TY = fused_lds_bytes<T, M, TB, 16, 64>() <= kHalf ? 16 : 8;
    static_assert(fused_lds_bytes<T, M, TB, TY, 64>() <= kFull, "LDS overflow");
};

constexpr int kFusedMinN = 64;

template <class T, class M>
inline bool fused_supported(int n)
{
    return n >= kFusedMinN && (n & (n - 1)) == 0;
}

// Kernel launches made for `count` sweeps with temporal block tb.
inline int fused_launches(int count, int tb) { return tb >= 2 ? (count + 1) / 2 : count; }

inline int fused_chunk(int n)
{
    // planes streamed per workgroup: long enough to amortise the 2*H-plane
    // pipeline fill, short enough to give >= 1024 workgroups at 512^3
    return n >= 512 ? 64 : (n >= 256 ? 32 : 16);
}

// Chunks along x per tile column.  When the device holds a whole number
// (<= 16) of workgroups per tile column at once and the chunks stay at least
// 16 planes long, one round of that many chunks: every workgroup slot busy,
// no partly filled last round (measured: 512^3, 3 per tile column, 3-5%
// faster than 64-plane chunks; 256^3, 12 per tile column, FP32 f(R) 9% faster
// than 32-plane chunks, which filled two thirds of the slots).  Otherwise, or
// when the occupancy is unknown (resident <= 0), fused_chunk() planes per
// chunk.
inline int fused_chunks(int n, int tiles, int resident)
{
    if (resident > 0 && resident % tiles == 0 && resident / tiles <= 16 &&
        resident / tiles <= n / 16)
        return resident / tiles;
    return n / fused_chunk(n);
}

template <class T, class M, int TB, bool SIG, bool PROL = false, class TI = T>
int launch_fused_pass(const M& m, int n, double h, const TI* in, T* out, const T* eta,
                      const T* sigma, hipStream_t s, char* err, const T* cphi = nullptr,
                      const T* cphat = nullptr, double in_scale = 1.0, double in_offset = 0.0)
{
    using Tile = FusedTile<T, M, TB>;
    constexpr int TY = Tile::TY, TZ = Tile::TZ, NT = Tile::NT;
    constexpr int lds = fused_lds_bytes<T, M, TB, TY, TZ, PROL>();
    static_assert(lds <= Tile::kFull, "LDS overflow");
    auto kern = k_sweep_fused<T, M, TB, TY, TZ, NT, SIG, PROL, TI>;
    static std::atomic<unsigned> lds_done{0};  // per instantiation: devices set up
    if (ensure_dynamic_lds((const void*)kern, lds, lds_done) != hipSuccess) {
        snprintf(err, 512, "hipFuncSetAttribute(shared %d B) failed", lds);
        return -4;
    }
    static std::atomic<int> resident[kMaxDevices];  // per instantiation and device
    const int res = resident_blocks((const void*)kern, NT, lds, resident);
    const int tiles = (n / TZ) * (n / TY);
    const int nxc = fused_chunks(n, tiles, res);
    const int blocks = tiles * nxc;
    T ih2 = (T)(1.0 / (h * h));
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(NT), lds, s, m, n, nxc, ih2, in, out, eta, sigma,
                       cphi, cphat, (T)in_scale, (T)in_offset);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        snprintf(err, 512, "k_sweep_fused: %s", hipGetErrorString(e));
        return -4;
    }
    return 0;
}

template <class T, class M, int TB, bool PROL>
int launch_fused_pass_sig(const M& m, int n, double h, const T* in, T* out, const T* eta,
                          const T* sigma, hipStream_t s, char* err, const T* cphi,
                          const T* cphat)
{
    return sigma ? launch_fused_pass<T, M, TB, true, PROL>(m, n, h, in, out, eta, sigma, s, err,
                                                           cphi, cphat)
                 : launch_fused_pass<T, M, TB, false, PROL>(m, n, h, in, out, eta, sigma, s, err,
                                                            cphi, cphat);
}

// Sweeps in the first fused pass of `count` sweeps with temporal block tb.
inline int fused_first_pass(int count, int tb) { return (tb >= 2 && count >= 2) ? 2 : 1; }

// `count` sweeps of phi through the fused kernels, ping-ponging between *phi
// and *tmp.  On return *phi points at the buffer holding the result (the two
// pointers are swapped when the number of passes is odd).  With cphi (and
// cphat, side n/2), phi += P(cphi - cphat) first, inside the first pass,
// which must then be a single sweep (fused_first_pass == 1): in a two-sweep
// pass the extra registers cost a third of the workgroups per CU, more than
// the separate prolongation pass saves.  With in32 (double passes, no cphi,
// count >= 1, no FAS source), the first pass reads the field from in32 (its
// values times in_scale plus in_offset) instead of *phi, which it only
// writes to through the ping-pong.
template <class T, class M>
int launch_fused_sweeps(const M& m, int n, double h, T** phi, T** tmp, const T* eta,
                        const T* sigma, int count, int tb, hipStream_t s, char* err,
                        const T* cphi = nullptr, const T* cphat = nullptr,
                        const float* in32 = nullptr, double in_scale = 1.0, double in_offset = 0.0)
{
    if (cphi && fused_first_pass(count, tb) != 1) {
        snprintf(err, 512, "fused prolongation needs a single-sweep first pass");
        return -4;
    }
    if (in32 && (sizeof(T) != 8 || cphi || sigma || count < 1)) {
        snprintf(err, 512, "a single-precision input needs a double pass without prolongation "
                           "or FAS source");
        return -4;
    }
    int done = 0;
    if constexpr (sizeof(T) == 8) {
        if (in32) {  // the first pass, from the single-precision field
            const int step = fused_first_pass(count, tb);
            const int r = step == 2
                              ? launch_fused_pass<T, M, 2, false, false, float>(
                                    m, n, h, in32, *tmp, eta, nullptr, s, err, nullptr, nullptr,
                                    in_scale, in_offset)
                              : launch_fused_pass<T, M, 1, false, false, float>(
                                    m, n, h, in32, *tmp, eta, nullptr, s, err, nullptr, nullptr,
                                    in_scale, in_offset);
            if (r) return r;
            T* t = *phi;
            *phi = *tmp;
            *tmp = t;
            done = step;
        }
    }
    while (done < count) {
        const int step = (tb >= 2 && count - done >= 2) ? 2 : 1;
        const bool prol = cphi && done == 0;
        int r;
        if (step == 2)
            r = launch_fused_pass_sig<T, M, 2, false>(m, n, h, *phi, *tmp, eta, sigma, s, err,
                                                      nullptr, nullptr);
        else
            r = prol ? launch_fused_pass_sig<T, M, 1, true>(m, n, h, *phi, *tmp, eta, sigma, s, err,
                                                            cphi, cphat)
                     : launch_fused_pass_sig<T, M, 1, false>(m, n, h, *phi, *tmp, eta, sigma, s,
                                                             err, nullptr, nullptr);
        if (r) return r;
        T* t = *phi;
        *phi = *tmp;
        *tmp = t;
        done += step;
    }
    return 0;
}

}  // namespace isis
