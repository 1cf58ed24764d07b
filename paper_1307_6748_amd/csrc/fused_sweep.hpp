// Fused red-black Newton-Gauss-Seidel sweeps: TB full sweeps (2*TB colour
// stages) per pass over HBM, out of place (in -> out).
//
// Each workgroup owns a TY x TZ tile of the y-z plane and streams along x over
// a chunk of XC planes.  Planes of phi (with a y/z halo of H = 2*TB cells)
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
    static constexpr int items(int k) { return (EY - 2 * k) * ((EZ - 2 * k) / 2); }
    static constexpr int ipt(int k) { return (items(k) + NT - 1) / NT; }
    static constexpr int MAXI = (items(1) + NT - 1) / NT;
};

// Compile-time loop: f(std::integral_constant<int, i>) for i in [B, E).
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

template <class G, class T>
__device__ __forceinline__ void load_plane_regs(const T* __restrict__ src, int n, int x, int y0,
                                                int z0, typename Vec2<T>::type* regs)
{
    using V = typename Vec2<T>::type;
    const int msk = n - 1;
    const long xoff = (long)(x & msk) * n;
    // Unconditional, branch-free loads (the tail is clamped to a valid pair):
    // the compiler can then count outstanding loads exactly and wait only
    // for the ones a use needs, instead of draining all of them.
#pragma unroll
    for (int q = 0; q < G::LPT; ++q) {
        int it = min((int)threadIdx.x + q * G::NT, G::PAIRS - 1);
        int r = it / G::NP, cp = it - r * G::NP;
        int y = (y0 - G::H + r) & msk;
        int z = (z0 - G::H + 2 * cp) & msk;  // even: the pair (z, z+1) is contiguous
        regs[q] = *reinterpret_cast<const V*>(src + (xoff + y) * n + z);
    }
}

// Shared-memory footprint of one workgroup, in bytes.
template <class T, class M, int TB, int TY, int TZ>
constexpr int fused_lds_bytes()
{
    using G = FusedGeom<T, TB, TY, TZ, 256>;
    int planes = G::NR * (StageOp<T, M>::kStaged ? 2 : 1);
    return planes * G::PLANE * (int)sizeof(T);
}

template <class T, class M, int TB, int TY, int TZ, int NT, bool SIG>
__global__ __launch_bounds__(NT) void k_sweep_fused(M m, int n, int xc, T ih2,
                                                    const T* __restrict__ in, T* __restrict__ out,
                                                    const T* __restrict__ eta,
                                                    const T* __restrict__ sigma)
{
    using G = FusedGeom<T, TB, TY, TZ, NT>;
    using V = typename Vec2<T>::type;
    constexpr bool STAGED = StageOp<T, M>::kStaged;
    constexpr int NK = 2 * TB;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* ring = reinterpret_cast<T*>(smem_raw);  // NR planes of phi
    T* xring = ring + G::NR * G::PLANE;        // NR planes of e^phi (f(R) only)

    // XCD-aware tile order: ids are dealt round-robin to 8 XCDs; give each
    // XCD a contiguous range of tiles.
    const int nb = gridDim.x;
    int b = blockIdx.x;
    if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
    const int ntz = n / TZ, nty = n / TY;
    const int zt = b % ntz;
    const int yt = (b / ntz) % nty;
    const int xt = b / (ntz * nty);
    const int x0 = xt * xc, y0 = yt * TY, z0 = zt * TZ;
    const int sbeg = x0 - G::H, send = x0 + xc - 1 + G::H;
    const int msk = n - 1;
    const int tid = threadIdx.x;

    auto slot = [&](int p) __attribute__((always_inline)) { return (p - sbeg) % G::NR; };
    auto stage_valid = [&](int p, int k) __attribute__((always_inline)) { return p >= sbeg + k && p <= send - k; };
    // Plane row r, column c of a plane in LDS.  Rows are stored colour-split
    // (even columns, then odd columns): the cells one stage updates have one
    // column parity per row, so consecutive lanes touch consecutive words and
    // the LDS accesses are free of bank conflicts.
    auto lds = [&](int r, int c) __attribute__((always_inline)) {
        return r * G::EZ + (c & 1) * G::HZ + (c >> 1);
    };
    // Row and column of the it-th cell updated by stage k on plane p.
    auto item_rc = [&](int p, int k, int it, int& r, int& c) __attribute__((always_inline)) {
        const int colour = (k - 1) & 1;  // stages 1, 3: red; 2, 4: black
        const int pairs = (G::EZ - 2 * k) / 2;
        const int rr = it / pairs, cp = it - rr * pairs;
        r = k + rr;
        const int par = (p + y0 + z0 + k + colour + r) & 1;
        c = k + 2 * cp + par;
    };

    V pA[G::LPT], pB[G::LPT];
    T eA[NK][G::MAXI], eB[NK][G::MAXI];
    T sA[SIG ? NK : 1][SIG ? G::MAXI : 1], sB[SIG ? NK : 1][SIG ? G::MAXI : 1];

    // Density (and FAS source) of the cells this thread updates at step s.
    // Loaded unconditionally (clamped items, wrapped planes; unused values are
    // discarded) so that the loads carry no branches -- see load_plane_regs.
    auto fetch_cells = [&](int s, T (&e)[NK][G::MAXI], T (&sg)[SIG ? NK : 1][SIG ? G::MAXI : 1]) __attribute__((always_inline)) {
        static_for<0, NK>([&](auto kc) {
            constexpr int k = decltype(kc)::value + 1;
            const int p = s - k;
            const long xoff = (long)(p & msk) * n;
            static_for<0, G::ipt(k)>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                const int it = min(tid + q * NT, G::items(k) - 1);
                int r, c;
                item_rc(p, k, it, r, c);
                const long g = (xoff + ((y0 - G::H + r) & msk)) * n + ((z0 - G::H + c) & msk);
                e[k - 1][q] = eta[g];
                if constexpr (SIG) sg[k - 1][q] = sigma[g];
            });
        });
    };

    auto deposit = [&](int s, const V (&regs)[G::LPT]) __attribute__((always_inline)) {
        T* dst = ring + slot(s) * G::PLANE;
        T* xd = xring + slot(s) * G::PLANE;
#pragma unroll
        for (int q = 0; q < G::LPT; ++q) {
            int it = tid + q * NT;
            if (it < G::PAIRS) {
                int r = it / G::NP, cp = it - r * G::NP;
                const int oe = r * G::EZ + cp;  // column 2cp (even half)
                const int oo = oe + G::HZ;        // column 2cp+1 (odd half)
                dst[oe] = regs[q].x;
                dst[oo] = regs[q].y;
                if constexpr (STAGED) {
                    xd[oe] = StageOp<T, M>::stage(regs[q].x);
                    xd[oo] = StageOp<T, M>::stage(regs[q].y);
                }
            }
        }
    };

    auto stages = [&](int s, const T (&e)[NK][G::MAXI],
                      const T (&sg)[SIG ? NK : 1][SIG ? G::MAXI : 1]) __attribute__((always_inline)) {
        static_for<0, NK>([&](auto kc) {
            constexpr int k = decltype(kc)::value + 1;
            const int p = s - k;
            if (stage_valid(p, k)) {
                T* cur = ring + slot(p) * G::PLANE;
                const T* prv = ring + slot(p - 1) * G::PLANE;
                const T* nxt = ring + slot(p + 1) * G::PLANE;
                T* xcur = xring + slot(p) * G::PLANE;
                const T* xprv = xring + slot(p - 1) * G::PLANE;
                const T* xnxt = xring + slot(p + 1) * G::PLANE;
                static_for<0, G::ipt(k)>([&](auto qc) {
                    constexpr int q = decltype(qc)::value;
                    const int it = tid + q * NT;
                    if (it < G::items(k)) {
                        int r, c;
                        item_rc(p, k, it, r, c);
                        const int o = lds(r, c);
                        const int ozm = lds(r, c - 1), ozp = lds(r, c + 1);
                        T nb[6];
                        nb[0] = prv[o];
                        nb[1] = nxt[o];
                        nb[2] = cur[o - G::EZ];
                        nb[3] = cur[o + G::EZ];
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
                            StageOp<T, M>::eval(m, pc, nb, xcur[o], enb, e[k - 1][q], ih2, L, D);
                        } else {
                            StageOp<T, M>::eval(m, pc, nb, T(0), nullptr, e[k - 1][q], ih2, L, D);
                        }
                        T eps = L;
                        if constexpr (SIG) eps -= sg[k - 1][q];
                        const T nv = pc - eps / D;
                        cur[o] = nv;
                        if constexpr (STAGED) {
                            if (k < NK) xcur[o] = StageOp<T, M>::stage(nv);
                        }
                    }
                });
            }
            __syncthreads();
        });
    };

    auto write_out = [&](int s) __attribute__((always_inline)) {
        const int pw = s - NK;
        if (pw >= x0 && pw < x0 + xc) {
            const T* src = ring + slot(pw) * G::PLANE;
            const long xoff = (long)(pw & msk) * n;
            constexpr int OP = TZ / 2;  // output pairs per row
            for (int it = tid; it < TY * OP; it += NT) {
                const int rr = it / OP, cp = it - rr * OP;
                const int o = lds(G::H + rr, G::H + 2 * cp);  // even column (H is even)
                V v;
                v.x = src[o];
                v.y = src[o + G::HZ];
                *reinterpret_cast<V*>(out + (xoff + y0 + rr) * n + z0 + 2 * cp) = v;
            }
        }
    };

    // One step: planes up to s are in LDS, plane s+1 is in `ready`; `spare`
    // (which held plane s) receives plane s+2.  ec/sc hold this step's cell
    // data, en/sn receive the next step's.
    auto step = [&](int s, V (&spare)[G::LPT], const V (&ready)[G::LPT],
                    const T (&ec)[NK][G::MAXI], const T (&sc)[SIG ? NK : 1][SIG ? G::MAXI : 1],
                    T (&en)[NK][G::MAXI], T (&sn)[SIG ? NK : 1][SIG ? G::MAXI : 1]) __attribute__((always_inline)) {
        // (past the chunk end these load wrapped, unused planes: branch-free)
        load_plane_regs<G, T>(in, n, s + 2, y0, z0, spare);
        fetch_cells(s + 1, en, sn);
        stages(s, ec, sc);  // ends with a barrier: the slot of plane s+1-NR is free
        write_out(s);
        if (s + 1 <= send) deposit(s + 1, ready);
        __syncthreads();
    };

    load_plane_regs<G, T>(in, n, sbeg, y0, z0, pA);
    load_plane_regs<G, T>(in, n, sbeg + 1, y0, z0, pB);
    deposit(sbeg, pA);
    fetch_cells(sbeg, eA, sA);
    __syncthreads();
    for (int s = sbeg; s <= send; s += 2) {
        step(s, pA, pB, eA, sA, eB, sB);
        if (s + 1 <= send) step(s + 1, pB, pA, eB, sB, eA, sA);
    }
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

template <class T, class M, int TB, bool SIG>
int launch_fused_pass(const M& m, int n, double h, const T* in, T* out, const T* eta,
                      const T* sigma, hipStream_t s, char* err)
{
    using Tile = FusedTile<T, M, TB>;
    constexpr int TY = Tile::TY, TZ = Tile::TZ, NT = Tile::NT;
    constexpr int lds = fused_lds_bytes<T, M, TB, TY, TZ>();
    const int xc = fused_chunk(n);
    const int blocks = (n / TZ) * (n / TY) * (n / xc);
    auto kern = k_sweep_fused<T, M, TB, TY, TZ, NT, SIG>;
    static bool attr_done = false;  // per instantiation
    if (!attr_done) {
        if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                lds) != hipSuccess) {
            snprintf(err, 512, "hipFuncSetAttribute(shared %d B) failed", lds);
            return -4;
        }
        attr_done = true;
    }
    T ih2 = (T)(1.0 / (h * h));
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(NT), lds, s, m, n, xc, ih2, in, out, eta, sigma);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        snprintf(err, 512, "k_sweep_fused: %s", hipGetErrorString(e));
        return -4;
    }
    return 0;
}

// `count` sweeps of phi through the fused kernels, ping-ponging between *phi
// and *tmp.  On return *phi points at the buffer holding the result (the two
// pointers are swapped when the number of passes is odd).
template <class T, class M>
int launch_fused_sweeps(const M& m, int n, double h, T** phi, T** tmp, const T* eta,
                        const T* sigma, int count, int tb, hipStream_t s, char* err)
{
    int done = 0;
    while (done < count) {
        const int step = (tb >= 2 && count - done >= 2) ? 2 : 1;
        int r;
        if (step == 2)
            r = sigma ? launch_fused_pass<T, M, 2, true>(m, n, h, *phi, *tmp, eta, sigma, s, err)
                      : launch_fused_pass<T, M, 2, false>(m, n, h, *phi, *tmp, eta, sigma, s, err);
        else
            r = sigma ? launch_fused_pass<T, M, 1, true>(m, n, h, *phi, *tmp, eta, sigma, s, err)
                      : launch_fused_pass<T, M, 1, false>(m, n, h, *phi, *tmp, eta, sigma, s, err);
        if (r) return r;
        T* t = *phi;
        *phi = *tmp;
        *tmp = t;
        done += step;
    }
    return 0;
}

}  // namespace isis
