// Learned warm start: a 3D U-Net in BF16 with FP32 accumulation on MFMA.
//
// The network maps (log density, expansion factor, cold-start field) to the
// correction phi* - phi_cold; its prediction initialises the FAS solve, which
// stays the judge of its error (the caller falls back to the cold start when
// the predicted field's residual is not below the cold start's).
//
// Architecture (4 levels, channels 16/32/64/64, periodic 3x3x3 convolutions,
// ReLU, 2x2x2 average pooling, nearest upsampling, skip concatenation
// [upsampled, skip], 1x1x1 head):
//   enc0 16->16, 16->16 | enc1 pool, 16->32, 32->32 | enc2 pool, 32->64, 64->64
//   bot pool, 64->64, 64->64 | dec2 up+cat 128->64, 64->64
//   dec1 up+cat 96->32, 32->32 | dec0 up+cat 48->16, 16->16 | head 16->1
// Tensors are channels-last [x][y][z][c] in bfloat16 (raw uint16 bits).
// Convolution weights W[t][cout][cin], t = (di+1)*9 + (dj+1)*3 + (dk+1) for
// the input read at (i+di, j+dj, k+dk); the flat FP32 parameter vector holds
// the 14 convolutions (weights then bias) in the order above, then the head.
//
// Convolutions are implicit GEMMs: M = voxels, N = output channels,
// K = 27 * input channels, on v_mfma_f32_16x16x16_bf16.  One wave owns 64
// consecutive voxels along z (four 16-voxel M tiles) and all output channels.
// The data gradient is the same kernel on flipped, transposed weights; the
// weight gradient is a split-K GEMM over voxel chunks with a fixed-order
// reduction of the partial sums (deterministic).  On sides >= 64 the input is
// staged in LDS (k_conv3_lds; k_conv3_ring streams along x for 16 input
// channels), and the prediction's last decoder convolution reads its
// upsampled and skip inputs directly instead of a materialised concatenation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "../../include/isis_mg.h"

namespace {

thread_local char u_err[512];

void uerr(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(u_err, sizeof(u_err), fmt, ap);
    va_end(ap);
}

using bf16_t = uint16_t;
typedef short s4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kMaxGrid = 65536;

int grid_of(long work) { return (int)std::max(1L, std::min((work + kThreads - 1) / kThreads, (long)kMaxGrid)); }

__device__ __forceinline__ float bf2f(bf16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Round to nearest even (NaN kept quiet).
__device__ __forceinline__ bf16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (bf16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}

// ---------------------------------------------------------------------------
// Convolution (forward; also the data gradient with prepared weights).
// ---------------------------------------------------------------------------

// y[v][co] = sum_t sum_ci x[v + d_t][ci] * w[t][co][ci] (+ bias, ReLU).
// Any power-of-two side n >= 2; grid = ceil(n^3 / 256) workgroups of four
// waves, each wave 64 consecutive voxels (four M tiles of 16).  Lanes past the
// last voxel load voxel 0 and store nothing.
template <int CIN, int COUT>
__global__ __launch_bounds__(kThreads) void k_conv3(const bf16_t* __restrict__ x, int n,
                                                    const bf16_t* __restrict__ w,
                                                    const float* __restrict__ bias, int relu,
                                                    bf16_t* __restrict__ y, float* __restrict__ yf)
{
    constexpr int NT = COUT / 16;
    const int lane = threadIdx.x & 63;
    const long wave = (long)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    const long v0 = wave * 64;  // first voxel of this wave
    const long nvox = (long)n * n * n;
    const int msk = n - 1;
    const int m = lane & 15, g = lane >> 4;
    // coordinates of this lane's voxel in each M tile (A operand row m)
    int ci_[4], cj_[4], ck_[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        long v = v0 + 16 * t + m;
        if (v >= nvox) v = 0;
        ck_[t] = (int)(v % n);
        const long r = v / n;
        cj_[t] = (int)(r % n);
        ci_[t] = (int)(r / n);
    }

    f4 acc[4][NT];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < NT; ++u) acc[t][u] = f4{0.f, 0.f, 0.f, 0.f};

    for (int tap = 0; tap < 27; ++tap) {
        const int di = tap / 9 - 1, dj = (tap / 3) % 3 - 1, dk = tap % 3 - 1;
        const bf16_t* wt = w + (long)tap * COUT * CIN;
        long src[4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
            src[t] = ((long)((ci_[t] + di) & msk) * n + ((cj_[t] + dj) & msk)) * n +
                     ((ck_[t] + dk) & msk);
#pragma unroll
        for (int c0 = 0; c0 < CIN; c0 += 16) {
            s4 a[4], b[NT];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                a[t] = *reinterpret_cast<const s4*>(x + src[t] * CIN + c0 + 4 * g);
#pragma unroll
            for (int u = 0; u < NT; ++u)
                b[u] = *reinterpret_cast<const s4*>(wt + (long)(16 * u + m) * CIN + c0 + 4 * g);
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int u = 0; u < NT; ++u)
                    acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[t], b[u], acc[t][u], 0,
                                                                          0, 0);
        }
    }
    // D[row = 4g + r][col = m]: voxel v0 + 16t + 4g + r, channel 16u + m
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            const int co = 16 * u + m;
            const float bb = bias ? bias[co] : 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const long v = v0 + 16 * t + 4 * g + r;
                if (v >= nvox) continue;
                float val = acc[t][u][r] + bb;
                if (relu) val = fmaxf(val, 0.f);
                if (y) y[v * COUT + co] = f2bf(val);
                if (yf) yf[v * COUT + co] = val;
            }
        }
}

// The same convolution with its input staged in LDS (sides n >= 64).  A
// workgroup computes a 4 (y) x 64 (z) tile of one x-plane, one z-row of 64
// voxels per wave (four M tiles of 16).  For each 16-channel slice of the
// input it stages the 3 x 6 x 66 voxels its 27 taps read (38 KB), so every
// input value comes from L2 about 4.6 times per convolution instead of once
// per tap.  LDS holds a slice as two arrays of 16-byte units, one per half
// of 8 channels ([half][plane][row][z]), read by the 16x16x32 BF16 MFMA two
// taps at a time: lane g = lane / 16 takes channel half g & 1 of tap 2p + (g
// >> 1), so the 16 lanes of one (half, tap) group read 256 contiguous bytes
// (a voxel-major layout put lanes m, m+4, m+8, m+12 on one bank).  The 27th
// tap is a 14th pair whose second half is zero, so every product runs on the
// 16x16x32 MFMA.  Tiles are dealt to the 8 XCDs in contiguous ranges with x
// fastest, so neighbouring planes share an L2.
constexpr int kLY = 4, kLZ = 64;                   // output tile (y, z)
constexpr int kLPY = kLY + 2, kLPZ = kLZ + 2;      // with the halo
constexpr int kLVox = 3 * kLPY * kLPZ;             // staged voxels per slice

//
// CLO > 0: the input is the concatenation [nearest upsampling of lo, x] of a
// coarse [(n/2)^3][CLO] tensor and a fine [n^3][CIN - CLO] tensor (the
// decoder's skip), read directly instead of materialised.
template <int CIN, int COUT, int CLO = 0>
__global__ __launch_bounds__(kThreads) void k_conv3_lds(const bf16_t* __restrict__ x, int n,
                                                        const bf16_t* __restrict__ w,
                                                        const float* __restrict__ bias, int relu,
                                                        bf16_t* __restrict__ y,
                                                        float* __restrict__ yf,
                                                        const bf16_t* __restrict__ lo = nullptr)
{
    static_assert(CIN % 16 == 0 && COUT % 16 == 0 && CLO % 16 == 0 && CLO < CIN,
                  "whole 16-channel slices");
    constexpr int NT = COUT / 16;
    __shared__ uint4 tile[2 * kLVox];  // [8-channel half][plane][row][z]
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = lane & 15, g = lane >> 4;
    const int msk = n - 1, nyt = n / kLY;
    const int nb = gridDim.x;
    int b = blockIdx.x;
    if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
    const int x0 = b % n, yt = (b / n) % nyt, zt = b / (n * nyt);
    const int y0 = yt * kLY, z0 = zt * kLZ;

    f4 acc[4][NT];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < NT; ++u) acc[t][u] = f4{0.f, 0.f, 0.f, 0.f};

    // k of the 16x16x32 MFMA = two taps of one slice: lanes g = 0, 1 carry
    // channels 8g..8g+7 of tap 2p, lanes g = 2, 3 those of tap 2p + 1.  The
    // 27th tap is the 14th pair with zeros in the second half: every product
    // runs on the one MFMA shape.  (Mixing in the 16x16x16 MFMA for the 27th
    // tap measured wrong sums for the 32 -> 16 instantiation, whose schedule
    // interleaves the two shapes on renamed accumulators.)
    const int hh = g & 1, side = g >> 1;
    const uint4* th = tile + hh * kLVox;  // this lane's 8-channel half
    for (int c0 = 0; c0 < CIN; c0 += 16) {
        if (c0) __syncthreads();  // the previous slice has been consumed
        for (int e = tid; e < kLVox * 2; e += kThreads) {
            const int vox = e >> 1, h = e & 1;
            const int zz = vox % kLPZ, rr = (vox / kLPZ) % kLPY, pp = vox / (kLPZ * kLPY);
            const int xf = (x0 - 1 + pp) & msk, yf_ = (y0 - 1 + rr) & msk, zf = (z0 - 1 + zz) & msk;
            const bf16_t* src;
            if constexpr (CLO > 0) {
                if (c0 < CLO) {
                    const int nc = n >> 1;
                    const long V = ((long)(xf >> 1) * nc + (yf_ >> 1)) * nc + (zf >> 1);
                    src = lo + V * CLO + c0 + 8 * h;
                } else {
                    src = x + (((long)xf * n + yf_) * n + zf) * (CIN - CLO) + (c0 - CLO) + 8 * h;
                }
            } else {
                src = x + (((long)xf * n + yf_) * n + zf) * CIN + c0 + 8 * h;
            }
            tile[h * kLVox + vox] = *reinterpret_cast<const uint4*>(src);
        }
        __syncthreads();
#pragma unroll
        for (int pr = 0; pr < 14; ++pr) {
            // pair 13: taps 26 and (nonexistent) 27; lanes of the second half
            // read tap 26's (valid) addresses and zero what they loaded
            const bool live = pr < 13 || side == 0;
            const int tap = live ? 2 * pr + side : 26;
            const int off = ((tap / 9) * kLPY + wv + (tap / 3) % 3) * kLPZ + m + tap % 3;
            const bf16_t* wt = w + (long)tap * COUT * CIN;
            bf8v bw[NT];
#pragma unroll
            for (int u = 0; u < NT; ++u) {
                bw[u] = *reinterpret_cast<const bf8v*>(wt + (long)(16 * u + m) * CIN + c0 + 8 * hh);
                if (!live) bw[u] = bf8v{};
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                bf8v a = *reinterpret_cast<const bf8v*>(th + off + 16 * t);
                if (!live) a = bf8v{};
#pragma unroll
                for (int u = 0; u < NT; ++u)
                    acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[u], acc[t][u], 0, 0, 0);
            }
        }
    }
    // D[row = 4g + r][col = m]: voxel z0 + 16t + 4g + r of row y0 + wv, channel 16u + m
    const long v0 = ((long)x0 * n + (y0 + wv)) * n + z0;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            const int co = 16 * u + m;
            const float bb = bias ? bias[co] : 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const long v = v0 + 16 * t + 4 * g + r;
                float val = acc[t][u][r] + bb;
                if (relu) val = fmaxf(val, 0.f);
                if (y) y[v * COUT + co] = f2bf(val);
                if (yf) yf[v * COUT + co] = val;
            }
        }
}

// 16 input channels (sides n >= 64): the 4 x 64 tile streams along x over
// xc planes through a ring of three staged planes (6 x 66 voxels, 32 B
// each), so each output plane stages one new input plane instead of three;
// the next plane is loaded into registers while the current one is computed.
template <int COUT>
__global__ __launch_bounds__(kThreads) void k_conv3_ring(const bf16_t* __restrict__ x, int n,
                                                         int xc, const bf16_t* __restrict__ w,
                                                         const float* __restrict__ bias, int relu,
                                                         bf16_t* __restrict__ y,
                                                         float* __restrict__ yf)
{
    constexpr int CIN = 16, NT = COUT / 16;
    constexpr int PVOX = kLPY * kLPZ;                   // voxels per staged plane
    constexpr int PV = PVOX * 2;                        // 16-byte input vectors per plane
    constexpr int PER = (PV + kThreads - 1) / kThreads;  // of them per thread
    __shared__ uint2 ring[3 * 4 * PVOX];  // [slot][4-channel group][row][z] (see k_conv3_lds)
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = lane & 15, g = lane >> 4;
    const int msk = n - 1, nyt = n / kLY, nzt = n / kLZ;
    const int nb = gridDim.x;
    int b = blockIdx.x;
    if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
    const int yt = b % nyt, zt = (b / nyt) % nzt, xq = b / (nyt * nzt);
    const int y0 = yt * kLY, z0 = zt * kLZ, x0 = xq * xc;
    const size_t plane = (size_t)n * n * CIN;
    // in-plane element offsets of this thread's vectors (tail clamped; its
    // stores are skipped)
    unsigned poff[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = min(tid + q * kThreads, PV - 1);
        const int vox = e >> 1, h = e & 1;
        const int zz = vox % kLPZ, rr = vox / kLPZ;
        poff[q] = (unsigned)((((y0 - 1 + rr) & msk) * n + ((z0 - 1 + zz) & msk)) * CIN + 8 * h);
    }
    uint4 pre[PER];
    auto load = [&](int xp) __attribute__((always_inline)) {
        const bf16_t* pl = x + (size_t)(xp & msk) * plane;
#pragma unroll
        for (int q = 0; q < PER; ++q) pre[q] = *reinterpret_cast<const uint4*>(pl + poff[q]);
    };
    auto put = [&](int xp) __attribute__((always_inline)) {
        uint2* dst = ring + ((xp - x0 + 1) % 3) * 4 * PVOX;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * kThreads;
            if ((q + 1) * kThreads <= PV || e < PV) {
                const int vox = e >> 1, h = e & 1;
                dst[(2 * h) * PVOX + vox] = uint2{pre[q].x, pre[q].y};
                dst[(2 * h + 1) * PVOX + vox] = uint2{pre[q].z, pre[q].w};
            }
        }
    };
    load(x0 - 1);
    put(x0 - 1);
    load(x0);
    put(x0);
    load(x0 + 1);
    for (int xi = x0; xi < x0 + xc; ++xi) {
        put(xi + 1);  // into the slot of plane xi - 2, free since the last barrier
        __syncthreads();
        if (xi + 2 <= x0 + xc) load(xi + 2);  // in flight during this plane's taps
        f4 acc[4][NT];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int u = 0; u < NT; ++u) acc[t][u] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int tap = 0; tap < 27; ++tap) {
            const int pi = tap / 9, rj = (tap / 3) % 3, zk = tap % 3;
            const bf16_t* wt = w + (long)tap * COUT * CIN;
            s4 bw[NT];
#pragma unroll
            for (int u = 0; u < NT; ++u)
                bw[u] = *reinterpret_cast<const s4*>(wt + (16 * u + m) * CIN + 4 * g);
            const int slot = (xi - 1 + pi - x0 + 1) % 3;
            const uint2* tg = ring + (slot * 4 + g) * PVOX;  // this lane's k-group
            const int base = (wv + rj) * kLPZ + m + zk;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const s4 a = *reinterpret_cast<const s4*>(tg + base + 16 * t);
#pragma unroll
                for (int u = 0; u < NT; ++u)
                    acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bw[u], acc[t][u], 0,
                                                                          0, 0);
            }
        }
        const long v0 = ((long)xi * n + (y0 + wv)) * n + z0;
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int u = 0; u < NT; ++u) {
                const int co = 16 * u + m;
                const float bb = bias ? bias[co] : 0.f;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const long v = v0 + 16 * t + 4 * g + r;
                    float val = acc[t][u][r] + bb;
                    if (relu) val = fmaxf(val, 0.f);
                    if (y) y[v * COUT + co] = f2bf(val);
                    if (yf) yf[v * COUT + co] = val;
                }
            }
        __syncthreads();  // the slot of plane xi - 1 is free for the next put
    }
}

// dW partials: part[chunk][t][co][ci] = sum over the chunk's voxels v of
// dy[v][co] * x[v + d_t][ci].  One workgroup per (tap, chunk); its waves
// split the 16x16 output tiles.  K (voxels) advances 16 at a time.
template <int CIN, int COUT>
__global__ __launch_bounds__(kThreads) void k_conv3_dw(const bf16_t* __restrict__ x, int n,
                                                       const bf16_t* __restrict__ dy,
                                                       int chunk, float* __restrict__ part)
{
    constexpr int TM = COUT / 16, TN = CIN / 16, TILES = TM * TN;
    constexpr int WAVES = kThreads / 64;
    constexpr int TPW = (TILES + WAVES - 1) / WAVES;  // tiles per wave
    const int tap = blockIdx.x % 27;
    const int ch = blockIdx.x / 27;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, g = lane >> 4;
    const int di = tap / 9 - 1, dj = (tap / 3) % 3 - 1, dk = tap % 3 - 1;
    const int msk = n - 1;
    const long vbeg = (long)ch * chunk, vend = vbeg + chunk;

    f4 acc[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};

    for (long vb = vbeg; vb < vend; vb += 16) {
        // K index k = 4g + r  ->  voxel vb + 4g + r
        long vx[4], vy[4];
        bool live[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            long v = vb + 4 * g + r;
            live[r] = v < vend;  // chunks shorter than 16 voxels (tiny grids)
            if (!live[r]) v = vbeg;
            vy[r] = v;
            const int kk = (int)(v % n);
            const long rw = v / n;
            const int jj = (int)(rw % n), ii = (int)(rw / n);
            vx[r] = ((long)((ii + di) & msk) * n + ((jj + dj) & msk)) * n + ((kk + dk) & msk);
        }
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            const int tile = wave + q * WAVES;
            if (tile < TILES) {
                const int tm = tile / TN, tn = tile % TN;
                s4 a, b;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    a[r] = live[r] ? (short)dy[vy[r] * COUT + 16 * tm + m] : (short)0;  // A[co][v]
                    b[r] = (short)x[vx[r] * CIN + 16 * tn + m];                          // B[v][ci]
                }
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[q], 0, 0, 0);
            }
        }
    }
    float* out = part + ((long)ch * 27 + tap) * COUT * CIN;
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        const int tile = wave + q * WAVES;
        if (tile < TILES) {
            const int tm = tile / TN, tn = tile % TN;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                out[(long)(16 * tm + 4 * g + r) * CIN + 16 * tn + m] = acc[q][r];
        }
    }
}

// out[e] = sum_c part[c][e] in chunk order (deterministic), optionally added.
__global__ __launch_bounds__(kThreads) void k_sum_chunks(const float* __restrict__ part,
                                                         int nchunk, long elems,
                                                         float* __restrict__ out)
{
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < elems;
         e += (long)gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int c = 0; c < nchunk; ++c) s += part[(long)c * elems + e];
        out[e] = s;
    }
}

// Per-channel sums of a [nvox][C] bf16 tensor: partial sums per block of
// voxels (fixed chunking), reduced by k_sum_chunks.
__global__ __launch_bounds__(kThreads) void k_chan_sum(const bf16_t* __restrict__ a, long nvox,
                                                       int C, int chunk, float* __restrict__ part)
{
    // block b handles voxels [b*chunk, (b+1)*chunk); thread t sums channel t
    const long v0 = (long)blockIdx.x * chunk;
    for (int c = threadIdx.x; c < C; c += blockDim.x) {
        float s = 0.f;
        for (long v = v0; v < v0 + chunk && v < nvox; ++v) s += bf2f(a[v * C + c]);
        part[(long)blockIdx.x * C + c] = s;
    }
}

// Weights for the data gradient: wt[t'][ci][co] = w[26 - t][co][ci] (bf16).
__global__ void k_flip_weights(const float* __restrict__ w, int cin, int cout,
                               bf16_t* __restrict__ wt)
{
    const long total = 27L * cin * cout;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const int co = (int)(e % cout);
        const long r = e / cout;
        const int ci = (int)(r % cin);
        const int tp = (int)(r / cin);
        wt[e] = f2bf(w[((long)(26 - tp) * cout + co) * cin + ci]);
    }
}

__global__ void k_to_bf16(const float* __restrict__ src, long total, bf16_t* __restrict__ dst)
{
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x)
        dst[e] = f2bf(src[e]);
}

// ---------------------------------------------------------------------------
// Pooling, upsampling, concatenation, masks, head, loss, Adam.
// ---------------------------------------------------------------------------

// y[V][c] = mean of the 8 children (reading channels [c0, c0+C) of a tensor
// with channel stride cs); nf = fine side (a power of two).  One 16-byte
// vector of 8 channels per thread (C, cs, c0 multiples of 8, C / 8 a power
// of two).
__global__ void k_pool2(const bf16_t* __restrict__ x, int nf, int cs, int c0, int C,
                        bf16_t* __restrict__ y)
{
    const int nc = nf / 2, lc = __builtin_ctz(nc), lq = __builtin_ctz(C / 8);
    const long total = ((long)nc * nc * nc) << lq;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const int q = (int)(e & ((C / 8) - 1));
        const long V = e >> lq;
        const int K = (int)(V & (nc - 1)), J = (int)((V >> lc) & (nc - 1)), I = (int)(V >> (2 * lc));
        float sum[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int d = 0; d < 2; ++d) {
                    const long vf = ((long)(2 * I + a) * nf + (2 * J + b)) * nf + (2 * K + d);
                    const uint4 u = *reinterpret_cast<const uint4*>(x + vf * cs + c0 + 8 * q);
                    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        sum[2 * i] += bf2f((bf16_t)(w[i] & 0xffffu));
                        sum[2 * i + 1] += bf2f((bf16_t)(w[i] >> 16));
                    }
                }
        uint32_t o[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            o[i] = (uint32_t)f2bf(sum[2 * i] * 0.125f) | ((uint32_t)f2bf(sum[2 * i + 1] * 0.125f) << 16);
        reinterpret_cast<uint4*>(y)[e] = uint4{o[0], o[1], o[2], o[3]};
    }
}

// Nearest upsampling of a [nc^3][C] tensor into channels [0, C) of a
// [(2nc)^3][C+S] tensor, and copy of skip [(2nc)^3][S] into channels
// [C, C+S).  One 16-byte vector of 8 output channels per thread, so a wave
// writes 1 KiB of contiguous output (C and S are multiples of 8, the tensors
// 256-byte aligned); coordinates by shifts (the side is a power of two).
template <int C, int S>
__global__ void k_up2_cat(const bf16_t* __restrict__ lo, int nc, const bf16_t* __restrict__ skip,
                          bf16_t* __restrict__ out)
{
    static_assert(C % 8 == 0 && S % 8 == 0, "channels in whole 16-byte vectors");
    constexpr int VC = C / 8, VS = S / 8, VT = VC + VS;
    const int nf = 2 * nc, lf = __builtin_ctz(nf);
    const long total = (long)nf * nf * nf * VT;
    const uint4* lov = reinterpret_cast<const uint4*>(lo);
    const uint4* skv = reinterpret_cast<const uint4*>(skip);
    uint4* outv = reinterpret_cast<uint4*>(out);
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const long v = e / VT;
        const int q = (int)(e - v * VT);
        if (q < VC) {
            const int k = (int)(v & (nf - 1)), j = (int)((v >> lf) & (nf - 1));
            const int i = (int)(v >> (2 * lf));
            const long V = ((long)(i >> 1) * nc + (j >> 1)) * nc + (k >> 1);
            outv[e] = lov[V * VC + q];
        } else {
            outv[e] = skv[v * VS + (q - VC)];
        }
    }
}

// Gradient through upsampling: y[V][c] = sum of the 8 children's
// dcat[v][c] (channels [0, C) of the concat gradient, stride cs).
__global__ void k_up2_bwd(const bf16_t* __restrict__ dcat, int nf, int cs, int C,
                          bf16_t* __restrict__ y)
{
    const int nc = nf / 2;
    const long total = (long)nc * nc * nc * C;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const int c = (int)(e % C);
        const long V = e / C;
        const int K = (int)(V % nc);
        const long r = V / nc;
        const int J = (int)(r % nc), I = (int)(r / nc);
        float s = 0.f;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int d = 0; d < 2; ++d) {
                    const long vf = ((long)(2 * I + a) * nf + (2 * J + b)) * nf + (2 * K + d);
                    s += bf2f(dcat[vf * cs + c]);
                }
        y[e] = f2bf(s);
    }
}

// Gradient into a skip tensor: out[v][c] = bf16(dcat[v][C + c] + bf16(dlo[V][c] / 8))
// where dlo is the gradient at the pooled (coarse) level.
__global__ void k_skip_grad(const bf16_t* __restrict__ dcat, int nf, int cs, int C, int S,
                            const bf16_t* __restrict__ dlo, bf16_t* __restrict__ out)
{
    const int nc = nf / 2;
    const long total = (long)nf * nf * nf * S;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const int c = (int)(e % S);
        const long v = e / S;
        const int k = (int)(v % nf);
        const long r = v / nf;
        const int j = (int)(r % nf), i = (int)(r / nf);
        const long V = ((long)(i / 2) * nc + j / 2) * nc + k / 2;
        const float pb = bf2f(f2bf(bf2f(dlo[V * S + c]) * 0.125f));
        out[e] = f2bf(bf2f(dcat[v * cs + C + c]) + pb);
    }
}

// g = g * (o > 0) (ReLU gradient; exact in bf16).
__global__ void k_relu_mask(bf16_t* __restrict__ g, const bf16_t* __restrict__ o, long total)
{
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x)
        if (!(bf2f(o[e]) > 0.f)) g[e] = 0;
}

// Input channels: log(eta)/2, a, phi_cold, zeros (16 channels).
__global__ void k_make_input(const double* __restrict__ eta, const double* __restrict__ cold,
                             double a, long nvox, bf16_t* __restrict__ x)
{
    for (long v = (long)blockIdx.x * blockDim.x + threadIdx.x; v < nvox;
         v += (long)gridDim.x * blockDim.x) {
        // channels 0, 1, 2 = log(eta)/2, a, cold; 3..15 zero (two 16-byte stores)
        uint4* o = reinterpret_cast<uint4*>(x + v * 16);
        const uint32_t c01 = (uint32_t)f2bf((float)(log(eta[v]) * 0.5)) |
                             ((uint32_t)f2bf((float)a) << 16);
        o[0] = uint4{c01, (uint32_t)f2bf((float)cold[v]), 0u, 0u};
        o[1] = uint4{0u, 0u, 0u, 0u};
    }
}

// out[v] = sum_c d[v][c] wh[c] + bh (fp32); guess[v] = cold[v] + out[v] if
// guess != NULL.
__global__ void k_head(const bf16_t* __restrict__ d, const float* __restrict__ wh, long nvox,
                       float* __restrict__ out, const double* __restrict__ cold,
                       double* __restrict__ guess)
{
    for (long v = (long)blockIdx.x * blockDim.x + threadIdx.x; v < nvox;
         v += (long)gridDim.x * blockDim.x) {
        const uint4* dv = reinterpret_cast<const uint4*>(d + v * 16);
        const uint4 u0 = dv[0], u1 = dv[1];
        const uint32_t w[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
        float s = wh[16];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            s += bf2f((bf16_t)(w[i] & 0xffffu)) * wh[2 * i];
            s += bf2f((bf16_t)(w[i] >> 16)) * wh[2 * i + 1];
        }
        if (out) out[v] = s;
        if (guess) guess[v] = cold[v] + (double)s;
    }
}

// Loss pieces: dout[v] = 2 (out - target) / nvox; per-block partials of
// (out - target)^2 and of dout and of dout * d[v][c] (head gradient).
__global__ __launch_bounds__(kThreads) void k_head_bwd(const float* __restrict__ out,
                                                       const double* __restrict__ phi_t,
                                                       const double* __restrict__ cold,
                                                       const bf16_t* __restrict__ d,
                                                       const float* __restrict__ wh, long nvox,
                                                       int chunk, float* __restrict__ part,
                                                       bf16_t* __restrict__ dh)
{
    // part[b][0..15] = sum dout*d[:,c], part[b][16] = sum dout, part[b][17] = sum err^2
    __shared__ float red[kThreads][18];
    float acc[18];
    for (int q = 0; q < 18; ++q) acc[q] = 0.f;
    const long v0 = (long)blockIdx.x * chunk;
    const float scale = 2.0f / (float)nvox;
    for (long v = v0 + threadIdx.x; v < v0 + chunk && v < nvox; v += blockDim.x) {
        const float err = out[v] - (float)(phi_t[v] - cold[v]);
        const float go = scale * err;
        for (int c = 0; c < 16; ++c) {
            acc[c] += go * bf2f(d[v * 16 + c]);
            dh[v * 16 + c] = f2bf(go * wh[c]);
        }
        acc[16] += go;
        acc[17] += err * err;
    }
    for (int q = 0; q < 18; ++q) red[threadIdx.x][q] = acc[q];
    __syncthreads();
    if (threadIdx.x < 18) {
        float s = 0.f;
        for (int t = 0; t < blockDim.x; ++t) s += red[t][threadIdx.x];
        part[(long)blockIdx.x * 18 + threadIdx.x] = s;
    }
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long total, float lr, float b1, float b2, float eps,
                       float c1, float c2)
{
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const float gg = g[e];
        const float mm = b1 * m[e] + (1.f - b1) * gg;
        const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
        m[e] = mm;
        v[e] = vv;
        p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------

struct ConvSpec {
    int cin, cout;
};
constexpr ConvSpec kConvs[14] = {{16, 16},  {16, 16}, {16, 32}, {32, 32}, {32, 64},
                                 {64, 64},  {64, 64}, {64, 64}, {128, 64}, {64, 64},
                                 {96, 32},  {32, 32}, {48, 16}, {16, 16}};
constexpr int kHeadIn = 16;

long param_offset(int layer)
{
    long off = 0;
    for (int l = 0; l < layer; ++l) off += 27L * kConvs[l].cin * kConvs[l].cout + kConvs[l].cout;
    return off;
}
long param_total() { return param_offset(14) + kHeadIn + 1; }

#define UCHECK(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            uerr("%s: %s", #call, hipGetErrorString(e_));                             \
            return ISIS_ERR_HIP;                                                      \
        }                                                                             \
    } while (0)
#define ULAUNCH(name)                                                                 \
    do {                                                                              \
        hipError_t e_ = hipGetLastError();                                            \
        if (e_ != hipSuccess) {                                                       \
            uerr("%s: %s", name, hipGetErrorString(e_));                              \
            return ISIS_ERR_HIP;                                                      \
        }                                                                             \
    } while (0)

int launch_conv(const bf16_t* x, int n, int cin, const bf16_t* w, const float* bias, int cout,
                int relu, bf16_t* y, float* yf, hipStream_t s)
{
    const long nvox = (long)n * n * n;
    const int blocks = (int)((nvox + 255) / 256);
    // sides >= 64 (powers of two): the LDS-staged kernel, one workgroup per
    // 4 x 64 tile of an x-plane
    const bool lds = n >= kLZ;
    const long lblocks = (long)n * (n / kLY) * (n / kLZ);
    // 16 input channels: planes per workgroup for the ring kernel, a power of
    // two up to 16 that leaves >= 2048 workgroups
    const long tiles2d = (long)(n / kLY) * (n / kLZ);
    int xc = 1;
    while (xc < 16 && tiles2d * (n / (2 * xc)) >= 2048) xc *= 2;
#define CONV_CASE(CI, CO)                                                                   \
    if (cin == CI && cout == CO) {                                                          \
        if (lds && CI == 16)                                                                \
            hipLaunchKernelGGL((k_conv3_ring<CO>), dim3((unsigned)(tiles2d * (n / xc))),     \
                               dim3(kThreads), 0, s, x, n, xc, w, bias, relu, y, yf);       \
        else if (lds)                                                                       \
            hipLaunchKernelGGL((k_conv3_lds<CI, CO>), dim3((unsigned)lblocks), dim3(kThreads), \
                               0, s, x, n, w, bias, relu, y, yf);                           \
        else                                                                                \
            hipLaunchKernelGGL((k_conv3<CI, CO>), dim3(blocks), dim3(kThreads), 0, s, x, n, \
                               w, bias, relu, y, yf);                                       \
        ULAUNCH("k_conv3");                                                                 \
        return ISIS_OK;                                                                     \
    }
    CONV_CASE(16, 16) CONV_CASE(16, 32) CONV_CASE(32, 32) CONV_CASE(32, 64) CONV_CASE(64, 64)
    CONV_CASE(128, 64) CONV_CASE(96, 32) CONV_CASE(48, 16)
    // data-gradient shapes (channels swapped)
    CONV_CASE(32, 16) CONV_CASE(64, 32) CONV_CASE(64, 128) CONV_CASE(32, 96) CONV_CASE(16, 48)
#undef CONV_CASE
    uerr("no convolution kernel for %d -> %d channels", cin, cout);
    return ISIS_ERR_UNSUPPORTED;
}

// Convolution of [nearest upsampling of lo (n/2)^3 x clo, skip n^3 x (cin -
// clo)] without materialising the concatenation (sides n >= 64).
int launch_conv_cat(const bf16_t* lo, const bf16_t* skip, int n, int cin, int clo,
                    const bf16_t* w, const float* bias, int cout, int relu, bf16_t* y,
                    hipStream_t s)
{
    if (n < kLZ || !(cin == 48 && clo == 32 && cout == 16)) {
        uerr("no fused decoder convolution for %d (%d upsampled) -> %d channels at side %d", cin,
             clo, cout, n);
        return ISIS_ERR_UNSUPPORTED;
    }
    const long lblocks = (long)n * (n / kLY) * (n / kLZ);
    hipLaunchKernelGGL((k_conv3_lds<48, 16, 32>), dim3((unsigned)lblocks), dim3(kThreads), 0, s,
                       skip, n, w, bias, relu, y, nullptr, lo);
    ULAUNCH("k_conv3_lds (concatenated input)");
    return ISIS_OK;
}

int dw_chunk(long nvox) { return (int)std::min<long>(nvox, 4096); }

size_t dw_part_floats(long nvox, int cin, int cout)
{
    return (size_t)(nvox / dw_chunk(nvox)) * 27 * cin * cout;
}

int launch_conv_dw(const bf16_t* x, int n, int cin, const bf16_t* dy, int cout, float* part,
                   float* dw, hipStream_t s)
{
    const long nvox = (long)n * n * n;
    const int chunk = dw_chunk(nvox);
    const int nchunk = (int)(nvox / chunk);
    bool ok = false;
#define DW_CASE(CI, CO)                                                                     \
    if (cin == CI && cout == CO) {                                                          \
        hipLaunchKernelGGL((k_conv3_dw<CI, CO>), dim3(27 * nchunk), dim3(kThreads), 0, s, x, \
                           n, dy, chunk, part);                                             \
        ok = true;                                                                          \
    }
    DW_CASE(16, 16) DW_CASE(16, 32) DW_CASE(32, 32) DW_CASE(32, 64) DW_CASE(64, 64)
    DW_CASE(128, 64) DW_CASE(96, 32) DW_CASE(48, 16)
#undef DW_CASE
    if (!ok) {
        uerr("no weight-gradient kernel for %d -> %d channels", cin, cout);
        return ISIS_ERR_UNSUPPORTED;
    }
    ULAUNCH("k_conv3_dw");
    const long elems = 27L * cin * cout;
    hipLaunchKernelGGL(k_sum_chunks, dim3(grid_of(elems)), dim3(kThreads), 0, s, part, nchunk,
                       elems, dw);
    ULAUNCH("k_sum_chunks");
    return ISIS_OK;
}

int launch_chan_sum(const bf16_t* a, long nvox, int C, float* part, float* out, hipStream_t s)
{
    const int chunk = 4096;
    const int nb = (int)((nvox + chunk - 1) / chunk);
    hipLaunchKernelGGL(k_chan_sum, dim3(nb), dim3(kThreads), 0, s, a, nvox, C, chunk, part);
    ULAUNCH("k_chan_sum");
    hipLaunchKernelGGL(k_sum_chunks, dim3(1), dim3(kThreads), 0, s, part, nb, (long)C, out);
    ULAUNCH("k_sum_chunks");
    return ISIS_OK;
}


// ---------------------------------------------------------------------------
// The network: workspace plan, forward, backward.
// ---------------------------------------------------------------------------

int level_of(int layer)
{
    static const int lv[14] = {0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0};
    return lv[layer];
}

struct Plan {
    int n[4];
    long nv[4];
    bf16_t *in, *o[14], *p1, *p2, *p3, *c8, *c10, *c12;  // forward tensors
    float* out;                                            // head output (fp32)
    bf16_t* wf[14];                                        // bf16 weights
    // training only
    bf16_t *ga, *gb;            // ping-pong gradients (largest: nv0 x 16)
    bf16_t *gc8, *gc10, *gc12;  // gradients of the concatenations (kept for the skips)
    bf16_t* wb[14];             // flipped, transposed bf16 weights (data gradient)
    float *part, *grad, *hpart, *hsum, *loss;
    size_t bytes;
};

Plan make_plan(int n, int training, char* base)
{
    Plan P;
    memset(&P, 0, sizeof(P));
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        off = (off + 255) & ~(size_t)255;
        char* p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    for (int l = 0; l < 4; ++l) {
        P.n[l] = n >> l;
        P.nv[l] = (long)P.n[l] * P.n[l] * P.n[l];
    }
    P.in = (bf16_t*)take(P.nv[0] * 16 * 2);
    for (int c = 0; c < 14; ++c) P.o[c] = (bf16_t*)take(P.nv[level_of(c)] * kConvs[c].cout * 2);
    P.p1 = (bf16_t*)take(P.nv[1] * 16 * 2);
    P.p2 = (bf16_t*)take(P.nv[2] * 32 * 2);
    P.p3 = (bf16_t*)take(P.nv[3] * 64 * 2);
    P.c8 = (bf16_t*)take(P.nv[2] * 128 * 2);
    P.c10 = (bf16_t*)take(P.nv[1] * 96 * 2);
    P.c12 = (bf16_t*)take(P.nv[0] * 48 * 2);
    P.out = (float*)take(P.nv[0] * 4);
    for (int c = 0; c < 14; ++c) P.wf[c] = (bf16_t*)take(27L * kConvs[c].cin * kConvs[c].cout * 2);
    if (training) {
        P.ga = (bf16_t*)take(P.nv[0] * 16 * 2);
        P.gb = (bf16_t*)take(P.nv[0] * 16 * 2);
        P.gc8 = (bf16_t*)take(P.nv[2] * 128 * 2);
        P.gc10 = (bf16_t*)take(P.nv[1] * 96 * 2);
        P.gc12 = (bf16_t*)take(P.nv[0] * 48 * 2);
        for (int c = 0; c < 14; ++c)
            P.wb[c] = (bf16_t*)take(27L * kConvs[c].cin * kConvs[c].cout * 2);
        size_t part = 0;
        for (int c = 0; c < 14; ++c)
            part = std::max(part, dw_part_floats(P.nv[level_of(c)], kConvs[c].cin, kConvs[c].cout));
        for (int l = 0; l < 4; ++l) part = std::max(part, (size_t)((P.nv[l] + 4095) / 4096) * 128);
        P.part = (float*)take(part * 4);
        P.grad = (float*)take(param_total() * 4);
        P.hpart = (float*)take((size_t)((P.nv[0] + 4095) / 4096) * 18 * 4);
        P.hsum = (float*)take(18 * 4);
        P.loss = (float*)take(4);
    }
    P.bytes = off + 256;
    return P;
}

#define TRY(x)                       \
    do {                             \
        int r_ = (x);                \
        if (r_ != ISIS_OK) return r_; \
    } while (0)

// fuse_cat: the last decoder stage reads its upsampled and skip inputs
// directly (prediction; training keeps the concatenation for the weight
// gradient).
int run_forward(const Plan& P, const float* params, hipStream_t s, bool fuse_cat = false)
{
    for (int c = 0; c < 14; ++c) {
        const long e = 27L * kConvs[c].cin * kConvs[c].cout;
        hipLaunchKernelGGL(k_to_bf16, dim3(grid_of(e)), dim3(kThreads), 0, s,
                           params + param_offset(c), e, P.wf[c]);
        ULAUNCH("k_to_bf16");
    }
    auto conv = [&](int c, const bf16_t* x) -> int {
        const int lv = level_of(c);
        return launch_conv(x, P.n[lv], kConvs[c].cin, P.wf[c],
                           params + param_offset(c) + 27L * kConvs[c].cin * kConvs[c].cout,
                           kConvs[c].cout, 1, P.o[c], nullptr, s);
    };
    auto pool = [&](const bf16_t* x, int lvf, int C, bf16_t* y) -> int {
        hipLaunchKernelGGL(k_pool2, dim3(grid_of(P.nv[lvf + 1] * C / 8)), dim3(kThreads), 0, s, x,
                           P.n[lvf], C, 0, C, y);
        ULAUNCH("k_pool2");
        return (int)ISIS_OK;
    };
    auto upcat = [&](const bf16_t* lo, int lvc, int C, const bf16_t* skip, int S, bf16_t* out) -> int {
        const dim3 g(grid_of(P.nv[lvc - 1] * (C + S) / 8));
        if (C == 64 && S == 64)
            hipLaunchKernelGGL((k_up2_cat<64, 64>), g, dim3(kThreads), 0, s, lo, P.n[lvc], skip, out);
        else if (C == 64 && S == 32)
            hipLaunchKernelGGL((k_up2_cat<64, 32>), g, dim3(kThreads), 0, s, lo, P.n[lvc], skip, out);
        else if (C == 32 && S == 16)
            hipLaunchKernelGGL((k_up2_cat<32, 16>), g, dim3(kThreads), 0, s, lo, P.n[lvc], skip, out);
        else {
            uerr("k_up2_cat: no instance for %d + %d channels", C, S);
            return (int)ISIS_ERR_INVALID_ARG;
        }
        ULAUNCH("k_up2_cat");
        return (int)ISIS_OK;
    };
    TRY(conv(0, P.in));
    TRY(conv(1, P.o[0]));
    TRY(pool(P.o[1], 0, 16, P.p1));
    TRY(conv(2, P.p1));
    TRY(conv(3, P.o[2]));
    TRY(pool(P.o[3], 1, 32, P.p2));
    TRY(conv(4, P.p2));
    TRY(conv(5, P.o[4]));
    TRY(pool(P.o[5], 2, 64, P.p3));
    TRY(conv(6, P.p3));
    TRY(conv(7, P.o[6]));
    TRY(upcat(P.o[7], 3, 64, P.o[5], 64, P.c8));
    TRY(conv(8, P.c8));
    TRY(conv(9, P.o[8]));
    TRY(upcat(P.o[9], 2, 64, P.o[3], 32, P.c10));
    TRY(conv(10, P.c10));
    TRY(conv(11, P.o[10]));
    if (fuse_cat && P.n[0] >= kLZ) {
        TRY(launch_conv_cat(P.o[11], P.o[1], P.n[0], 48, 32, P.wf[12],
                            params + param_offset(12) + 27L * 48 * 16, 16, 1, P.o[12], s));
    } else {
        TRY(upcat(P.o[11], 1, 32, P.o[1], 16, P.c12));
        TRY(conv(12, P.c12));
    }
    TRY(conv(13, P.o[12]));
    return ISIS_OK;
}

// Backward from d(o13) in P.ga; writes the 14 convolutions' gradients into
// P.grad (the head's part is written by the caller).
int run_backward(const Plan& P, const float* params, hipStream_t s)
{
    for (int c = 1; c < 14; ++c) {
        hipLaunchKernelGGL(k_flip_weights, dim3(grid_of(27L * kConvs[c].cin * kConvs[c].cout)),
                           dim3(kThreads), 0, s, params + param_offset(c), kConvs[c].cin,
                           kConvs[c].cout, P.wb[c]);
        ULAUNCH("k_flip_weights");
    }
    // back(c, g, x, dx): g = d(o_c) (masked in place), weight and bias
    // gradients from the layer input x, dx = d(x) (skipped when NULL).
    auto back = [&](int c, bf16_t* g, const bf16_t* x, bf16_t* dx) -> int {
        const int lv = level_of(c);
        const long nv = P.nv[lv];
        const int ci = kConvs[c].cin, co = kConvs[c].cout;
        hipLaunchKernelGGL(k_relu_mask, dim3(grid_of(nv * co)), dim3(kThreads), 0, s, g, P.o[c],
                           nv * co);
        ULAUNCH("k_relu_mask");
        float* gw = P.grad + param_offset(c);
        int rr = launch_conv_dw(x, P.n[lv], ci, g, co, P.part, gw, s);
        if (rr) return rr;
        rr = launch_chan_sum(g, nv, co, P.part, gw + 27L * ci * co, s);
        if (rr) return rr;
        if (!dx) return ISIS_OK;
        return launch_conv(g, P.n[lv], co, P.wb[c], nullptr, ci, 0, dx, nullptr, s);
    };
    // gradient of the upsampled half of a concatenation (level lvf fine)
    auto upb = [&](const bf16_t* dcat, int lvf, int cs, int C, bf16_t* y) -> int {
        hipLaunchKernelGGL(k_up2_bwd, dim3(grid_of(P.nv[lvf + 1] * C)), dim3(kThreads), 0, s, dcat,
                           P.n[lvf], cs, C, y);
        ULAUNCH("k_up2_bwd");
        return (int)ISIS_OK;
    };
    // gradient of a skip tensor: concat part + pooled path
    auto skipg = [&](const bf16_t* dcat, int lvf, int cs, int C, int S, const bf16_t* dlo,
                     bf16_t* y) -> int {
        hipLaunchKernelGGL(k_skip_grad, dim3(grid_of(P.nv[lvf] * S)), dim3(kThreads), 0, s, dcat,
                           P.n[lvf], cs, C, S, dlo, y);
        ULAUNCH("k_skip_grad");
        return (int)ISIS_OK;
    };
    TRY(back(13, P.ga, P.o[12], P.gb));               // gb = d o12
    TRY(back(12, P.gb, P.c12, P.gc12));               // gc12 = d c12 [nv0][48]
    TRY(upb(P.gc12, 0, 48, 32, P.ga));                // ga = d o11 [nv1][32]
    TRY(back(11, P.ga, P.o[10], P.gb));               // gb = d o10
    TRY(back(10, P.gb, P.c10, P.gc10));               // gc10 = d c10 [nv1][96]
    TRY(upb(P.gc10, 1, 96, 64, P.ga));                // ga = d o9 [nv2][64]
    TRY(back(9, P.ga, P.o[8], P.gb));                 // gb = d o8
    TRY(back(8, P.gb, P.c8, P.gc8));                  // gc8 = d c8 [nv2][128]
    TRY(upb(P.gc8, 2, 128, 64, P.ga));                // ga = d o7 [nv3][64]
    TRY(back(7, P.ga, P.o[6], P.gb));                 // gb = d o6
    TRY(back(6, P.gb, P.p3, P.ga));                   // ga = d p3 [nv3][64]
    TRY(skipg(P.gc8, 2, 128, 64, 64, P.ga, P.gb));    // gb = d o5 [nv2][64]
    TRY(back(5, P.gb, P.o[4], P.ga));                 // ga = d o4
    TRY(back(4, P.ga, P.p2, P.gb));                   // gb = d p2 [nv2][32]
    TRY(skipg(P.gc10, 1, 96, 64, 32, P.gb, P.ga));    // ga = d o3 [nv1][32]
    TRY(back(3, P.ga, P.o[2], P.gb));                 // gb = d o2
    TRY(back(2, P.gb, P.p1, P.ga));                   // ga = d p1 [nv1][16]
    TRY(skipg(P.gc12, 0, 48, 32, 16, P.ga, P.gb));    // gb = d o1 [nv0][16]
    TRY(back(1, P.gb, P.o[0], P.ga));                 // ga = d o0
    TRY(back(0, P.ga, P.in, nullptr));
    return ISIS_OK;
}

bool valid_unet_n(int n) { return n >= 16 && n <= 2048 && (n & (n - 1)) == 0; }

}  // namespace

// ---------------------------------------------------------------------------
// C ABI.
// ---------------------------------------------------------------------------

extern "C" {

size_t isis_unet_param_count(void) { return (size_t)param_total(); }

size_t isis_unet_workspace_size(int n, int training)
{
    if (!valid_unet_n(n)) return 0;
    return make_plan(n, training, nullptr).bytes;
}

const char* isis_unet_last_error(void) { return u_err; }

int isis_unet_predict(const float* params, const double* eta, const double* phi_cold, double a,
                      int n, double* guess, float* out, void* workspace, size_t workspace_bytes,
                      void* stream)
{
    u_err[0] = 0;
    if (!valid_unet_n(n) || !params || !eta || !phi_cold || !workspace || !(a > 0.0)) {
        uerr("unet_predict: need n a power of two in [16, 2048], a > 0, non-NULL arrays");
        return ISIS_ERR_INVALID_ARG;
    }
    Plan P = make_plan(n, 0, (char*)workspace);
    if (workspace_bytes < P.bytes || ((uintptr_t)workspace & 255)) {
        uerr("unet_predict: workspace must be 256-byte aligned and >= %zu bytes", P.bytes);
        return ISIS_ERR_INVALID_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_make_input, dim3(grid_of(P.nv[0])), dim3(kThreads), 0, s, eta, phi_cold,
                       a, P.nv[0], P.in);
    ULAUNCH("k_make_input");
    TRY(run_forward(P, params, s, true));
    hipLaunchKernelGGL(k_head, dim3(grid_of(P.nv[0])), dim3(kThreads), 0, s, P.o[13],
                       params + param_offset(14), P.nv[0], out, phi_cold, guess);
    ULAUNCH("k_head");
    return ISIS_OK;
}

int isis_unet_forward(const float* params, const double* eta, const double* phi_cold, double a,
                      int n, float* out, void* workspace, size_t workspace_bytes, void* stream)
{
    u_err[0] = 0;
    if (!valid_unet_n(n) || !params || !eta || !phi_cold || !workspace || !(a > 0.0)) {
        uerr("unet_forward: need n a power of two in [16, 2048], a > 0, non-NULL arrays");
        return ISIS_ERR_INVALID_ARG;
    }
    Plan P = make_plan(n, 1, (char*)workspace);
    if (workspace_bytes < P.bytes || ((uintptr_t)workspace & 255)) {
        uerr("unet_forward: workspace must be 256-byte aligned and >= %zu bytes (training size)",
             P.bytes);
        return ISIS_ERR_INVALID_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_make_input, dim3(grid_of(P.nv[0])), dim3(kThreads), 0, s, eta, phi_cold,
                       a, P.nv[0], P.in);
    ULAUNCH("k_make_input");
    TRY(run_forward(P, params, s));
    hipLaunchKernelGGL(k_head, dim3(grid_of(P.nv[0])), dim3(kThreads), 0, s, P.o[13],
                       params + param_offset(14), P.nv[0], P.out, nullptr, nullptr);
    ULAUNCH("k_head");
    if (out) UCHECK(hipMemcpyAsync(out, P.out, P.nv[0] * sizeof(float), hipMemcpyDeviceToDevice, s));
    return ISIS_OK;
}

int isis_unet_backward(const float* params, const double* phi_cold, const double* phi_target,
                       int n, void* workspace, size_t workspace_bytes, float* grad,
                       float* loss_out, void* stream)
{
    u_err[0] = 0;
    if (!valid_unet_n(n) || !params || !phi_cold || !phi_target || !workspace) {
        uerr("unet_backward: need n a power of two in [16, 2048] and non-NULL arrays");
        return ISIS_ERR_INVALID_ARG;
    }
    Plan P = make_plan(n, 1, (char*)workspace);
    if (workspace_bytes < P.bytes || ((uintptr_t)workspace & 255)) {
        uerr("unet_backward: workspace must be 256-byte aligned and >= %zu bytes (training size)",
             P.bytes);
        return ISIS_ERR_INVALID_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    const float* head = params + param_offset(14);
    const int hchunk = 4096;
    const int hb = (int)((P.nv[0] + hchunk - 1) / hchunk);
    hipLaunchKernelGGL(k_head_bwd, dim3(hb), dim3(kThreads), 0, s, P.out, phi_target, phi_cold,
                       P.o[13], head, P.nv[0], hchunk, P.hpart, P.ga);
    ULAUNCH("k_head_bwd");
    hipLaunchKernelGGL(k_sum_chunks, dim3(1), dim3(kThreads), 0, s, P.hpart, hb, 18L, P.hsum);
    ULAUNCH("k_sum_chunks");
    // head gradient (16 weights, 1 bias) into the flat gradient
    UCHECK(hipMemcpyAsync(P.grad + param_offset(14), P.hsum, 17 * sizeof(float),
                          hipMemcpyDeviceToDevice, s));
    TRY(run_backward(P, params, s));
    if (grad && grad != P.grad)
        UCHECK(hipMemcpyAsync(grad, P.grad, param_total() * sizeof(float), hipMemcpyDeviceToDevice,
                              s));
    if (loss_out) {
        float h[18];
        UCHECK(hipMemcpyAsync(h, P.hsum, sizeof(h), hipMemcpyDeviceToHost, s));
        UCHECK(hipStreamSynchronize(s));
        *loss_out = h[17] / (float)P.nv[0];
    }
    return ISIS_OK;
}

int isis_unet_adam_step(float* params, const float* grad, float* adam_m, float* adam_v,
                        long count, int step, float lr, void* stream)
{
    u_err[0] = 0;
    if (!params || !grad || !adam_m || !adam_v || count < 0 || step < 1 || !(lr >= 0.f)) {
        uerr("unet_adam_step: invalid arguments");
        return ISIS_ERR_INVALID_ARG;
    }
    if (count == 0) return ISIS_OK;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(grid_of(count)), dim3(kThreads), 0, (hipStream_t)stream,
                       params, grad, adam_m, adam_v, count, lr, b1, b2, 1e-8f, c1, c2);
    ULAUNCH("k_adam");
    return ISIS_OK;
}

int isis_unet_train_step(float* params, float* adam_m, float* adam_v, int step, float lr,
                         const double* eta, const double* phi_cold, const double* phi_target,
                         double a, int n, void* workspace, size_t workspace_bytes,
                         float* loss_out, float* grad_out, void* stream)
{
    u_err[0] = 0;
    if (!valid_unet_n(n) || !params || !adam_m || !adam_v || step < 1 || !(lr >= 0.f) || !eta ||
        !phi_cold || !phi_target || !workspace || !(a > 0.0)) {
        uerr("unet_train_step: invalid arguments");
        return ISIS_ERR_INVALID_ARG;
    }
    TRY(isis_unet_forward(params, eta, phi_cold, a, n, nullptr, workspace, workspace_bytes,
                          stream));
    Plan P = make_plan(n, 1, (char*)workspace);
    TRY(isis_unet_backward(params, phi_cold, phi_target, n, workspace, workspace_bytes, grad_out,
                           loss_out, stream));
    return isis_unet_adam_step(params, P.grad, adam_m, adam_v, param_total(), step, lr, stream);
}

int isis_unet_tensor(void* workspace, int n, int id, void** ptr, long* voxels, int* channels)
{
    u_err[0] = 0;
    if (!valid_unet_n(n) || !workspace || !ptr || id < 0 || id > 21) {
        uerr("unet_tensor: need n a power of two in [16, 2048], a workspace and 0 <= id <= 21");
        return ISIS_ERR_INVALID_ARG;
    }
    Plan P = make_plan(n, 1, (char*)workspace);
    void* q = nullptr;
    int lv = 0, C = 0;
    if (id < 14) {
        q = P.o[id];
        lv = level_of(id);
        C = kConvs[id].cout;
    } else if (id == 14) {
        q = P.in;
        C = 16;
    } else if (id <= 17) {
        lv = id - 14;
        q = id == 15 ? P.p1 : id == 16 ? P.p2 : P.p3;
        C = id == 15 ? 16 : id == 16 ? 32 : 64;
    } else if (id == 18) {
        q = P.c8;
        lv = 2;
        C = 128;
    } else if (id == 19) {
        q = P.c10;
        lv = 1;
        C = 96;
    } else if (id == 20) {
        q = P.c12;
        lv = 0;
        C = 48;
    } else {
        q = P.out;
        lv = 0;
        C = 1;
    }
    *ptr = q;
    if (voxels) *voxels = P.nv[lv];
    if (channels) *channels = C;
    return ISIS_OK;
}

int isis_conv3_fwd(const uint16_t* x, int n, int cin, const uint16_t* w, const float* bias,
                   int cout, int relu, uint16_t* y, float* yf, void* stream)
{
    u_err[0] = 0;
    if (!valid_unet_n(n) && !(n >= 2 && (n & (n - 1)) == 0)) {
        uerr("conv3_fwd: n must be a power of two >= 2");
        return ISIS_ERR_INVALID_ARG;
    }
    if (!x || !w || (!y && !yf)) {
        uerr("conv3_fwd: NULL array");
        return ISIS_ERR_INVALID_ARG;
    }
    return launch_conv(x, n, cin, w, bias, cout, relu, y, yf, (hipStream_t)stream);
}

size_t isis_conv3_bwd_weight_workspace(int n, int cin, int cout)
{
    if (n < 2 || (n & (n - 1))) return 0;
    const long nv = (long)n * n * n;
    return std::max(dw_part_floats(nv, cin, cout), (size_t)((nv + 4095) / 4096) * cout) * 4 + 256;
}

int isis_conv3_bwd_weight(const uint16_t* x, int n, int cin, const uint16_t* dy, int cout,
                          float* dw, float* db, void* workspace, size_t workspace_bytes,
                          void* stream)
{
    u_err[0] = 0;
    if (n < 2 || (n & (n - 1)) || !x || !dy || !dw || !workspace) {
        uerr("conv3_bwd_weight: invalid arguments");
        return ISIS_ERR_INVALID_ARG;
    }
    if (workspace_bytes < isis_conv3_bwd_weight_workspace(n, cin, cout)) {
        uerr("conv3_bwd_weight: workspace too small");
        return ISIS_ERR_INVALID_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    TRY(launch_conv_dw(x, n, cin, dy, cout, (float*)workspace, dw, s));
    if (db) TRY(launch_chan_sum(dy, (long)n * n * n, cout, (float*)workspace, db, s));
    return ISIS_OK;
}

int isis_conv3_flip_weights(const float* w, int cin, int cout, uint16_t* wt, void* stream)
{
    u_err[0] = 0;
    if (!w || !wt || cin <= 0 || cout <= 0) {
        uerr("conv3_flip_weights: invalid arguments");
        return ISIS_ERR_INVALID_ARG;
    }
    hipLaunchKernelGGL(k_flip_weights, dim3(grid_of(27L * cin * cout)), dim3(kThreads), 0,
                       (hipStream_t)stream, w, cin, cout, wt);
    ULAUNCH("k_flip_weights");
    return ISIS_OK;
}

}  // extern "C"
