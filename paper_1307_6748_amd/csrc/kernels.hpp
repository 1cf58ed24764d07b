// Level kernels of the FAS V-cycle: red-black Newton-Gauss-Seidel half-sweep,
// defect, fused defect + restriction, FAS coarse source, trilinear
// prolongation + correction, restriction, coarsest-grid solve, cold start,
// deterministic norm reductions and precision conversions.
//
// Grid layout: n^3 cells, index (i*n + j)*n + k with z (k) contiguous,
// periodic.  Every kernel is a grid-stride loop over its output cells, so any
// grid size is safe; launches use 256-thread blocks (four wave64s).
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>

#include "model.hpp"

namespace isis {

constexpr int kBlock = 256;
constexpr int kReduceBlocks = 8192;  // partial sums per reduction (fixed: deterministic)

// Raises a kernel's dynamic LDS limit to `bytes` on the current device, once
// per device (the attribute is per device); `done` is the kernel's bitmask of
// devices already set up.
inline hipError_t ensure_dynamic_lds(const void* kern, int bytes, std::atomic<unsigned>& done)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const unsigned bit = dev < 32 ? 1u << dev : 0u;
    if (bit && (done.load(std::memory_order_acquire) & bit)) return hipSuccess;
    e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess && bit) done.fetch_or(bit, std::memory_order_release);
    return e;
}

// Workgroups of `kern` (nt threads, `lds` bytes of dynamic LDS) that the
// current device holds at once: workgroups per CU times the CU count.  Cached
// per device in cache[dev] (0 = not yet queried); 0 on failure, with the
// runtime's last-error state cleared so that later launch checks are not
// confused by it.
constexpr int kMaxDevices = 64;
inline int resident_blocks(const void* kern, int nt, int lds, std::atomic<int>* cache)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) {
        (void)hipGetLastError();
        return 0;
    }
    if (dev < kMaxDevices) {
        const int v = cache[dev].load(std::memory_order_acquire);
        if (v > 0) return v;
    }
    int per_cu = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, nt, (size_t)lds) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    const int v = per_cu * ncu;
    if (dev < kMaxDevices && v > 0) cache[dev].store(v, std::memory_order_release);
    return v;
}

// Native two-element vectors (16- or 8-byte loads and stores).  Clang's
// ext_vector_type keeps them in registers; HIP's struct-based double2 is
// copied with memcpy, which pins arrays of it to scratch memory.
template <class T>
struct Vec2 {
    using type = T __attribute__((ext_vector_type(2)));
};

__device__ __forceinline__ int wrap_dec(int i, int n) { return i == 0 ? n - 1 : i - 1; }
__device__ __forceinline__ int wrap_inc(int i, int n) { return i == n - 1 ? 0 : i + 1; }
__device__ __forceinline__ long cell(int n, int i, int j, int k)
{
    return ((long)i * n + j) * n + k;
}

// Gather the cell value and its six periodic neighbours (x-, x+, y-, y+, z-, z+).
template <class T>
__device__ __forceinline__ T gather(const T* __restrict__ f, int n, int i, int j, int k, T nb[6])
{
    nb[0] = f[cell(n, wrap_dec(i, n), j, k)];
    nb[1] = f[cell(n, wrap_inc(i, n), j, k)];
    nb[2] = f[cell(n, i, wrap_dec(j, n), k)];
    nb[3] = f[cell(n, i, wrap_inc(j, n), k)];
    nb[4] = f[cell(n, i, j, wrap_dec(k, n))];
    nb[5] = f[cell(n, i, j, wrap_inc(k, n))];
    return f[cell(n, i, j, k)];
}

// Adds this wave's safeguard activations (per-lane counts) to the model's
// device counter: a wave64 sum, then one 64-bit atomic per wave.  Integer
// sums do not depend on the order, so the total is deterministic.  Every lane
// of the wave must call it.
template <class M>
__device__ __forceinline__ void guard_flush(const M& m, unsigned cnt)
{
    if constexpr (M::kGuard) {
        if (!m.hits) return;
        for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
        if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(m.hits, (unsigned long long)cnt);
    }
}

// One colour of a red-black Newton-Gauss-Seidel sweep, in place (Sec. 3.2).
// Cells of one colour only read cells of the other colour, so the update is
// race-free and independent of the order.
template <class T, class M>
__global__ __launch_bounds__(kBlock) void k_halfsweep(M m, int n, T ih2, T* __restrict__ phi,
                                                      const T* __restrict__ eta,
                                                      const T* __restrict__ sigma, int colour)
{
    const int hn = n >> 1;
    const long total = (long)n * n * hn;
    unsigned hits = 0;
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (long)gridDim.x * blockDim.x) {
        int kk = (int)(t % hn);
        long r = t / hn;
        int j = (int)(r % n);
        int i = (int)(r / n);
        int k = 2 * kk + ((i + j + colour) & 1);
        T nb[6];
        T p = gather(phi, n, i, j, k, nb);
        long c = cell(n, i, j, k);
        T L, D;
        const T e = eta[c];
        m.op(p, nb, e, ih2, L, D);
        if constexpr (M::kGuard) hits += m.guarded(p, e);
        T eps = L - (sigma ? sigma[c] : T(0));
        phi[c] = p - m.limit(eps / D);
    }
    guard_flush(m, hits);
}

// out = L(phi) - sigma.
template <class T, class M>
__global__ __launch_bounds__(kBlock) void k_defect(M m, int n, T ih2, const T* __restrict__ phi,
                                                   const T* __restrict__ eta,
                                                   const T* __restrict__ sigma, T* __restrict__ out)
{
    const long total = (long)n * n * n;
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < total;
         c += (long)gridDim.x * blockDim.x) {
        int k = (int)(c % n);
        long r = c / n;
        int j = (int)(r % n);
        int i = (int)(r / n);
        T nb[6];
        T p = gather(phi, n, i, j, k, nb);
        T L, D;
        m.op(p, nb, eta[c], ih2, L, D);
        out[c] = L - (sigma ? sigma[c] : T(0));
    }
}

// Block sum of a double (wave64 shuffles, then across the block's waves).
// Every thread of the block must call it; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double part[kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) part[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kBlock / 64; ++w) s += part[w];
    __syncthreads();
    return s;
}

// Finest-level defect in double precision with per-block partial sums of r^2
// (and of r, for diagnostics).  TF is the field's storage type: double, or
// float for the FP64 defect of the FP32 iterate in mixed precision.  The model
// M works in double.  res may be NULL.
template <class TF, class M>
__global__ __launch_bounds__(kBlock) void k_defect_norm(M m, int n, double ih2,
                                                        const TF* __restrict__ phi,
                                                        const double* __restrict__ eta,
                                                        double* __restrict__ res,
                                                        double* __restrict__ partial)
{
    const long total = (long)n * n * n;
    double acc = 0.0;
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < total;
         c += (long)gridDim.x * blockDim.x) {
        int k = (int)(c % n);
        long r = c / n;
        int j = (int)(r % n);
        int i = (int)(r / n);
        double nb[6];
        nb[0] = (double)phi[cell(n, wrap_dec(i, n), j, k)];
        nb[1] = (double)phi[cell(n, wrap_inc(i, n), j, k)];
        nb[2] = (double)phi[cell(n, i, wrap_dec(j, n), k)];
        nb[3] = (double)phi[cell(n, i, wrap_inc(j, n), k)];
        nb[4] = (double)phi[cell(n, i, j, wrap_dec(k, n))];
        nb[5] = (double)phi[cell(n, i, j, wrap_inc(k, n))];
        double p = (double)phi[c];
        double L, D;
        m.op(p, nb, eta[c], ih2, L, D);
        if (res) res[c] = L;
        acc += L * L;
    }
    double s = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Sum of a field (for the mean of the singular linear problem).
template <class T>
__global__ __launch_bounds__(kBlock) void k_sum(long total, const T* __restrict__ f,
                                                double* __restrict__ partial)
{
    double acc = 0.0;
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < total;
         c += (long)gridDim.x * blockDim.x)
        acc += (double)f[c];
    double s = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// out[0] = sum of partial[0..count) in a fixed order (one block).
__global__ __launch_bounds__(kBlock) void k_reduce(const double* __restrict__ partial, int count,
                                                   double* __restrict__ out)
{
    // Each thread sums fixed runs of 8 consecutive partials (loads issued
    // together, added in order): deterministic, and a few load latencies
    // instead of count / blockDim dependent ones.
    double acc = 0.0;
    for (int q0 = threadIdx.x * 8; q0 < count; q0 += blockDim.x * 8) {
        double v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = q0 + j < count ? partial[q0 + j] : 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j) acc += v[j];
    }
    double s = block_sum(acc);
    if (threadIdx.x == 0) out[0] = s;
}

// f -= sum[0] / total (removes the mean of the singular linear problem).
template <class T>
__global__ __launch_bounds__(kBlock) void k_sub_mean(long total, T* __restrict__ f,
                                                     const double* __restrict__ sum)
{
    const T mu = (T)(sum[0] / (double)total);
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < total;
         c += (long)gridDim.x * blockDim.x)
        f[c] -= mu;
}

// coarse = mean of 8 children.
template <class T>
__global__ __launch_bounds__(kBlock) void k_restrict(int nf, const T* __restrict__ fine,
                                                     T* __restrict__ coarse,
                                                     float* __restrict__ fine32)
{
    const int nc = nf >> 1;
    const long total = (long)nc * nc * nc;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (long)gridDim.x * blockDim.x) {
        int K = (int)(q % nc);
        long r = q / nc;
        int J = (int)(r % nc);
        int I = (int)(r / nc);
        T s = T(0);
#pragma unroll
        for (int di = 0; di < 2; ++di)
#pragma unroll
            for (int dj = 0; dj < 2; ++dj)
#pragma unroll
                for (int dk = 0; dk < 2; ++dk) {
                    const long c = cell(nf, 2 * I + di, 2 * J + dj, 2 * K + dk);
                    const T v = fine[c];
                    s += v;
                    if (fine32) fine32[c] = (float)v;  // the fine level's FP32 copy, same pass
                }
        coarse[q] = s / T(8);
    }
}

// FAS descent, first half (Sec. 3.2): for each coarse cell, the fine defect
// eps = L_f(phi_f) - sigma_f at its 8 children, restricted (rr_c = R eps),
// and the restricted approximation phi_c = phihat_c = R phi_f.
template <class T, class M>
__global__ __launch_bounds__(kBlock) void k_defect_restrict(M m, int nf, T ih2,
                                                            const T* __restrict__ phi,
                                                            const T* __restrict__ eta,
                                                            const T* __restrict__ sigma,
                                                            T* __restrict__ phi_c,
                                                            T* __restrict__ phihat_c,
                                                            T* __restrict__ rr_c)
{
    const int nc = nf >> 1;
    const long total = (long)nc * nc * nc;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (long)gridDim.x * blockDim.x) {
        int K = (int)(q % nc);
        long r = q / nc;
        int J = (int)(r % nc);
        int I = (int)(r / nc);
        T sr = T(0), sp = T(0);
#pragma unroll
        for (int di = 0; di < 2; ++di)
#pragma unroll
            for (int dj = 0; dj < 2; ++dj)
#pragma unroll
                for (int dk = 0; dk < 2; ++dk) {
                    int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
                    long c = cell(nf, i, j, k);
                    T nb[6];
                    T p = gather(phi, nf, i, j, k, nb);
                    T L, D;
                    m.op(p, nb, eta[c], ih2, L, D);
                    sr += L - (sigma ? sigma[c] : T(0));
                    sp += p;
                }
        T pc = sp / T(8);
        phi_c[q] = pc;
        phihat_c[q] = pc;
        rr_c[q] = sr / T(8);
    }
}

// FAS descent, second half: sigma_c = L_c(phi_c, eta_c) - rr_c.
template <class T, class M>
__global__ __launch_bounds__(kBlock) void k_fas_sigma(M m, int nc, T ih2,
                                                      const T* __restrict__ phi_c,
                                                      const T* __restrict__ eta_c,
                                                      const T* __restrict__ rr_c,
                                                      T* __restrict__ sigma_c)
{
    const long total = (long)nc * nc * nc;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (long)gridDim.x * blockDim.x) {
        int K = (int)(q % nc);
        long r = q / nc;
        int J = (int)(r % nc);
        int I = (int)(r / nc);
        T nb[6];
        T p = gather(phi_c, nc, I, J, K, nb);
        T L, D;
        m.op(p, nb, eta_c[q], ih2, L, D);
        sigma_c[q] = L - rr_c[q];
    }
}

// Prolongation weight of the other coarse cell N along one axis (the
// parent P takes 1 minus it).  PW = 0: trilinear, 1/4.  PW = 1, 2: weighted by
// the flux coefficient b of the flux-form operators (Sec. 3.4), read from the
// restricted field coarse_hat: 1 / (2 (1 + b_P / b_N)), which keeps the flux
// b de/dx continuous across the face between P and N when b is constant over
// each coarse cell and the correction linear between the centres; b = e^x for
// PW = 1 (fields in u), 2^x for PW = 2 (single-precision f(R), carried as
// w = u / ln 2).  Only the difference of the two values enters, so extreme
// contrasts give 0 or 1/2, never an overflow.
template <int PW, class T>
__device__ __forceinline__ T prolong_weight(T xp, T xn)
{
    if constexpr (PW == 0) {
        return T(0.25);
    } else {
        const T d = xp - xn;
        T e;
        if constexpr (PW == 2)
            e = exp2(d);
        else
            e = exp(d);
        return T(1) / (T(2) * (T(1) + e));
    }
}

// fine += P(coarse - coarse_hat), cell-centred: along each axis the parent
// I = i/2 and its neighbour I + s (s = +1 for odd i, -1 for even i); weights
// 3/4 and 1/4 (trilinear, PW = 0) or from prolong_weight (PW = 1, 2).
template <class T, int PW = 0>
__global__ __launch_bounds__(kBlock) void k_prolong_correct(int nf, T* __restrict__ fine,
                                                            const T* __restrict__ coarse,
                                                            const T* __restrict__ coarse_hat)
{
    const int nc = nf >> 1;
    const long total = (long)nf * nf * nf;
    const T w[2] = {T(0.75), T(0.25)};
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < total;
         c += (long)gridDim.x * blockDim.x) {
        int k = (int)(c % nf);
        long r = c / nf;
        int j = (int)(r % nf);
        int i = (int)(r / nf);
        int I[2], J[2], K[2];
        I[0] = i >> 1;
        I[1] = (i & 1) ? wrap_inc(I[0], nc) : wrap_dec(I[0], nc);
        J[0] = j >> 1;
        J[1] = (j & 1) ? wrap_inc(J[0], nc) : wrap_dec(J[0], nc);
        K[0] = k >> 1;
        K[1] = (k & 1) ? wrap_inc(K[0], nc) : wrap_dec(K[0], nc);
        T wx[2] = {w[0], w[1]}, wy[2] = {w[0], w[1]}, wz[2] = {w[0], w[1]};
        if constexpr (PW != 0) {
            const T hp = coarse_hat[cell(nc, I[0], J[0], K[0])];
            wx[1] = prolong_weight<PW>(hp, coarse_hat[cell(nc, I[1], J[0], K[0])]);
            wy[1] = prolong_weight<PW>(hp, coarse_hat[cell(nc, I[0], J[1], K[0])]);
            wz[1] = prolong_weight<PW>(hp, coarse_hat[cell(nc, I[0], J[0], K[1])]);
            wx[0] = T(1) - wx[1];
            wy[0] = T(1) - wy[1];
            wz[0] = T(1) - wz[1];
        }
        T s = T(0);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int d = 0; d < 2; ++d) {
                    long q = cell(nc, I[a], J[b], K[d]);
                    s += wx[a] * wy[b] * wz[d] * (coarse[q] - coarse_hat[q]);
                }
        fine[c] += s;
    }
}

// nu_c red-black sweeps on the 4^3 coarsest grid: one wave64, one cell per
// lane, the grid held in LDS.
template <class T, class M>
__global__ __launch_bounds__(64) void k_coarse_solve(M m, T ih2, T* __restrict__ phi,
                                                     const T* __restrict__ eta,
                                                     const T* __restrict__ sigma, int nu_c)
{
    __shared__ T f[64];
    const int t = threadIdx.x;
    const int i = t >> 4, j = (t >> 2) & 3, k = t & 3;
    f[t] = phi[t];
    const T e = eta[t];
    const T s = sigma ? sigma[t] : T(0);
    __syncthreads();
    unsigned hits = 0;
    for (int it = 0; it < nu_c; ++it) {
        for (int colour = 0; colour < 2; ++colour) {
            if (((i + j + k) & 1) == colour) {
                T nb[6];
                T p = gather(f, 4, i, j, k, nb);
                T L, D;
                m.op(p, nb, e, ih2, L, D);
                if constexpr (M::kGuard) hits += m.guarded(p, e);
                f[t] = p - m.limit((L - s) / D);
            }
            __syncthreads();
        }
    }
    phi[t] = f[t];
    guard_flush(m, hits);
}

// The cold start written into phi64, its FP32 copy (cold - shift) * kVar into
// phi32 (if not NULL) and per-block partial sums of cold^2, in one pass.
template <class M>
__global__ __launch_bounds__(kBlock) void k_cold_start_sumsq(M m, long total,
                                                             const double* __restrict__ eta,
                                                             double* __restrict__ phi64,
                                                             float* __restrict__ phi32,
                                                             double scale32, double offset32,
                                                             double* __restrict__ partial)
{
    double acc = 0.0;
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < total;
         c += (long)gridDim.x * blockDim.x) {
        const double v = (double)m.cold(eta[c]);
        phi64[c] = v;
        if (phi32) phi32[c] = (float)(v * scale32 + offset32);
        acc += v * v;
    }
    double s = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <class T, class M>
__global__ __launch_bounds__(kBlock) void k_cold_start(M m, long total,
                                                       const double* __restrict__ eta,
                                                       T* __restrict__ phi)
{
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < total;
         c += (long)gridDim.x * blockDim.x)
        phi[c] = (T)m.cold((double)eta[c]);
}

template <class TO, class TI>
__global__ __launch_bounds__(kBlock) void k_convert(long total, const TI* __restrict__ in,
                                                    TO* __restrict__ out, double scale,
                                                    double offset)
{
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < total;
         c += (long)gridDim.x * blockDim.x)
        out[c] = (TO)((double)in[c] * scale + offset);
}

}  // namespace isis
