// The bottom of a V-cycle in one workgroup: from the first level of side
// <= 16 down to the 4^3 coarsest grid and back (Sec. 3.2), with every array
// these levels touch held in LDS.  On the device each of these levels is a
// dozen launches of a few microseconds each, almost all launch and drain;
// here they are one launch whose phases are separated by workgroup barriers.
// Each phase computes per cell what the per-level kernels compute, with the
// same terms in the same order: k_halfsweep, k_defect_restrict (or the fine
// defect then k_restrict_fw for full weighting), k_fas_sigma,
// k_prolong_correct (with its weights PW) and the coarsest grid's sweeps of
// k_coarse_solve.  Only the first level's field is written back; the coarser
// levels' fields are rebuilt by every descent.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace isis {

constexpr int kBottomMaxN = 16;      // side of the first level handled
constexpr int kBottomMaxLevels = 3;  // 16, 8, 4
// threads: 1024 in single precision (16 waves hide LDS latency on the one
// CU; every model's update fits 128 registers), 512 in double (up to 218)
template <class T>
constexpr int bottom_threads()
{
    return sizeof(T) == 4 ? 1024 : 512;
}

template <class T>
struct BottomArgs {
    int nlev;                        // levels handled, 2 or 3; sides 4 << (nlev - 1 - q)
    int nu_pre, nu_post, nu_coarse;
    T* phi0;                         // the first level's field, updated in place
    const T* sigma0;                 // the first level's FAS source (may be NULL: zero)
    const T* eta[kBottomMaxLevels];  // densities
    T ih2[kBottomMaxLevels];         // 1/h^2 per level
};

// LDS elements: per level field, density and FAS source, plus the first
// level's fine-defect buffer and each coarser level's restricted field.
__host__ __device__ constexpr int bottom_lds_elems(int nlev)
{
    int e = 0;
    for (int q = 0; q < nlev; ++q) {
        const int n = 4 << (nlev - 1 - q);
        e += 4 * n * n * n;
    }
    return e;
}

// PW: the prolongation's weights (k_prolong_correct).
template <class T, class M, bool FW, int PW = 0>
__global__ __launch_bounds__(bottom_threads<T>()) void k_bottom_cycle(M m, BottomArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* base = reinterpret_cast<T*>(smem_raw);
    const int tid = threadIdx.x;
    constexpr int NT = bottom_threads<T>();
    const int nlev = a.nlev;
    // level q: phi, eta, sig, then aux (first level: the fine defect; coarser
    // levels: phihat)
    T *phi[kBottomMaxLevels], *eta[kBottomMaxLevels], *sig[kBottomMaxLevels],
        *aux[kBottomMaxLevels];
    int side[kBottomMaxLevels];
    {
        int off = 0;
        for (int q = 0; q < kBottomMaxLevels; ++q) {
            const int n = q < nlev ? 4 << (nlev - 1 - q) : 0;
            const int n3 = n * n * n;
            side[q] = n;
            phi[q] = base + off;
            eta[q] = base + off + n3;
            sig[q] = base + off + 2 * n3;
            aux[q] = base + off + 3 * n3;
            off += 4 * n3;
        }
    }
    {
        const int n3 = side[0] * side[0] * side[0];
        for (int c = tid; c < n3; c += NT) {
            phi[0][c] = a.phi0[c];
            eta[0][c] = a.eta[0][c];
            sig[0][c] = a.sigma0 ? a.sigma0[c] : T(0);
        }
        for (int q = 1; q < nlev; ++q) {
            const int m3 = side[q] * side[q] * side[q];
            for (int c = tid; c < m3; c += NT) eta[q][c] = a.eta[q][c];
        }
    }
    __syncthreads();
    unsigned hits = 0;

    // one colour of level q; cells t = tid, tid + stride, ...
    auto colour_pass = [&](int q, int colour, int stride) __attribute__((always_inline)) {
        const int n = side[q], hn = n >> 1;
        const int total = n * n * hn;
        T* f = phi[q];
        const T ih2 = a.ih2[q];
        for (int t = tid; t < total; t += stride) {
            const int kk = t % hn, r = t / hn;
            const int j = r % n, i = r / n;
            const int k = 2 * kk + ((i + j + colour) & 1);
            T nb[6];
            const T p = gather(f, n, i, j, k, nb);
            const long c = cell(n, i, j, k);
            T L, D;
            const T e = eta[q][c];
            m.op(p, nb, e, ih2, L, D);
            if constexpr (M::kGuard) hits += m.guarded(p, e);
            const T eps = L - sig[q][c];
            f[c] = p - m.limit(eps / D);
        }
    };
    auto halfsweep = [&](int q, int colour) __attribute__((always_inline)) {
        colour_pass(q, colour, NT);
        __syncthreads();
    };

    auto descend = [&](int q) __attribute__((always_inline)) {
        const int nf = side[q], nc = nf >> 1;
        const int c3 = nc * nc * nc;
        const T ih2 = a.ih2[q];
        T* pc_ = phi[q + 1];
        T* ph_ = aux[q + 1];
        T* rr = sig[q + 1];  // the restricted defect, then Sigma in place
        if constexpr (FW) {
            // the fine defect into the first level's buffer (nf^3 <= its size)
            T* dfine = aux[0];
            const int f3 = nf * nf * nf;
            for (int c = tid; c < f3; c += NT) {
                const int k = c % nf, r = c / nf;
                const int j = r % nf, i = r / nf;
                T nb[6];
                const T p = gather(phi[q], nf, i, j, k, nb);
                T L, D;
                m.op(p, nb, eta[q][c], ih2, L, D);
                dfine[c] = L - sig[q][c];
            }
            __syncthreads();
            const T w[4] = {T(0.125), T(0.375), T(0.375), T(0.125)};
            for (int Q = tid; Q < c3; Q += NT) {
                const int K = Q % nc, r = Q / nc;
                const int J = r % nc, I = r / nc;
                T sp = T(0);
#pragma unroll
                for (int di = 0; di < 2; ++di)
#pragma unroll
                    for (int dj = 0; dj < 2; ++dj)
#pragma unroll
                        for (int dk = 0; dk < 2; ++dk)
                            sp += phi[q][cell(nf, 2 * I + di, 2 * J + dj, 2 * K + dk)];
                T sx = T(0);
#pragma unroll
                for (int aa = 0; aa < 4; ++aa) {
                    const int i = (2 * I - 1 + aa + nf) % nf;
                    T sy = T(0);
#pragma unroll
                    for (int bb = 0; bb < 4; ++bb) {
                        const int j = (2 * J - 1 + bb + nf) % nf;
                        const T* row = dfine + (i * nf + j) * nf;
                        T sz = T(0);
#pragma unroll
                        for (int cc = 0; cc < 4; ++cc) sz += w[cc] * row[(2 * K - 1 + cc + nf) % nf];
                        sy += w[bb] * sz;
                    }
                    sx += w[aa] * sy;
                }
                const T pcv = sp / T(8);
                pc_[Q] = pcv;
                ph_[Q] = pcv;
                rr[Q] = sx;
            }
        } else {
            for (int Q = tid; Q < c3; Q += NT) {
                const int K = Q % nc, r = Q / nc;
                const int J = r % nc, I = r / nc;
                T sr = T(0), sp = T(0);
#pragma unroll
                for (int di = 0; di < 2; ++di)
#pragma unroll
                    for (int dj = 0; dj < 2; ++dj)
#pragma unroll
                        for (int dk = 0; dk < 2; ++dk) {
                            const int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
                            const long c = cell(nf, i, j, k);
                            T nb[6];
                            const T p = gather(phi[q], nf, i, j, k, nb);
                            T L, D;
                            m.op(p, nb, eta[q][c], ih2, L, D);
                            sr += L - sig[q][c];
                            sp += p;
                        }
                const T pcv = sp / T(8);
                pc_[Q] = pcv;
                ph_[Q] = pcv;
                rr[Q] = sr / T(8);
            }
        }
        __syncthreads();
        // Sigma_c = L_c(phi_c) - rr_c, cell by cell in place
        const T ih2c = a.ih2[q + 1];
        for (int Q = tid; Q < c3; Q += NT) {
            const int K = Q % nc, r = Q / nc;
            const int J = r % nc, I = r / nc;
            T nb[6];
            const T p = gather(pc_, nc, I, J, K, nb);
            T L, D;
            m.op(p, nb, eta[q + 1][Q], ih2c, L, D);
            rr[Q] = L - rr[Q];
        }
        __syncthreads();
    };

    auto prolong = [&](int q) __attribute__((always_inline)) {
        const int nf = side[q], nc = nf >> 1;
        const int f3 = nf * nf * nf;
        const T* co = phi[q + 1];
        const T* ch = aux[q + 1];
        const T w[2] = {T(0.75), T(0.25)};
        for (int c = tid; c < f3; c += NT) {
            const int k = c % nf, r = c / nf;
            const int j = r % nf, i = r / nf;
            int I[2], J[2], K[2];
            I[0] = i >> 1;
            I[1] = (i & 1) ? wrap_inc(I[0], nc) : wrap_dec(I[0], nc);
            J[0] = j >> 1;
            J[1] = (j & 1) ? wrap_inc(J[0], nc) : wrap_dec(J[0], nc);
            K[0] = k >> 1;
            K[1] = (k & 1) ? wrap_inc(K[0], nc) : wrap_dec(K[0], nc);
            T wx[2] = {w[0], w[1]}, wy[2] = {w[0], w[1]}, wz[2] = {w[0], w[1]};
            if constexpr (PW != 0) {
                const T hp = ch[cell(nc, I[0], J[0], K[0])];
                wx[1] = prolong_weight<PW>(hp, ch[cell(nc, I[1], J[0], K[0])]);
                wy[1] = prolong_weight<PW>(hp, ch[cell(nc, I[0], J[1], K[0])]);
                wz[1] = prolong_weight<PW>(hp, ch[cell(nc, I[0], J[0], K[1])]);
                wx[0] = T(1) - wx[1];
                wy[0] = T(1) - wy[1];
                wz[0] = T(1) - wz[1];
            }
            T s = T(0);
#pragma unroll
            for (int aa = 0; aa < 2; ++aa)
#pragma unroll
                for (int bb = 0; bb < 2; ++bb)
#pragma unroll
                    for (int dd = 0; dd < 2; ++dd) {
                        const long qq = cell(nc, I[aa], J[bb], K[dd]);
                        s += wx[aa] * wy[bb] * wz[dd] * (co[qq] - ch[qq]);
                    }
            phi[q][c] += s;
        }
        __syncthreads();
    };

    for (int q = 0; q + 1 < nlev; ++q) {
        for (int it = 0; it < a.nu_pre; ++it) {
            halfsweep(q, 0);
            halfsweep(q, 1);
        }
        descend(q);
    }
    // The 4^3 grid (32 cells per colour) in the first wave alone: a wave's
    // LDS operations complete in issue order, so between colours it needs
    // only the fences that keep the compiler from reordering its LDS accesses
    // and wait for its writes; the other waves wait at the barrier below.
    if (tid < 64) {
        for (int it = 0; it < a.nu_coarse; ++it) {
#pragma unroll
            for (int colour = 0; colour < 2; ++colour) {
                colour_pass(nlev - 1, colour, 64);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            }
        }
    }
    __syncthreads();
    for (int q = nlev - 2; q >= 0; --q) {
        prolong(q);
        for (int it = 0; it < a.nu_post; ++it) {
            halfsweep(q, 0);
            halfsweep(q, 1);
        }
    }
    {
        const int n3 = side[0] * side[0] * side[0];
        for (int c = tid; c < n3; c += NT) a.phi0[c] = phi[0][c];
    }
    guard_flush(m, hits);
}

}  // namespace isis
