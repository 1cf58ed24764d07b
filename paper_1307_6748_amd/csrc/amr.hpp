// Refinement boundaries with masks (Sec. 3.3.1, 3.4.1): the operator, its
// Newton-Gauss-Seidel smoother and its defect on a refinement patch.
//
// A patch is an n^3 grid (spacing h, indices periodic) whose cells carry a
// mask: m > 0 inside the refinement (these cells are relaxed), m <= 0 outside
// (m = -1: the cell does not exist on this level, its value u^Int comes from
// the coarser grid; -1 < m <= 0: it exists with its centre outside the
// boundary, u^Int is its own pre-iteration value).  An inside cell c with a
// masked neighbour f sees the ghost value
//     u_G = u_f^Int + (m_f / m_c) (u_c - u_c^Pre)          (eq. ueq),
// the linear extrapolation through u_c and the boundary value at the mask's
// zero crossing; u^Pre is the field when the boundary values were set.  The
// model's operator then runs on the ghost-substituted neighbours (for the
// non-canonical models the face coefficient is b(u_G)), and the Newton
// denominator gains each ghost's dependence on u_c (model.ghost_dD).  Cells
// with m <= 0 are neither relaxed nor counted in the defect.  Patches keep a
// layer of m = -1 cells around their inside, so the periodic wrap never joins
// inside cells.  Double precision; per-cell grid-stride kernels (patches are
// small next to the uniform grid).
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace isis {

template <class M>
__device__ __forceinline__ void masked_op(const M& m, int n, double ih2,
                                          const double* __restrict__ phi,
                                          const double* __restrict__ eta,
                                          const double* __restrict__ mask,
                                          const double* __restrict__ u_int,
                                          const double* __restrict__ u_pre, int i, int j, int k,
                                          double& L, double& D)
{
    const long c = cell(n, i, j, k);
    const long q[6] = {cell(n, wrap_dec(i, n), j, k), cell(n, wrap_inc(i, n), j, k),
                       cell(n, i, wrap_dec(j, n), k), cell(n, i, wrap_inc(j, n), k),
                       cell(n, i, j, wrap_dec(k, n)), cell(n, i, j, wrap_inc(k, n))};
    const double p = phi[c], mc = mask[c], pre = u_pre[c];
    double v[6], r[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const double mf = mask[q[f]];
        if (mf > 0.0) {
            v[f] = phi[q[f]];
            r[f] = 0.0;
        } else {
            const double ui = mf > -1.0 ? u_pre[q[f]] : u_int[q[f]];  // eq. bpsi
            r[f] = mf / mc;
            v[f] = ui + r[f] * (p - pre);                               // eq. ueq
        }
    }
    m.op(p, v, eta[c], ih2, L, D);
#pragma unroll
    for (int f = 0; f < 6; ++f)
        if (r[f] != 0.0) D += m.ghost_dD(p, v[f], r[f], ih2);
}

// One colour of the red-black Newton-Gauss-Seidel sweep over the inside
// cells; masked cells keep their values.
template <class M>
__global__ __launch_bounds__(kBlock) void k_masked_halfsweep(
    M m, int n, double ih2, double* __restrict__ phi, const double* __restrict__ eta,
    const double* __restrict__ sigma, const double* __restrict__ mask,
    const double* __restrict__ u_int, const double* __restrict__ u_pre, int colour)
{
    const int hn = n >> 1;
    const long total = (long)n * n * hn;
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (long)gridDim.x * blockDim.x) {
        const int kk = (int)(t % hn);
        const long r = t / hn;
        const int j = (int)(r % n), i = (int)(r / n);
        const int k = 2 * kk + ((i + j + colour) & 1);
        const long c = cell(n, i, j, k);
        if (!(mask[c] > 0.0)) continue;
        double L, D;
        masked_op(m, n, ih2, phi, eta, mask, u_int, u_pre, i, j, k, L, D);
        const double eps = L - (sigma ? sigma[c] : 0.0);
        phi[c] = phi[c] - m.limit(eps / D);
    }
}

// out = L - sigma at inside cells, 0 elsewhere (out may be NULL); with
// partial, per-block sums of out^2 in partial[block] and of the inside cells
// in partial[nblocks + block] (for the RMS over the inside).
template <class M>
__global__ __launch_bounds__(kBlock) void k_masked_defect(
    M m, int n, double ih2, const double* __restrict__ phi, const double* __restrict__ eta,
    const double* __restrict__ sigma, const double* __restrict__ mask,
    const double* __restrict__ u_int, const double* __restrict__ u_pre, double* __restrict__ out,
    double* __restrict__ partial)
{
    const long total = (long)n * n * n;
    double acc = 0.0, cnt = 0.0;
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < total;
         c += (long)gridDim.x * blockDim.x) {
        double res = 0.0;
        if (mask[c] > 0.0) {
            const int k = (int)(c % n);
            const long r = c / n;
            const int j = (int)(r % n), i = (int)(r / n);
            double L, D;
            masked_op(m, n, ih2, phi, eta, mask, u_int, u_pre, i, j, k, L, D);
            res = L - (sigma ? sigma[c] : 0.0);
            cnt += 1.0;
        }
        if (out) out[c] = res;
        acc += res * res;
    }
    if (partial) {
        const double s = block_sum(acc);
        const double q = block_sum(cnt);
        if (threadIdx.x == 0) {
            partial[blockIdx.x] = s;
            partial[gridDim.x + blockIdx.x] = q;
        }
    }
}

}  // namespace isis
