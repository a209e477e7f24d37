// HIP kernels of EXACT with an explicit measurement matrix (the Gaussian
// measurement model, paper Sec. 2.2, and its experiment in Sec. 5) for CDNA4
// (gfx950, wave64).
//
// F(x) = (1/n) A^T r with r_i = Y_i - sum_k J_k exp(-mu_k max(<a_i, x>, 0))
// costs one pass over A: a workgroup streams a block of rows, forms each
// row's inner product with x (a fixed-order block reduction), its residual,
// and adds r_i a_i to a per-workgroup partial gradient held in registers,
// so every element of A is read from HBM once per evaluation.  The partial
// gradients are then summed in a fixed order.  No atomics.
#include "exact_internal.h"

#include <cmath>

namespace exact {
namespace {

constexpr int kDT = 256;          // threads of the streaming and reduction blocks
constexpr int kSumRows = 32;      // partial gradients summed per reduction block
constexpr int kFinT = 1024;       // threads of the single-block finish

__device__ __forceinline__ bool dskip(const int32_t *skip)
{
    return skip != nullptr && *skip != 0;
}

// Rows [blockIdx.x * rpb, min(n, (blockIdx.x + 1) * rpb)) of A (n x d,
// row-major); thread t owns columns t + 256 c, c < C.  linear: r_i = s_i
// (the power iteration's A^T A x), else the spectral residual.  Rows go in
// batches of RB; later batches' loads are issued before the current
// batch's block reduction, so they stay in flight across its barrier.
template <int C, int RB>
__device__ __forceinline__ void dense_load(const float *__restrict__ A, long row0, long i1, int d,
                                           int t, float (&a)[RB][C])
{
#pragma unroll
    for (int q = 0; q < RB; ++q) {
        const long row = row0 + q;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const int j = c * kDT + t;
            a[q][c] = (row < i1 && j < d) ? A[(size_t)row * d + j] : 0.f;
        }
    }
}

template <int C>
__global__ __launch_bounds__(kDT) void k_dense_F(const float *__restrict__ A, long n, int d,
                                                 const float *__restrict__ x,
                                                 const float *__restrict__ Y,
                                                 const float *__restrict__ J,
                                                 const float *__restrict__ mu, int K, int linear,
                                                 long rpb, float *__restrict__ parts,
                                                 const int32_t *__restrict__ skip)
{
    constexpr int RB = C >= 16 ? 2 : 4;
    if (dskip(skip))
        return;
    __shared__ float red[2][RB][kDT / 64];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    float xr[C], g[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j = c * kDT + t;
        xr[c] = j < d ? x[j] : 0.f;
        g[c] = 0.f;
    }
    const long i0 = (long)blockIdx.x * rpb;
    const long i1 = min(n, i0 + rpb);
    int buf = 0;
    // rows i .. i + RB - 1 (held in a): inner products with x (a fixed-order
    // block reduction: the wave's lanes, then the four waves in order), the
    // residual, and r_i a_i into the partial gradient; one barrier, with the
    // LDS slots alternating between batches
    auto sum_batch = [&](const float(&a)[RB][C], long i) {
        float dot[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            float s = 0.f;
#pragma unroll
            for (int c = 0; c < C; ++c)
                s = fmaf(a[q][c], xr[c], s);
            for (int off = 32; off > 0; off >>= 1)
                s += __shfl_xor(s, off);
            dot[q] = s;
        }
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < RB; ++q)
                red[buf][q][wave] = dot[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const long row = i + q;
            const float s = ((red[buf][q][0] + red[buf][q][1]) + red[buf][q][2]) + red[buf][q][3];
            float r = 0.f;
            if (row < i1) {
                if (linear) {
                    r = s;
                } else {
                    const float sp = fmaxf(s, 0.f);
                    float m = 0.f;
                    for (int k = 0; k < K; ++k)
                        m = fmaf(J[k], expf(-mu[k] * sp), m);
                    r = Y[row] - m;
                }
            }
#pragma unroll
            for (int c = 0; c < C; ++c)
                g[c] = fmaf(a[q][c], r, g[c]);
        }
        buf ^= 1;
    };
    // two register sets used alternately, without copies: one batch's loads
    // stay in flight while the other is summed (a third set, with two
    // batches in flight, measured 10 % slower: its registers cost more
    // occupancy than the deeper prefetch gains)
    float a0[RB][C], a1[RB][C];
    dense_load<C, RB>(A, i0, i1, d, t, a0);
    for (long i = i0; i < i1; i += 2 * RB) {
        dense_load<C, RB>(A, i + RB, i1, d, t, a1);
        sum_batch(a0, i);
        __builtin_amdgcn_sched_barrier(0);
        if (i + RB >= i1)
            break;
        dense_load<C, RB>(A, i + 2 * RB, i1, d, t, a0);
        sum_batch(a1, i + RB);
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j = c * kDT + t;
        if (j < d)
            parts[(size_t)blockIdx.x * d + j] = g[c];
    }
}

// parts2[by][j] = sum over row blocks b in [by*kSumRows, ...) of parts[b][j],
// in order.
__global__ __launch_bounds__(kDT) void k_dense_sum(const float *__restrict__ parts, int nb, int d,
                                                   float *__restrict__ parts2,
                                                   const int32_t *__restrict__ skip)
{
    if (dskip(skip))
        return;
    const int j = blockIdx.x * kDT + threadIdx.x;
    if (j >= d)
        return;
    const int b0 = blockIdx.y * kSumRows, b1 = min(nb, b0 + kSumRows);
    float s = 0.f;
    for (int b = b0; b < b1; ++b)
        s += parts[(size_t)b * d + j];
    parts2[(size_t)blockIdx.y * d + j] = s;
}

// g[j] = inv_n * sum over groups of parts2[by][j], in order.
__global__ __launch_bounds__(kDT) void k_dense_sum2(const float *__restrict__ parts2, int ng, int d,
                                                    float inv_n, float *__restrict__ g,
                                                    const int32_t *__restrict__ skip)
{
    if (dskip(skip))
        return;
    const int j = blockIdx.x * kDT + threadIdx.x;
    if (j >= d)
        return;
    float s = 0.f;
    for (int by = 0; by < ng; ++by)
        s += parts2[(size_t)by * d + j];
    g[j] = s * inv_n;
}

__device__ __forceinline__ double fin_sum(double v, double *lds)
{
    const int t = threadIdx.x;
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off);
    __syncthreads();
    if ((t & 63) == 0)
        lds[t >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kFinT / 64; ++w)
        s += lds[w];
    return s;
}

// One block, on g = F (the summed gradient).  mode 0: z = g.
// mode 1 (half step) / 2 (full step): z = P(x - gamma g) with P the ball of
// the given radius (radius <= 0: none); mode 1 also sets rho_t from
// ||z - x||, ||x|| in the state; mode 2 advances t and applies the stop
// test, as the CT finish does.  mode 3 (power iteration): u = g, then
// lam = <v,u>/<v,v>, v = u / ||u||.  Columns j = t + kFinT c.
__global__ __launch_bounds__(kFinT) void k_dense_finish(const float *__restrict__ g, int d,
                                                        int mode, const float *x, float gamma,
                                                        double radius, float *z, SolveState *st)
{
    if (mode != 0 && mode != 3 && st->done)
        return;
    __shared__ double lds[kFinT / 64];
    const int t = threadIdx.x;
    double zz = 0.0, vu = 0.0, vv = 0.0;
    for (int j = t; j < d; j += kFinT) {
        const float gj = g[j];
        if (mode == 0) {
            z[j] = gj;
        } else if (mode == 3) {
            const double xv = x[j];
            vu = fma(xv, (double)gj, vu);
            vv = fma(xv, xv, vv);
            zz = fma((double)gj, (double)gj, zz);
            z[j] = gj;
        } else {
            const float zj = fmaf(-gamma, gj, x[j]);
            z[j] = zj;
            zz = fma((double)zj, (double)zj, zz);
        }
    }
    if (mode == 0)
        return;
    if (mode == 3) {
        vu = fin_sum(vu, lds);
        vv = fin_sum(vv, lds);
        zz = fin_sum(zz, lds);
        __syncthreads();
        const double nrm = sqrt(zz);
        for (int j = t; j < d; j += kFinT)
            z[j] = nrm > 0.0 ? (float)(z[j] / nrm) : 0.f;
        if (t == 0) {
            st->lam = vv > 0.0 ? vu / vv : 0.0;
            st->unorm = nrm;
        }
        return;
    }
    zz = fin_sum(zz, lds);
    __syncthreads();
    const double nz = sqrt(zz);
    const float alpha = (radius > 0.0 && nz > radius) ? (float)(radius / nz) : 1.f;
    double num = 0.0, den = 0.0;
    for (int j = t; j < d; j += kFinT) {
        const float zj = alpha == 1.f ? z[j] : z[j] * alpha;
        z[j] = zj;
        if (mode == 1) {
            const double xv = x[j], dz = (double)zj - xv;
            num = fma(dz, dz, num);
            den = fma(xv, xv, den);
        }
    }
    if (mode == 1) {
        num = fin_sum(num, lds);
        __syncthreads();
        den = fin_sum(den, lds);
        if (t == 0)
            st->rho = den > 0.0 ? sqrt(num / den) : -1.0;
        return;
    }
    if (t == 0) {
        const int tt = st->t + 1;
        st->t = tt;
        const double rho = st->rho;
        if (st->tol > 0.0 && rho >= 0.0 && rho <= st->tol) {
            st->converged = 1;
            st->done = 1;
        } else if (tt >= st->max_iters) {
            st->done = 1;
        }
    }
}

}  // namespace

int dense_cols(int d)
{
    int C = 1;
    while (C * kDT < d)
        C *= 2;
    return C;
}

// Row blocks: one resident round of the streaming kernel (its register use
// allows 3 blocks per CU at 16 column chunks, 4 at 8, 8 below), at least
// 64 rows each.
int dense_blocks(long n, int d)
{
    const int C = dense_cols(d);
    const long cap = 256L * (C >= 16 ? 3 : (C == 8 ? 4 : 8));
    const long want = (n + 63) / 64;
    return (int)(want < 1 ? 1 : (want > cap ? cap : want));
}

int dense_sum_groups(long n, int d) { return (dense_blocks(n, d) + kSumRows - 1) / kSumRows; }

hipError_t launch_dense_F(const float *A, long n, int d, const float *x, const float *Y,
                          const float *J, const float *mu, int K, bool linear, float *parts,
                          float *parts2, float *g, const int32_t *skip, hipStream_t st)
{
    const int nb = dense_blocks(n, d);
    const long rpb = (n + nb - 1) / nb;
    const int C = dense_cols(d);
    const dim3 grid(nb), blk(kDT);
    const int lin = linear ? 1 : 0;
    switch (C) {
    case 1: hipLaunchKernelGGL(k_dense_F<1>, grid, blk, 0, st, A, n, d, x, Y, J, mu, K, lin, rpb, parts, skip); break;
    case 2: hipLaunchKernelGGL(k_dense_F<2>, grid, blk, 0, st, A, n, d, x, Y, J, mu, K, lin, rpb, parts, skip); break;
    case 4: hipLaunchKernelGGL(k_dense_F<4>, grid, blk, 0, st, A, n, d, x, Y, J, mu, K, lin, rpb, parts, skip); break;
    case 8: hipLaunchKernelGGL(k_dense_F<8>, grid, blk, 0, st, A, n, d, x, Y, J, mu, K, lin, rpb, parts, skip); break;
    case 16: hipLaunchKernelGGL(k_dense_F<16>, grid, blk, 0, st, A, n, d, x, Y, J, mu, K, lin, rpb, parts, skip); break;
    default: return hipErrorInvalidValue;
    }
    const int ng = dense_sum_groups(n, d);
    hipLaunchKernelGGL(k_dense_sum, dim3((d + kDT - 1) / kDT, ng), dim3(kDT), 0, st, parts, nb, d,
                       parts2, skip);
    hipLaunchKernelGGL(k_dense_sum2, dim3((d + kDT - 1) / kDT), dim3(kDT), 0, st, parts2, ng, d,
                       (float)(1.0 / (double)n), g, skip);
    return hipGetLastError();
}

hipError_t launch_dense_finish(const float *g, int d, int mode, const float *x, float gamma,
                               double radius, float *z, SolveState *state, hipStream_t st)
{
    hipLaunchKernelGGL(k_dense_finish, dim3(1), dim3(kFinT), 0, st, g, d, mode, x, gamma, radius,
                       z, state);
    return hipGetLastError();
}

}  // namespace exact
