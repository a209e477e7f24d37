// HIP kernels of the TV-ball and orthant projection (the constraint set of
// the paper's experiments, Sec. 5) for CDNA4 (gfx950, wave64).
//
// The TV-regularized point argmin ||x - b||^2 + lam TV(x) (eq.
// TV-regularization) is computed by fast gradient projection on the dual of
// TV denoising (Beck and Teboulle 2009): a fixed number of stencil steps on
// a pair of dual fields.  TV is the isotropic total variation with forward
// differences.  The binary search on lam and Dykstra's alternation with the
// orthant (eq. projection-intersection) are driven from the host, one
// captured graph per proximal solve.  Reductions are fixed-order doubles.
#include "exact_internal.h"

#include <algorithm>
#include <cmath>

namespace exact {
namespace {

constexpr int kTvX = 32, kTvY = 8;          // 256-thread stencil blocks
constexpr int kTvRed = 256;

// x = b - l L(r, s) at pixel (i, j):
// L(r, s)_ij = r_ij + s_ij - r_{i-1,j} - s_{i,j-1} (terms outside are 0).
__device__ __forceinline__ float primal_at(const float *__restrict__ b,
                                           const float *__restrict__ r,
                                           const float *__restrict__ s, float l, int N, int i,
                                           int j)
{
    const size_t c = (size_t)i * N + j;
    float L = r[c] + s[c];
    if (i > 0)
        L -= r[c - N];
    if (j > 0)
        L -= s[c - 1];
    return fmaf(-l, L, b[c]);
}

// FGP steps from the extrapolated dual point (r, s) to the new dual point
// (p, q) and the next extrapolated point, each
//   x = b - l L(r, s);  (p', q') = P_disc((r, s) + L^T(x) / (8 l));
//   (r, s) <- (p', q') + w_t ((p', q') - (p, q));  (p, q) <- (p', q'),
// with momentum weight w_t for step t.  L^T(x) = (x_ij - x_{i+1,j},
// x_ij - x_{i,j+1}); the last row of p and the last column of q stay zero.
// lam (device) is the TV weight; l = lam / 2.
//
// Temporal blocking: a step at a pixel reads the previous state within
// Chebyshev distance 1, so a workgroup that holds its 32 x 32 tile and a
// halo of kFgpHalo pixels in LDS (r, s, x) and registers (p, q, b) can take
// up to kFgpHalo steps before its tile's values depend on anything outside:
// after step t the cells within t of the region's edge are stale, the tile
// is not.  Pixels outside the image hold zero state.  Each step's arithmetic
// per pixel is the single-step formula's, so the result does not depend on
// the blocking.  The state is read from one set of fields and written to
// another (neighbouring workgroups read the halo).
constexpr int kFgpTile = 32, kFgpHalo = 8, kFgpReg = kFgpTile + 2 * kFgpHalo;
constexpr int kFgpThreads = 768;
constexpr int kFgpCells = kFgpReg * kFgpReg / kFgpThreads;
static_assert(kFgpReg * kFgpReg % kFgpThreads == 0, "region cells per thread");

struct FgpSteps {
    float w[kFgpHalo];   // momentum weight of each step of this launch
    int32_t n;           // steps, 1..kFgpHalo
};

__global__ __launch_bounds__(kFgpThreads) void k_fgp_steps(
    const float *__restrict__ b, const float *__restrict__ p, const float *__restrict__ q,
    const float *__restrict__ r, const float *__restrict__ s, float *__restrict__ po,
    float *__restrict__ qo, float *__restrict__ ro, float *__restrict__ so,
    const double *__restrict__ lam, FgpSteps W, int N)
{
    __shared__ float R[kFgpReg][kFgpReg + 1], S[kFgpReg][kFgpReg + 1], X[kFgpReg][kFgpReg + 1];
    const int i0 = blockIdx.y * kFgpTile - kFgpHalo, j0 = blockIdx.x * kFgpTile - kFgpHalo;
    const float l = (float)(*lam * 0.5);
    const float inv8l = (float)(1.0 / (8.0 * (*lam * 0.5)));
    float pc[kFgpCells], qc[kFgpCells], bc[kFgpCells];
#pragma unroll
    for (int c = 0; c < kFgpCells; ++c) {
        const int k = threadIdx.x + c * kFgpThreads;
        const int a = k / kFgpReg, e = k % kFgpReg, gi = i0 + a, gj = j0 + e;
        const bool in = gi >= 0 && gi < N && gj >= 0 && gj < N;
        const size_t g = in ? (size_t)gi * N + gj : 0;
        R[a][e] = in ? r[g] : 0.f;
        S[a][e] = in ? s[g] : 0.f;
        pc[c] = in ? p[g] : 0.f;
        qc[c] = in ? q[g] : 0.f;
        bc[c] = in ? b[g] : 0.f;
    }
    __syncthreads();
    for (int t = 0; t < W.n; ++t) {
        // x = b - l (r + s - r_up - s_left) on the whole region (terms beyond
        // the region's edge are taken as zero: those cells go stale)
#pragma unroll
        for (int c = 0; c < kFgpCells; ++c) {
            const int k = threadIdx.x + c * kFgpThreads;
            const int a = k / kFgpReg, e = k % kFgpReg;
            const float up = a > 0 ? R[a - 1][e] : 0.f, left = e > 0 ? S[a][e - 1] : 0.f;
            const float L = ((R[a][e] + S[a][e]) - up) - left;
            X[a][e] = fmaf(-l, L, bc[c]);
        }
        __syncthreads();
        const float w = W.w[t];
#pragma unroll
        for (int c = 0; c < kFgpCells; ++c) {
            const int k = threadIdx.x + c * kFgpThreads;
            const int a = k / kFgpReg, e = k % kFgpReg, gi = i0 + a, gj = j0 + e;
            const bool in = gi >= 0 && gi < N && gj >= 0 && gj < N;
            const float xc = X[a][e];
            float av = 0.f, bv = 0.f;
            if (gi + 1 < N && a + 1 < kFgpReg)
                av = fmaf(xc - X[a + 1][e], inv8l, R[a][e]);
            if (gj + 1 < N && e + 1 < kFgpReg)
                bv = fmaf(xc - X[a][e + 1], inv8l, S[a][e]);
            // projection onto the unit disc: (a, b) / max(|(a, b)|, 1), with
            // the hardware square root and reciprocal (1 ulp each; the
            // reciprocal is 1 exactly when the point is inside the disc)
            const float nrm = __builtin_amdgcn_sqrtf(fmaf(av, av, bv * bv));
            const float inv = __builtin_amdgcn_rcpf(fmaxf(nrm, 1.f));
            const float pn = in ? av * inv : 0.f, qn = in ? bv * inv : 0.f;
            // only this cell's r, s are read in this phase: update in place
            R[a][e] = fmaf(w, pn - pc[c], pn);
            S[a][e] = fmaf(w, qn - qc[c], qn);
            pc[c] = pn;
            qc[c] = qn;
        }
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < kFgpCells; ++c) {
        const int k = threadIdx.x + c * kFgpThreads;
        const int a = k / kFgpReg, e = k % kFgpReg, gi = i0 + a, gj = j0 + e;
        if (a < kFgpHalo || a >= kFgpHalo + kFgpTile || e < kFgpHalo || e >= kFgpHalo + kFgpTile)
            continue;
        if (gi >= N || gj >= N)
            continue;
        const size_t g = (size_t)gi * N + gj;
        po[g] = pc[c];
        qo[g] = qc[c];
        ro[g] = R[a][e];
        so[g] = S[a][e];
    }
}

// x = b - l L(p, q), the primal point of the final dual iterate.
__global__ __launch_bounds__(kTvX *kTvY) void k_fgp_final(const float *__restrict__ b,
                                                          const float *__restrict__ p,
                                                          const float *__restrict__ q,
                                                          const double *__restrict__ lam,
                                                          float *__restrict__ x, int N)
{
    const int j = blockIdx.x * kTvX + threadIdx.x;
    const int i = blockIdx.y * kTvY + threadIdx.y;
    if (i >= N || j >= N)
        return;
    x[(size_t)i * N + j] = primal_at(b, p, q, (float)(*lam * 0.5), N, i, j);
}

// Four fields set to zero (a fill kernel, so that a captured graph holds no
// memset node).
__global__ void k_zero4(float *__restrict__ a, float *__restrict__ b, float *__restrict__ c,
                        float *__restrict__ d, long n)
{
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n;
         k += (long)gridDim.x * blockDim.x) {
        a[k] = 0.f;
        b[k] = 0.f;
        c[k] = 0.f;
        d[k] = 0.f;
    }
}

__device__ __forceinline__ double block_sum1(double v, double *lds)
{
    const int t = threadIdx.x + threadIdx.y * blockDim.x;
    lds[t] = v;
    __syncthreads();
    for (int w = kTvRed / 2; w > 0; w >>= 1) {
        if (t < w)
            lds[t] += lds[t + w];
        __syncthreads();
    }
    return lds[0];
}

// Per-block double sums of |grad x| (isotropic, forward differences, zero
// across the last row and column).
__global__ __launch_bounds__(kTvX *kTvY) void k_tv_parts(const float *__restrict__ x, int N,
                                                         double *__restrict__ parts)
{
    __shared__ double red[kTvRed];
    const int j = blockIdx.x * kTvX + threadIdx.x;
    const int i = blockIdx.y * kTvY + threadIdx.y;
    double v = 0.0;
    if (i < N && j < N) {
        const size_t c = (size_t)i * N + j;
        const double xc = x[c];
        const double dx = j + 1 < N ? (double)x[c + 1] - xc : 0.0;
        const double dy = i + 1 < N ? (double)x[c + N] - xc : 0.0;
        v = sqrt(dx * dx + dy * dy);
    }
    v = block_sum1(v, red);
    if (threadIdx.x == 0 && threadIdx.y == 0)
        parts[blockIdx.y * gridDim.x + blockIdx.x] = v;
}

// out[0] = fixed-order sum of parts[0..n).
__global__ __launch_bounds__(kTvRed) void k_sum_finish(const double *__restrict__ parts, int n,
                                                       double *__restrict__ out)
{
    __shared__ double red[kTvRed];
    double v = 0.0;
    for (int k = threadIdx.x; k < n; k += kTvRed)
        v += parts[k];
    v = block_sum1(v, red);
    if (threadIdx.x == 0)
        out[0] = v;
}

// w = z + p.
__global__ void k_dyk_pre(const float *__restrict__ z, const float *__restrict__ p,
                          float *__restrict__ w, long d)
{
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < d;
         k += (long)gridDim.x * blockDim.x)
        w[k] = z[k] + p[k];
}

// One Dykstra round after y = P_TV(w), w = z + p:
// p = w - y; zn = max(0, y + q); q = y + q - zn; z = zn; and per-block
// double sums of (zn - z_old)^2.  Blocks of 256 cover d in a grid-stride
// loop, so the partial sums are in a fixed order.
__global__ __launch_bounds__(kTvRed) void k_dyk_post(const float *__restrict__ w,
                                                     const float *__restrict__ y,
                                                     float *__restrict__ p, float *__restrict__ q,
                                                     float *__restrict__ z, long d,
                                                     double *__restrict__ parts)
{
    __shared__ double red[kTvRed];
    double acc = 0.0;
    for (long k = blockIdx.x * (long)kTvRed + threadIdx.x; k < d; k += (long)gridDim.x * kTvRed) {
        const float yk = y[k], t = yk + q[k];
        const float zn = fmaxf(t, 0.f);
        p[k] = w[k] - yk;
        q[k] = t - zn;
        const double dz = (double)zn - (double)z[k];
        acc = fma(dz, dz, acc);
        z[k] = zn;
    }
    acc = block_sum1(acc, red);
    if (threadIdx.x == 0)
        parts[blockIdx.x] = acc;
}

// z = x - gamma g (the unprojected extragradient point).
__global__ void k_axpy(const float *__restrict__ x, const float *__restrict__ g, float gamma,
                       float *__restrict__ z, long d)
{
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < d;
         k += (long)gridDim.x * blockDim.x)
        z[k] = fmaf(-gamma, g[k], x[k]);
}

// Per-block double sums of (a - b)^2 and b^2.
__global__ __launch_bounds__(kTvRed) void k_diff2(const float *__restrict__ a,
                                                  const float *__restrict__ b, long d,
                                                  double *__restrict__ parts)
{
    __shared__ double red[kTvRed];
    double s0 = 0.0, s1 = 0.0;
    for (long k = blockIdx.x * (long)kTvRed + threadIdx.x; k < d; k += (long)gridDim.x * kTvRed) {
        const double bv = b[k], dv = (double)a[k] - bv;
        s0 = fma(dv, dv, s0);
        s1 = fma(bv, bv, s1);
    }
    s0 = block_sum1(s0, red);
    __syncthreads();
    s1 = block_sum1(s1, red);
    if (threadIdx.x == 0) {
        parts[2 * blockIdx.x] = s0;
        parts[2 * blockIdx.x + 1] = s1;
    }
}

__global__ __launch_bounds__(kTvRed) void k_sum2_finish(const double *__restrict__ parts, int n,
                                                        double *__restrict__ out)
{
    __shared__ double red[kTvRed];
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < n; k += kTvRed) {
        a += parts[2 * k];
        b += parts[2 * k + 1];
    }
    a = block_sum1(a, red);
    __syncthreads();
    b = block_sum1(b, red);
    if (threadIdx.x == 0) {
        out[0] = a;
        out[1] = b;
    }
}

dim3 tv_grid(int N) { return dim3((N + kTvX - 1) / kTvX, (N + kTvY - 1) / kTvY); }

int flat_blocks(long d)
{
    long b = (d + kTvRed * 4 - 1) / (kTvRed * 4);
    return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

}  // namespace

int num_tv_parts(int N)
{
    const dim3 g = tv_grid(N);
    return (int)(g.x * g.y);
}

int num_flat_parts(long d) { return flat_blocks(d); }

hipError_t launch_prox_graph_body(const float *b, float *p, float *q, float *r, float *s,
                                  float *p2, float *q2, float *r2, float *s2, const double *lam,
                                  int iters, float *x, int N, hipStream_t st)
{
    const long d = (long)N * N;
    hipLaunchKernelGGL(k_zero4, dim3(flat_blocks(d)), dim3(kTvRed), 0, st, p, q, r, s, d);
    const dim3 grid((N + kFgpTile - 1) / kFgpTile, (N + kFgpTile - 1) / kFgpTile);
    double t = 1.0;
    for (int k = 0; k < iters;) {
        FgpSteps W;
        W.n = std::min(kFgpHalo, iters - k);
        for (int u = 0; u < kFgpHalo; ++u)
            W.w[u] = 0.f;
        for (int u = 0; u < W.n; ++u) {
            const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
            W.w[u] = (float)((t - 1.0) / tn);
            t = tn;
        }
        hipLaunchKernelGGL(k_fgp_steps, grid, dim3(kFgpThreads), 0, st, b, p, q, r, s, p2, q2,
                           r2, s2, lam, W, N);
        std::swap(p, p2);
        std::swap(q, q2);
        std::swap(r, r2);
        std::swap(s, s2);
        k += W.n;
    }
    hipLaunchKernelGGL(k_fgp_final, tv_grid(N), dim3(kTvX, kTvY), 0, st, b, p, q, lam, x, N);
    return hipGetLastError();
}

hipError_t launch_tv_norm(const float *x, int N, double *parts, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_tv_parts, tv_grid(N), dim3(kTvX, kTvY), 0, st, x, N, parts);
    hipLaunchKernelGGL(k_sum_finish, dim3(1), dim3(kTvRed), 0, st, parts, num_tv_parts(N), out);
    return hipGetLastError();
}

hipError_t launch_dyk_pre(const float *z, const float *p, float *w, long d, hipStream_t st)
{
    hipLaunchKernelGGL(k_dyk_pre, dim3(flat_blocks(d)), dim3(kTvRed), 0, st, z, p, w, d);
    return hipGetLastError();
}

hipError_t launch_dyk_post(const float *w, const float *y, float *p, float *q, float *z, long d,
                           double *parts, double *out, hipStream_t st)
{
    const int nb = flat_blocks(d);
    hipLaunchKernelGGL(k_dyk_post, dim3(nb), dim3(kTvRed), 0, st, w, y, p, q, z, d, parts);
    hipLaunchKernelGGL(k_sum_finish, dim3(1), dim3(kTvRed), 0, st, parts, nb, out);
    return hipGetLastError();
}

hipError_t launch_axpy(const float *x, const float *g, float gamma, float *z, long d,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_axpy, dim3(flat_blocks(d)), dim3(kTvRed), 0, st, x, g, gamma, z, d);
    return hipGetLastError();
}

hipError_t launch_diff2(const float *a, const float *b, long d, double *parts, double *out,
                        hipStream_t st)
{
    const int nb = flat_blocks(d);
    hipLaunchKernelGGL(k_diff2, dim3(nb), dim3(kTvRed), 0, st, a, b, d, parts);
    hipLaunchKernelGGL(k_sum2_finish, dim3(1), dim3(kTvRed), 0, st, parts, nb, out);
    return hipGetLastError();
}

}  // namespace exact
