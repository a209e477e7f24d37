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

// One FGP step: from the extrapolated dual point (r, s) to the new dual
// point (p, q) (in place: each lane owns its pixel's p, q) and the next
// extrapolated point (r2, s2) with momentum weight w:
//   x = b - l L(r, s);  (p', q') = P_disc((r, s) + L^T(x) / (8 l));
//   (r2, s2) = (p', q') + w ((p', q') - (p, q)).
// L^T(x) = (x_ij - x_{i+1,j}, x_ij - x_{i,j+1}); the last row of p and the
// last column of q stay zero.  lam (device) is the TV weight; l = lam / 2.
//
// A 32 x 8 block stages r (one row above), s (one column left) and b for its
// tile plus one row below and one column right in LDS (zeros outside the
// image), forms x on that extended tile, then updates its own pixels.
__global__ __launch_bounds__(kTvX *kTvY) void k_fgp_step(
    const float *__restrict__ b, const float *__restrict__ r, const float *__restrict__ s,
    float *__restrict__ p, float *__restrict__ q, float *__restrict__ r2,
    float *__restrict__ s2, const double *__restrict__ lam, float w, int N)
{
    constexpr int RY = kTvY + 2, RX = kTvX + 1;     // r: rows i0-1 .. i0+8
    constexpr int SY = kTvY + 1, SX = kTvX + 2;     // s: cols j0-1 .. j0+32
    constexpr int XY = kTvY + 1, XX = kTvX + 1;     // b, x: tile + 1 row + 1 column
    __shared__ float Rl[RY][RX], Sl[SY][SX], Bl[XY][XX], Xl[XY][XX];
    const int tid = threadIdx.x + threadIdx.y * kTvX;
    const int i0 = blockIdx.y * kTvY, j0 = blockIdx.x * kTvX;
    const float l = (float)(*lam * 0.5);
    const float inv8l = (float)(1.0 / (8.0 * (*lam * 0.5)));
    for (int k = tid; k < RY * RX; k += kTvX * kTvY) {
        const int gi = i0 - 1 + k / RX, gj = j0 + k % RX;
        Rl[k / RX][k % RX] = (gi >= 0 && gi < N && gj < N) ? r[(size_t)gi * N + gj] : 0.f;
    }
    for (int k = tid; k < SY * SX; k += kTvX * kTvY) {
        const int gi = i0 + k / SX, gj = j0 - 1 + k % SX;
        Sl[k / SX][k % SX] = (gi < N && gj >= 0 && gj < N) ? s[(size_t)gi * N + gj] : 0.f;
    }
    for (int k = tid; k < XY * XX; k += kTvX * kTvY) {
        const int gi = i0 + k / XX, gj = j0 + k % XX;
        Bl[k / XX][k % XX] = (gi < N && gj < N) ? b[(size_t)gi * N + gj] : 0.f;
    }
    __syncthreads();
    // x = b - l (r + s - r_up - s_left) on the extended tile
    for (int k = tid; k < XY * XX; k += kTvX * kTvY) {
        const int a = k / XX, c = k % XX;
        const float L = ((Rl[a + 1][c] + Sl[a][c + 1]) - Rl[a][c]) - Sl[a][c];
        Xl[a][c] = fmaf(-l, L, Bl[a][c]);
    }
    __syncthreads();
    const int i = i0 + threadIdx.y, j = j0 + threadIdx.x;
    if (i >= N || j >= N)
        return;
    const int ty = threadIdx.y, tx = threadIdx.x;
    const float xc = Xl[ty][tx];
    float av = 0.f, bv = 0.f;
    if (i + 1 < N)
        av = fmaf(xc - Xl[ty + 1][tx], inv8l, Rl[ty + 1][tx]);
    if (j + 1 < N)
        bv = fmaf(xc - Xl[ty][tx + 1], inv8l, Sl[ty][tx + 1]);
    const float nrm = sqrtf(fmaf(av, av, bv * bv));
    const float den = fmaxf(nrm, 1.f);
    const float pn = av / den, qn = bv / den;
    const size_t c = (size_t)i * N + j;
    const float po = p[c], qo = q[c];
    p[c] = pn;
    q[c] = qn;
    r2[c] = fmaf(w, pn - po, pn);
    s2[c] = fmaf(w, qn - qo, qn);
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
                                  float *r2, float *s2, const double *lam, int iters, float *x,
                                  int N, hipStream_t st)
{
    const long d = (long)N * N;
    hipLaunchKernelGGL(k_zero4, dim3(flat_blocks(d)), dim3(kTvRed), 0, st, p, q, r, s, d);
    double t = 1.0;
    for (int k = 0; k < iters; ++k) {
        const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
        const float w = (float)((t - 1.0) / tn);
        hipLaunchKernelGGL(k_fgp_step, tv_grid(N), dim3(kTvX, kTvY), 0, st, b, r, s, p, q, r2,
                           s2, lam, w, N);
        std::swap(r, r2);
        std::swap(s, s2);
        t = tn;
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
