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

// Fixed-order sum of the kTvRed threads' v (every thread gets it).
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

// FGP steps from the extrapolated dual point (r, s) to the new dual point
// (p, q) and the next extrapolated point, each
//   x = b - l L(r, s);  (p', q') = P_disc((r, s) + L^T(x) / (8 l));
//   (r, s) <- (p', q') + w_t ((p', q') - (p, q));  (p, q) <- (p', q'),
// with momentum weight w_t for step t.  L^T(x) = (x_ij - x_{i+1,j},
// x_ij - x_{i,j+1}); the last row of p and the last column of q stay zero.
// lam is the TV weight; l = lam / 2.
//
// Temporal blocking: a step at a pixel reads the previous state within
// Chebyshev distance 1, so a workgroup that holds its 32 x 32 tile and a
// halo of kFgpHalo pixels can take up to kFgpHalo steps before its tile's
// values depend on anything outside: after step t the cells within t of the
// region's edge are stale, the tile is not.  Pixels outside the image hold
// zero state.  Each step's arithmetic per pixel is the single-step
// formula's, so the result does not depend on the blocking.  The state is
// read from one set of fields and written to another (neighbouring
// workgroups read the halo).
//
// A thread owns kFgpCells cells of the region and keeps their whole state
// (p, q, r, s, b and the step's x) in registers; r, s and x also go to LDS
// for the neighbours' reads.  The LDS fields carry a zero border, so that
// the up and left neighbours of the region's first row and column read the
// zeros the formula takes there, and the reads need no branch; the down and
// right neighbours beyond the region are read from the border and masked.
constexpr int kFgpTile = 32, kFgpHalo = 8, kFgpReg = kFgpTile + 2 * kFgpHalo;
constexpr int kFgpLd = kFgpReg + 2;       // LDS row: a border cell on each side
constexpr int kFgpThreads = 768;
constexpr int kFgpCells = kFgpReg * kFgpReg / kFgpThreads;
static_assert(kFgpReg * kFgpReg % kFgpThreads == 0, "region cells per thread");

struct FgpSteps {
    float w[kFgpHalo];   // momentum weight of each step of this launch
    int32_t n;           // steps, 1..kFgpHalo
    int32_t zero;        // the dual state starts at zero (p, q, r, s are not read)
};

__global__ __launch_bounds__(kFgpThreads) void k_fgp_steps(
    const float *__restrict__ b, const float *__restrict__ p, const float *__restrict__ q,
    const float *__restrict__ r, const float *__restrict__ s, float *__restrict__ po,
    float *__restrict__ qo, float *__restrict__ ro, float *__restrict__ so, double lam,
    FgpSteps W, int N)
{
    // region cell (a, e) at [a + 1][e + 1]; rows 0 and kFgpLd - 1 and
    // columns 0 and kFgpLd - 1 stay zero
    __shared__ float R[kFgpLd][kFgpLd], S[kFgpLd][kFgpLd], X[kFgpLd][kFgpLd];
    const int i0 = blockIdx.y * kFgpTile - kFgpHalo, j0 = blockIdx.x * kFgpTile - kFgpHalo;
    const float l = (float)(lam * 0.5);
    const float inv8l = (float)(1.0 / (8.0 * (lam * 0.5)));
    for (int k = threadIdx.x; k < 4 * kFgpLd; k += kFgpThreads) {
        const int side = k / kFgpLd, m = k % kFgpLd;
        const int a = side == 0 ? 0 : side == 1 ? kFgpLd - 1 : m;
        const int e = side == 0 || side == 1 ? m : side == 2 ? 0 : kFgpLd - 1;
        R[a][e] = 0.f;
        S[a][e] = 0.f;
        X[a][e] = 0.f;
    }
    float pc[kFgpCells], qc[kFgpCells], bc[kFgpCells], rc[kFgpCells], sc[kFgpCells];
    float xc[kFgpCells];
    int ca[kFgpCells], ce[kFgpCells];       // LDS row and column of the cell
    bool in[kFgpCells], dn[kFgpCells], rt[kFgpCells];
#pragma unroll
    for (int c = 0; c < kFgpCells; ++c) {
        const int k = threadIdx.x + c * kFgpThreads;
        const int a = k / kFgpReg, e = k % kFgpReg, gi = i0 + a, gj = j0 + e;
        ca[c] = a + 1;
        ce[c] = e + 1;
        in[c] = gi >= 0 && gi < N && gj >= 0 && gj < N;
        dn[c] = gi + 1 < N && a + 1 < kFgpReg;    // the pixel below exists and is in the region
        rt[c] = gj + 1 < N && e + 1 < kFgpReg;    // likewise the pixel to the right
        const size_t g = in[c] ? (size_t)gi * N + gj : 0;
        const bool ld = in[c] && !W.zero;
        rc[c] = ld ? r[g] : 0.f;
        sc[c] = ld ? s[g] : 0.f;
        pc[c] = ld ? p[g] : 0.f;
        qc[c] = ld ? q[g] : 0.f;
        bc[c] = in[c] ? b[g] : 0.f;
        R[ca[c]][ce[c]] = rc[c];
        S[ca[c]][ce[c]] = sc[c];
    }
    __syncthreads();
    for (int t = 0; t < W.n; ++t) {
        // x = b - l (r + s - r_up - s_left) on the whole region (terms beyond
        // the region's edge are taken as zero: those cells go stale)
        float up[kFgpCells], left[kFgpCells];
#pragma unroll
        for (int c = 0; c < kFgpCells; ++c) {
            up[c] = R[ca[c] - 1][ce[c]];
            left[c] = S[ca[c]][ce[c] - 1];
        }
#pragma unroll
        for (int c = 0; c < kFgpCells; ++c) {
            const float L = ((rc[c] + sc[c]) - up[c]) - left[c];
            xc[c] = fmaf(-l, L, bc[c]);
            X[ca[c]][ce[c]] = xc[c];
        }
        __syncthreads();
        const float w = W.w[t];
        float xd[kFgpCells], xr[kFgpCells];
#pragma unroll
        for (int c = 0; c < kFgpCells; ++c) {
            xd[c] = X[ca[c] + 1][ce[c]];
            xr[c] = X[ca[c]][ce[c] + 1];
        }
#pragma unroll
        for (int c = 0; c < kFgpCells; ++c) {
            const float av = dn[c] ? fmaf(xc[c] - xd[c], inv8l, rc[c]) : 0.f;
            const float bv = rt[c] ? fmaf(xc[c] - xr[c], inv8l, sc[c]) : 0.f;
            // projection onto the unit disc: (a, b) / max(|(a, b)|, 1), with
            // the hardware square root and reciprocal (1 ulp each; the
            // reciprocal is 1 exactly when the point is inside the disc)
            const float nrm = __builtin_amdgcn_sqrtf(fmaf(av, av, bv * bv));
            const float inv = __builtin_amdgcn_rcpf(fmaxf(nrm, 1.f));
            const float pn = in[c] ? av * inv : 0.f, qn = in[c] ? bv * inv : 0.f;
            rc[c] = fmaf(w, pn - pc[c], pn);
            sc[c] = fmaf(w, qn - qc[c], qn);
            pc[c] = pn;
            qc[c] = qn;
            // only this cell's r, s are written in this phase, and no cell's
            // r, s are read in it
            R[ca[c]][ce[c]] = rc[c];
            S[ca[c]][ce[c]] = sc[c];
        }
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < kFgpCells; ++c) {
        const int a = ca[c] - 1, e = ce[c] - 1, gi = i0 + a, gj = j0 + e;
        if (a < kFgpHalo || a >= kFgpHalo + kFgpTile || e < kFgpHalo || e >= kFgpHalo + kFgpTile)
            continue;
        if (gi >= N || gj >= N)
            continue;
        const size_t g = (size_t)gi * N + gj;
        po[g] = pc[c];
        qo[g] = qc[c];
        ro[g] = rc[c];
        so[g] = sc[c];
    }
}

// x = b - l L(p, q), the primal point of the final dual iterate, and
// per-block double sums of |grad x| as k_tv_parts forms them (the
// neighbours' x recomputed by the same formula: the same floats).
__global__ __launch_bounds__(kTvX *kTvY) void k_fgp_final(const float *__restrict__ b,
                                                          const float *__restrict__ p,
                                                          const float *__restrict__ q,
                                                          double lam, float *__restrict__ x,
                                                          int N, double *__restrict__ parts)
{
    __shared__ double red[kTvRed];
    const int j = blockIdx.x * kTvX + threadIdx.x;
    const int i = blockIdx.y * kTvY + threadIdx.y;
    const float l = (float)(lam * 0.5);
    double v = 0.0;
    if (i < N && j < N) {
        const float xv = primal_at(b, p, q, l, N, i, j);
        x[(size_t)i * N + j] = xv;
        const double xc = xv;
        const double dx = j + 1 < N ? (double)primal_at(b, p, q, l, N, i, j + 1) - xc : 0.0;
        const double dy = i + 1 < N ? (double)primal_at(b, p, q, l, N, i + 1, j) - xc : 0.0;
        v = sqrt(dx * dx + dy * dy);
    }
    v = block_sum1(v, red);
    if (threadIdx.x == 0 && threadIdx.y == 0)
        parts[blockIdx.y * gridDim.x + blockIdx.x] = v;
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

// After a finish kernel's results: with flag not null, seq to *flag, ordered
// after the results at system scope, so that a host polling pinned memory
// for seq can read the results as soon as it sees it.
__device__ __forceinline__ void post_seq(unsigned *flag, unsigned seq)
{
    if (flag) {
        __threadfence_system();
        __hip_atomic_store(flag, seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// out[0] = fixed-order sum of parts[0..n); then post_seq.
__global__ __launch_bounds__(kTvRed) void k_sum_finish(const double *__restrict__ parts, int n,
                                                       double *__restrict__ out, unsigned *flag,
                                                       unsigned seq)
{
    __shared__ double red[kTvRed];
    double v = 0.0;
    for (int k = threadIdx.x; k < n; k += kTvRed)
        v += parts[k];
    v = block_sum1(v, red);
    if (threadIdx.x == 0) {
        out[0] = v;
        post_seq(flag, seq);
    }
}

// w = z + p, and per-block double sums of |grad w| as k_tv_parts forms
// them (the neighbours' w recomputed from z and p: the same floats).
__global__ __launch_bounds__(kTvX *kTvY) void k_dyk_pre(const float *__restrict__ z,
                                                        const float *__restrict__ p, int N,
                                                        float *__restrict__ w,
                                                        double *__restrict__ parts)
{
    __shared__ double red[kTvRed];
    const int j = blockIdx.x * kTvX + threadIdx.x;
    const int i = blockIdx.y * kTvY + threadIdx.y;
    double v = 0.0;
    if (i < N && j < N) {
        const size_t c = (size_t)i * N + j;
        const float wc = z[c] + p[c];
        w[c] = wc;
        const double xc = wc;
        const double dx = j + 1 < N ? (double)(z[c + 1] + p[c + 1]) - xc : 0.0;
        const double dy = i + 1 < N ? (double)(z[c + N] + p[c + N]) - xc : 0.0;
        v = sqrt(dx * dx + dy * dy);
    }
    v = block_sum1(v, red);
    if (threadIdx.x == 0 && threadIdx.y == 0)
        parts[blockIdx.y * gridDim.x + blockIdx.x] = v;
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

// out[0..1] = fixed-order sums of parts[2k] and parts[2k + 1]; then post_seq.
__global__ __launch_bounds__(kTvRed) void k_sum2_finish(const double *__restrict__ parts, int n,
                                                        double *__restrict__ out, unsigned *flag,
                                                        unsigned seq)
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
        post_seq(flag, seq);
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

hipError_t launch_prox(const float *b, float *p, float *q, float *r, float *s, float *p2,
                       float *q2, float *r2, float *s2, double lam, int iters, float *x, int N,
                       double *parts, double *out, hipStream_t st, unsigned *flag, unsigned seq)
{
    const dim3 grid((N + kFgpTile - 1) / kFgpTile, (N + kFgpTile - 1) / kFgpTile);
    double t = 1.0;
    for (int k = 0; k < iters;) {
        FgpSteps W;
        W.n = std::min(kFgpHalo, iters - k);
        W.zero = k == 0;
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
    hipLaunchKernelGGL(k_fgp_final, tv_grid(N), dim3(kTvX, kTvY), 0, st, b, p, q, lam, x, N,
                       parts);
    hipLaunchKernelGGL(k_sum_finish, dim3(1), dim3(kTvRed), 0, st, parts, num_tv_parts(N), out,
                       flag, seq);
    return hipGetLastError();
}

hipError_t launch_tv_norm(const float *x, int N, double *parts, double *out, hipStream_t st,
                          unsigned *flag, unsigned seq)
{
    hipLaunchKernelGGL(k_tv_parts, tv_grid(N), dim3(kTvX, kTvY), 0, st, x, N, parts);
    hipLaunchKernelGGL(k_sum_finish, dim3(1), dim3(kTvRed), 0, st, parts, num_tv_parts(N), out,
                       flag, seq);
    return hipGetLastError();
}

hipError_t launch_dyk_pre(const float *z, const float *p, float *w, int N, double *parts,
                          double *out, hipStream_t st, unsigned *flag, unsigned seq)
{
    hipLaunchKernelGGL(k_dyk_pre, tv_grid(N), dim3(kTvX, kTvY), 0, st, z, p, N, w, parts);
    hipLaunchKernelGGL(k_sum_finish, dim3(1), dim3(kTvRed), 0, st, parts, num_tv_parts(N), out,
                       flag, seq);
    return hipGetLastError();
}

hipError_t launch_dyk_post(const float *w, const float *y, float *p, float *q, float *z, long d,
                           double *parts, double *out, hipStream_t st, unsigned *flag,
                           unsigned seq)
{
    const int nb = flat_blocks(d);
    hipLaunchKernelGGL(k_dyk_post, dim3(nb), dim3(kTvRed), 0, st, w, y, p, q, z, d, parts);
    hipLaunchKernelGGL(k_sum_finish, dim3(1), dim3(kTvRed), 0, st, parts, nb, out, flag, seq);
    return hipGetLastError();
}

hipError_t launch_axpy(const float *x, const float *g, float gamma, float *z, long d,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_axpy, dim3(flat_blocks(d)), dim3(kTvRed), 0, st, x, g, gamma, z, d);
    return hipGetLastError();
}

hipError_t launch_diff2(const float *a, const float *b, long d, double *parts, double *out,
                        hipStream_t st, unsigned *flag, unsigned seq)
{
    const int nb = flat_blocks(d);
    hipLaunchKernelGGL(k_diff2, dim3(nb), dim3(kTvRed), 0, st, a, b, d, parts);
    hipLaunchKernelGGL(k_sum2_finish, dim3(1), dim3(kTvRed), 0, st, parts, nb, out, flag, seq);
    return hipGetLastError();
}

}  // namespace exact
