// HIP kernels of libexact for CDNA4 (gfx950, wave64).
//
// Joseph forward projector with the polychromatic residual fused in, the
// gather back-projector that applies the identical transposed weights, the
// projected extragradient update and the double-precision reductions behind
// the step size and the stop test.  Everything here is deterministic: no
// atomics, fixed summation orders.
#include "exact_internal.h"

#include <cmath>

namespace exact {
namespace {

constexpr int kFwdThreads = 64;     // one wave: 64 consecutive bins of a view
constexpr int kBackX = 16, kBackY = 16;
constexpr int kRedThreads = 256;

__device__ __forceinline__ bool skipped(const int32_t *skip)
{
    return skip != nullptr && *skip != 0;
}

// Kahan-compensated accumulation.
struct Kahan {
    float s = 0.f, c = 0.f;
    __device__ __forceinline__ void add(float t)
    {
        const float y = t - c;
        const float u = s + y;
        c = (u - s) - y;
        s = u;
    }
    __device__ __forceinline__ float value() const { return s - c; }
};

// Fixed-order sum of one double per thread over kRedThreads threads (the
// x-y plane of the block); threads with active = false (other z planes)
// only take part in the barriers.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*lds)[kRedThreads],
                                          bool active = true)
{
    const int t = threadIdx.x + threadIdx.y * blockDim.x;
    if (active) {
#pragma unroll
        for (int q = 0; q < NV; ++q)
            lds[q][t] = v[q];
    }
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if (active && t < w) {
#pragma unroll
            for (int q = 0; q < NV; ++q)
                lds[q][t] += lds[q][t + w];
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < NV; ++q)
        v[q] = lds[q][0];
}

// 1.5 * 2^52: adding it to a double x with |x| < 2^31 rounds x to the
// nearest integer (ties to even) and leaves that integer, in two's
// complement, in the low 32 bits of the sum.
constexpr double kRoundMagic = 6755399441055744.0;

__device__ __forceinline__ int low_int(double m)
{
    return __double2loint(m);
}

// min(max(v, kLo), hi) for kLo <= hi in one instruction (the compiler
// forms v_med3_i32 only for constant bounds).
template <int kLo>
__device__ __forceinline__ int clamp_int(int v, int hi)
{
    int r;
    asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(v), "n"(kLo), "v"(hi));
    return r;
}

// Fixed-order sum over the kRedThreads threads of the block's x-y plane
// with one barrier: a butterfly within each wave, then the four wave sums in
// order.  Threads with active = false (other z planes) contribute nothing
// and only take part in the barrier; every thread gets the sum.
template <int NV>
__device__ __forceinline__ void plane_sum(double (&v)[NV], double (*lds)[kRedThreads / 64],
                                          bool active)
{
    const int t = threadIdx.x + threadIdx.y * blockDim.x;
#pragma unroll
    for (int q = 0; q < NV; ++q)
        for (int off = 32; off > 0; off >>= 1)
            v[q] += __shfl_xor(v[q], off);
    if (active && (t & 63) == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q)
            lds[q][t >> 6] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = 0.0;
        for (int w = 0; w < kRedThreads / 64; ++w)
            s += lds[q][w];
        v[q] = s;
    }
}

// Fixed-order reduction of a run's update partials, rho_t, and the stop test
// (with stop_mode 1 also the averaged-iterate partials and their criterion).
// With kGated it runs only while a finish is pending (the single-scan path,
// where the next step's first kernel or the host settles it) and clears the
// flag; the batched path runs it unconditionally after every step.
//
// The summation order is that of kRedThreads virtual lanes and does not
// depend on the launching block's size kThreads (a 1-D block, a multiple
// of 64 threads): virtual lane l adds partials l, l + kRedThreads, ... in
// that order (eight loads in flight at a time), a butterfly sums each 64
// consecutive virtual lanes, and the four group sums are added in order.
// A block of kThreads < kRedThreads threads runs kRedThreads / kThreads
// virtual lanes per thread; in a larger block the threads past
// kRedThreads only take part in the barrier.  So the result is bitwise the
// same wherever the finish runs (the forward's last workgroup, the host's
// settle kernel, the batched finish) and whatever the forward's tile knobs.
template <bool kGated, int kThreads>
__device__ __forceinline__ void finish_block(const double *__restrict__ partials, int nparts,
                                             const double *__restrict__ avg_parts, int n_avg,
                                             SolveState *st)
{
    static_assert(kThreads % 64 == 0 &&
                      (kThreads >= kRedThreads || kRedThreads % kThreads == 0),
                  "finish_block: block size");
    constexpr int kSets = kThreads >= kRedThreads ? 1 : kRedThreads / kThreads;
    if (st->done || (kGated && !st->pending))
        return;
    __shared__ double red[3][kRedThreads / 64];
    const int t = threadIdx.x;
#pragma unroll
    for (int set = 0; set < kSets; ++set) {
        const int l = t + set * kThreads;           // virtual lane
        const bool active = l < kRedThreads;
        double v3[3] = {0.0, 0.0, 0.0};
        // an absent partial adds +0.0: the sums are of squares, so this
        // changes no bit
        constexpr int kU = 8;
        if (active) {
            for (int q0 = l; q0 < nparts; q0 += kU * kRedThreads) {
                double a[kU], b[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int q = q0 + u * kRedThreads;
                    a[u] = q < nparts ? partials[2 * q] : 0.0;
                    b[u] = q < nparts ? partials[2 * q + 1] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    v3[0] += a[u];
                    v3[1] += b[u];
                }
            }
            for (int q0 = l; q0 < n_avg; q0 += kU * kRedThreads) {
                double a[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int q = q0 + u * kRedThreads;
                    a[u] = q < n_avg ? avg_parts[q] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < kU; ++u)
                    v3[2] += a[u];
            }
        }
        // every lane of the wave takes part in the butterfly; the group's
        // first lane keeps the sum in the group's fixed order
#pragma unroll
        for (int q = 0; q < 3; ++q)
            for (int off = 32; off > 0; off >>= 1)
                v3[q] += __shfl_xor(v3[q], off);
        if (active && (l & 63) == 0) {
#pragma unroll
            for (int q = 0; q < 3; ++q)
                red[q][l >> 6] = v3[q];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double v3[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            double s = 0.0;
            for (int w = 0; w < kRedThreads / 64; ++w)
                s += red[q][w];
            v3[q] = s;
        }
        const double rho = v3[1] > 0.0 ? sqrt(v3[0] / v3[1]) : -1.0;
        const int tt = st->t + 1;
        st->rho = rho;
        st->t = tt;
        bool met;
        if (st->stop_mode == 1) {
            const double crit = sqrt(v3[2]);
            st->crit = crit;
            met = crit <= st->tol;
        } else {
            met = rho >= 0.0 && rho <= st->tol;
        }
        if (st->tol > 0.0 && met) {
            st->converged = 1;
            st->done = 1;
        } else if (tt >= st->max_iters) {
            st->done = 1;
        }
        if (kGated)
            st->pending = 0;
    }
}

// ---------------------------------------------------------------- forward

constexpr int kSegs = kFwdSegs;   // waves per forward workgroup, each a share of the lines
static_assert(kFwdRays == 2 * kFwdThreads, "a forward lane takes two rays");
static_assert(kSegs % 2 == 0 && kSegs >= 2, "the epilogue pairs the waves");
// The residual's energies of one ray are split over kEPhase waves.
constexpr int kEPhase = kSegs / 2;

// Bin block of rank r when the blocks of a view are taken centre-out (the
// central blocks hold the longest chords): c, c-1, c+1, c-2, ... with
// c = nbb / 2.  A bijection of [0, nbb).
__device__ __host__ __forceinline__ int centre_out(int r, int nbb)
{
    const int c = nbb / 2;
    return (r % 2 == 0) ? c + r / 2 : c - (r + 1) / 2;
}

#ifndef EXACT_VIEW_BATCH
#define EXACT_VIEW_BATCH 4
#endif
constexpr int kLineBatch = kFwdLineBatch;      // lines whose loads are in flight together
constexpr int kViewBatch = EXACT_VIEW_BATCH;   // views likewise in the back-projector

// Element i of a float array through a 32-bit byte offset: with a
// wave-uniform base this is a scalar-base + vector-offset load.
__device__ __forceinline__ float at(const float *__restrict__ base, unsigned i)
{
    return *(const float *)((const char *)base + (i << 2));
}

// A forward lane takes two adjacent rays of a view.  On every line the ray
// with the lower crossing (in columns) is at flo and the other at fhi =
// flo + |P|, both advanced exactly by Q per line (kMode 2 keeps both; kMode
// 0 and 1 keep flo only and derive the other, below).  The crossings lie on
// the 2^-32 grid with |f| < 2^20, so the lane holds them as 64-bit integers
// F = f 2^32: the high word is floor(f) and the low word is 2^32 (f -
// floor(f)), and F += Q 2^32 is exact.  Each ray's taps are the single-ray
// rule's: columns floor(f) and floor(f) + 1 with weights (float)(1 - e) and
// (float)e, e = f - floor(f), the column clamped into the padded row (every
// crossing with a tap inside the image has f >= 1; any other reads padding
// zeros, as do lines the ray does not reach).  The lane forms the weights
// times 2^32, (float)(2^32 - lo) and (float)lo: the exact values rounded
// once, so each is the unit weight times 2^32 exactly, and the ray's sums
// carry that factor until forward_pair_end removes it (every step of the
// sums scales exactly).
//
// kMode 0 (|P| < 1) and 1 (1 <= |P| < 2): the four taps lie in the four
// columns c .. c + 3 from the lower ray's column c, which one 16-byte load
// (at a 4-byte-aligned address) reads.  The lane keeps only the lower
// crossing: with |P| 2^32 = kMode 2^32 + p (p < 2^32), the upper ray's low
// word is lo + p mod 2^32 and its column is c + d, d = kMode + the carry of
// that add, so the carry selects between the two offsets.  If c is clamped
// (floor(f) < 0 or floor(f) > cmax), both rays' taps lie in the padding, and
// the columns c + d, c + d + 1 read in place of the upper ray's are padding
// too (at the row's start kPadX >= 3 zero columns; at its end the last two
// padded columns and the next row's first, or the buffer's zero tail).  An
// unclamped c whose upper ray passes cmax reads the same padding columns
// the clamped column would.
// Lanes read neighbouring columns, and this one load serves two rays: the
// address unit takes about a third less time per tap than with one 8-byte
// load per ray (measured on MI355X with the forward's access pattern).
// kMode 2 (|P| >= 2): one 8-byte load per ray.
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));   // 4-byte aligned
typedef float f2u __attribute__((ext_vector_type(2), aligned(4)));

struct PairTaps {
    float l0, l1, h0, h1;   // weights times 2^32: lower ray, upper ray
    // modes 0, 1: columns c .. c + 3; mode 2: lower pair, upper pair (one
    // vector, so that the loop-carried set stays one register tuple)
    f4 v;
    bool up;                // modes 0, 1: d = kMode + 1
};

// x 2^32 as a 64-bit integer, for x on the 2^-32 grid with |x| < 2^20 (exact).
__device__ __forceinline__ long long fixed32(double x)
{
    return (long long)(x * 4294967296.0);
}

// (float)(2^32 - w) for a low word w = 2^32 e: the weight 1 - e times 2^32,
// rounded once.  For w > 0 the exact value is the 32-bit integer -w, whose
// conversion rounds to nearest even as the float cast of the real does; w =
// 0 gives 2^32 exactly.
__device__ __forceinline__ float weight_lo(unsigned w)
{
    unsigned n;
    const bool borrow = __builtin_usub_overflow(0u, w, &n);   // w > 0
    return borrow ? (float)n : 4294967296.0f;
}

template <int kMode>
__device__ __forceinline__ void pair_fetch(long long &flo, long long &fhi, unsigned pfrac,
                                           int cmax, long long Q,
                                           const float *__restrict__ img, int rowoff,
                                           PairTaps &t)
{
    const unsigned elo = (unsigned)flo;                        // 2^32 (f - floor(f))
    const int clo = clamp_int<0>((int)(flo >> 32), cmax);     // floor(f), clamped
    unsigned ehi;
    int chi = 0;
    if (kMode < 2) {
        t.up = __builtin_uadd_overflow(elo, pfrac, &ehi);     // upper ray: d = kMode + carry
    } else {
        ehi = (unsigned)fhi;
        chi = clamp_int<0>((int)(fhi >> 32), cmax);
        t.up = false;
        fhi += Q;
    }
    flo += Q;                                                  // exact
    // one running crossing per ray (kept opaque: otherwise the compiler
    // forms every unrolled line's crossing from the first and keeps them all
    // live)
    if (kMode < 2)
        asm("" : "+v"(flo));
    else
        asm("" : "+v"(flo), "+v"(fhi));
    t.l0 = weight_lo(elo);                                     // 2^32 (1 - e), rounded once
    t.l1 = (float)elo;                                         // 2^32 e, rounded once
    t.h0 = weight_lo(ehi);
    t.h1 = (float)ehi;
    const unsigned i = (unsigned)(rowoff + clo);
    if (kMode < 2) {
        const float *p = (const float *)((const char *)img + (i << 2));
        t.v = *(const f4u *)p;
    } else {
        const unsigned j = (unsigned)(rowoff + chi);
        const f2u a = *(const f2u *)((const char *)img + (i << 2));
        const f2u b = *(const f2u *)((const char *)img + (j << 2));
        t.v = f4{a.x, a.y, b.x, b.y};
    }
}

// Adds the line's contributions: s += w1 v1 + w0 v0 (as fma(w1, v1,
// fma(w0, v0, s))) for each ray.
template <int kMode>
__device__ __forceinline__ void pair_apply(const PairTaps &t, float &slo, float &shi)
{
    slo = fmaf(t.l1, t.v.y, fmaf(t.l0, t.v.x, slo));
    float a, b;
    if (kMode == 0) {
        a = t.up ? t.v.y : t.v.x;
        b = t.up ? t.v.z : t.v.y;
    } else if (kMode == 1) {
        a = t.up ? t.v.z : t.v.y;
        b = t.up ? t.v.w : t.v.z;
    } else {
        a = t.v.z;
        b = t.v.w;
    }
    shi = fmaf(t.h1, b, fmaf(t.h0, a, shi));
}

// The lines kw0 .. kw1 of the padded image img for a lane's two rays,
// from crossings flo, fhi on line kw0, into Kahan sums (lower ray, upper
// ray).  Batches of kLineBatch lines are summed in float before one Kahan
// step.  Software-pipelined with one register set: each line's taps are
// used and the slot is at once refilled with the next batch's line, so a
// batch of loads is in flight while the current batch is summed, and no
// value moves between registers from one batch to the next.
template <int kMode>
__device__ __forceinline__ void pair_lines(long long flo, long long fhi, unsigned pfrac, int kw0,
                                           int kw1, int cmax, long long Q, int Np,
                                           const float *__restrict__ img, Kahan &alo, Kahan &ahi)
{
    PairTaps t[kLineBatch];
    int k = kw0;
    const int nb = kw1 >= kw0 ? (kw1 - kw0 + 1) / kLineBatch : 0;
    if (nb > 0) {
#pragma unroll
        for (int q = 0; q < kLineBatch; ++q)
            pair_fetch<kMode>(flo, fhi, pfrac, cmax, Q, img, (k + q) * Np, t[q]);
        k += kLineBatch;
        for (int i = 1; i < nb; ++i) {
            float slo = 0.f, shi = 0.f;
#pragma unroll
            for (int q = 0; q < kLineBatch; ++q) {
                pair_apply<kMode>(t[q], slo, shi);
                pair_fetch<kMode>(flo, fhi, pfrac, cmax, Q, img, (k + q) * Np, t[q]);
            }
            k += kLineBatch;
            alo.add(slo);
            ahi.add(shi);
        }
        float slo = 0.f, shi = 0.f;
#pragma unroll
        for (int q = 0; q < kLineBatch; ++q)
            pair_apply<kMode>(t[q], slo, shi);
        alo.add(slo);
        ahi.add(shi);
    }
    for (; k <= kw1; ++k) {
        PairTaps u;
        pair_fetch<kMode>(flo, fhi, pfrac, cmax, Q, img, k * Np, u);
        float slo = 0.f, shi = 0.f;
        pair_apply<kMode>(u, slo, shi);
        alo.add(slo);
        ahi.add(shi);
    }
}

// Spectrum read through device pointers (the batched kernels); mu2 holds
// mu log2(e), as in SpecArg.
struct SpecPtr {
    int32_t K;
    const float *__restrict__ J;
    const float *__restrict__ mu2;
    const float *__restrict__ bg;
};

// End of a forward block: lane l of wave seg holds the Kahan partials of
// rays 2l (e) and 2l + 1 (o) of the block over its share of the lines.  Ray
// r's partials are combined in segment order, times the view's path length;
// with kResid the spectral residual replaces the line integral:
// r_i = Y_i - sum_k J_k exp(-mu_k (bg_i + max(s_i, 0))), with exp(-mu t) =
// 2^(-mu log2(e) t) by the hardware exp2 (whose result is exp2f's except
// below 2^-126, where it flushes a term that no count could register).
// Ray r = lane + 64 (seg mod 2) is finished by the waves seg with that
// parity: wave seg sums the energies k = q, q + kEPhase, ... (q = seg / 2)
// and the sums are added in q order.  Ray i = vidx B + b goes to
// out[vidx ostride + ooff + b], times wstep when weighted, and unweighted to
// plain[i] when plain is not null.  Every thread of the workgroup calls this
// (it holds barriers).
template <bool kResid, class Spec>
__device__ __forceinline__ void forward_pair_end(const Kahan &ae, const Kahan &ao, int seg,
                                                 int lane, const ViewGeom &G, int b0, int B,
                                                 float (*ps)[kFwdRays], float (*pc)[kFwdRays],
                                                 float (*pm)[kFwdRays],
                                                 const float *__restrict__ Y, const Spec &sp,
                                                 float *__restrict__ out, int ostride, int ooff,
                                                 bool weighted, float *__restrict__ plain)
{
    ps[seg][2 * lane] = ae.s;
    pc[seg][2 * lane] = ae.c;
    ps[seg][2 * lane + 1] = ao.s;
    pc[seg][2 * lane + 1] = ao.c;
    __syncthreads();
    const int r = lane + kFwdThreads * (seg & 1), q = seg >> 1;
    const int b = b0 + r;
    const bool ray = b < B;
    const size_t i = (size_t)G.vidx * B + (ray ? b : 0);
    Kahan tot;
#pragma unroll
    for (int u = 0; u < kSegs; ++u) {
        tot.add(ps[u][r]);
        tot.add(-pc[u][r]);
    }
    // the sums carry the weights' factor 2^32 (removed exactly)
    float val = (tot.value() * 0x1p-32f) * G.wstep;
    if (kResid) {
        const float sp0 = fmaxf(val, 0.f) + ((sp.bg && ray) ? sp.bg[i] : 0.f);
        float m = 0.f;
#pragma unroll 4
        for (int k = q; k < sp.K; k += kEPhase)
            m = fmaf(sp.J[k], __builtin_amdgcn_exp2f(-sp.mu2[k] * sp0), m);
        pm[q][r] = m;
        __syncthreads();
        if (q == 0) {
            float mt = pm[0][r];
#pragma unroll
            for (int u = 1; u < kEPhase; ++u)
                mt += pm[u][r];
            val = Y[i] - mt;
        }
    }
    if (q != 0 || !ray)
        return;
    const size_t o = (size_t)G.vidx * ostride + ooff + b;
    out[o] = weighted ? val * G.wstep : val;
    if (plain)
        plain[i] = val;
}

// Forward projection of rays [128 bblock, 128 bblock + 128) of table view
// `slot` by one workgroup of kFwdThreads * kSegs threads, reading the padded
// image pair; with kResid the spectral residual replaces the line integral.
// Lane l takes rays 2l and 2l + 1 of the block; the kSegs waves take the
// same rays and split the image lines any of them reaches (from the
// geometry's block table blk[2 (slot nbb + bblock) + {0, 1}]) into equal
// shares, walked in a wave-uniform loop (the line's address is scalar).
// Column-stepping views read the transposed image so that the lanes of a
// wave touch neighbouring addresses on every line.  Ray i = vidx B + b goes
// to out[vidx * ostride + ooff + b], times the view's wstep when weighted,
// and unweighted to plain[i] when plain is not null.
template <bool kResid, class Spec>
__device__ __forceinline__ void forward_block(const ViewGeom *__restrict__ views,
                                              const int32_t *__restrict__ blk, int N, int B,
                                              int nrow, const float *__restrict__ xp,
                                              const float *__restrict__ xTp,
                                              const float *__restrict__ Y, const Spec &sp,
                                              float *__restrict__ out, int ostride, int ooff,
                                              bool weighted, float *__restrict__ plain,
                                              int slot, int bblock)
{
    __shared__ float part_s[kSegs][kFwdRays], part_c[kSegs][kFwdRays];
    __shared__ float part_m[kEPhase][kFwdRays];
    const int lane = threadIdx.x % kFwdThreads;
    const int seg = __builtin_amdgcn_readfirstlane(threadIdx.x / kFwdThreads);  // wave-uniform
    const int b0 = bblock * kFwdRays;
    const ViewGeom G = views[slot];
    const float *__restrict__ img = slot < nrow ? xp : xTp;
    const int Np = padded_cols(N);
    const int cmax = N + 2 * kPadX - 2;

    // the waves hold the same 128 rays: split the lines any of them reaches
    // into equal shares
    const int bi = 2 * (slot * ((B + kFwdRays - 1) / kFwdRays) + bblock);
    const int kmin = blk[bi], kmax = blk[bi + 1];
    int kw0 = 0, kw1 = -1;
    if (kmin <= kmax) {
        const int per = (kmax - kmin + kSegs) / kSegs;
        kw0 = kmin + seg * per;
        kw1 = min(kmax, kw0 + per - 1);
    }
    // padded column coordinates of the lane's rays on line kw0 (exact), as
    // 2^-32 fixed point
    const double fe = fma((double)kw0, G.Q, fma((double)(b0 + 2 * lane), G.P, G.A)) + (double)kPadX;
    const double fo = fma((double)kw0, G.Q, fma((double)(b0 + 2 * lane + 1), G.P, G.A)) + (double)kPadX;
    const long long Fe = fixed32(fe), Fo = fixed32(fo), Qf = fixed32(G.Q);
    const bool rising = G.P >= 0.0;                 // ray 2l + 1 crosses to the right of ray 2l
    const double aP = fabs(G.P);
    const unsigned pfrac = (unsigned)fixed32(aP);   // |P| 2^32 mod 2^32
    const long long Flo = rising ? Fe : Fo, Fhi = rising ? Fo : Fe;
    Kahan alo, ahi;
    if (aP < 1.0)
        pair_lines<0>(Flo, Fhi, pfrac, kw0, kw1, cmax, Qf, Np, img, alo, ahi);
    else if (aP < 2.0)
        pair_lines<1>(Flo, Fhi, pfrac, kw0, kw1, cmax, Qf, Np, img, alo, ahi);
    else
        pair_lines<2>(Flo, Fhi, pfrac, kw0, kw1, cmax, Qf, Np, img, alo, ahi);
    forward_pair_end<kResid>(rising ? alo : ahi, rising ? ahi : alo, seg, lane, G, b0, B, part_s,
                             part_c, part_m, Y, sp, out, ostride, ooff, weighted, plain);
}

// Workgroup i projects ray block order[i] (the geometry's dispatch order:
// longest blocks first, with the ones a CU holds at once balanced in lines).
template <bool kResid>
__global__ __launch_bounds__(kFwdThreads *kSegs) void k_forward(
    const ViewGeom *__restrict__ views, const int32_t *__restrict__ blk,
    const int32_t *__restrict__ order, int N, int V, int B, int nrow,
    const float *__restrict__ xp, const float *__restrict__ xTp, const float *__restrict__ Y,
    SpecArg sp, float *__restrict__ out, int ostride, int ooff, int weighted,
    float *__restrict__ plain, const int32_t *__restrict__ skip, FinishArgs fin)
{
    if (skipped(skip))
        return;
    // The step's first kernel hides the previous step's finish in one more
    // workgroup after the projection's, dispatched last: the finish runs if
    // one is pending, and this step's is marked pending unless the run has
    // just stopped.  Nothing that reads the stop flag runs before this
    // kernel ends; its other workgroups may compute a residual that no
    // later kernel uses.
    if (kResid && fin.state && blockIdx.x == gridDim.x - 1) {
        finish_block<true, kFwdThreads * kSegs>(fin.partials, fin.nparts, fin.avg_parts,
                                                 fin.n_avg, fin.state);
        if (threadIdx.x == 0 && !fin.state->done)
            fin.state->pending = 1;
        return;
    }
    const int nbb = (B + kFwdRays - 1) / kFwdRays;
    const int it = order[blockIdx.x];
    forward_block<kResid>(views, blk, N, B, nrow, xp, xTp, Y, sp, out, ostride, ooff,
                          weighted != 0, plain, it / nbb, it % nbb);
}

// Number of positive matrix entries on each ray, summed per workgroup:
// the forward walk with the same weights, counting w > 0.
__global__ __launch_bounds__(kFwdThreads) void k_count_nnz(const ViewGeom *__restrict__ views,
                                                           int N, int B,
                                                           long long *__restrict__ parts)
{
    __shared__ long long red[kFwdThreads];
    const int v = blockIdx.y;
    const int b = blockIdx.x * kFwdThreads + threadIdx.x;
    long long cnt = 0;
    if (b < B) {
        const ViewGeom G = views[v];
        double f = fma((double)b, G.P, G.A);
        for (int k = 0; k < N; ++k) {
            const double fl = floor(f);
            const double e0 = f - fl;
            f += G.Q;
            if (fl < -1.0 || fl > (double)(N - 1))
                continue;
            const int j0 = (int)fl;
            cnt += (j0 >= 0 && (float)(1.0 - e0) > 0.f) ? 1 : 0;
            cnt += (j0 + 1 <= N - 1 && (float)e0 > 0.f) ? 1 : 0;
        }
    }
    red[threadIdx.x] = cnt;
    __syncthreads();
    for (int w = kFwdThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        parts[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

// ------------------------------------------------------------------- back

// Taps of view G for pixel (line k, pixel j of that line): the sum over
// bins b within one pixel of (float)(1 - |f(b, k) - j|) times the weighted
// padded residual at bin b (padded-bin numbers; the path-length factor is in
// the residual already), formed as u0 r0 + u1 r1 by tap_fetch and tap_apply.
//
// Pair rule (every |P| >= 1).  Let t be the real solution of f(t, k) = j.
// Bin b has positive weight iff |b - t| |P| < 1, so only b_f = floor(t)
// and b_f + 1 can.  With d = f(b_f, k) - j = (b_f - t) P (exact), b_f's
// weight is (float)(1 - |d|) and, as |d| <= |P|, b_f + 1 is at distance
// |P| - |d| (exact), so its weight is (float)(|d| + (1 - |P|)): the same
// floats the forward projector forms for these (bin, pixel) pairs.
//
// t is computed as -T (1/P) and truncated.  Its error is at most
// |T| 2^-52 < 2^-32 (|T| < 2^20 by the geometry check), so when t lies
// within that error of an integer n the truncation may give n where floor
// gives n - 1 or the reverse.  For |P| = 1 there is no error (1/P = +-1);
// otherwise |P| - 1 >= 2^-32 (P is a multiple of 2^-32), and the bin lost
// (n - 1 or n + 1) is at distance >= 1 - error from t, hence weight <= 0,
// while the pair still formed gets weights that round to the exact ones
// (the far one to <= 0, the near one to the float of 1 - (error) |P|,
// which is 1 as the exact one is).
//
// The pair (b_f, b_f + 1) is clamped into [0, B + 2 kPadB - 1]: a truncated t below 1
// (negative t truncates upwards) or above the detector lands on two
// padding bins, which read zero whatever their weights; a pair holding a
// detector bin has t >= 1, where truncation is floor.
struct PairTap {
    float u0, u1, r0, r1;
};

// The pair's weights and residual values (the loads are issued here and
// waited for where the values are used).  r is the weighted padded
// sinogram; the view's row offset goes into the per-lane element index, so
// the base stays the same scalar pointer for every view.  Without kClamp
// the caller guarantees 0 <= trunc(t) <= B + 2 kPadB - 2 for every pixel of
// the image (the geometry's coverage test), so the clamp is the identity.
template <bool kClamp>
__device__ __forceinline__ PairTap tap_fetch(const ViewGeom &G, double kd, double jd, int B,
                                             const float *__restrict__ r)
{
    const double T = fma(kd, G.Q, G.Ab - jd);                  // f(0, k) - j, padded; exact
    const double t = -T * G.invP;
    const int bf = kClamp ? clamp_int<0>((int)t, B + 2 * kPadB - 2) : (int)t;
    const double d = fma((double)bf, G.P, T);                  // exact
    PairTap p;
    p.u0 = __builtin_amdgcn_fmed3f((float)(1.0 - fabs(d)), 0.f, 1.f);
    p.u1 = __builtin_amdgcn_fmed3f((float)(fabs(d) + G.omP), 0.f, 1.f);
    const unsigned i = (unsigned)(G.roff + bf);
    // Two 4-byte loads rather than one 8-byte load at a 4-byte-aligned
    // address: a wave's lanes read few, repeated bins, and the split loads
    // go through the address unit faster (measured: 10 % faster kernel at
    // 512^2 and 1024^2).  Hiding the second base from the compiler keeps it
    // from merging them.
    const float EXACT_GLOBAL *r1 = (const float EXACT_GLOBAL *)(r + 1);
    asm("" : "+s"(r1));
    p.r0 = at(r, i);
    p.r1 = *(const float EXACT_GLOBAL *)((const char EXACT_GLOBAL *)r1 + (i << 2));
    return p;
}

__device__ __forceinline__ float tap_apply(const PairTap &p, float acc)
{
    return fmaf(p.u1, p.r1, fmaf(p.u0, p.r0, acc));
}

// General rule (bins narrower than pixels): every bin within `reach` of b0.
// Works in true bin numbers with explicit range tests (the padding is too
// narrow for the reach); rv points at bin 0 of a weighted row.
__device__ __forceinline__ float taps_reach(const ViewGeom &G, double kd, double jd, int B,
                                            int reach, const float *__restrict__ rv, float acc)
{
    const double T = fma(kd, G.Q, G.A) - jd;                        // exact
    const double m = fma(-T, G.invP, kRoundMagic);
    const int b0 = min(max(low_int(m), -2 - reach), B + 1 + reach);
    const double d0 = fma((double)b0, G.P, T);                      // exact
    float s = acc;
    for (int q = -reach; q <= reach; ++q) {
        const int bb = b0 + q;
        const float u = (float)(1.0 - fabs(fma((double)q, G.P, d0)));   // exact distance
        const bool ok = u > 0.f && (unsigned)bb < (unsigned)B;
        s = fmaf(ok ? u : 0.f, rv[ok ? bb : 0], s);
    }
    return s;
}

// Sum over views [v0, v1) of the taps for pixel (kd, jd) of each view's
// stepping line, from the weighted padded sinogram r.  Batches of views,
// each summed in float (in view order) before one Kahan step.  With the
// pair rule the loop is software-pipelined: the next batch's weights are
// formed and its loads issued before the current batch is summed, so a
// wave keeps two batches of loads in flight.
template <bool kTwo, bool kClamp>
__device__ __forceinline__ void gather_views(const ViewGeom *__restrict__ views, int v0, int v1,
                                             double kd, double jd, int B, int reach,
                                             const float *__restrict__ r, Kahan &acc)
{
    const int rstride = padded_bins(B);
    int v = v0;
    if (kTwo) {
        // two register sets used alternately: a copy between them would
        // make the compiler wait for the loads at the copy
        PairTap ta[kViewBatch], tb[kViewBatch];
        auto fetch = [&](PairTap(&t)[kViewBatch], int vb) {
            // the batch's table pointer (constant address space: scalar
            // loads), opaque to the loop optimiser so that the views' fields
            // are read at small positive immediate offsets
            using CView = const ViewGeom EXACT_CONSTANT;
            CView *gp = (CView *)(views + vb);
            asm("" : "+s"(gp));
#pragma unroll
            for (int q = 0; q < kViewBatch; ++q) {
                const ViewGeom G = gp[q];
                t[q] = tap_fetch<kClamp>(G, kd, jd, B, r);
            }
        };
        auto apply = [&](const PairTap(&t)[kViewBatch]) {
            float sb = 0.f;
#pragma unroll
            for (int q = 0; q < kViewBatch; ++q)
                sb = tap_apply(t[q], sb);
            acc.add(sb);
        };
        const int nb = (v1 - v0) / kViewBatch;
        if (nb > 0) {
            fetch(ta, v);
            int i = 1;
            // the scheduling barriers keep each batch's loads ahead of the
            // previous batch's sum and the next batch's loads behind it
            for (; i + 1 < nb; i += 2) {
                fetch(tb, v + i * kViewBatch);
                apply(ta);
                __builtin_amdgcn_sched_barrier(0);
                fetch(ta, v + (i + 1) * kViewBatch);
                apply(tb);
                __builtin_amdgcn_sched_barrier(0);
            }
            if (i < nb) {
                fetch(tb, v + i * kViewBatch);
                apply(ta);
                apply(tb);
            } else {
                apply(ta);
            }
            v += nb * kViewBatch;
        }
        for (; v < v1; ++v) {
            const ViewGeom G = views[v];
            acc.add(tap_apply(tap_fetch<kClamp>(G, kd, jd, B, r), 0.f));
        }
        return;
    }
    for (; v + kViewBatch <= v1; v += kViewBatch) {
        float sb = 0.f;
#pragma unroll
        for (int q = 0; q < kViewBatch; ++q) {
            const ViewGeom G = views[v + q];
            sb = taps_reach(G, kd, jd, B, reach, r + (size_t)G.vidx * rstride + kPadB, sb);
        }
        acc.add(sb);
    }
    for (; v < v1; ++v) {
        const ViewGeom G = views[v];
        acc.add(taps_reach(G, kd, jd, B, reach, r + (size_t)G.vidx * rstride + kPadB, 0.f));
    }
}

// (A^T r) at pixel (ix, iy) with the views split over the block's two z
// planes: plane 0 gathers the row-stepping views, plane 1 the
// column-stepping views (each about half of them), so a 16 x 16 tile runs
// as 8 waves.  Plane 1 hands its sum to plane 0 through LDS; the result
// (row part + column part, a fixed order) is meaningful in plane 0.  Every
// thread of the block calls this (it holds a barrier).
template <bool kTwo, bool kClamp>
__device__ __forceinline__ float back_pixel_split(const ViewGeom *__restrict__ views, int V,
                                                  int B, int nrow, int reach,
                                                  const float *__restrict__ r, int ix, int iy,
                                                  bool inside)
{
    __shared__ float part[kBackY][kBackX];
    float v = 0.f;
    if (inside) {
        Kahan acc;
        if (threadIdx.z == 0)
            gather_views<kTwo, kClamp>(views, 0, nrow, (double)iy, (double)ix, B, reach, r, acc);
        else
            gather_views<kTwo, kClamp>(views, nrow, V, (double)ix, (double)iy, B, reach, r, acc);
        v = acc.value();
    }
    if (threadIdx.z == 1)
        part[threadIdx.y][threadIdx.x] = v;
    __syncthreads();
    return threadIdx.z == 0 ? v + part[threadIdx.y][threadIdx.x] : 0.f;
}

template <bool kTwo, bool kClamp>
__global__ __launch_bounds__(kBackX *kBackY * 2) void k_back(
    const ViewGeom *__restrict__ views, int N, int V, int B, int nrow, int reach,
    const float *__restrict__ r, float *__restrict__ img, float scale,
    const int32_t *__restrict__ skip)
{
    if (skipped(skip))
        return;
    const int ix = blockIdx.x * kBackX + threadIdx.x;
    const int iy = blockIdx.y * kBackY + threadIdx.y;
    const bool inside = ix < N && iy < N;
    const float g = back_pixel_split<kTwo, kClamp>(views, V, B, nrow, reach, r, ix, iy, inside);
    if (inside && threadIdx.z == 0)
        img[(size_t)iy * N + ix] = g * scale;
}

// rw[vidx][kPadB + b] = wstep * r[vidx][b] for the view in table slot
// blockIdx.y, and the row's 2 kPadB padding bins set to zero (by the row's
// first block), so rw needs no clearing before.
__global__ __launch_bounds__(256) void k_weigh_rows(const ViewGeom *__restrict__ views, int B,
                                                    const float *__restrict__ r,
                                                    float *__restrict__ rw)
{
    const ViewGeom G = views[blockIdx.y];
    const int b = blockIdx.x * 256 + threadIdx.x;
    float *row = rw + (size_t)G.vidx * padded_bins(B);
    if (b < B)
        row[kPadB + b] = r[(size_t)G.vidx * B + b] * G.wstep;
    if (blockIdx.x == 0 && threadIdx.x < 2 * kPadB)
        row[threadIdx.x < kPadB ? threadIdx.x : B + threadIdx.x] = 0.f;
}

// The projected update on one 16 x 16 tile once g = scale (A^T r) is known
// for the lane's pixel (paper Sec. 1.2, eq. extragrad-method, with the
// orthant projection of Sec. 3.1): z = max(0, x_p - gamma g), written to
// the padded pair (zp and, through an LDS tile, zTp) and, when z is not
// null, to z; with kPartials the tile's double sums of (z - x)^2 and x^2 go
// to part2[0..1].  z may alias x (each lane reads and writes only its own
// pixel of x).  Every thread of the block calls this (it holds barriers);
// the work is done by z plane 0, and lanes outside the image pass
// inside = false.
template <bool kPartials>
__device__ __forceinline__ void update_epilogue(bool inside, float g, int N, const float *x,
                                                float gamma, float *z, float *__restrict__ zp,
                                                float *__restrict__ zTp,
                                                double *__restrict__ part2, int tx, int ty)
{
    __shared__ float tile[kBackY][kBackX + 1];
    __shared__ double red[2][kRedThreads / 64];
    const bool plane0 = threadIdx.z == 0;
    const int Np = padded_cols(N);
    const int ix = tx * kBackX + threadIdx.x;
    const int iy = ty * kBackY + threadIdx.y;
    double num = 0.0, den = 0.0;
    if (inside && plane0) {
        const size_t p = (size_t)iy * N + ix;
        const float xv = x[p];
        const float zv = fmaxf(0.f, fmaf(-gamma, g, xv));
        if (z)
            z[p] = zv;
        zp[(size_t)iy * Np + kPadX + ix] = zv;
        tile[threadIdx.y][threadIdx.x] = zv;
        if (kPartials) {
            const double dz = (double)zv - (double)xv;
            num = dz * dz;
            den = (double)xv * (double)xv;
        }
    }
    __syncthreads();
    const int ixT = tx * kBackX + threadIdx.y, iyT = ty * kBackY + threadIdx.x;
    if (plane0 && ixT < N && iyT < N)
        zTp[(size_t)ixT * Np + kPadX + iyT] = tile[threadIdx.x][threadIdx.y];
    if (kPartials) {
        double v2[2] = {num, den};
        plane_sum<2>(v2, red, plane0);
        if (plane0 && threadIdx.x == 0 && threadIdx.y == 0) {
            part2[0] = v2[0];
            part2[1] = v2[1];
        }
    }
}

// Back-projection fused with the update: the block's two z planes gather
// the pixel's gradient from the padded residual, then plane 0 runs the
// update epilogue.
template <bool kTwo, bool kPartials, bool kClamp>
__global__ __launch_bounds__(kBackX *kBackY * 2) void k_back_update(
    const ViewGeom *__restrict__ views, int N, int V, int B, int nrow, int reach,
    const float *__restrict__ r, float scale, const float *x, float gamma, float *z,
    float *__restrict__ zp, float *__restrict__ zTp, double *__restrict__ partials,
    const int32_t *__restrict__ skip)
{
    if (skipped(skip))
        return;
    const int ix = blockIdx.x * kBackX + threadIdx.x;
    const int iy = blockIdx.y * kBackY + threadIdx.y;
    const bool inside = ix < N && iy < N;
    const float g =
        back_pixel_split<kTwo, kClamp>(views, V, B, nrow, reach, r, ix, iy, inside) * scale;
    const int blk = blockIdx.y * gridDim.x + blockIdx.x;
    update_epilogue<kPartials>(inside, g, N, x, gamma, z, zp, zTp,
                               kPartials ? partials + 2 * blk : nullptr, blockIdx.x, blockIdx.y);
}

// ------------------------------------------------------ elementwise / tiles

// x into the padded pair: row-major copy xp and transpose xTp, the
// transpose through an LDS tile; the padding (kPadX columns at each end of
// every row, and the kImgTail floats after the last row) is set to zero
// too, grid-stride over its N 2 kPadX + kImgTail floats per buffer, so the
// pair needs no clearing before.
__global__ __launch_bounds__(kTile * 8) void k_pad_pair(const float *__restrict__ x,
                                                        float *__restrict__ xp,
                                                        float *__restrict__ xTp, int N)
{
    __shared__ float tile[kTile][kTile + 1];
    const int Np = padded_cols(N);
    const int bx = blockIdx.x * kTile, by = blockIdx.y * kTile;
    {
        const long edge = (long)N * 2 * kPadX, pad = edge + kImgTail;
        const long nthr = (long)gridDim.x * gridDim.y * blockDim.x * blockDim.y;
        for (long k = ((long)blockIdx.y * gridDim.x + blockIdx.x) * (blockDim.x * blockDim.y) +
                      threadIdx.y * blockDim.x + threadIdx.x;
             k < pad; k += nthr) {
            long a;
            if (k < edge) {
                const long row = k / (2 * kPadX);
                const int c = (int)(k % (2 * kPadX));
                a = row * Np + (c < kPadX ? c : N + c);   // right padding: kPadX + N + (c - kPadX)
            } else {
                a = (long)N * Np + (k - edge);
            }
            xp[a] = 0.f;
            xTp[a] = 0.f;
        }
    }
    for (int rr = threadIdx.y; rr < kTile; rr += 8) {
        const int iy = by + rr, ix = bx + threadIdx.x;
        if (iy < N && ix < N) {
            const float v = x[(size_t)iy * N + ix];
            xp[(size_t)iy * Np + kPadX + ix] = v;
            tile[rr][threadIdx.x] = v;
        }
    }
    __syncthreads();
    for (int rr = threadIdx.y; rr < kTile; rr += 8) {
        const int ixT = bx + rr, iyT = by + threadIdx.x;
        if (ixT < N && iyT < N)
            xTp[(size_t)ixT * Np + kPadX + iyT] = tile[threadIdx.x][rr];
    }
}

__global__ void k_fill(float *__restrict__ x, float value, long count)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < count;
         i += (long)gridDim.x * blockDim.x)
        x[i] = value;
}

__global__ void k_window_sum(const float *__restrict__ y, int Wn, long n,
                             float *__restrict__ Y, int32_t *__restrict__ bad)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x) {
        float s = 0.f;
        bool ok = true;
        for (int j = 0; j < Wn; ++j) {
            const float yv = y[(size_t)j * n + i];
            ok = ok && isfinite(yv) && yv >= 0.f;
            s += yv;
        }
        Y[i] = s;
        if (!ok && bad)
            *bad = 1;
    }
}

__global__ void k_count_bad(const float *__restrict__ x, long count, int32_t *__restrict__ bad)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < count;
         i += (long)gridDim.x * blockDim.x) {
        const float v = x[i];
        if (!(isfinite(v) && v >= 0.f))
            *bad = 1;
    }
}

__global__ void k_state_init(SolveState *st, double tol, int max_iters, int stop_mode)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->rho = -1.0;
        st->lam = 0.0;
        st->unorm = 0.0;
        st->tol = tol;
        st->t = 0;
        st->done = max_iters <= 0 ? 1 : 0;
        st->converged = 0;
        st->max_iters = max_iters;
        st->stop_mode = stop_mode;
        st->pending = 0;
        st->crit = -1.0;
    }
}

template <bool kGated>
__global__ __launch_bounds__(kRedThreads) void k_eg_finish(const double *__restrict__ partials,
                                                           int nparts,
                                                           const double *__restrict__ avg_parts,
                                                           int n_avg, SolveState *st)
{
    finish_block<kGated, kRedThreads>(partials, nparts, avg_parts, n_avg, st);
}

// ------------------------------------------------------ averaged iterate

constexpr int kAvgThreads = 256;

__global__ __launch_bounds__(kAvgThreads) void k_avg_init(const float *__restrict__ x,
                                                          float *__restrict__ ring, int R, int J,
                                                          double *__restrict__ S, long d)
{
    const long p = (long)blockIdx.x * kAvgThreads + threadIdx.x;
    if (p >= d)
        return;
    const float v = x[p];
    S[p] = (double)v;
    if (J >= 1)
        ring[(size_t)(1 % R) * (size_t)d + (size_t)p] = v;
}

// One pixel per lane.  Window of index s: j = floor(s/2)+1 .. s, c_s =
// s - floor(s/2) iterates.  Odd s adds x_s; even s adds x_s and drops
// x_{s/2}.
__global__ __launch_bounds__(kAvgThreads) void k_avg_step(
    const float *__restrict__ x, float *__restrict__ ring, int R, int J, double *__restrict__ S,
    long d, double *__restrict__ partials, const SolveState *__restrict__ st)
{
    if (st->done)
        return;
    __shared__ double red[1][kRedThreads];
    const int s = st->t + 2;
    const double c_new = (double)(s - s / 2), c_old = (double)((s - 1) - (s - 1) / 2);
    const long p = (long)blockIdx.x * kAvgThreads + threadIdx.x;
    double sq = 0.0;
    if (p < d) {
        const float xs = x[p];
        const double so = S[p];
        double sn = so + (double)xs;
        if ((s & 1) == 0)
            sn -= (double)ring[(size_t)((s / 2) % R) * (size_t)d + (size_t)p];
        const double diff = sn / c_new - so / c_old;
        sq = diff * diff;
        S[p] = sn;
        if (s <= J)
            ring[(size_t)(s % R) * (size_t)d + (size_t)p] = xs;
    }
    double v1[1] = {sq};
    block_sum<1>(v1, red);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = v1[0];
}

__global__ __launch_bounds__(kAvgThreads) void k_avg_output(const double *__restrict__ S,
                                                            float *__restrict__ x, long d,
                                                            const SolveState *__restrict__ st)
{
    const int s = st->t + 1;
    const double c = (double)(s - s / 2);
    const long p = (long)blockIdx.x * kAvgThreads + threadIdx.x;
    if (p < d)
        x[p] = (float)(S[p] / c);
}

// ------------------------------------------------------------- batched

// A descriptor's global-memory pointer as the generic pointer the shared
// device code takes (an address-space cast the compiler sees through).
template <class T>
__device__ __forceinline__ T *glob(T EXACT_GLOBAL *p)
{
    return (T *)p;
}

// One phase of the extragradient step for every problem of a batch: each
// workgroup takes one item (problem, a, b) of the phase's list; the
// problem's own buffers and parameters come from its descriptor.  Items of
// problems that have stopped return at once.  The per-item work is the
// single-problem kernels' own device code, so a problem gets bit-identical
// results alone and in a batch.
template <bool kAtHalf>
__global__ __launch_bounds__(kFwdThreads *kSegs) void kb_forward(const BatchProb *__restrict__ probs,
                                                                 const BatchItem *__restrict__ items)
{
    const BatchItem it = items[blockIdx.x];
    const BatchProb &P = probs[it.p];
    if (glob(P.state)->done)
        return;
    const SpecPtr sp{P.K, glob(P.J), glob(P.mu2), P.bg ? glob(P.bg) : nullptr};
    forward_block<true>(glob(P.views), glob(P.blk), P.N, P.B, P.nrow, glob(kAtHalf ? P.xhp : P.xp),
                        glob(kAtHalf ? P.xhTp : P.xTp), glob(P.Y), sp, glob(P.r),
                        padded_bins(P.B), kPadB, true, nullptr, it.a, it.b);
}

template <bool kHalf>
__global__ __launch_bounds__(kBackX *kBackY * 2) void kb_back_update(
    const BatchProb *__restrict__ probs, const BatchItem *__restrict__ items)
{
    const BatchItem it = items[blockIdx.x];
    const BatchProb &P = probs[it.p];
    if (glob(P.state)->done)
        return;
    const int ix = it.a * kBackX + threadIdx.x;
    const int iy = it.b * kBackY + threadIdx.y;
    const bool inside = ix < P.N && iy < P.N;
    // the gather of either projector variant comes before the epilogue's
    // stores, so its view-table loads stay scalar
    float g;
    if (P.reach == 0 && P.covers)
        g = back_pixel_split<true, false>(glob(P.views), P.V, P.B, P.nrow, 0, glob(P.r), ix, iy,
                                          inside);
    else if (P.reach == 0)
        g = back_pixel_split<true, true>(glob(P.views), P.V, P.B, P.nrow, 0, glob(P.r), ix, iy,
                                         inside);
    else
        g = back_pixel_split<false, true>(glob(P.views), P.V, P.B, P.nrow, P.reach, glob(P.r),
                                          ix, iy, inside);
    g *= P.inv_n;
    const int ntx = (P.N + kBackX - 1) / kBackX;
    double *part2 = kHalf ? glob(P.parts) + 2 * (it.b * ntx + it.a) : nullptr;
    update_epilogue<kHalf>(inside, g, P.N, glob(P.x), P.gamma, kHalf ? nullptr : glob(P.x),
                           glob(kHalf ? P.xhp : P.xp), glob(kHalf ? P.xhTp : P.xTp), part2, it.a,
                           it.b);
}

__global__ __launch_bounds__(kRedThreads) void kb_finish(const BatchProb *__restrict__ probs)
{
    const BatchProb &P = probs[blockIdx.x];
    finish_block<false, kRedThreads>(glob(P.parts), P.ntiles, nullptr, 0, glob(P.state));
}

__global__ __launch_bounds__(kRedThreads) void k_dot3(const float *__restrict__ v,
                                                      const float *__restrict__ u, long d,
                                                      double *__restrict__ partials,
                                                      const int32_t *__restrict__ skip)
{
    if (skipped(skip))
        return;
    __shared__ double red[3][kRedThreads];
    double a[3] = {0.0, 0.0, 0.0};
    for (long i = blockIdx.x * (long)kRedThreads + threadIdx.x; i < d;
         i += (long)gridDim.x * kRedThreads) {
        const double vv = v[i], uu = u[i];
        a[0] = fma(vv, uu, a[0]);
        a[1] = fma(vv, vv, a[1]);
        a[2] = fma(uu, uu, a[2]);
    }
    block_sum<3>(a, red);
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x] = a[0];
        partials[3 * blockIdx.x + 1] = a[1];
        partials[3 * blockIdx.x + 2] = a[2];
    }
}

// One power-iteration step's Rayleigh quotient lam = <v, u> / <v, v> and
// ||u|| into the state, and the stop test on the device: done once lam
// changes by at most rel_tol (relative) from the previous step's, once t
// reaches max_iters, or at once with converged = -1 if lam is not finite and
// positive.  No-op once done, so that steps enqueued past the stop change
// nothing.
__global__ __launch_bounds__(kRedThreads) void k_dot3_finish(const double *__restrict__ partials,
                                                             int nparts, SolveState *st,
                                                             double rel_tol)
{
    if (st->done)
        return;
    __shared__ double red[3][kRedThreads];
    double a[3] = {0.0, 0.0, 0.0};
    for (int q = threadIdx.x; q < nparts; q += kRedThreads) {
        a[0] += partials[3 * q];
        a[1] += partials[3 * q + 1];
        a[2] += partials[3 * q + 2];
    }
    block_sum<3>(a, red);
    if (threadIdx.x == 0) {
        const double lam = a[1] > 0.0 ? a[0] / a[1] : 0.0;
        st->unorm = sqrt(a[2]);
        if (!(isfinite(lam) && lam > 0.0)) {
            st->lam = lam;
            st->converged = -1;
            st->done = 1;
            return;
        }
        const bool conv = st->t >= 1 && fabs(lam - st->lam) <= rel_tol * fabs(lam);
        st->lam = lam;
        st->t += 1;
        if (conv) {
            st->converged = 1;
            st->done = 1;
        } else if (st->t >= st->max_iters) {
            st->done = 1;
        }
    }
}

__global__ __launch_bounds__(kTile * 8) void k_normalize(const float *__restrict__ u,
                                                         float *__restrict__ v,
                                                         float *__restrict__ vp,
                                                         float *__restrict__ vTp, int N,
                                                         const SolveState *__restrict__ st)
{
    if (st->done)
        return;
    __shared__ float tile[kTile][kTile + 1];
    const double nrm = st->unorm;
    const float inv = nrm > 0.0 ? (float)(1.0 / nrm) : 0.f;
    const int Np = padded_cols(N);
    const int bx = blockIdx.x * kTile, by = blockIdx.y * kTile;
    for (int rr = threadIdx.y; rr < kTile; rr += 8) {
        const int iy = by + rr, ix = bx + threadIdx.x;
        if (iy < N && ix < N) {
            const float zv = u[(size_t)iy * N + ix] * inv;
            v[(size_t)iy * N + ix] = zv;
            vp[(size_t)iy * Np + kPadX + ix] = zv;
            tile[rr][threadIdx.x] = zv;
        }
    }
    __syncthreads();
    for (int rr = threadIdx.y; rr < kTile; rr += 8) {
        const int ixT = bx + rr, iyT = by + threadIdx.x;
        if (ixT < N && iyT < N)
            vTp[(size_t)ixT * Np + kPadX + iyT] = tile[threadIdx.x][rr];
    }
}

inline dim3 tile_grid(int N)
{
    const int t = (N + kTile - 1) / kTile;
    return dim3(t, t);
}

inline int dot_blocks(long d)
{
    long b = (d + kRedThreads * 4 - 1) / (kRedThreads * 4);
    return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

}  // namespace

int num_tiles(int N)
{
    const int t = (N + kBackX - 1) / kBackX;
    return t * t;
}

int num_dot_parts(long d) { return dot_blocks(d); }

int num_count_parts(const Geo &g) { return ((g.B + kFwdThreads - 1) / kFwdThreads) * g.V; }

hipError_t launch_count_nonzeros(const Geo &g, long long *parts, hipStream_t st)
{
    dim3 grid((g.B + kFwdThreads - 1) / kFwdThreads, g.V);
    hipLaunchKernelGGL(k_count_nnz, grid, dim3(kFwdThreads), 0, st, g.views, g.N, g.B, parts);
    return hipGetLastError();
}

hipError_t launch_pad_pair(const float *x, float *xp, float *xTp, int N, hipStream_t st)
{
    hipLaunchKernelGGL(k_pad_pair, tile_grid(N), dim3(kTile, 8), 0, st, x, xp, xTp, N);
    return hipGetLastError();
}

hipError_t launch_fill(float *x, float value, long count, hipStream_t st)
{
    long blocks = (count + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    if (blocks < 1)
        blocks = 1;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, st, x, value, count);
    return hipGetLastError();
}

// The forward launch over every ray block of the geometry, in its dispatch
// order; with a step finish (fin) one more workgroup runs it.
template <bool kResid>
hipError_t launch_forward_any(const Geo &g, const float *xp, const float *xTp, const float *Y,
                              const SpecArg &sp, float *out, int ostride, int ooff, bool weighted,
                              float *plain, const int32_t *skip, hipStream_t st,
                              const FinishArgs &fin)
{
    const int nblocks = ((g.B + kFwdRays - 1) / kFwdRays) * g.V;
    // with a finish, one more workgroup (the last) runs it
    hipLaunchKernelGGL(k_forward<kResid>, dim3(nblocks + (fin.state ? 1 : 0)),
                       dim3(kFwdThreads * kSegs), 0, st, g.views, g.blk, g.order, g.N, g.V, g.B,
                       g.nrow, xp, xTp, Y, sp, out, ostride, ooff, weighted ? 1 : 0, plain, skip,
                       fin);
    return hipGetLastError();
}

hipError_t launch_forward(const Geo &g, const float *xp, const float *xTp, float *s,
                          int s_stride, int s_off, bool weighted, const int32_t *skip,
                          hipStream_t st)
{
    SpecArg none;
    none.K = 0;
    none.bg = nullptr;
    const FinishArgs nofin{nullptr, 0, nullptr, 0, nullptr};
    return launch_forward_any<false>(g, xp, xTp, nullptr, none, s, s_stride, s_off, weighted,
                                     nullptr, skip, st, nofin);
}

hipError_t launch_forward_residual(const Geo &g, const float *xp, const float *xTp,
                                   const float *Y, const SpecArg &sp, float *r, float *r_plain,
                                   const int32_t *skip, hipStream_t st, const FinishArgs *fin)
{
    const FinishArgs f = fin ? *fin : FinishArgs{nullptr, 0, nullptr, 0, nullptr};
    return launch_forward_any<true>(g, xp, xTp, Y, sp, r, padded_bins(g.B), kPadB, true, r_plain,
                                    skip, st, f);
}

hipError_t launch_weigh_rows(const Geo &g, const float *r, float *rw, hipStream_t st)
{
    dim3 grid((g.B + 255) / 256, g.V);
    hipLaunchKernelGGL(k_weigh_rows, grid, dim3(256), 0, st, g.views, g.B, r, rw);
    return hipGetLastError();
}

hipError_t launch_back(const Geo &g, const float *rw, float *img, float scale,
                       const int32_t *skip, hipStream_t st)
{
    dim3 grid((g.N + kBackX - 1) / kBackX, (g.N + kBackY - 1) / kBackY);
    dim3 blk(kBackX, kBackY, 2);
    if (g.reach == 0 && g.covers)
        hipLaunchKernelGGL((k_back<true, false>), grid, blk, 0, st, g.views, g.N, g.V, g.B,
                           g.nrow, 0, rw, img, scale, skip);
    else if (g.reach == 0)
        hipLaunchKernelGGL((k_back<true, true>), grid, blk, 0, st, g.views, g.N, g.V, g.B,
                           g.nrow, 0, rw, img, scale, skip);
    else
        hipLaunchKernelGGL((k_back<false, true>), grid, blk, 0, st, g.views, g.N, g.V, g.B,
                           g.nrow, g.reach, rw, img, scale, skip);
    return hipGetLastError();
}

hipError_t launch_window_sum(const float *y, int Wn, long n, float *Y, int32_t *bad,
                             hipStream_t st)
{
    long blocks = (n + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    if (blocks < 1)
        blocks = 1;
    hipLaunchKernelGGL(k_window_sum, dim3((unsigned)blocks), dim3(256), 0, st, y, Wn, n, Y, bad);
    return hipGetLastError();
}

hipError_t launch_count_bad(const float *x, long count, int32_t *bad, hipStream_t st)
{
    long blocks = (count + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    if (blocks < 1)
        blocks = 1;
    hipLaunchKernelGGL(k_count_bad, dim3((unsigned)blocks), dim3(256), 0, st, x, count, bad);
    return hipGetLastError();
}

hipError_t launch_state_init(SolveState *state, double tol, int max_iters, int stop_mode,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, st, state, tol, max_iters, stop_mode);
    return hipGetLastError();
}

int avg_last_kept(int max_iters) { return max_iters < 0 ? 0 : (int)(((long)max_iters + 1) / 2); }
int avg_ring_slots(int max_iters) { return avg_last_kept(max_iters) / 2 + 2; }
int num_avg_parts(long d) { return (int)((d + kAvgThreads - 1) / kAvgThreads); }

hipError_t launch_avg_init(const float *x, float *ring, int R, int J, double *S, long d,
                           hipStream_t st)
{
    if (d <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_avg_init, dim3(num_avg_parts(d)), dim3(kAvgThreads), 0, st, x, ring, R,
                       J, S, d);
    return hipGetLastError();
}

hipError_t launch_avg_step(const float *x, float *ring, int R, int J, double *S, long d,
                           double *partials, const SolveState *state, hipStream_t st)
{
    hipLaunchKernelGGL(k_avg_step, dim3(num_avg_parts(d)), dim3(kAvgThreads), 0, st, x, ring, R,
                       J, S, d, partials, state);
    return hipGetLastError();
}

hipError_t launch_avg_output(const double *S, float *x, long d, const SolveState *state,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_avg_output, dim3(num_avg_parts(d)), dim3(kAvgThreads), 0, st, S, x, d,
                       state);
    return hipGetLastError();
}

hipError_t launch_back_update(const Geo &g, const float *r, float scale, const float *x,
                              float gamma, float *z, float *zp, float *zTp, double *partials,
                              const int32_t *skip, hipStream_t st)
{
    dim3 grid((g.N + kBackX - 1) / kBackX, (g.N + kBackY - 1) / kBackY);
    dim3 blk(kBackX, kBackY, 2);
#define EXACT_BU(TWO, PART, CLAMP)                                                              \
    hipLaunchKernelGGL((k_back_update<TWO, PART, CLAMP>), grid, blk, 0, st, g.views, g.N, g.V, \
                       g.B, g.nrow, TWO ? 0 : g.reach, r, scale, x, gamma, z, zp, zTp,         \
                       partials, skip)
    if (g.reach == 0 && g.covers) {
        if (partials)
            EXACT_BU(true, true, false);
        else
            EXACT_BU(true, false, false);
    } else if (g.reach == 0) {
        if (partials)
            EXACT_BU(true, true, true);
        else
            EXACT_BU(true, false, true);
    } else {
        if (partials)
            EXACT_BU(false, true, true);
        else
            EXACT_BU(false, false, true);
    }
#undef EXACT_BU
    return hipGetLastError();
}

hipError_t launch_eg_finish(const double *partials, int nparts, const double *avg_parts,
                            int n_avg, SolveState *state, hipStream_t st)
{
    hipLaunchKernelGGL(k_eg_finish<false>, dim3(1), dim3(kRedThreads), 0, st, partials, nparts,
                       avg_parts, n_avg, state);
    return hipGetLastError();
}

hipError_t launch_eg_finish_pending(const FinishArgs &fin, hipStream_t st)
{
    hipLaunchKernelGGL(k_eg_finish<true>, dim3(1), dim3(kRedThreads), 0, st, fin.partials,
                       fin.nparts, fin.avg_parts, fin.n_avg, fin.state);
    return hipGetLastError();
}

hipError_t launch_batch_step(const BatchProb *probs, int nprobs, const BatchItem *fwd, int nfwd,
                             const BatchItem *back, int nback, hipStream_t st)
{
    if (nprobs == 0)
        return hipSuccess;
    const dim3 fb(kFwdThreads * kSegs), bb(kBackX, kBackY, 2), rb(kRedThreads);
    hipLaunchKernelGGL(kb_forward<false>, dim3(nfwd), fb, 0, st, probs, fwd);
    hipLaunchKernelGGL(kb_back_update<true>, dim3(nback), bb, 0, st, probs, back);
    hipLaunchKernelGGL(kb_forward<true>, dim3(nfwd), fb, 0, st, probs, fwd);
    hipLaunchKernelGGL(kb_back_update<false>, dim3(nback), bb, 0, st, probs, back);
    hipLaunchKernelGGL(kb_finish, dim3(nprobs), rb, 0, st, probs);
    return hipGetLastError();
}

int fwd_items_per_view(int B) { return (B + kFwdRays - 1) / kFwdRays; }
int fwd_resident_blocks_per_cu()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_forward<true>, kFwdThreads * kSegs, 0) !=
            hipSuccess ||
        n < 1)
        return 1;
    return n;
}
int fwd_block_centre_out(int r, int nbb) { return centre_out(r, nbb); }
int back_tiles_per_side(int N) { return (N + kBackX - 1) / kBackX; }

hipError_t launch_dot3(const float *v, const float *u, int N, double *partials,
                       const int32_t *skip, hipStream_t st)
{
    const long d = (long)N * N;
    hipLaunchKernelGGL(k_dot3, dim3(dot_blocks(d)), dim3(kRedThreads), 0, st, v, u, d, partials,
                       skip);
    return hipGetLastError();
}

hipError_t launch_dot3_finish(const double *partials, int nparts, SolveState *state,
                              double rel_tol, hipStream_t st)
{
    hipLaunchKernelGGL(k_dot3_finish, dim3(1), dim3(kRedThreads), 0, st, partials, nparts, state,
                       rel_tol);
    return hipGetLastError();
}

hipError_t launch_normalize(const float *u, float *v, float *vp, float *vTp, int N,
                            const SolveState *state, hipStream_t st)
{
    hipLaunchKernelGGL(k_normalize, tile_grid(N), dim3(kTile, 8), 0, st, u, v, vp, vTp, N, state);
    return hipGetLastError();
}

}  // namespace exact
