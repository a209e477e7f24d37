// Internal declarations shared by the HIP kernels and the C-ABI layer of
// libexact.  Not installed; the public interface is include/exact.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace exact {

// Largest number of energy bins the fused epilogue takes by value.
constexpr int kMaxEnergies = 128;

// One view of the Joseph projector, in pixel-index units.
//
// A ray (v, b) crosses stepping line k (row iy for row-stepping views,
// column ix otherwise) at the fractional pixel index
//     f(b, k) = A + b P + k Q
// and puts weight wstep * (float)(1 - |f - j|) on pixel j of that line when
// positive.  A, P and Q are rounded to multiples of 2^-32 and every crossing
// stays below 2^20 in magnitude, so f and f - j are integers times 2^-32 with
// at most 53 significant bits: double arithmetic on them is exact in any
// order (incremental stepping in the forward, direct evaluation in the
// back-projector).  Both kernels therefore apply bit-identical weights.
//
// The back-projector takes, for a pixel, the bins floor(t) and floor(t) + 1
// around the solution t of f(t, k) = j; invP = 1/P (rounded), Ab = A -
// kPadB P is A in padded-bin coordinates (bin b of a padded sinogram row
// sits at index b + kPadB), omP = 1 - |P| (exact) and roff = vidx (B + 2
// kPadB) is the first element of the view's padded sinogram row.  The
// fields the back-projector reads come first.
//
// The geometry's table lists the row-stepping views first and the
// column-stepping views after them (Geo::nrow of each); vidx is the view's
// index v in the sinogram.
struct alignas(8) ViewGeom {
    double Ab, P, Q, invP, omP;
    int32_t roff;
    int32_t vidx;
    double A;
    float wstep;
    int32_t pad1_;
};
static_assert(sizeof(ViewGeom) == 64, "ViewGeom layout");

// Padded layouts read by the projectors.  An image row (or a row of the
// transposed image) holds kPadX zeros, the N pixels, kPadX zeros; a
// sinogram row holds kPadB zero bins, the B bins, kPadB zero bins.  Taps
// that fall outside the image or the detector then read zeros at in-bounds
// addresses, so the inner loops need no range tests.  The padding is zeroed
// when a buffer is created and never written afterwards.  A padded image
// buffer holds kImgTail zero floats after its last row: the forward reads
// four consecutive columns from a column at most Np - 2, so a read at the
// last row's end stays in the buffer.  kPadX is four so that the three
// columns a clamped lane reads at a row's start are all padding.
//
// A padded sinogram that the back-projector reads is **weighted**: row v
// holds wstep_v r[v][b], the path-length factor of the view applied once
// per ray by its producer instead of once per pixel and view.
constexpr int kPadX = 4;
constexpr int kPadB = 2;
constexpr int kImgTail = 64;
__host__ __device__ inline int padded_cols(int N) { return N + 2 * kPadX; }
// Floats of one padded image buffer (N rows of padded_cols(N), and the tail).
__host__ __device__ inline long padded_image_floats(int N)
{
    return (long)N * padded_cols(N) + kImgTail;
}
__host__ __device__ inline int padded_bins(int B) { return B + 2 * kPadB; }

// Spectrum collapsed over windows, passed to kernels by value; bg (device,
// [V][B], or null) holds known materials' line integrals per ray.  The CT
// residual evaluates exp(-mu_k t) as 2^(-mu2_k t) with mu2_k = mu_k log2(e)
// (rounded once on the host).
struct SpecArg {
    int32_t K;
    float J[kMaxEnergies];    // J_k = sum_j weight[j][k]
    float mu[kMaxEnergies];
    float mu2[kMaxEnergies];
    const float *bg;
};

// Device-side state of one extragradient run.
struct SolveState {
    double rho;          // last natural residual (-1 if undefined)
    double lam;          // power iteration: Rayleigh quotient
    double unorm;        // power iteration: ||u||
    double tol;
    int32_t t;           // steps completed
    int32_t done;        // nonzero: every later kernel of the run is a no-op
    int32_t converged;
    int32_t max_iters;
    int32_t stop_mode;   // 0: natural residual rho; 1: averaged iterate
    int32_t pending;     // a completed step's finish (reduction, stop test) not yet run
    double crit;         // stop_mode 1: last ||xbar_s - xbar_{s-1}|| (-1 if none)
};

// Tile knobs of the forward projector (compile-time): waves per ray block,
// each a share of the block's lines (EXACT_FWD_SEGS), and lines per batch
// summed in float before one Kahan step (EXACT_LINE_BATCH), both swept by
// the autotuner.  A workgroup projects kFwdRays = 128 adjacent rays, two per
// lane.
#ifndef EXACT_FWD_SEGS
#define EXACT_FWD_SEGS 4
#endif
#ifndef EXACT_LINE_BATCH
#define EXACT_LINE_BATCH 4
#endif
constexpr int kFwdSegs = EXACT_FWD_SEGS;
constexpr int kFwdLineBatch = EXACT_LINE_BATCH;
constexpr int kFwdRays = 128;

struct Geo {
    const ViewGeom *views;
    // Per (table slot, block of kFwdRays bins): first and last image line
    // any of the block's rays reaches (first > last if none), conservative
    // by one line; 2 ints each, slot-major.
    const int32_t *blk;
    // Dispatch order of the forward projector's workgroups: workgroup i
    // projects the rays of block order[i] = slot * nbb + block (a
    // permutation of the V * nbb blocks, nbb = ceil(B / kFwdRays)).
    const int32_t *order;
    int N, V, B;
    int nrow;        // views[0, nrow) step along rows, views[nrow, V) along columns
    // Bins examined on each side of the nearest one in the back-projector's
    // general rule; 0 when every |P| >= 1 (bins at least as wide as
    // pixels), where the bin-pair rule applies.
    int reach;
    // Nonzero when, for every view and every pixel of the image, the pair
    // rule's first bin trunc(t) lies in the padded row without clamping
    // (the detector covers the image's projection with half a bin to spare).
    int covers;
};

// Device code sees the descriptor's pointers as global-memory pointers
// (otherwise pointers loaded from memory are generic and every access
// through them becomes a flat load); host code (and exact_capi.hip, which
// defines EXACT_HOST_SIDE) sees plain pointers.  The layout is the same.
#if defined(__HIP_DEVICE_COMPILE__) && !defined(EXACT_HOST_SIDE)
#define EXACT_GLOBAL __attribute__((address_space(1)))
#else
#define EXACT_GLOBAL
#endif

// Device code reads wave-uniform read-only tables through constant-address-
// space pointers, which the compiler loads with scalar loads.
#if defined(__HIP_DEVICE_COMPILE__)
#define EXACT_CONSTANT __attribute__((address_space(4)))
#else
#define EXACT_CONSTANT
#endif

// One problem of a batch, as the batched kernels see it.
struct BatchProb {
    const ViewGeom EXACT_GLOBAL *views;
    int32_t N, V, B, nrow, reach, K, ntiles, covers;
    const float EXACT_GLOBAL *Y;       // window sums of y
    const int32_t EXACT_GLOBAL *blk;   // the geometry's block line table
    const float EXACT_GLOBAL *J;       // spectrum (device copies; mu2 = mu log2(e))
    const float EXACT_GLOBAL *mu2;
    const float EXACT_GLOBAL *bg;      // known materials' line integrals, or null
    float EXACT_GLOBAL *x;             // iterate (the caller's buffer)
    float EXACT_GLOBAL *xp;            // iterate and its transpose, padded rows
    float EXACT_GLOBAL *xTp;
    float EXACT_GLOBAL *xhp;           // half-step iterate and its transpose, padded
    float EXACT_GLOBAL *xhTp;
    float EXACT_GLOBAL *r;             // residual, padded rows
    double EXACT_GLOBAL *parts;        // update partials, 2 per 16x16 tile
    SolveState EXACT_GLOBAL *state;
    float gamma, inv_n;
};

// One workgroup's work: problem p and two coordinates (forward: table view
// slot, bin block; back-projection and update: tile column, tile row).
struct BatchItem {
    int32_t p, a, b, pad;
};

// Tile side of the padding/transposition and normalisation kernels.
constexpr int kTile = 32;

// 16 x 16 tiles of an N x N image (the update partials are per tile).
int num_tiles(int N);
int num_dot_parts(long d);
int num_count_parts(const Geo &g);

hipError_t launch_count_nonzeros(const Geo &g, long long *parts, hipStream_t st);

// Batched step: the five phases of one extragradient step over the item
// lists (forward items; back-projection + update tiles).
hipError_t launch_batch_step(const BatchProb *probs, int nprobs, const BatchItem *fwd, int nfwd,
                             const BatchItem *back, int nback, hipStream_t st);
int fwd_items_per_view(int B);
// Forward-projector workgroups one CU holds at once (from the kernel's
// occupancy on the current device).
int fwd_resident_blocks_per_cu();
int fwd_block_centre_out(int r, int nbb);
int back_tiles_per_side(int N);

// xp, xTp (padded, padding already zero) <- x and its transpose.
hipError_t launch_pad_pair(const float *x, float *xp, float *xTp, int N, hipStream_t st);
hipError_t launch_fill(float *x, float value, long count, hipStream_t st);
// s = A x from the padded pair; s[vidx * s_stride + s_off + b] (times the
// view's wstep when weighted: the weighted padded sinogram the
// back-projector reads).
hipError_t launch_forward(const Geo &g, const float *xp, const float *xTp, float *s,
                          int s_stride, int s_off, bool weighted, const int32_t *skip,
                          hipStream_t st);
// r = Y - sum_k J_k exp(-mu_k (A x)_+) into a weighted padded residual and,
// when r_plain is not null, unweighted into the plain [V][B] layout.
// With fin (nullable), the kernel's last workgroup also runs the previous
// step's finish when one is pending and marks this step's as pending (the
// step's first kernel hides the finish; see k_forward).
struct FinishArgs {
    const double *partials;
    int nparts;
    const double *avg_parts;
    int n_avg;
    SolveState *state;
};
hipError_t launch_forward_residual(const Geo &g, const float *xp, const float *xTp,
                                   const float *Y, const SpecArg &sp, float *r, float *r_plain,
                                   const int32_t *skip, hipStream_t st,
                                   const FinishArgs *fin = nullptr);
// rw (padded, padding already zero) <- the plain [V][B] sinogram r,
// weighted row by row.
hipError_t launch_weigh_rows(const Geo &g, const float *r, float *rw, hipStream_t st);
// img = scale A^T r from a weighted padded sinogram.
hipError_t launch_back(const Geo &g, const float *rw, float *img, float scale,
                       const int32_t *skip, hipStream_t st);
hipError_t launch_window_sum(const float *y, int Wn, long n, float *Y,
                             int32_t *bad, hipStream_t st);
hipError_t launch_count_bad(const float *x, long count, int32_t *bad,
                            hipStream_t st);
hipError_t launch_state_init(SolveState *state, double tol, int max_iters, int stop_mode,
                             hipStream_t st);
// Back-projection fused with the update: g = scale A^T r (r weighted and
// padded) and z = max(0, x - gamma g) for every pixel, written to zp and
// (transposed) zTp in the padded layout and, when z is not null, to z.  With
// partials != nullptr also writes per-tile double partial sums of
// ||z - x||^2 and ||x||^2 (2 per 16x16 tile, num_tiles of them).  z may
// alias x.
hipError_t launch_back_update(const Geo &g, const float *r, float scale, const float *x,
                              float gamma, float *z, float *zp, float *zTp, double *partials,
                              const int32_t *skip, hipStream_t st);
// Fixed-order reduction of the update partials; sets rho_t, advances t and
// raises done when t reaches max_iters or the run's stop rule holds: rho_t
// <= tol (stop_mode 0), or, from the averaged-iterate partials (n_avg of
// them), ||xbar_s - xbar_{s-1}|| <= tol (stop_mode 1).
// The finish of a step whose finish is pending (no-op otherwise): settles
// the state before the host reads it.
hipError_t launch_eg_finish_pending(const FinishArgs &fin, hipStream_t st);
hipError_t launch_eg_finish(const double *partials, int nparts, const double *avg_parts,
                            int n_avg, SolveState *state, hipStream_t st);

// Averaged iterate xbar_s = mean of x_j, j = floor(s/2)+1 .. s, kept as the
// double running sum S of its window.  Iterates that a later window move
// drops are kept in a ring of R image slots (slot j mod R holds x_j for
// j <= J = floor((max_iters+1)/2), the largest index ever dropped);
// R = floor(J/2) + 2 slots suffice.
int avg_ring_slots(int max_iters);
int avg_last_kept(int max_iters);
int num_avg_parts(long d);
// s = 1: S = x_1 and x_1 into its ring slot.
hipError_t launch_avg_init(const float *x, float *ring, int R, int J, double *S, long d,
                           hipStream_t st);
// After the step that produced x_s (s = t + 2 with t the steps completed
// before it): moves the window, S += x_s (- x_{s/2} for even s), stores x_s
// if it will be dropped later, and writes per-block partials of
// (S_new/c_s - S_old/c_{s-1})^2.  No-op once the run is done.
hipError_t launch_avg_step(const float *x, float *ring, int R, int J, double *S, long d,
                           double *partials, const SolveState *state, hipStream_t st);
// x = xbar at the last index reached (s = t + 1).
hipError_t launch_avg_output(const double *S, float *x, long d, const SolveState *state,
                             hipStream_t st);
// Power iteration helpers: partials of <v,u>, <v,v>, <u,u> (no-op while
// *skip); reduction into state->lam and state->unorm with the stop test
// (state->t counts the steps; done at relative change <= rel_tol, at
// state->max_iters, or with converged = -1 for a non-positive estimate);
// v = u / unorm (and its transpose), a no-op once done.
hipError_t launch_dot3(const float *v, const float *u, int N, double *partials,
                       const int32_t *skip, hipStream_t st);
hipError_t launch_dot3_finish(const double *partials, int nparts, SolveState *state,
                              double rel_tol, hipStream_t st);
// v = u / ||u|| (the norm from the state), also into the padded pair.
hipError_t launch_normalize(const float *u, float *v, float *vp, float *vTp, int N,
                            const SolveState *state, hipStream_t st);

// ---- TV-ball and orthant projection (exact_tv.hip)

int num_tv_parts(int N);        // partial sums of k_tv_parts
int num_flat_parts(long d);     // partial sums of the flat reductions
// One TV-regularized point x = argmin ||x - b||^2 + lam TV(x) by `iters`
// (>= 1) FGP steps from zero, and out[0] = TV(x) in double (parts:
// num_tv_parts(N)).  p, q, r, s and p2, q2, r2, s2 are work fields of N*N
// floats (the state alternates between the two sets); out may be pinned
// host memory's device address.  Launch sequence only.  Here and in the
// launchers below that write a result to out: with flag not null (pinned
// host memory's device address), the last kernel then writes seq to *flag,
// ordered after the result at system scope, for a host that polls.
hipError_t launch_prox(const float *b, float *p, float *q, float *r, float *s, float *p2,
                       float *q2, float *r2, float *s2, double lam, int iters, float *x, int N,
                       double *parts, double *out, hipStream_t st, unsigned *flag = nullptr,
                       unsigned seq = 0);
// out[0] = TV(x) in double (parts: num_tv_parts(N) doubles; out may be
// pinned host memory's device address, as for the Dykstra sums below).
hipError_t launch_tv_norm(const float *x, int N, double *parts, double *out, hipStream_t st,
                          unsigned *flag = nullptr, unsigned seq = 0);
// Dykstra's round around the TV projection: w = z + p and out[0] = TV(w)
// before it (parts: num_tv_parts(N)); after it p = w - y, z = max(0, y + q),
// q = y + q - z and out[0] = ||z_new - z_old||^2.
hipError_t launch_dyk_pre(const float *z, const float *p, float *w, int N, double *parts,
                          double *out, hipStream_t st, unsigned *flag = nullptr,
                          unsigned seq = 0);
hipError_t launch_dyk_post(const float *w, const float *y, float *p, float *q, float *z, long d,
                           double *parts, double *out, hipStream_t st, unsigned *flag = nullptr,
                           unsigned seq = 0);
// z = x - gamma g.
hipError_t launch_axpy(const float *x, const float *g, float gamma, float *z, long d,
                       hipStream_t st);
// out[0] = ||a - b||^2, out[1] = ||b||^2 in double (parts: 2 num_flat_parts(d)).
hipError_t launch_diff2(const float *a, const float *b, long d, double *parts, double *out,
                        hipStream_t st, unsigned *flag = nullptr, unsigned seq = 0);

// ---- dense measurement matrix (exact_dense.hip)

constexpr int kDenseMaxCols = 4096;   // columns of A the streaming kernel holds
int dense_cols(int d);                // column chunks per thread (power of two)
int dense_blocks(long n, int d);      // row blocks (partial gradients)
int dense_sum_groups(long n, int d);  // groups of partial gradients after the first sum
// g = (1/n) A^T r, r_i = <a_i, x> (linear) or Y_i - sum_k J_k exp(-mu_k
// max(<a_i, x>, 0)), by one streaming pass over A and two fixed-order sums.
// parts: dense_blocks * d floats; parts2: dense_sum_groups * d; g: d.
hipError_t launch_dense_F(const float *A, long n, int d, const float *x, const float *Y,
                          const float *J, const float *mu, int K, bool linear, float *parts,
                          float *parts2, float *g, const int32_t *skip, hipStream_t st);
// Single-block finish on g: mode 0 z = g; 1 half step z = P(x - gamma g)
// and rho into the state; 2 full step (z may alias x), t and the stop test;
// 3 power iteration (x = v in, z = v out, lam and ||u|| into the state).
hipError_t launch_dense_finish(const float *g, int d, int mode, const float *x, float gamma,
                               double radius, float *z, SolveState *state, hipStream_t st);

}  // namespace exact
