// C ABI of libexact (declared in include/exact.h): argument checks, the
// per-view geometry tables, and the host drivers of the operator, the power
// iteration and the extragradient solve.  All arithmetic of the path runs
// in the kernels of exact_kernels.hip.
#define EXACT_HOST_SIDE 1
#include "exact.h"
#include "exact_internal.h"
#include "exact_tables.h"

#include <cerrno>
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using exact::Geo;
using exact::SolveState;
using exact::SpecArg;
using exact::ViewGeom;
using exact::balanced_order;
using exact::block_lines;
using exact::block_weight;

struct exact_geometry_s {
    int N, V, B, half_turns, reach, nrow, covers;
    double pixel_cm, bin_cm;
    int device;
    ViewGeom *d_views;
    int32_t *d_blk, *d_order;
    std::vector<ViewGeom> h_views;
};

namespace {

thread_local std::string g_last_error;

struct Fail {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const std::string &msg) { throw Fail{code, msg}; }

void hip_check(hipError_t e, const char *what)
{
    if (e != hipSuccess)
        fail(e == hipErrorOutOfMemory ? -ENOMEM : -EIO,
             std::string(what) + ": " + hipGetErrorString(e));
}

template <class F>
int guarded(F &&body)
{
    try {
        g_last_error.clear();
        return body();
    } catch (const Fail &f) {
        g_last_error = f.msg;
        return f.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return -ENOMEM;
    } catch (...) {
        g_last_error = "unexpected internal error";
        return -EIO;
    }
}

Geo geo_of(const exact_geometry_s *g)
{
    return Geo{g->d_views, g->d_blk, g->d_order, g->N,     g->V,
               g->B,       g->nrow,  g->reach,   g->covers};
}

void check_geometry(const exact_geometry_s *g)
{
    if (!g)
        fail(-EINVAL, "geometry handle is NULL");
}

// Collapses the window weights (J_k = sum_j weight[j][k]) and validates the
// spectrum as the paper's parameter domain requires (Sec. 1.2: intensities
// positive, sensitivities nonnegative, attenuation positive).
SpecArg make_spec(const exact_spectrum *sp, double *sum_J_mu)
{
    if (!sp)
        fail(-EINVAL, "spectrum is NULL");
    const int K = sp->n_energies, Wn = sp->n_windows;
    if (K < 1 || K > exact::kMaxEnergies)
        fail(-EINVAL, "n_energies must be in [1, " + std::to_string(exact::kMaxEnergies) + "]");
    if (Wn < 1)
        fail(-EINVAL, "n_windows must be >= 1");
    if (!sp->mu || !sp->weight)
        fail(-EINVAL, "spectrum arrays are NULL");
    SpecArg a;
    std::memset(&a, 0, sizeof(a));
    a.K = K;
    double sjm = 0.0;
    for (int k = 0; k < K; ++k) {
        const double mu = sp->mu[k];
        if (!(std::isfinite(mu) && mu > 0.0))
            fail(-EINVAL, "mu[" + std::to_string(k) + "] must be finite and > 0");
        double J = 0.0;
        for (int j = 0; j < Wn; ++j) {
            const double w = sp->weight[(size_t)j * K + k];
            if (!(std::isfinite(w) && w >= 0.0))
                fail(-EINVAL, "weight[" + std::to_string(j) + "][" + std::to_string(k) +
                                  "] must be finite and >= 0");
            J += w;
        }
        a.J[k] = (float)J;
        a.mu[k] = (float)mu;
        a.mu2[k] = (float)((long double)mu * 1.44269504088896340735992468100189214L);
        sjm += J * mu;
    }
    for (int j = 0; j < Wn; ++j) {
        double row = 0.0;
        for (int k = 0; k < K; ++k)
            row += sp->weight[(size_t)j * K + k];
        if (!(row > 0.0))
            fail(-EINVAL, "window " + std::to_string(j) + " has zero total weight");
    }
    if (sum_J_mu)
        *sum_J_mu = sjm;
    a.bg = sp->background;
    return a;
}

// Rounds to the nearest multiple of 2^-32.
long double fixed32(long double v) { return roundl(ldexpl(v, 32)) / 4294967296.0L; }

// Per-view parameters of the Joseph projector (see ViewGeom).  Computed in
// long double; A, P, Q are rounded once to multiples of 2^-32 pixel, which
// moves any crossing by at most (1 + b + k) 2^-33 pixel.  Sets *reach for the
// back-projector and fails if a crossing could leave the exact range.
std::vector<ViewGeom> build_views(int N, int V, int B, int half_turns, double pixel_cm,
                                  double bin_cm, int *reach, int *nrow)
{
    const long double pi = 3.14159265358979323846264338327950288L;
    const long double c = (N - 1) / 2.0L;
    const long double half = (B - 1) / 2.0L;
    const long double ratio = (long double)bin_cm / (long double)pixel_cm;
    std::vector<ViewGeom> rows, cols;
    long double pmin = 1e30L;
    for (int v = 0; v < V; ++v) {
        const long q = ((long)half_turns * v) % V;
        const bool row = 4 * q <= V || 4 * q >= 3L * V;
        const long double th = (long double)half_turns * pi * (long double)v / (long double)V;
        const long double ct = cosl(th), st = sinl(th);
        const long double cs = row ? ct : st;       // cosine along the stepping axis
        const long double sn = row ? st : ct;
        const long double P = fixed32(ratio / cs);
        const long double Q = fixed32(-sn / cs);
        const long double A = fixed32(c + c * sn / cs - half * ratio / cs);
        // largest crossing (or crossing minus pixel index) the kernels form:
        // b up to B + 64 (candidate bins beyond the detector are formed, then
        // discarded), k and j up to N
        const long double span = fabsl(A) + (B + 64) * fabsl(P) + N * fabsl(Q) + N + 4.0L;
        if (!(span < 1048576.0L))
            fail(-EINVAL, "geometry too large for exact crossing arithmetic (|crossing| >= 2^20)");
        ViewGeom G;
        std::memset(&G, 0, sizeof(G));
        G.A = (double)A;
        G.Ab = (double)(A - (long double)exact::kPadB * P);   // exact: multiples of 2^-32
        G.P = (double)P;
        G.Q = (double)Q;
        G.invP = (double)(1.0L / P);
        G.omP = (double)(1.0L - fabsl(P));                        // exact
        G.wstep = (float)((long double)pixel_cm / fabsl(cs));
        G.vidx = v;
        G.roff = v * exact::padded_bins(B);
        (row ? rows : cols).push_back(G);
        pmin = std::min(pmin, fabsl(P));
    }
    *nrow = (int)rows.size();
    std::vector<ViewGeom> out(rows);
    out.insert(out.end(), cols.begin(), cols.end());
    // Bins within one pixel of a pixel's crossing satisfy |b - b*| < 1/|P|;
    // the nearest bin b0 is within 1/2 (+ rounding) of b*.
    *reach = pmin >= 1.0L ? 0 : (int)floorl(1.0L / pmin + 0.5L + 0.01L);
    if (*reach > 32)
        fail(-EINVAL, "bins narrower than 1/32 of a pixel are not supported");
    return out;
}


// CUs of the current device and forward workgroups each holds at once.
void forward_residency(int device, int *cus, int *per_cu)
{
    hip_check(hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, device),
              "hipDeviceGetAttribute");
    *per_cu = exact::fwd_resident_blocks_per_cu();
}

// Whether the bin-pair rule needs no clamp: for every view and every pixel
// (j, k) of the image, t = -(A_b - j + k Q) / P (padded bin coordinate) lies
// in [-1/2, B + 2 kPadB - 3/2], so that trunc(t) is a bin of the padded row
// whose neighbour is too.  t is affine in (j, k), so the image's corners
// bound it; the half-bin margins dwarf the device's rounding of t.
int pair_covers(const std::vector<ViewGeom> &views, int N, int B, int reach)
{
    if (reach != 0)
        return 0;
    const long double lo = -0.5L, hi = (long double)(B + 2 * exact::kPadB) - 1.5L;
    for (const ViewGeom &G : views) {
        for (int cj = 0; cj < 2; ++cj)
            for (int ck = 0; ck < 2; ++ck) {
                const long double j = cj ? N - 1 : 0, k = ck ? N - 1 : 0;
                const long double t = -((long double)G.Ab - j + k * (long double)G.Q) /
                                      (long double)G.P;
                if (!(t >= lo && t <= hi))
                    return 0;
            }
    }
    return 1;
}

// Stream-ordered scratch buffer, released on the same stream.
struct AsyncBuf {
    void *p = nullptr;
    hipStream_t st = nullptr;
    AsyncBuf(size_t bytes, hipStream_t s) : st(s)
    {
        hip_check(hipMallocAsync(&p, bytes > 0 ? bytes : 16, st), "hipMallocAsync");
    }
    ~AsyncBuf()
    {
        if (p)
            (void)hipFreeAsync(p, st);
    }
    template <class T>
    T *as() const { return static_cast<T *>(p); }
    AsyncBuf(const AsyncBuf &) = delete;
    AsyncBuf &operator=(const AsyncBuf &) = delete;
};

// Plain device buffer for the blocking drivers.
struct DevBuf {
    void *p = nullptr;
    explicit DevBuf(size_t bytes) { hip_check(hipMalloc(&p, bytes > 0 ? bytes : 16), "hipMalloc"); }
    ~DevBuf()
    {
        if (p)
            (void)hipFree(p);
    }
    template <class T>
    T *as() const { return static_cast<T *>(p); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
};

struct PinnedState {
    SolveState *h = nullptr;
    PinnedState() { hip_check(hipHostMalloc((void **)&h, sizeof(SolveState), hipHostMallocDefault), "hipHostMalloc"); }
    ~PinnedState()
    {
        if (h)
            (void)hipHostFree(h);
    }
};

// A private non-blocking stream ordered after `user` (graph capture is not
// allowed on the legacy null stream, which torch may hand us).
struct OwnStream {
    hipStream_t st = nullptr;
    explicit OwnStream(hipStream_t user)
    {
        hip_check(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
        hipEvent_t ev;
        hip_check(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate");
        hip_check(hipEventRecord(ev, user), "hipEventRecord");
        hip_check(hipStreamWaitEvent(st, ev, 0), "hipStreamWaitEvent");
        (void)hipEventDestroy(ev);
    }
    ~OwnStream()
    {
        if (st) {
            (void)hipStreamSynchronize(st);
            (void)hipStreamDestroy(st);
        }
    }
};

void read_state(const SolveState *d, PinnedState &h, hipStream_t st)
{
    hip_check(hipMemcpyAsync(h.h, d, sizeof(SolveState), hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
}

// Power iteration for lambda_max(A^T A / n) on stream st (blocking).
double power_iteration(const exact_geometry_s *g, int max_iters, hipStream_t st, int *iters_out)
{
    const Geo G = geo_of(g);
    const long d = (long)g->N * g->N, n = (long)g->V * g->B;
    const int nparts = exact::num_dot_parts(d);
    const size_t dp = (size_t)exact::padded_image_floats(g->N);
    const size_t np = (size_t)g->V * exact::padded_bins(g->B);
    DevBuf v(d * 4), vp(dp * 4), vTp(dp * 4), u(d * 4), s(np * 4), parts(nparts * 3 * 8),
        state(sizeof(SolveState));
    PinnedState hs;
    hip_check(hipMemsetAsync(vp.p, 0, dp * 4, st), "hipMemsetAsync");
    hip_check(hipMemsetAsync(vTp.p, 0, dp * 4, st), "hipMemsetAsync");
    hip_check(hipMemsetAsync(s.p, 0, np * 4, st), "hipMemsetAsync");
    hip_check(exact::launch_fill(v.as<float>(), (float)(1.0 / std::sqrt((double)d)), d, st), "fill");
    hip_check(exact::launch_pad_pair(v.as<float>(), vp.as<float>(), vTp.as<float>(), g->N, st),
              "pad_pair");
    SolveState *S = state.as<SolveState>();
    hip_check(exact::launch_state_init(S, 0.0, max_iters, 0, st), "state_init");
    // steps go to the device in chunks; the stop test runs there (every
    // kernel of a step after the stop is a no-op), and the host reads the
    // state once per chunk
    constexpr int kChunk = 16;
    const int32_t *skip = &S->done;
    for (int it = 0; it < max_iters;) {
        for (int c = 0; c < kChunk && it < max_iters; ++c, ++it) {
            hip_check(exact::launch_forward(G, vp.as<float>(), vTp.as<float>(), s.as<float>(),
                                            exact::padded_bins(g->B), exact::kPadB, true, skip,
                                            st),
                      "forward");
            hip_check(exact::launch_back(G, s.as<float>(), u.as<float>(), (float)(1.0 / (double)n),
                                         skip, st),
                      "back");
            hip_check(exact::launch_dot3(v.as<float>(), u.as<float>(), g->N, parts.as<double>(),
                                         skip, st),
                      "dot3");
            hip_check(exact::launch_dot3_finish(parts.as<double>(), nparts, S, 1e-7, st),
                      "dot3_finish");
            hip_check(exact::launch_normalize(u.as<float>(), v.as<float>(), vp.as<float>(),
                                              vTp.as<float>(), g->N, S, st),
                      "normalize");
        }
        read_state(S, hs, st);
        if (hs.h->done)
            break;
    }
    if (hs.h->converged < 0)
        fail(-EIO, "power iteration produced a non-positive eigenvalue estimate");
    if (iters_out)
        *iters_out = hs.h->t;
    return hs.h->lam;
}
}  // namespace

extern "C" {

void exact_solve_opts_default(exact_solve_opts *o)
{
    if (!o)
        return;
    o->gamma = 0.0;
    o->gamma_scale = 0.25;
    o->max_iters = 500;
    o->tol = 0.0;
    o->stop_mode = EXACT_STOP_NATURAL_RESIDUAL;
    o->check_every = 16;
    o->power_iters = 100;
    o->lambda_hat = 0.0;
}

const char *exact_last_error(void) { return g_last_error.c_str(); }

int exact_geometry_create(int32_t n_pix, int32_t n_views, int32_t n_bins, int32_t half_turns,
                          double pixel_cm, double bin_cm, exact_geometry *out)
{
    return guarded([&]() -> int {
        if (!out)
            fail(-EINVAL, "out is NULL");
        *out = nullptr;
        if (n_pix < 1 || n_pix > 16384)
            fail(-EINVAL, "n_pix must be in [1, 16384]");
        // every element of the padded residual (n_views rows of n_bins + 4)
        // must have a 32-bit byte offset: the gather forms them that way
        if (n_views < 1 || n_bins < 1 ||
            (long long)n_views * ((long long)n_bins + 2 * exact::kPadB) >= (1LL << 30))
            fail(-EINVAL, "n_views, n_bins must be >= 1 with n_views*(n_bins+4) < 2^30");
        if (half_turns != 1 && half_turns != 2)
            fail(-EINVAL, "half_turns must be 1 (180 degrees) or 2 (360 degrees)");
        if (!(std::isfinite(pixel_cm) && pixel_cm > 0.0 && std::isfinite(bin_cm) && bin_cm > 0.0))
            fail(-EINVAL, "pixel_cm and bin_cm must be finite and > 0");
        auto *g = new exact_geometry_s();
        g->N = n_pix;
        g->V = n_views;
        g->B = n_bins;
        g->half_turns = half_turns;
        g->pixel_cm = pixel_cm;
        g->bin_cm = bin_cm;
        g->d_views = nullptr;
        g->d_blk = nullptr;
        g->d_order = nullptr;
        try {
            hip_check(hipGetDevice(&g->device), "hipGetDevice");
            g->h_views = build_views(n_pix, n_views, n_bins, half_turns, pixel_cm, bin_cm,
                                     &g->reach, &g->nrow);
            g->covers = pair_covers(g->h_views, n_pix, n_bins, g->reach);
            const size_t bytes = sizeof(ViewGeom) * (size_t)n_views;
            hip_check(hipMalloc((void **)&g->d_views, bytes), "hipMalloc");
            hip_check(hipMemcpy(g->d_views, g->h_views.data(), bytes, hipMemcpyHostToDevice),
                      "hipMemcpy");
            const std::vector<int32_t> blk = block_lines(g->h_views, n_pix, n_bins);
            hip_check(hipMalloc((void **)&g->d_blk, blk.size() * sizeof(int32_t)), "hipMalloc");
            hip_check(hipMemcpy(g->d_blk, blk.data(), blk.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice),
                      "hipMemcpy");
            int cus = 0, per_cu = 0;
            forward_residency(g->device, &cus, &per_cu);
            std::vector<long> w(blk.size() / 2);
            for (size_t i = 0; i < w.size(); ++i)
                w[i] = block_weight(blk, i);
            const std::vector<int32_t> order = balanced_order(w, cus, per_cu);
            hip_check(hipMalloc((void **)&g->d_order, order.size() * sizeof(int32_t)), "hipMalloc");
            hip_check(hipMemcpy(g->d_order, order.data(), order.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice),
                      "hipMemcpy");
        } catch (...) {
            if (g->d_views)
                (void)hipFree(g->d_views);
            if (g->d_blk)
                (void)hipFree(g->d_blk);
            if (g->d_order)
                (void)hipFree(g->d_order);
            delete g;
            throw;
        }
        *out = g;
        return 0;
    });
}

int exact_geometry_destroy(exact_geometry g)
{
    return guarded([&]() -> int {
        if (!g)
            return 0;
        // the handle and its tables are released whatever a free reports
        std::unique_ptr<exact_geometry_s> own(g);
        (void)hipDeviceSynchronize();
        const hipError_t e[3] = {g->d_views ? hipFree(g->d_views) : hipSuccess,
                                 g->d_blk ? hipFree(g->d_blk) : hipSuccess,
                                 g->d_order ? hipFree(g->d_order) : hipSuccess};
        for (hipError_t x : e)
            hip_check(x, "hipFree");
        return 0;
    });
}

int exact_forward(exact_geometry g, const float *x_dev, float *s_dev, void *stream)
{
    return guarded([&]() -> int {
        check_geometry(g);
        if (!x_dev || !s_dev)
            fail(-EINVAL, "NULL buffer");
        hipStream_t st = (hipStream_t)stream;
        const size_t dp = (size_t)exact::padded_image_floats(g->N);
        AsyncBuf xp(dp * sizeof(float), st), xTp(dp * sizeof(float), st);
        // the pad kernel writes the pair's zero padding too
        hip_check(exact::launch_pad_pair(x_dev, xp.as<float>(), xTp.as<float>(), g->N, st),
                  "pad_pair");
        hip_check(exact::launch_forward(geo_of(g), xp.as<float>(), xTp.as<float>(), s_dev, g->B, 0,
                                        false, nullptr, st),
                  "forward");
        return 0;
    });
}

int exact_backproject(exact_geometry g, const float *r_dev, float *img_dev, void *stream)
{
    return guarded([&]() -> int {
        check_geometry(g);
        if (!r_dev || !img_dev)
            fail(-EINVAL, "NULL buffer");
        hipStream_t st = (hipStream_t)stream;
        const size_t np = (size_t)g->V * exact::padded_bins(g->B);
        AsyncBuf rw(np * sizeof(float), st);
        // the weighing kernel writes the rows' zero padding too
        hip_check(exact::launch_weigh_rows(geo_of(g), r_dev, rw.as<float>(), st), "weigh_rows");
        hip_check(exact::launch_back(geo_of(g), rw.as<float>(), img_dev, 1.0f, nullptr, st),
                  "back");
        return 0;
    });
}

int exact_operator(exact_geometry g, const exact_spectrum *sp, const float *y_dev,
                   const float *x_dev, float *F_dev, float *r_dev, void *stream)
{
    return guarded([&]() -> int {
        check_geometry(g);
        if (!y_dev || !x_dev || !F_dev)
            fail(-EINVAL, "NULL buffer");
        const SpecArg a = make_spec(sp, nullptr);
        hipStream_t st = (hipStream_t)stream;
        const long n = (long)g->V * g->B;
        const size_t dp = (size_t)exact::padded_image_floats(g->N);
        const size_t np = (size_t)g->V * exact::padded_bins(g->B);
        AsyncBuf Y(n * sizeof(float), st), xp(dp * sizeof(float), st), xTp(dp * sizeof(float), st),
            rp(np * sizeof(float), st);
        // the pad kernel writes the image pair's zero padding; the forward
        // writes only the residual's interior bins, so its padding is cleared
        hip_check(hipMemsetAsync(rp.p, 0, np * sizeof(float), st), "hipMemsetAsync");
        hip_check(exact::launch_window_sum(y_dev, sp->n_windows, n, Y.as<float>(), nullptr, st),
                  "window_sum");
        hip_check(exact::launch_pad_pair(x_dev, xp.as<float>(), xTp.as<float>(), g->N, st),
                  "pad_pair");
        hip_check(exact::launch_forward_residual(geo_of(g), xp.as<float>(), xTp.as<float>(),
                                                 Y.as<float>(), a, rp.as<float>(), r_dev, nullptr,
                                                 st),
                  "forward_residual");
        hip_check(exact::launch_back(geo_of(g), rp.as<float>(), F_dev, (float)(1.0 / (double)n),
                                     nullptr, st),
                  "back");
        return 0;
    });
}

}  // extern "C"

// Scratch of exact_operator_noalloc: a file-scope device array, one copy per
// GPU, held until the process ends.  Host code never uses the array's name
// as an address (in host code it is a stand-in, not device memory): the
// device address comes from hipGetSymbolAddress, once per device, with that
// device current, and is kept below.
namespace {
constexpr size_t kNoAllocBytes = (size_t)EXACT_NOALLOC_SCRATCH_MIB << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;      // per device ordinal, null until looked up

// The calling thread's current device's copy of `scratch`.
unsigned char *scratch_on(int device)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((size_t)device >= g_scratch_ptr.size())
        g_scratch_ptr.resize((size_t)device + 1, nullptr);
    if (!g_scratch_ptr[(size_t)device]) {
        void *ptr = nullptr;
        hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
        if (!ptr)
            fail(-EIO, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_ptr[(size_t)device] = ptr;
    }
    return static_cast<unsigned char *>(g_scratch_ptr[(size_t)device]);
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
}  // namespace

extern "C" {

int exact_operator_noalloc(exact_geometry g, const exact_spectrum *sp, const float *y_dev,
                           const float *x_dev, float *F_dev, float *r_dev, void *stream)
{
    return guarded([&]() -> int {
        check_geometry(g);
        if (!y_dev || !x_dev || !F_dev)
            fail(-EINVAL, "NULL buffer");
        const SpecArg a = make_spec(sp, nullptr);
        int device = -1;
        hip_check(hipGetDevice(&device), "hipGetDevice");
        if (device != g->device)
            fail(-EINVAL, "the geometry was created on device " + std::to_string(g->device) +
                              ", the current device is " + std::to_string(device));
        const long n = (long)g->V * g->B;
        const size_t dp = (size_t)exact::padded_image_floats(g->N);
        const size_t np = (size_t)g->V * exact::padded_bins(g->B);
        const size_t oY = 0, oxp = align256(4 * (size_t)n), oxTp = oxp + align256(4 * dp),
                     orp = oxTp + align256(4 * dp), need = orp + align256(4 * np);
        if (need > kNoAllocBytes)
            fail(-ENOSPC, "exact_operator_noalloc needs " + std::to_string(need) +
                              " bytes of scratch; the static array holds " +
                              std::to_string(kNoAllocBytes));
        unsigned char *base = scratch_on(device);
        float *Y = reinterpret_cast<float *>(base + oY);
        float *xp = reinterpret_cast<float *>(base + oxp);
        float *xTp = reinterpret_cast<float *>(base + oxTp);
        float *rp = reinterpret_cast<float *>(base + orp);
        hipStream_t st = (hipStream_t)stream;
        // the array keeps the previous call's contents: the padding the
        // projectors read must be zero again.  The pad kernel writes the
        // image pair's padding; the residual's is cleared by a fill kernel
        // (not a memset, so that the call can be captured into a graph).
        hip_check(exact::launch_fill(rp, 0.f, (long)np, st), "fill");
        hip_check(exact::launch_window_sum(y_dev, sp->n_windows, n, Y, nullptr, st), "window_sum");
        hip_check(exact::launch_pad_pair(x_dev, xp, xTp, g->N, st), "pad_pair");
        hip_check(exact::launch_forward_residual(geo_of(g), xp, xTp, Y, a, rp, r_dev, nullptr, st),
                  "forward_residual");
        hip_check(exact::launch_back(geo_of(g), rp, F_dev, (float)(1.0 / (double)n), nullptr, st),
                  "back");
        return 0;
    });
}

int exact_step_size(exact_geometry g, const exact_spectrum *sp, int32_t max_iters,
                    double gamma_scale, double *lambda_out, double *gamma_out, void *stream)
{
    return guarded([&]() -> int {
        check_geometry(g);
        if (!lambda_out)
            fail(-EINVAL, "lambda_out is NULL");
        if (max_iters < 1)
            fail(-EINVAL, "max_iters must be >= 1");
        double sjm = 0.0;
        if (sp)
            make_spec(sp, &sjm);
        OwnStream own((hipStream_t)stream);
        const double lam = power_iteration(g, max_iters, own.st, nullptr);
        *lambda_out = lam;
        if (gamma_out)
            *gamma_out = sp ? gamma_scale / (lam * sjm) : 0.0;
        return 0;
    });
}

int exact_count_nonzeros(exact_geometry g, int64_t *nnz_out, void *stream)
{
    return guarded([&]() -> int {
        check_geometry(g);
        if (!nnz_out)
            fail(-EINVAL, "nnz_out is NULL");
        OwnStream own((hipStream_t)stream);
        const int nparts = exact::num_count_parts(geo_of(g));
        DevBuf parts((size_t)nparts * 8);
        std::vector<long long> h((size_t)nparts);
        hip_check(exact::launch_count_nonzeros(geo_of(g), parts.as<long long>(), own.st), "count");
        hip_check(hipMemcpyAsync(h.data(), parts.p, (size_t)nparts * 8, hipMemcpyDeviceToHost, own.st),
                  "hipMemcpyAsync");
        hip_check(hipStreamSynchronize(own.st), "hipStreamSynchronize");
        long long total = 0;
        for (long long c : h)
            total += c;
        *nnz_out = (int64_t)total;
        return 0;
    });
}

}  // extern "C"

// One extragradient run's device state: the spectrum, the window sums of
// y, the iterate and the half-step iterate with their transposes in the
// projectors' padded layout, the padded residual, the update partials.  The
// iterate itself
// is the caller's buffer.  `state` points at the run's SolveState (owned by
// the solver or the batch).
struct Problem {
    const exact_geometry_s *g = nullptr;
    SpecArg spec;
    double gamma = 0.0, lam = 0.0;
    int max_iters = 0;
    int stop_mode = EXACT_STOP_NATURAL_RESIDUAL;
    int avg_R = 0, avg_J = 0;                       // averaged-iterate ring (stop_mode 1)
    std::unique_ptr<DevBuf> avg_ring, avg_S, avg_parts;
    float *x = nullptr;
    std::unique_ptr<DevBuf> Y, r, xp, xTp, xhp, xhTp, parts, specd, bg;
    SolveState *state = nullptr;
    size_t footprint = 0;

    exact::BatchProb desc() const
    {
        exact::BatchProb d;
        std::memset(&d, 0, sizeof(d));
        d.views = g->d_views;
        d.blk = g->d_blk;
        d.N = g->N;
        d.V = g->V;
        d.B = g->B;
        d.nrow = g->nrow;
        d.reach = g->reach;
        d.covers = g->covers;
        d.K = spec.K;
        d.ntiles = exact::num_tiles(g->N);
        d.Y = Y->as<float>();
        d.J = specd->as<float>();
        d.mu2 = specd->as<float>() + exact::kMaxEnergies;
        d.bg = bg ? bg->as<float>() : nullptr;
        d.x = x;
        d.xp = xp->as<float>();
        d.xTp = xTp->as<float>();
        d.xhp = xhp->as<float>();
        d.xhTp = xhTp->as<float>();
        d.r = r->as<float>();
        d.parts = parts->as<double>();
        d.state = state;
        d.gamma = (float)gamma;
        d.inv_n = (float)(1.0 / ((double)g->V * g->B));
        return d;
    }
};

namespace {

// Device bytes one run allocates (besides the caller's x and y).
size_t run_footprint(int N, int V, int B)
{
    const size_t n = (size_t)V * B;
    const size_t dp = (size_t)exact::padded_image_floats(N), np = (size_t)V * exact::padded_bins(B);
    return 4 * (n + np + 4 * dp) + 16 * (size_t)exact::num_tiles(N) + 8 * exact::kMaxEnergies +
           sizeof(SolveState);
}

void validate_opts(exact_solve_opts &o)
{
    if (o.max_iters < 0)
        fail(-EINVAL, "max_iters must be >= 0");
    if (!(std::isfinite(o.tol) && o.tol >= 0.0))
        fail(-EINVAL, "tol must be finite and >= 0");
    if (o.stop_mode != EXACT_STOP_NATURAL_RESIDUAL && o.stop_mode != EXACT_STOP_AVERAGED_ITERATE)
        fail(-EINVAL, "unsupported stop_mode");
    if (!std::isfinite(o.gamma))
        fail(-EINVAL, "gamma must be finite");
    if (o.gamma <= 0.0 && !(std::isfinite(o.gamma_scale) && o.gamma_scale > 0.0))
        fail(-EINVAL, "gamma_scale must be > 0 when gamma is automatic");
    if (!(std::isfinite(o.lambda_hat) && o.lambda_hat >= 0.0))
        fail(-EINVAL, "lambda_hat must be finite and >= 0");
    if (o.check_every < 1)
        o.check_every = 1;
    if (o.power_iters < 1)
        o.power_iters = 1;
}

// Validates the inputs, sums the windows of y, checks y and x_1 on the
// device, picks the step size (Theorem 2's rule by power iteration unless
// given), writes x_1's transpose and initialises the device state.  Blocks.
void problem_init(Problem &p, const exact_geometry_s *g, const exact_spectrum *sp,
                  const float *y_dev, float *x_dev, exact_solve_opts o, SolveState *state,
                  hipStream_t st)
{
    check_geometry(g);
    if (!y_dev || !x_dev)
        fail(-EINVAL, "NULL buffer");
    validate_opts(o);
    double sjm = 0.0;
    p.g = g;
    p.spec = make_spec(sp, &sjm);
    p.x = x_dev;
    p.max_iters = o.max_iters;
    p.stop_mode = o.stop_mode;
    p.state = state;
    const long d = (long)g->N * g->N, n = (long)g->V * g->B;
    p.footprint = run_footprint(g->N, g->V, g->B) + (sp->background ? (size_t)n * 4 : 0);
    const size_t dp = (size_t)exact::padded_image_floats(g->N);
    const size_t np = (size_t)g->V * exact::padded_bins(g->B);
    p.Y.reset(new DevBuf(n * 4));
    p.r.reset(new DevBuf(np * 4));
    p.xp.reset(new DevBuf(dp * 4));
    p.xTp.reset(new DevBuf(dp * 4));
    p.xhp.reset(new DevBuf(dp * 4));
    p.xhTp.reset(new DevBuf(dp * 4));
    // the padding of these buffers must read zero; kernels never write it
    for (DevBuf *b : {p.r.get(), p.xp.get(), p.xTp.get(), p.xhp.get(), p.xhTp.get()})
        hip_check(hipMemsetAsync(b->p, 0, (b == p.r.get() ? np : dp) * 4, st), "hipMemsetAsync");
    p.parts.reset(new DevBuf((size_t)exact::num_tiles(g->N) * 2 * 8));
    p.specd.reset(new DevBuf(2 * exact::kMaxEnergies * 4));
    hip_check(hipMemcpyAsync(p.specd->p, p.spec.J, exact::kMaxEnergies * 4, hipMemcpyHostToDevice, st),
              "hipMemcpyAsync");
    hip_check(hipMemcpyAsync(p.specd->as<float>() + exact::kMaxEnergies, p.spec.mu2,
                             exact::kMaxEnergies * 4, hipMemcpyHostToDevice, st),
              "hipMemcpyAsync");

    // the run keeps its own copy of the known background
    if (sp->background) {
        p.bg.reset(new DevBuf(n * 4));
        hip_check(hipMemcpyAsync(p.bg->p, sp->background, n * 4, hipMemcpyDeviceToDevice, st),
                  "hipMemcpyAsync");
        p.spec.bg = p.bg->as<float>();
    }

    DevBuf bad(12);
    int32_t *badp = bad.as<int32_t>();
    hip_check(hipMemsetAsync(bad.p, 0, 12, st), "hipMemsetAsync");
    hip_check(exact::launch_window_sum(y_dev, sp->n_windows, n, p.Y->as<float>(), badp, st),
              "window_sum");
    hip_check(exact::launch_count_bad(x_dev, d, badp + 1, st), "count_bad");
    if (p.bg)
        hip_check(exact::launch_count_bad(p.bg->as<float>(), n, badp + 2, st), "count_bad");
    int32_t hbad[3] = {0, 0, 0};
    hip_check(hipMemcpyAsync(hbad, badp, 12, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    if (hbad[0])
        fail(-EINVAL, "y contains negative or non-finite counts");
    if (hbad[1])
        fail(-EINVAL, "x_1 contains negative or non-finite values");
    if (hbad[2])
        fail(-EINVAL, "background contains negative or non-finite values");

    p.gamma = o.gamma;
    if (p.gamma <= 0.0) {
        // Theorem 2: gamma = c / (lambda_max(A^T A / n) sum_k J_k mu_k)
        p.lam = o.lambda_hat > 0.0 ? o.lambda_hat : power_iteration(g, o.power_iters, st, nullptr);
        p.gamma = o.gamma_scale / (p.lam * sjm);
    }
    hip_check(exact::launch_pad_pair(x_dev, p.xp->as<float>(), p.xTp->as<float>(), g->N, st),
              "pad_pair");
    hip_check(exact::launch_state_init(state, o.tol, o.max_iters, o.stop_mode, st), "state_init");
    if (o.stop_mode == EXACT_STOP_AVERAGED_ITERATE) {
        p.avg_J = exact::avg_last_kept(o.max_iters);
        p.avg_R = exact::avg_ring_slots(o.max_iters);
        p.avg_ring.reset(new DevBuf((size_t)p.avg_R * (size_t)d * 4));
        p.avg_S.reset(new DevBuf((size_t)d * 8));
        p.avg_parts.reset(new DevBuf((size_t)exact::num_avg_parts(d) * 8));
        hip_check(exact::launch_avg_init(x_dev, p.avg_ring->as<float>(), p.avg_R, p.avg_J,
                                         p.avg_S->as<double>(), d, st),
                  "avg_init");
    }
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
}

void fill_info(const Problem &p, const SolveState &h, exact_solve_info *info,
               std::chrono::steady_clock::time_point t0)
{
    if (!info)
        return;
    info->iters = p.max_iters == 0 ? 0 : h.t;
    info->resid = p.max_iters == 0 ? -1.0
                  : p.stop_mode == EXACT_STOP_AVERAGED_ITERATE ? h.crit
                                                                : h.rho;
    info->gamma = p.gamma;
    info->lambda_hat = p.lam;
    info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// Steps per replay of a multi-step graph (a solver's or a batch's): a graph
// launch costs the host and the GPU a fixed overhead, which the steps of one
// graph share.  Steps after a run stops are no-ops on the device either way.
#ifndef EXACT_GRAPH_STEPS
#define EXACT_GRAPH_STEPS 8
#endif
constexpr int kGraphSteps = EXACT_GRAPH_STEPS;
static_assert(kGraphSteps >= 1, "steps per graph");

// n steps on stream own, ordered after the work on `user` and before what
// `user` enqueues next: replays of `multi` (kGraphSteps steps each), then of
// `one` for the rest.
void replay_steps(hipGraphExec_t one, hipGraphExec_t multi, int n, hipStream_t own,
                  hipStream_t user)
{
    hipEvent_t ev;
    hip_check(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate");
    hipError_t e = hipEventRecord(ev, user);
    if (e == hipSuccess)
        e = hipStreamWaitEvent(own, ev, 0);
    for (int c = 0; c + kGraphSteps <= n && e == hipSuccess; c += kGraphSteps)
        e = hipGraphLaunch(multi, own);
    for (int c = n - n % kGraphSteps; c < n && e == hipSuccess; ++c)
        e = hipGraphLaunch(one, own);
    if (e == hipSuccess)
        e = hipEventRecord(ev, own);
    if (e == hipSuccess)
        e = hipStreamWaitEvent(user, ev, 0);
    (void)hipEventDestroy(ev);
    hip_check(e, "graph replay");
}

struct Graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void reset()
    {
        if (exec)
            (void)hipGraphExecDestroy(exec);
        if (graph)
            (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
    ~Graph() { reset(); }
    // Captures whatever `enqueue` launches on st.
    template <class F>
    void capture(hipStream_t st, F &&enqueue)
    {
        reset();
        hip_check(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        const hipError_t ce = enqueue();
        const hipError_t ee = hipStreamEndCapture(st, &graph);
        hip_check(ce, "kernel launch during capture");
        hip_check(ee, "hipStreamEndCapture");
        hip_check(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    }
};

// The step finish's inputs: the update partials (and with the averaged
// rule its partials) and the run's state.
exact::FinishArgs finish_args(const Problem &p)
{
    const bool avg = p.stop_mode == EXACT_STOP_AVERAGED_ITERATE;
    const long d = (long)p.g->N * p.g->N;
    return exact::FinishArgs{p.parts->as<double>(), exact::num_tiles(p.g->N),
                             avg ? p.avg_parts->as<double>() : nullptr,
                             avg ? exact::num_avg_parts(d) : 0, p.state};
}

// Enqueue order of one extragradient step (paper Sec. 1.2, eq.
// extragrad-method): F at x_t, half-step from x_t, F at x_{t+1/2}, full step
// again from x_t, then the fixed-order residual reduction and stop test.
// In the captured graph (marks == nullptr) that finish runs inside the next
// step's first kernel, and the host settles the last one before it reads
// the state (settle_finish); with marks, for per-phase timing, it runs as
// its own kernel at the end of the step.
hipError_t enqueue_step(const Problem &p, hipStream_t st, hipEvent_t *marks = nullptr)
{
    const exact_geometry_s *g = p.g;
    const Geo G = geo_of(g);
    const long n = (long)g->V * g->B;
    const float gf = (float)p.gamma;
    const float inv_n = (float)(1.0 / (double)n);
    SolveState *S = p.state;
    const int32_t *skip = &S->done;
    float *Y = p.Y->as<float>(), *r = p.r->as<float>();
    float *xp = p.xp->as<float>(), *xTp = p.xTp->as<float>();
    float *xhp = p.xhp->as<float>(), *xhTp = p.xhTp->as<float>();
    double *parts = p.parts->as<double>();
    hipError_t e = hipSuccess;
    auto cap = [&](hipError_t x) {
        if (e == hipSuccess && x != hipSuccess)
            e = x;
    };
    int phase = 0;
    auto mark = [&]() {           // event before phase `phase` (and after the last)
        if (marks)
            cap(hipEventRecord(marks[phase], st));
        ++phase;
    };
    const exact::FinishArgs fin = finish_args(p);
    mark();
    cap(exact::launch_forward_residual(G, xp, xTp, Y, p.spec, r, nullptr, skip, st,
                                       marks ? nullptr : &fin));
    mark();
    cap(exact::launch_back_update(G, r, inv_n, p.x, gf, nullptr, xhp, xhTp, parts, skip, st));
    mark();
    cap(exact::launch_forward_residual(G, xhp, xhTp, Y, p.spec, r, nullptr, skip, st));
    mark();
    cap(exact::launch_back_update(G, r, inv_n, p.x, gf, p.x, xp, xTp, nullptr, skip, st));
    mark();
    if (p.stop_mode == EXACT_STOP_AVERAGED_ITERATE) {
        const long d = (long)g->N * g->N;
        cap(exact::launch_avg_step(p.x, p.avg_ring->as<float>(), p.avg_R, p.avg_J,
                                   p.avg_S->as<double>(), d, p.avg_parts->as<double>(), S, st));
    }
    if (marks)
        cap(exact::launch_eg_finish(fin.partials, fin.nparts, fin.avg_parts, fin.n_avg, S, st));
    mark();
    return e;
}

// Runs the last step's finish if the graph left it pending.
void settle_finish(const Problem &p, hipStream_t st)
{
    hip_check(exact::launch_eg_finish_pending(finish_args(p), st), "finish");
}

}  // namespace

// A resident extragradient run: its Problem, its state, a private stream
// and the captured step graph.
struct exact_solver_s {
    std::unique_ptr<OwnStream> own;
    std::unique_ptr<DevBuf> state;
    std::unique_ptr<PinnedState> hs;
    Problem prob;
    Graph step;       // one step
    Graph steps;      // kGraphSteps steps
    std::chrono::steady_clock::time_point t0;

    ~exact_solver_s()
    {
        if (own && own->st)
            (void)hipStreamSynchronize(own->st);
        step.reset();
        steps.reset();
    }
};

namespace {

exact_solver_s *solver_build(exact_geometry_s *g, const exact_spectrum *sp, const float *y_dev,
                             float *x_dev, const exact_solve_opts &o, hipStream_t user)
{
    std::unique_ptr<exact_solver_s> s(new exact_solver_s());
    s->t0 = std::chrono::steady_clock::now();
    check_geometry(g);
    s->own.reset(new OwnStream(user));
    s->state.reset(new DevBuf(sizeof(SolveState)));
    s->hs.reset(new PinnedState());
    problem_init(s->prob, g, sp, y_dev, x_dev, o, s->state->as<SolveState>(), s->own->st);
    const Problem &p = s->prob;
    s->step.capture(s->own->st, [&]() { return enqueue_step(p, s->own->st); });
    s->steps.capture(s->own->st, [&]() {
        hipError_t e = hipSuccess;
        for (int k = 0; k < kGraphSteps && e == hipSuccess; ++k)
            e = enqueue_step(p, s->own->st);
        return e;
    });
    return s.release();
}



int solver_poll(exact_solver_s *s, exact_solve_info *info)
{
    settle_finish(s->prob, s->own->st);
    read_state(s->prob.state, *s->hs, s->own->st);
    fill_info(s->prob, *s->hs->h, info, s->t0);
    return s->hs->h->done ? 1 : 0;
}

}  // namespace

// A batch: many runs of different shapes advanced together, one captured
// graph of five batched phase kernels per step.  Runs occupy slots; the
// device descriptors and item lists are rebuilt (and the graph recaptured)
// at the next step after a run joins or leaves.
struct exact_batch_s {
    size_t budget = 0, used = 0;
    int capacity = 0;
    std::unique_ptr<OwnStream> own;
    std::unique_ptr<DevBuf> states;                 // SolveState[capacity]
    SolveState *hstates = nullptr;                   // pinned host copy
    std::vector<std::unique_ptr<Problem>> slots;     // nullptr: free
    std::vector<std::chrono::steady_clock::time_point> started;
    std::vector<char> stopped;                       // host view, from the last sync
    bool dirty = true;
    std::unique_ptr<DevBuf> descs, fwd, back;
    int nprob = 0, nfwd = 0, nback = 0;
    Graph step;       // one step of every running scan
    Graph steps;      // kGraphSteps such steps

    ~exact_batch_s()
    {
        if (own && own->st)
            (void)hipStreamSynchronize(own->st);
        step.reset();
        steps.reset();
        if (hstates)
            (void)hipHostFree(hstates);
    }
};

namespace {

// Item lists of the runs still running (as of the last sync), heaviest
// first so the long tiles start early: runs by decreasing N, and each run's
// forward items centre-out (central bin blocks hold the longest chords).
// Items of one run stay together, so that the XCDs' L2 holds few runs'
// images at a time.  A run that stopped is left out: its workgroups would
// only return at once.
void batch_rebuild(exact_batch_s *b)
{
    std::vector<int> order;
    for (int i = 0; i < (int)b->slots.size(); ++i)
        if (b->slots[(size_t)i] && !b->stopped[(size_t)i])
            order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        return b->slots[(size_t)a]->g->N > b->slots[(size_t)c]->g->N;
    });
    std::vector<exact::BatchProb> descs;
    std::vector<exact::BatchItem> fwd, back;
    for (int slot : order) {
        const Problem &p = *b->slots[(size_t)slot];
        const int pi = (int)descs.size();
        descs.push_back(p.desc());
        const int nbb = exact::fwd_items_per_view(p.g->B);
        for (int rk = 0; rk < nbb; ++rk)
            for (int v = 0; v < p.g->V; ++v)
                fwd.push_back(exact::BatchItem{pi, v, exact::fwd_block_centre_out(rk, nbb), 0});
        const int bt = exact::back_tiles_per_side(p.g->N);
        for (int ty = 0; ty < bt; ++ty)
            for (int tx = 0; tx < bt; ++tx)
                back.push_back(exact::BatchItem{pi, tx, ty, 0});
    }
    hipStream_t st = b->own->st;
    auto upload = [&](std::unique_ptr<DevBuf> &buf, const void *src, size_t bytes) {
        buf.reset(new DevBuf(bytes));
        if (bytes)
            hip_check(hipMemcpyAsync(buf->p, src, bytes, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    };
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    upload(b->descs, descs.data(), descs.size() * sizeof(exact::BatchProb));
    upload(b->fwd, fwd.data(), fwd.size() * sizeof(exact::BatchItem));
    upload(b->back, back.data(), back.size() * sizeof(exact::BatchItem));
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    b->nprob = (int)descs.size();
    b->nfwd = (int)fwd.size();
    b->nback = (int)back.size();
    const exact::BatchProb *dp = b->descs->as<exact::BatchProb>();
    const exact::BatchItem *f = b->fwd->as<exact::BatchItem>(), *bk = b->back->as<exact::BatchItem>();
    b->step.capture(st, [&]() {
        return exact::launch_batch_step(dp, b->nprob, f, b->nfwd, bk, b->nback, st);
    });
    b->steps.capture(st, [&]() {
        hipError_t e = hipSuccess;
        for (int k = 0; k < kGraphSteps && e == hipSuccess; ++k)
            e = exact::launch_batch_step(dp, b->nprob, f, b->nfwd, bk, b->nback, st);
        return e;
    });
    b->dirty = false;
}

exact_batch_s *batch_of(exact_batch b)
{
    if (!b)
        fail(-EINVAL, "batch is NULL");
    return b;
}

Problem &slot_of(exact_batch_s *b, int32_t slot)
{
    if (slot < 0 || slot >= (int)b->slots.size() || !b->slots[(size_t)slot])
        fail(-EINVAL, "no run in slot " + std::to_string(slot));
    return *b->slots[(size_t)slot];
}

}  // namespace

extern "C" {

int exact_solver_create(exact_geometry g, const exact_spectrum *sp, const float *y_dev,
                        float *x_dev, const exact_solve_opts *opts, exact_solver *out,
                        void *stream)
{
    return guarded([&]() -> int {
        if (!out)
            fail(-EINVAL, "out is NULL");
        *out = nullptr;
        exact_solve_opts o;
        exact_solve_opts_default(&o);
        if (opts)
            o = *opts;
        if (o.stop_mode == EXACT_STOP_AVERAGED_ITERATE)
            fail(-EINVAL, "the averaged-iterate stop rule is available in exact_solve only");
        *out = solver_build(g, sp, y_dev, x_dev, o, (hipStream_t)stream);
        return 0;
    });
}

int exact_solver_profile(exact_solver s, int32_t n_steps, double *phase_ms, void *stream)
{
    return guarded([&]() -> int {
        if (!s)
            fail(-EINVAL, "solver is NULL");
        if (!phase_ms)
            fail(-EINVAL, "phase_ms is NULL");
        if (n_steps < 1 || n_steps > 4096)
            fail(-EINVAL, "n_steps must be in [1, 4096]");
        constexpr int kMarks = EXACT_STEP_PHASES + 1;
        std::vector<hipEvent_t> ev((size_t)n_steps * kMarks, nullptr);
        struct Events {
            std::vector<hipEvent_t> &v;
            ~Events()
            {
                for (hipEvent_t e : v)
                    if (e)
                        (void)hipEventDestroy(e);
            }
        } guard{ev};
        for (hipEvent_t &e : ev)
            hip_check(hipEventCreate(&e), "hipEventCreate");
        hipStream_t own = s->own->st, user = (hipStream_t)stream;
        hipEvent_t order;
        hip_check(hipEventCreateWithFlags(&order, hipEventDisableTiming), "hipEventCreate");
        hipError_t e = hipEventRecord(order, user);
        if (e == hipSuccess)
            e = hipStreamWaitEvent(own, order, 0);
        // a finish the graph left pending runs first: each profiled step
        // then runs its own
        if (e == hipSuccess)
            e = exact::launch_eg_finish_pending(finish_args(s->prob), own);
        for (int t = 0; t < n_steps && e == hipSuccess; ++t)
            e = enqueue_step(s->prob, own, ev.data() + (size_t)t * kMarks);
        if (e == hipSuccess)
            e = hipEventRecord(order, own);
        if (e == hipSuccess)
            e = hipStreamWaitEvent(user, order, 0);
        if (e == hipSuccess)
            e = hipStreamSynchronize(own);
        (void)hipEventDestroy(order);
        hip_check(e, "profiled steps");
        for (int q = 0; q < EXACT_STEP_PHASES; ++q) {
            double sum = 0.0;
            for (int t = 0; t < n_steps; ++t) {
                float ms = 0.f;
                hip_check(hipEventElapsedTime(&ms, ev[(size_t)t * kMarks + q],
                                              ev[(size_t)t * kMarks + q + 1]),
                          "hipEventElapsedTime");
                sum += ms;
            }
            phase_ms[q] = sum / n_steps;
        }
        return 0;
    });
}

int exact_solver_time_kernels(exact_solver s, int32_t reps, double *kernel_ms, void *stream)
{
    return guarded([&]() -> int {
        if (!s)
            fail(-EINVAL, "solver is NULL");
        if (!kernel_ms)
            fail(-EINVAL, "kernel_ms is NULL");
        if (reps < 1 || reps > 4096)
            fail(-EINVAL, "reps must be in [1, 4096]");
        const Problem &p = s->prob;
        const exact_geometry_s *g = p.g;
        const Geo G = geo_of(g);
        const long d = (long)g->N * g->N, n = (long)g->V * g->B;
        const size_t dp = (size_t)exact::padded_image_floats(g->N);
        const float gf = (float)p.gamma;
        const float inv_n = (float)(1.0 / (double)n);
        hipStream_t own = s->own->st, user = (hipStream_t)stream;
        // scratch: the full step's image and padded pair, and a state copy
        // that the reduction may advance (never done, so no kernel skips)
        DevBuf z((size_t)d * 4), zp(dp * 4), zTp(dp * 4), state(sizeof(SolveState));
        SolveState *S = state.as<SolveState>();
        const int32_t *skip = &S->done;
        hipEvent_t order;
        hip_check(hipEventCreateWithFlags(&order, hipEventDisableTiming), "hipEventCreate");
        hipEvent_t ev[EXACT_STEP_PHASES + 1] = {};
        struct Events {
            hipEvent_t *v;
            hipEvent_t o;
            ~Events()
            {
                for (int i = 0; i <= EXACT_STEP_PHASES; ++i)
                    if (v[i])
                        (void)hipEventDestroy(v[i]);
                (void)hipEventDestroy(o);
            }
        } guard{ev, order};
        for (hipEvent_t &e : ev)
            hip_check(hipEventCreate(&e), "hipEventCreate");
        hip_check(hipEventRecord(order, user), "hipEventRecord");
        hip_check(hipStreamWaitEvent(own, order, 0), "hipStreamWaitEvent");
        // the graph's pending finish first, so the run's state is settled
        hip_check(exact::launch_eg_finish_pending(finish_args(p), own), "finish");
        hip_check(exact::launch_fill(zp.as<float>(), 0.f, (long)dp, own), "fill");
        hip_check(exact::launch_fill(zTp.as<float>(), 0.f, (long)dp, own), "fill");
        hip_check(exact::launch_state_init(S, 0.0, 0x7fffffff, 0, own), "state_init");
        const exact::FinishArgs fin = finish_args(p);
        float *Y = p.Y->as<float>(), *r = p.r->as<float>();
        float *xp = p.xp->as<float>(), *xTp = p.xTp->as<float>();
        float *xhp = p.xhp->as<float>(), *xhTp = p.xhTp->as<float>();
        double *parts = p.parts->as<double>();
        // one launch of the phase's kernel
        auto launch = [&](int q) -> hipError_t {
            switch (q) {
            case 0:
                return exact::launch_forward_residual(G, xp, xTp, Y, p.spec, r, nullptr, skip, own);
            case 1:
                return exact::launch_back_update(G, r, inv_n, p.x, gf, nullptr, xhp, xhTp, parts,
                                                 skip, own);
            case 2:
                return exact::launch_forward_residual(G, xhp, xhTp, Y, p.spec, r, nullptr, skip,
                                                      own);
            case 3:
                return exact::launch_back_update(G, r, inv_n, p.x, gf, z.as<float>(),
                                                 zp.as<float>(), zTp.as<float>(), nullptr, skip,
                                                 own);
            default:
                return exact::launch_eg_finish(fin.partials, fin.nparts, fin.avg_parts, fin.n_avg,
                                               S, own);
            }
        };
        // two passes over the phases, the first untimed (clocks and caches
        // settle), the second between the events
        for (int pass = 0; pass < 2; ++pass) {
            for (int q = 0; q < EXACT_STEP_PHASES; ++q) {
                if (pass == 1)
                    hip_check(hipEventRecord(ev[q], own), "hipEventRecord");
                for (int k = 0; k < reps; ++k)
                    hip_check(launch(q), "timed kernel");
            }
        }
        hip_check(hipEventRecord(ev[EXACT_STEP_PHASES], own), "hipEventRecord");
        hip_check(hipEventRecord(order, own), "hipEventRecord");
        hip_check(hipStreamWaitEvent(user, order, 0), "hipStreamWaitEvent");
        hip_check(hipStreamSynchronize(own), "hipStreamSynchronize");
        for (int q = 0; q < EXACT_STEP_PHASES; ++q) {
            float ms = 0.f;
            hip_check(hipEventElapsedTime(&ms, ev[q], ev[q + 1]), "hipEventElapsedTime");
            kernel_ms[q] = (double)ms / reps;
        }
        return 0;
    });
}

int exact_solver_step(exact_solver s, int32_t n_steps, void *stream)
{
    return guarded([&]() -> int {
        if (!s)
            fail(-EINVAL, "solver is NULL");
        if (n_steps < 0)
            fail(-EINVAL, "n_steps must be >= 0");
        replay_steps(s->step.exec, s->steps.exec, n_steps, s->own->st, (hipStream_t)stream);
        return 0;
    });
}

int exact_solver_poll(exact_solver s, exact_solve_info *info)
{
    return guarded([&]() -> int {
        if (!s)
            fail(-EINVAL, "solver is NULL");
        return solver_poll(s, info);
    });
}

int exact_solver_destroy(exact_solver s)
{
    return guarded([&]() -> int {
        delete s;
        return 0;
    });
}

int exact_solve(exact_geometry g, const exact_spectrum *sp, const float *y_dev, float *x_dev,
                const exact_solve_opts *opts, exact_solve_info *info, void *stream)
{
    return guarded([&]() -> int {
        const auto t0 = std::chrono::steady_clock::now();
        exact_solve_opts o;
        exact_solve_opts_default(&o);
        if (opts)
            o = *opts;
        std::unique_ptr<exact_solver_s> s(solver_build(g, sp, y_dev, x_dev, o, (hipStream_t)stream));
        validate_opts(o);
        int launched = 0;
        exact_solve_info local;
        while (launched < o.max_iters) {
            const int chunk = std::min(o.check_every, o.max_iters - launched);
            replay_steps(s->step.exec, s->steps.exec, chunk, s->own->st, (hipStream_t)stream);
            launched += chunk;
            if (solver_poll(s.get(), &local))
                break;
        }
        if (o.stop_mode == EXACT_STOP_AVERAGED_ITERATE) {
            const Problem &p = s->prob;
            hip_check(exact::launch_avg_output(p.avg_S->as<double>(), p.x,
                                               (long)p.g->N * p.g->N, p.state, s->own->st),
                      "avg_output");
        }
        solver_poll(s.get(), &local);
        const bool converged = s->hs->h->converged != 0;
        s.reset();
        local.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (info)
            *info = local;
        if (o.tol > 0.0 && !converged)
            return EXACT_ENOTCONV;
        return 0;
    });
}

size_t exact_run_footprint(int32_t n_pix, int32_t n_views, int32_t n_bins)
{
    if (n_pix < 1 || n_views < 1 || n_bins < 1)
        return 0;
    return run_footprint(n_pix, n_views, n_bins);
}

int exact_batch_create(size_t hbm_budget_bytes, int32_t capacity, exact_batch *out)
{
    return guarded([&]() -> int {
        if (!out)
            fail(-EINVAL, "out is NULL");
        *out = nullptr;
        if (capacity < 1 || capacity > 65536)
            fail(-EINVAL, "capacity must be in [1, 65536]");
        std::unique_ptr<exact_batch_s> b(new exact_batch_s());
        b->budget = hbm_budget_bytes;
        b->capacity = capacity;
        b->own.reset(new OwnStream(nullptr));
        b->states.reset(new DevBuf(sizeof(SolveState) * (size_t)capacity));
        hip_check(hipHostMalloc((void **)&b->hstates, sizeof(SolveState) * (size_t)capacity,
                                hipHostMallocDefault),
                  "hipHostMalloc");
        std::memset(b->hstates, 0, sizeof(SolveState) * (size_t)capacity);
        b->slots.resize((size_t)capacity);
        b->started.resize((size_t)capacity);
        b->stopped.assign((size_t)capacity, 0);
        *out = b.release();
        return 0;
    });
}

int exact_batch_add(exact_batch bh, exact_geometry g, const exact_spectrum *sp, const float *y_dev,
                    float *x_dev, const exact_solve_opts *opts, int32_t *slot_out, void *stream)
{
    return guarded([&]() -> int {
        exact_batch_s *b = batch_of(bh);
        check_geometry(g);
        if (!slot_out)
            fail(-EINVAL, "slot_out is NULL");
        *slot_out = -1;
        const size_t need = run_footprint(g->N, g->V, g->B) +
                            (sp && sp->background ? (size_t)g->V * g->B * 4 : 0);
        if (b->used + need > b->budget)
            fail(-ENOSPC, "run needs " + std::to_string(need) + " bytes, " +
                              std::to_string(b->budget - b->used) + " left in the batch budget");
        int slot = -1;
        for (int i = 0; i < b->capacity; ++i)
            if (!b->slots[(size_t)i]) {
                slot = i;
                break;
            }
        if (slot < 0)
            fail(-ENOSPC, "all " + std::to_string(b->capacity) + " slots are in use");
        exact_solve_opts o;
        exact_solve_opts_default(&o);
        if (opts)
            o = *opts;
        if (o.stop_mode == EXACT_STOP_AVERAGED_ITERATE)
            fail(-EINVAL, "the averaged-iterate stop rule is available in exact_solve only");
        std::unique_ptr<Problem> p(new Problem());
        // set-up runs on the batch's stream, after the caller's stream
        hip_check(hipStreamSynchronize(b->own->st), "hipStreamSynchronize");
        hip_check(hipStreamSynchronize((hipStream_t)stream), "hipStreamSynchronize");
        problem_init(*p, g, sp, y_dev, x_dev, o, b->states->as<SolveState>() + slot, b->own->st);
        b->used += p->footprint;
        b->slots[(size_t)slot] = std::move(p);
        b->started[(size_t)slot] = std::chrono::steady_clock::now();
        std::memset(&b->hstates[slot], 0, sizeof(SolveState));
        b->stopped[(size_t)slot] = 0;
        b->dirty = true;
        *slot_out = slot;
        return 0;
    });
}

int exact_batch_step(exact_batch bh, int32_t n_steps, void *stream)
{
    return guarded([&]() -> int {
        exact_batch_s *b = batch_of(bh);
        if (n_steps < 0)
            fail(-EINVAL, "n_steps must be >= 0");
        if (b->dirty)
            batch_rebuild(b);
        if (b->nprob == 0 || n_steps == 0)
            return 0;
        replay_steps(b->step.exec, b->steps.exec, n_steps, b->own->st, (hipStream_t)stream);
        return 0;
    });
}

int exact_batch_sync(exact_batch bh)
{
    return guarded([&]() -> int {
        exact_batch_s *b = batch_of(bh);
        hip_check(hipMemcpyAsync(b->hstates, b->states->p, sizeof(SolveState) * (size_t)b->capacity,
                                 hipMemcpyDeviceToHost, b->own->st),
                  "hipMemcpyAsync");
        hip_check(hipStreamSynchronize(b->own->st), "hipStreamSynchronize");
        int running = 0;
        for (int i = 0; i < b->capacity; ++i) {
            if (!b->slots[(size_t)i])
                continue;
            if (b->hstates[i].done) {
                if (!b->stopped[(size_t)i]) {
                    b->stopped[(size_t)i] = 1;
                    b->dirty = true;        // drop its items at the next step
                }
            } else {
                ++running;
            }
        }
        return running;
    });
}

int exact_batch_poll(exact_batch bh, int32_t slot, exact_solve_info *info)
{
    return guarded([&]() -> int {
        exact_batch_s *b = batch_of(bh);
        const Problem &p = slot_of(b, slot);
        const SolveState &h = b->hstates[slot];
        fill_info(p, h, info, b->started[(size_t)slot]);
        if (!h.done)
            return 0;
        return (h.converged || p.max_iters == 0 || h.tol <= 0.0) ? 1 : 2;
    });
}

int exact_batch_remove(exact_batch bh, int32_t slot)
{
    return guarded([&]() -> int {
        exact_batch_s *b = batch_of(bh);
        Problem &p = slot_of(b, slot);
        hip_check(hipStreamSynchronize(b->own->st), "hipStreamSynchronize");
        b->used -= p.footprint;
        b->slots[(size_t)slot].reset();
        if (!b->stopped[(size_t)slot])
            b->dirty = true;
        b->stopped[(size_t)slot] = 0;
        return 0;
    });
}

int exact_batch_destroy(exact_batch bh)
{
    return guarded([&]() -> int {
        delete bh;
        return 0;
    });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// TV ball and orthant (the constraint set of the paper's experiments)

namespace {

void validate_tv_opts(const exact_tv_opts &o)
{
    if (!(std::isfinite(o.tv_tol) && o.tv_tol >= 0.0))
        fail(-EINVAL, "tv_tol must be finite and >= 0");
    if (o.prox_iters < 1 || o.prox_iters > 100000)
        fail(-EINVAL, "prox_iters must be in [1, 100000]");
    if (o.max_bisect < 0 || o.max_bisect > 200)
        fail(-EINVAL, "max_bisect must be in [0, 200]");
    if (!(std::isfinite(o.dyk_tol) && o.dyk_tol >= 0.0))
        fail(-EINVAL, "dyk_tol must be finite and >= 0");
    if (o.max_outer < 1)
        fail(-EINVAL, "max_outer must be >= 1");
}

// Device work of the TV projection for one image size: the FGP fields, the
// TV-ball and Dykstra buffers and the reduction results.  A proximal solve
// is a short run of kernel launches (the weight a kernel argument) ending in
// the point's TV, which the last kernel writes to pinned host memory, and
// after it a sequence word; the host polls that word (no wake-up latency of
// a blocking stream wait) and reads the result.  A search keeps its current
// result in one of two output buffers and solves into the other, so keeping
// a point moves no data.
struct TvWork {
    int N = 0;
    long d = 0;
    exact_tv_opts o;
    std::unique_ptr<DevBuf> p, q, r, s, p2, q2, r2, s2, xb[2], w, z, dp, dq, parts;
    double *h = nullptr;       // pinned, coherent: [1..2] reduction results, [3] the sequence word
    double *hd = nullptr;      // its device address
    unsigned *fh = nullptr;    // the sequence word, host address
    unsigned *fd = nullptr;    // and device address
    unsigned seq = 0;          // the last sequence number handed out
    int solves = 0;

    TvWork(int n, const exact_tv_opts &opts, hipStream_t) : N(n), d((long)n * n), o(opts)
    {
        for (auto *b : {&p, &q, &r, &s, &p2, &q2, &r2, &s2, &xb[0], &xb[1], &w, &z, &dp, &dq})
            b->reset(new DevBuf((size_t)d * 4));
        const int np = std::max(exact::num_tv_parts(n), 2 * exact::num_flat_parts(d));
        parts.reset(new DevBuf((size_t)np * 8));
        hip_check(hipHostMalloc((void **)&h, 32, hipHostMallocMapped | hipHostMallocCoherent),
                  "hipHostMalloc");
        hip_check(hipHostGetDevicePointer((void **)&hd, h, 0), "hipHostGetDevicePointer");
        fh = reinterpret_cast<unsigned *>(h + 3);
        fd = reinterpret_cast<unsigned *>(hd + 3);
        __atomic_store_n(fh, 0u, __ATOMIC_RELEASE);
    }
    ~TvWork()
    {
        if (h)
            (void)hipHostFree(h);
    }

    // The next sequence number (never 0, the word's initial value).
    unsigned next()
    {
        if (++seq == 0)
            ++seq;
        return seq;
    }
    // Waits until the kernel that writes sequence number `want` has posted
    // it, by polling the pinned word.  After 2 s without it, a stream
    // synchronize waits for the stream and reports any error, and the word
    // must then hold `want`.
    void wait(unsigned want, hipStream_t st)
    {
        const auto t0 = std::chrono::steady_clock::now();
        for (long spin = 1;; ++spin) {
            if (__atomic_load_n(fh, __ATOMIC_ACQUIRE) == want)
                return;
            if (spin % 4096 == 0 &&
                std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) {
                hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
                if (__atomic_load_n(fh, __ATOMIC_ACQUIRE) != want)
                    fail(-EIO, "a TV reduction result was not posted");
                return;
            }
        }
    }
    // The reduction result the kernel posting `want` wrote to h[1].
    double sync1(unsigned want, hipStream_t st)
    {
        wait(want, st);
        return h[1];
    }
    double tv_of(const float *img, hipStream_t st)
    {
        const unsigned q1 = next();
        hip_check(exact::launch_tv_norm(img, N, parts->as<double>(), hd + 1, st, fd, q1),
                  "tv_norm");
        return sync1(q1, st);
    }
    // xb[k] = TV-regularized point of w for weight l; returns TV(xb[k]).
    double solve(int k, double l, hipStream_t st)
    {
        const unsigned q1 = next();
        hip_check(exact::launch_prox(w->as<float>(), p->as<float>(), q->as<float>(),
                                     r->as<float>(), s->as<float>(), p2->as<float>(),
                                     q2->as<float>(), r2->as<float>(), s2->as<float>(), l,
                                     o.prox_iters, xb[k]->as<float>(), N, parts->as<double>(),
                                     hd + 1, st, fd, q1),
                  "prox");
        ++solves;
        return sync1(q1, st);
    }
    void copy(float *dst, const float *src, hipStream_t st)
    {
        hip_check(hipMemcpyAsync(dst, src, (size_t)d * 4, hipMemcpyDeviceToDevice, st),
                  "hipMemcpyAsync");
    }

    // Weight of the last TV-ball point this work found (0: none yet); the
    // next search starts there.
    double lam_carry = 0.0;

    // Approximate projection of w onto {TV <= tau} (binary search on the TV
    // weight, cold or warm-started from lam_carry, the decisions of the
    // definition in the header), given tw = TV(w).  Returns the buffer that
    // holds the result: w itself, or xb[0] or xb[1].
    const float *tv_ball(double tau, double tw, hipStream_t st)
    {
        if (tw <= tau)
            return w->as<float>();
        int cur = 0;               // the buffer the next solve writes
        const float *res = nullptr;
        double lo = 0.0, hi = 1.0, t = 0.0, lam = 0.0;
        bool hit = false;
        auto sol = [&](double l) { return solve(cur, l, st); };
        auto keep = [&](double l) {   // the last solve's point is the result so far
            res = xb[cur]->as<float>();
            cur ^= 1;
            lam = l;
        };
        const double lam0 = lam_carry;
        if (lam0 <= 0.0) {
            t = sol(hi);
            for (int grow = 0; t > tau && grow < 60; ++grow) {
                lo = hi;
                hi = 2.0 * hi;
                t = sol(hi);
            }
            keep(hi);
        } else {
            t = sol(lam0);
            if (std::fabs(t - tau) <= o.tv_tol) {
                keep(lam0);
                hit = true;
            } else if (t > tau) {
                lo = lam0;
                hi = lam0 * 5.0 / 4.0;
                for (int grow = 0;; ++grow) {
                    t = sol(hi);
                    if (std::fabs(t - tau) <= o.tv_tol) {
                        keep(hi);
                        hit = true;
                        break;
                    }
                    if (t <= tau || grow + 1 >= 60)
                        break;
                    lo = hi;
                    hi = 2.0 * hi;
                }
                if (!hit)
                    keep(hi);
            } else {
                hi = lam0;
                keep(hi);
                lo = lam0 * 4.0 / 5.0;
                for (int shrink = 0;; ++shrink) {
                    t = sol(lo);
                    if (std::fabs(t - tau) <= o.tv_tol) {
                        keep(lo);
                        hit = true;
                        break;
                    }
                    if (t > tau)
                        break;
                    hi = lo;
                    keep(hi);
                    if (shrink + 1 >= 60) {
                        lo = 0.0;
                        break;
                    }
                    lo = lo / 2.0;
                }
            }
        }
        for (int it = 0; !hit && it < o.max_bisect; ++it) {
            const double mid = 0.5 * (lo + hi);
            t = sol(mid);
            if (std::fabs(t - tau) <= o.tv_tol) {
                keep(mid);
                break;
            }
            if (t > tau) {
                lo = mid;
            } else {
                hi = mid;
                keep(mid);
            }
        }
        lam_carry = lam;
        return res;
    }

    // out = projection of in onto {TV <= tau} and the orthant (Dykstra).
    // Returns the rounds taken.
    int project(const float *in, float *outp, double tau, hipStream_t st)
    {
        float *zp = z->as<float>(), *pp = dp->as<float>(), *qp = dq->as<float>();
        copy(zp, in, st);
        hip_check(hipMemsetAsync(pp, 0, (size_t)d * 4, st), "hipMemsetAsync");
        hip_check(hipMemsetAsync(qp, 0, (size_t)d * 4, st), "hipMemsetAsync");
        int k = 0;
        while (k < o.max_outer) {
            const unsigned q1 = next();
            hip_check(exact::launch_dyk_pre(zp, pp, w->as<float>(), N, parts->as<double>(),
                                            hd + 1, st, fd, q1),
                      "dyk_pre");
            const float *y = tv_ball(tau, sync1(q1, st), st);
            const unsigned q2 = next();
            hip_check(exact::launch_dyk_post(w->as<float>(), y, pp, qp, zp, d,
                                             parts->as<double>(), hd + 1, st, fd, q2),
                      "dyk_post");
            ++k;
            if (std::sqrt(sync1(q2, st)) <= o.dyk_tol)
                break;
        }
        copy(outp, zp, st);
        return k;
    }
};

exact_tv_opts tv_opts_of(const exact_tv_opts *opts)
{
    exact_tv_opts o;
    exact_tv_opts_default(&o);
    if (opts)
        o = *opts;
    validate_tv_opts(o);
    return o;
}

}  // namespace

extern "C" {

void exact_tv_opts_default(exact_tv_opts *o)
{
    if (!o)
        return;
    o->tv_tol = 0.01;
    o->prox_iters = 100;
    o->max_bisect = 40;
    o->dyk_tol = 1e-4;
    o->max_outer = 200;
}

int exact_tv_norm(int32_t n_pix, const float *x_dev, double *tv_out, void *stream)
{
    return guarded([&]() -> int {
        if (n_pix < 1 || n_pix > 16384)
            fail(-EINVAL, "n_pix must be in [1, 16384]");
        if (!x_dev || !tv_out)
            fail(-EINVAL, "NULL pointer");
        OwnStream own((hipStream_t)stream);
        DevBuf parts((size_t)exact::num_tv_parts(n_pix) * 8), out(8);
        hip_check(exact::launch_tv_norm(x_dev, n_pix, parts.as<double>(), out.as<double>(), own.st),
                  "tv_norm");
        hip_check(hipMemcpyAsync(tv_out, out.p, 8, hipMemcpyDeviceToHost, own.st), "hipMemcpyAsync");
        hip_check(hipStreamSynchronize(own.st), "hipStreamSynchronize");
        return 0;
    });
}

int exact_tv_prox(int32_t n_pix, const float *b_dev, double lam, int32_t iters, float *x_dev,
                  void *stream)
{
    return guarded([&]() -> int {
        if (n_pix < 1 || n_pix > 16384)
            fail(-EINVAL, "n_pix must be in [1, 16384]");
        if (!b_dev || !x_dev)
            fail(-EINVAL, "NULL pointer");
        if (!std::isfinite(lam))
            fail(-EINVAL, "lam must be finite");
        exact_tv_opts o;
        exact_tv_opts_default(&o);
        o.prox_iters = iters;
        validate_tv_opts(o);
        OwnStream own((hipStream_t)stream);
        const long d = (long)n_pix * n_pix;
        if (!(lam > 0.0)) {
            hip_check(hipMemcpyAsync(x_dev, b_dev, (size_t)d * 4, hipMemcpyDeviceToDevice, own.st),
                      "hipMemcpyAsync");
            hip_check(hipStreamSynchronize(own.st), "hipStreamSynchronize");
            return 0;
        }
        TvWork W(n_pix, o, own.st);
        W.copy(W.w->as<float>(), b_dev, own.st);
        W.solve(0, lam, own.st);
        W.copy(x_dev, W.xb[0]->as<float>(), own.st);
        hip_check(hipStreamSynchronize(own.st), "hipStreamSynchronize");
        return 0;
    });
}

int exact_project_tv(int32_t n_pix, const float *z_dev, double tau, const exact_tv_opts *opts,
                     float *out_dev, exact_tv_info *info, void *stream)
{
    return guarded([&]() -> int {
        const auto t0 = std::chrono::steady_clock::now();
        if (n_pix < 1 || n_pix > 16384)
            fail(-EINVAL, "n_pix must be in [1, 16384]");
        if (!z_dev || !out_dev)
            fail(-EINVAL, "NULL pointer");
        if (!(std::isfinite(tau) && tau > 0.0))
            fail(-EINVAL, "tau must be finite and > 0");
        const exact_tv_opts o = tv_opts_of(opts);
        OwnStream own((hipStream_t)stream);
        TvWork W(n_pix, o, own.st);
        const int rounds = W.project(z_dev, out_dev, tau, own.st);
        const double tv = W.tv_of(out_dev, own.st);
        hip_check(hipStreamSynchronize(own.st), "hipStreamSynchronize");
        if (info) {
            info->rounds = rounds;
            info->solves = W.solves;
            info->tv = tv;
            info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
        return 0;
    });
}

int exact_solve_tv(exact_geometry g, const exact_spectrum *sp, const float *y_dev, float *x_dev,
                   const exact_solve_opts *opts, double tau, const exact_tv_opts *tv,
                   exact_solve_info *info, exact_tv_info *tv_info, void *stream)
{
    return guarded([&]() -> int {
        const auto t0 = std::chrono::steady_clock::now();
        if (!(std::isfinite(tau) && tau > 0.0))
            fail(-EINVAL, "tau must be finite and > 0");
        exact_solve_opts o;
        exact_solve_opts_default(&o);
        if (opts)
            o = *opts;
        if (o.stop_mode != EXACT_STOP_NATURAL_RESIDUAL)
            fail(-EINVAL, "exact_solve_tv stops on the natural residual only");
        const exact_tv_opts to = tv_opts_of(tv);
        check_geometry(g);
        OwnStream own((hipStream_t)stream);
        hipStream_t st = own.st;
        DevBuf state(sizeof(SolveState));
        Problem p;
        problem_init(p, g, sp, y_dev, x_dev, o, state.as<SolveState>(), st);
        const Geo G = geo_of(g);
        const long d = (long)g->N * g->N, n = (long)g->V * g->B;
        const float gf = (float)p.gamma, inv_n = (float)(1.0 / (double)n);
        DevBuf grad((size_t)d * 4), v((size_t)d * 4), xh((size_t)d * 4);
        TvWork W(g->N, to, st);
        int t = 0, rounds = 0;
        double rho = -1.0;
        bool converged = false;
        // F(z) = (1/n) A^T r(z) from the padded pair of z, into grad
        auto gradient = [&](const float *zp, const float *zTp) {
            hip_check(exact::launch_forward_residual(G, zp, zTp, p.Y->as<float>(), p.spec,
                                                     p.r->as<float>(), nullptr, nullptr, st),
                      "forward_residual");
            hip_check(exact::launch_back(G, p.r->as<float>(), grad.as<float>(), inv_n, nullptr,
                                         st),
                      "back");
        };
        while (t < o.max_iters) {
            gradient(p.xp->as<float>(), p.xTp->as<float>());
            hip_check(exact::launch_axpy(x_dev, grad.as<float>(), gf, v.as<float>(), d, st), "axpy");
            rounds = W.project(v.as<float>(), xh.as<float>(), tau, st);
            hip_check(exact::launch_pad_pair(xh.as<float>(), p.xhp->as<float>(), p.xhTp->as<float>(),
                                             g->N, st),
                      "pad_pair");
            const unsigned q1 = W.next();
            hip_check(exact::launch_diff2(xh.as<float>(), x_dev, d, W.parts->as<double>(),
                                          W.hd + 1, st, W.fd, q1),
                      "diff2");
            W.wait(q1, st);
            rho = W.h[2] > 0.0 ? std::sqrt(W.h[1] / W.h[2]) : -1.0;
            gradient(p.xhp->as<float>(), p.xhTp->as<float>());
            hip_check(exact::launch_axpy(x_dev, grad.as<float>(), gf, v.as<float>(), d, st), "axpy");
            rounds = W.project(v.as<float>(), x_dev, tau, st);
            hip_check(exact::launch_pad_pair(x_dev, p.xp->as<float>(), p.xTp->as<float>(), g->N, st),
                      "pad_pair");
            ++t;
            if (o.tol > 0.0 && rho >= 0.0 && rho <= o.tol) {
                converged = true;
                break;
            }
        }
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
        if (info) {
            info->iters = t;
            info->resid = rho;
            info->gamma = p.gamma;
            info->lambda_hat = p.lam;
            info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
        if (tv_info) {
            tv_info->rounds = rounds;
            tv_info->solves = W.solves;
            tv_info->tv = W.tv_of(x_dev, st);
            tv_info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
        if (o.tol > 0.0 && !converged)
            return EXACT_ENOTCONV;
        return 0;
    });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Explicit measurement matrix (the Gaussian measurement model)

namespace {

// Device state of one dense problem: window sums of y, the collapsed
// spectrum, the partial gradients and the half-step iterate.
struct DenseWork {
    long n = 0;
    int d = 0, K = 0;
    std::unique_ptr<DevBuf> Y, J, mu, parts, parts2, g, xh;

    DenseWork(long n_, int d_, const exact_spectrum *sp, const float *y_dev, SpecArg &a,
              double *sjm, hipStream_t st)
        : n(n_), d(d_)
    {
        if (n < 1 || d < 1 || d > exact::kDenseMaxCols)
            fail(-EINVAL, "need n >= 1 and 1 <= d <= " + std::to_string(exact::kDenseMaxCols));
        if (!y_dev)
            fail(-EINVAL, "y is NULL");
        a = make_spec(sp, sjm);
        if (sp->background)
            fail(-EINVAL, "a known background applies to CT scans only");
        K = a.K;
        Y.reset(new DevBuf((size_t)n * 4));
        J.reset(new DevBuf((size_t)K * 4));
        mu.reset(new DevBuf((size_t)K * 4));
        parts.reset(new DevBuf((size_t)exact::dense_blocks(n, d) * d * 4));
        parts2.reset(new DevBuf((size_t)exact::dense_sum_groups(n, d) * d * 4));
        g.reset(new DevBuf((size_t)d * 4));
        xh.reset(new DevBuf((size_t)d * 4));
        hip_check(hipMemcpyAsync(J->p, a.J, (size_t)K * 4, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
        hip_check(hipMemcpyAsync(mu->p, a.mu, (size_t)K * 4, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
        DevBuf bad(4);
        hip_check(hipMemsetAsync(bad.p, 0, 4, st), "hipMemsetAsync");
        hip_check(exact::launch_window_sum(y_dev, sp->n_windows, n, Y->as<float>(), bad.as<int32_t>(), st),
                  "window_sum");
        int32_t hbad = 0;
        hip_check(hipMemcpyAsync(&hbad, bad.p, 4, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
        if (hbad)
            fail(-EINVAL, "y contains negative or non-finite counts");
    }

    hipError_t F(const float *A, const float *x, bool linear, const int32_t *skip, hipStream_t st)
    {
        return exact::launch_dense_F(A, n, d, x, Y->as<float>(), J->as<float>(), mu->as<float>(), K,
                                     linear, parts->as<float>(), parts2->as<float>(),
                                     g->as<float>(), skip, st);
    }
};

}  // namespace

extern "C" {

int exact_dense_operator(int32_t n, int32_t d, const float *A_dev, const exact_spectrum *sp,
                         const float *y_dev, const float *x_dev, float *F_dev, void *stream)
{
    return guarded([&]() -> int {
        if (!A_dev || !x_dev || !F_dev)
            fail(-EINVAL, "NULL buffer");
        OwnStream own((hipStream_t)stream);
        SpecArg a;
        DenseWork W(n, d, sp, y_dev, a, nullptr, own.st);
        hip_check(W.F(A_dev, x_dev, false, nullptr, own.st), "dense_F");
        hip_check(exact::launch_dense_finish(W.g->as<float>(), d, 0, x_dev, 0.f, 0.0, F_dev,
                                             nullptr, own.st),
                  "dense_finish");
        hip_check(hipStreamSynchronize(own.st), "hipStreamSynchronize");
        return 0;
    });
}

int exact_dense_solve(int32_t n, int32_t d, const float *A_dev, const exact_spectrum *sp,
                      const float *y_dev, float *x_dev, const exact_solve_opts *opts,
                      double radius, exact_solve_info *info, void *stream)
{
    return guarded([&]() -> int {
        const auto t0 = std::chrono::steady_clock::now();
        if (!A_dev || !x_dev)
            fail(-EINVAL, "NULL buffer");
        if (!std::isfinite(radius))
            fail(-EINVAL, "radius must be finite (<= 0 for no constraint)");
        exact_solve_opts o;
        exact_solve_opts_default(&o);
        if (opts)
            o = *opts;
        validate_opts(o);
        if (o.stop_mode != EXACT_STOP_NATURAL_RESIDUAL)
            fail(-EINVAL, "exact_dense_solve stops on the natural residual only");
        OwnStream own((hipStream_t)stream);
        hipStream_t st = own.st;
        SpecArg a;
        double sjm = 0.0;
        DenseWork W(n, d, sp, y_dev, a, &sjm, st);
        DevBuf state(sizeof(SolveState));
        PinnedState hs;
        SolveState *S = state.as<SolveState>();
        double gamma = o.gamma, lam = 0.0;
        if (gamma <= 0.0 && o.lambda_hat > 0.0) {
            lam = o.lambda_hat;
            gamma = o.gamma_scale / (lam * sjm);
        } else if (gamma <= 0.0) {
            // lambda_max(A^T A / n) by power iteration from the constant unit vector
            DevBuf v0((size_t)d * 4), v1((size_t)d * 4);
            hip_check(exact::launch_fill(v0.as<float>(), (float)(1.0 / std::sqrt((double)d)), d, st),
                      "fill");
            hip_check(exact::launch_state_init(S, 0.0, 0, 0, st), "state_init");
            float *vin = v0.as<float>(), *vout = v1.as<float>();
            for (int it = 1; it <= o.power_iters; ++it) {
                hip_check(W.F(A_dev, vin, true, nullptr, st), "dense_F");
                hip_check(exact::launch_dense_finish(W.g->as<float>(), d, 3, vin, 0.f, 0.0, vout,
                                                     S, st),
                          "dense_finish");
                std::swap(vin, vout);
                read_state(S, hs, st);
                const double lam_new = hs.h->lam;
                if (!(std::isfinite(lam_new) && lam_new > 0.0))
                    fail(-EIO, "power iteration produced a non-positive eigenvalue estimate");
                const bool done = it > 1 && std::fabs(lam_new - lam) <= 1e-7 * std::fabs(lam_new);
                lam = lam_new;
                if (done)
                    break;
            }
            gamma = o.gamma_scale / (lam * sjm);
        }
        hip_check(exact::launch_state_init(S, o.tol, o.max_iters, 0, st), "state_init");
        const float gf = (float)gamma;
        float *xh = W.xh->as<float>();
        Graph step;
        step.capture(st, [&]() {
            hipError_t e = W.F(A_dev, x_dev, false, &S->done, st);
            if (e == hipSuccess)
                e = exact::launch_dense_finish(W.g->as<float>(), d, 1, x_dev, gf, radius, xh, S,
                                               st);
            if (e == hipSuccess)
                e = W.F(A_dev, xh, false, &S->done, st);
            if (e == hipSuccess)
                e = exact::launch_dense_finish(W.g->as<float>(), d, 2, x_dev, gf, radius, x_dev,
                                               S, st);
            return e;
        });
        int launched = 0;
        while (launched < o.max_iters) {
            const int chunk = std::min(o.check_every, o.max_iters - launched);
            for (int c = 0; c < chunk; ++c)
                hip_check(hipGraphLaunch(step.exec, st), "graph launch");
            launched += chunk;
            read_state(S, hs, st);
            if (hs.h->done)
                break;
        }
        read_state(S, hs, st);
        step.reset();
        if (info) {
            info->iters = o.max_iters == 0 ? 0 : hs.h->t;
            info->resid = o.max_iters == 0 ? -1.0 : hs.h->rho;
            info->gamma = gamma;
            info->lambda_hat = lam;
            info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
        if (o.tol > 0.0 && !hs.h->converged)
            return EXACT_ENOTCONV;
        return 0;
    });
}

}  // extern "C"
