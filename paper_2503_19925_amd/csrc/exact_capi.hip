// C ABI of libexact (declared in include/exact.h): argument checks, the
// per-view geometry tables, and the host drivers of the operator, the power
// iteration and the extragradient solve.  All arithmetic of the path runs
// in the kernels of exact_kernels.hip.
#include "exact.h"
#include "exact_internal.h"

#include <cerrno>
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

using exact::Geo;
using exact::SolveState;
using exact::SpecArg;
using exact::ViewGeom;

struct exact_geometry_s {
    int N, V, B, half_turns, reach, nrow;
    double pixel_cm, bin_cm;
    int device;
    ViewGeom *d_views;
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
    return Geo{g->d_views, g->N, g->V, g->B, g->nrow, g->reach};
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
        // largest crossing the kernels form: b up to B + 64 (candidate bins
        // beyond the detector are formed, then discarded), k up to N
        const long double span = fabsl(A) + (B + 64) * fabsl(P) + N * fabsl(Q) + 2.0L;
        if (!(span < 1048576.0L))
            fail(-EINVAL, "geometry too large for exact crossing arithmetic (|crossing| >= 2^20)");
        ViewGeom G;
        std::memset(&G, 0, sizeof(G));
        G.A = (double)A;
        G.P = (double)P;
        G.Q = (double)Q;
        G.invP = (double)(1.0L / P);
        G.absP = (double)fabsl(P);
        G.wstep = (float)((long double)pixel_cm / fabsl(cs));
        G.vidx = v;
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
    DevBuf v(d * 4), vT(d * 4), u(d * 4), s(n * 4), parts(nparts * 3 * 8), state(sizeof(SolveState));
    PinnedState hs;
    hip_check(exact::launch_fill(v.as<float>(), (float)(1.0 / std::sqrt((double)d)), d, st), "fill");
    hip_check(exact::launch_fill(vT.as<float>(), (float)(1.0 / std::sqrt((double)d)), d, st), "fill");
    hip_check(exact::launch_state_init(state.as<SolveState>(), 0.0, 0, st), "state_init");
    double lam = 0.0;
    int it = 0;
    for (it = 1; it <= max_iters; ++it) {
        hip_check(exact::launch_forward(G, v.as<float>(), vT.as<float>(), s.as<float>(), nullptr, st), "forward");
        hip_check(exact::launch_back(G, s.as<float>(), u.as<float>(), (float)(1.0 / (double)n), nullptr, st), "back");
        hip_check(exact::launch_dot3(v.as<float>(), u.as<float>(), g->N, parts.as<double>(), st), "dot3");
        hip_check(exact::launch_dot3_finish(parts.as<double>(), nparts, state.as<SolveState>(), st), "dot3_finish");
        hip_check(exact::launch_normalize(u.as<float>(), v.as<float>(), vT.as<float>(), g->N,
                                          state.as<SolveState>(), st), "normalize");
        read_state(state.as<SolveState>(), hs, st);
        const double lam_new = hs.h->lam;
        if (!(std::isfinite(lam_new) && lam_new > 0.0))
            fail(-EIO, "power iteration produced a non-positive eigenvalue estimate");
        const bool done = it > 1 && std::fabs(lam_new - lam) <= 1e-7 * std::fabs(lam_new);
        lam = lam_new;
        if (done)
            break;
    }
    if (iters_out)
        *iters_out = it > max_iters ? max_iters : it;
    return lam;
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
        if (n_views < 1 || n_bins < 1 || (long long)n_views * n_bins >= (1LL << 31))
            fail(-EINVAL, "n_views, n_bins must be >= 1 with n_views*n_bins < 2^31");
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
        try {
            hip_check(hipGetDevice(&g->device), "hipGetDevice");
            g->h_views = build_views(n_pix, n_views, n_bins, half_turns, pixel_cm, bin_cm,
                                     &g->reach, &g->nrow);
            const size_t bytes = sizeof(ViewGeom) * (size_t)n_views;
            hip_check(hipMalloc((void **)&g->d_views, bytes), "hipMalloc");
            hip_check(hipMemcpy(g->d_views, g->h_views.data(), bytes, hipMemcpyHostToDevice),
                      "hipMemcpy");
        } catch (...) {
            if (g->d_views)
                (void)hipFree(g->d_views);
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
        (void)hipDeviceSynchronize();
        if (g->d_views)
            hip_check(hipFree(g->d_views), "hipFree");
        delete g;
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
        const long d = (long)g->N * g->N;
        AsyncBuf xT(d * sizeof(float), st);
        hip_check(exact::launch_transpose(x_dev, xT.as<float>(), g->N, st), "transpose");
        hip_check(exact::launch_forward(geo_of(g), x_dev, xT.as<float>(), s_dev, nullptr, st),
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
        hip_check(exact::launch_back(geo_of(g), r_dev, img_dev, 1.0f, nullptr, (hipStream_t)stream),
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
        const long d = (long)g->N * g->N, n = (long)g->V * g->B;
        AsyncBuf Y(n * sizeof(float), st), xT(d * sizeof(float), st);
        AsyncBuf rs(r_dev ? 0 : n * sizeof(float), st);
        float *r = r_dev ? r_dev : rs.as<float>();
        hip_check(exact::launch_window_sum(y_dev, sp->n_windows, n, Y.as<float>(), nullptr, st),
                  "window_sum");
        hip_check(exact::launch_transpose(x_dev, xT.as<float>(), g->N, st), "transpose");
        hip_check(exact::launch_forward_residual(geo_of(g), x_dev, xT.as<float>(), Y.as<float>(),
                                                 a, r, nullptr, st),
                  "forward_residual");
        hip_check(exact::launch_back(geo_of(g), r, F_dev, (float)(1.0 / (double)n), nullptr, st),
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

// A resident extragradient run: the spectrum, the window sums of y, the
// iterate's transpose, the half-step iterate, the gradient buffer, the
// partial sums and the device state stay allocated, and one full step is a
// captured graph replayed on a private stream.
struct exact_solver_s {
    const exact_geometry_s *g = nullptr;
    SpecArg spec;
    double gamma = 0.0, lam = 0.0;
    int max_iters = 0;
    float *x = nullptr;
    std::unique_ptr<OwnStream> own;
    std::unique_ptr<DevBuf> Y, r, gr, xT, xh, xhT, parts, state;
    std::unique_ptr<PinnedState> hs;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::chrono::steady_clock::time_point t0;

    ~exact_solver_s()
    {
        if (own && own->st)
            (void)hipStreamSynchronize(own->st);
        if (exec)
            (void)hipGraphExecDestroy(exec);
        if (graph)
            (void)hipGraphDestroy(graph);
    }
};

namespace {

void validate_opts(exact_solve_opts &o)
{
    if (o.max_iters < 0)
        fail(-EINVAL, "max_iters must be >= 0");
    if (!(std::isfinite(o.tol) && o.tol >= 0.0))
        fail(-EINVAL, "tol must be finite and >= 0");
    if (o.stop_mode != EXACT_STOP_NATURAL_RESIDUAL)
        fail(-EINVAL, "unsupported stop_mode");
    if (!std::isfinite(o.gamma))
        fail(-EINVAL, "gamma must be finite");
    if (o.gamma <= 0.0 && !(std::isfinite(o.gamma_scale) && o.gamma_scale > 0.0))
        fail(-EINVAL, "gamma_scale must be > 0 when gamma is automatic");
    if (o.check_every < 1)
        o.check_every = 1;
    if (o.power_iters < 1)
        o.power_iters = 1;
}

// Enqueue order of one extragradient step (paper Sec. 1.2, eq.
// extragrad-method): F at x_t, half-step from x_t, F at x_{t+1/2}, full step
// again from x_t, then the fixed-order residual reduction and stop test.
void capture_step(exact_solver_s *s)
{
    const exact_geometry_s *g = s->g;
    const Geo G = geo_of(g);
    const long n = (long)g->V * g->B;
    const int ntiles = exact::num_tiles(g->N);
    const float gf = (float)s->gamma;
    const float inv_n = (float)(1.0 / (double)n);
    hipStream_t st = s->own->st;
    SolveState *S = s->state->as<SolveState>();
    const int32_t *skip = &S->done;
    float *Y = s->Y->as<float>(), *r = s->r->as<float>(), *gr = s->gr->as<float>();
    float *xT = s->xT->as<float>(), *xh = s->xh->as<float>(), *xhT = s->xhT->as<float>();
    double *parts = s->parts->as<double>();

    hip_check(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    hipError_t ce = hipSuccess;
    auto cap = [&](hipError_t e) {
        if (ce == hipSuccess && e != hipSuccess)
            ce = e;
    };
    cap(exact::launch_forward_residual(G, s->x, xT, Y, s->spec, r, skip, st));
    cap(exact::launch_back(G, r, gr, inv_n, skip, st));
    cap(exact::launch_eg_update(s->x, gr, gf, xh, xhT, g->N, parts, skip, st));
    cap(exact::launch_forward_residual(G, xh, xhT, Y, s->spec, r, skip, st));
    cap(exact::launch_back(G, r, gr, inv_n, skip, st));
    cap(exact::launch_eg_update(s->x, gr, gf, s->x, xT, g->N, nullptr, skip, st));
    cap(exact::launch_eg_finish(parts, ntiles, S, st));
    hipError_t ee = hipStreamEndCapture(st, &s->graph);
    hip_check(ce, "kernel launch during capture");
    hip_check(ee, "hipStreamEndCapture");
    hip_check(hipGraphInstantiate(&s->exec, s->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
}

exact_solver_s *solver_build(exact_geometry_s *g, const exact_spectrum *sp, const float *y_dev,
                             float *x_dev, exact_solve_opts o, hipStream_t user)
{
    check_geometry(g);
    if (!y_dev || !x_dev)
        fail(-EINVAL, "NULL buffer");
    validate_opts(o);
    double sjm = 0.0;
    std::unique_ptr<exact_solver_s> s(new exact_solver_s());
    s->t0 = std::chrono::steady_clock::now();
    s->g = g;
    s->spec = make_spec(sp, &sjm);
    s->x = x_dev;
    s->max_iters = o.max_iters;
    const long d = (long)g->N * g->N, n = (long)g->V * g->B;
    s->own.reset(new OwnStream(user));
    hipStream_t st = s->own->st;
    s->Y.reset(new DevBuf(n * 4));
    s->r.reset(new DevBuf(n * 4));
    s->gr.reset(new DevBuf(d * 4));
    s->xT.reset(new DevBuf(d * 4));
    s->xh.reset(new DevBuf(d * 4));
    s->xhT.reset(new DevBuf(d * 4));
    s->parts.reset(new DevBuf((size_t)exact::num_tiles(g->N) * 2 * 8));
    s->state.reset(new DevBuf(sizeof(SolveState)));
    s->hs.reset(new PinnedState());

    // window sums of y and the domain checks on y and x_1
    DevBuf bad(8);
    int32_t *badp = bad.as<int32_t>();
    hip_check(hipMemsetAsync(bad.p, 0, 8, st), "hipMemsetAsync");
    hip_check(exact::launch_window_sum(y_dev, sp->n_windows, n, s->Y->as<float>(), badp, st),
              "window_sum");
    hip_check(exact::launch_count_bad(x_dev, d, badp + 1, st), "count_bad");
    int32_t hbad[2] = {0, 0};
    hip_check(hipMemcpyAsync(hbad, badp, 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    if (hbad[0])
        fail(-EINVAL, "y contains negative or non-finite counts");
    if (hbad[1])
        fail(-EINVAL, "x_1 contains negative or non-finite values");

    s->gamma = o.gamma;
    if (s->gamma <= 0.0) {
        s->lam = power_iteration(g, o.power_iters, st, nullptr);
        s->gamma = o.gamma_scale / (s->lam * sjm);
    }
    hip_check(exact::launch_transpose(x_dev, s->xT->as<float>(), g->N, st), "transpose");
    hip_check(exact::launch_state_init(s->state->as<SolveState>(), o.tol, o.max_iters, st),
              "state_init");
    capture_step(s.get());
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    return s.release();
}

void solver_enqueue(exact_solver_s *s, int n_steps, hipStream_t user)
{
    hipStream_t st = s->own->st;
    hipEvent_t ev;
    hip_check(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate");
    hipError_t e = hipEventRecord(ev, user);
    if (e == hipSuccess)
        e = hipStreamWaitEvent(st, ev, 0);
    for (int c = 0; c < n_steps && e == hipSuccess; ++c)
        e = hipGraphLaunch(s->exec, st);
    if (e == hipSuccess)
        e = hipEventRecord(ev, st);
    if (e == hipSuccess)
        e = hipStreamWaitEvent(user, ev, 0);
    (void)hipEventDestroy(ev);
    hip_check(e, "graph replay");
}

// Reads the device state (blocking on the solver's stream).
int solver_poll(exact_solver_s *s, exact_solve_info *info)
{
    read_state(s->state->as<SolveState>(), *s->hs, s->own->st);
    const SolveState &h = *s->hs->h;
    if (info) {
        info->iters = s->max_iters == 0 ? 0 : h.t;
        info->resid = s->max_iters == 0 ? -1.0 : h.rho;
        info->gamma = s->gamma;
        info->lambda_hat = s->lam;
        info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - s->t0)
                       .count();
    }
    return h.done ? 1 : 0;
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
        *out = solver_build(g, sp, y_dev, x_dev, o, (hipStream_t)stream);
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
        solver_enqueue(s, n_steps, (hipStream_t)stream);
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
            solver_enqueue(s.get(), chunk, (hipStream_t)stream);
            launched += chunk;
            if (solver_poll(s.get(), &local))
                break;
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

}  // extern "C"
