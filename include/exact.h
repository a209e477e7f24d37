/*
 * exact.h -- C ABI of libexact, the MI355X (gfx950) implementation of the
 * hot path of EXACT (EXtragradient Algorithm for Computed Tomography):
 * projected extragradient for single-material polychromatic CT,
 * arXiv 2503.19925.
 *
 * Conventions shared by every call
 * --------------------------------
 *  Geometry.  2-D parallel beam.  The image is N x N square pixels of side
 *  pixel_cm centred at the origin; pixel (iy, ix) has centre
 *  ((ix - c) pixel_cm, (iy - c) pixel_cm) with c = (N-1)/2 and iy = 0 the
 *  bottom row.  View v (0 <= v < V) is at theta_v = half_turns * pi * v / V;
 *  detector bin b (0 <= b < B) sits at u_b = (b - (B-1)/2) bin_cm; ray
 *  i = v*B + b is the line {p : p . (cos theta_v, sin theta_v) = u_b}.
 *  A is Joseph's matrix: a ray walks the image rows (views with
 *  |cos| >= |sin|, ties at 45/135 degrees decided by the integer test
 *  4q <= V or 4q >= 3V, q = half_turns*v mod V) or columns, and on each
 *  line puts tent weight max(0, 1 - |f - j|) on the pixels j next to its
 *  crossing f, times the path length per line pixel_cm/|cos| (rows) or
 *  pixel_cm/|sin| (columns).  Entries are nonnegative, as the paper
 *  requires of A (Sec. 1, forward model and the notation list below it).
 *
 *  Layouts (all device memory, float32, row-major, no padding):
 *    image   x[N*N]        p = iy*N + ix
 *    sinogram s[V*B]       i = v*B + b   (bins fastest)
 *    counts  y[Wn*V*B]     window-major: y[j*V*B + i]
 *
 *  Units: x in g/cm^3, lengths in cm, line integrals in g/cm^2, mu in
 *  cm^2/g, counts in photons.
 *
 *  Ownership.  The caller allocates and owns every device buffer passed in
 *  (the library never frees them).  The library owns the geometry handle
 *  and its device tables, and any scratch it needs (allocated stream-ordered
 *  and released before the call's work completes on the stream).  Host
 *  spectrum arrays are copied during the call.
 *
 *  Streams.  `stream` is a hipStream_t (NULL = the null stream).  The
 *  projector, operator and stepping calls (exact_forward, exact_backproject,
 *  exact_operator, exact_solver_step, exact_batch_step) are
 *  stream-ordered and return before the GPU work
 *  finishes; every other call that takes a stream orders its work after
 *  the stream's and blocks until done (its comment says so).  A geometry
 *  handle may be used from several streams at once.
 *
 *  Errors.  0 on success; a negative errno value on failure (-EINVAL bad
 *  argument, -ENOMEM out of memory, -ENOSPC a batch's budget or slots
 *  exhausted, -EIO a HIP runtime error); see
 *  exact_last_error() for a message.  exact_solve returns EXACT_ENOTCONV
 *  (+1) when max_iters ends the run before the tolerance is met.  No C++
 *  exception crosses this interface.
 */
#ifndef EXACT_H
#define EXACT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EXACT_ENOTCONV 1

typedef struct exact_geometry_s *exact_geometry;

/*
 * Known spectrum of the single material (paper Sec. 1, eq.
 * model:multi-material with one material; Sec. 1.2, eq. function-h-plus):
 * expected counts in window j on ray i are
 *     sum_k weight[j*K + k] * exp(-mu[k] * max(<a_i, x>, 0)),
 * weight[j][k] = Ibar_j * s_{jk} >= 0.  mu and weight are host pointers,
 * copied by each call.  Requirements: K >= 1, Wn >= 1, every mu[k] > 0 and
 * finite, every weight finite and >= 0, each window's row sum > 0.
 *
 * background (optional): when the scan's other materials are known (the
 * multi-material model of the paper's appendix, reparametrised there into
 * a single-material model with a per-ray spectrum), their line integrals
 * bg_i, one per ray ([V][B] float32, device pointer), and the expected
 * counts become sum_k weight[j*K + k] * exp(-mu[k] * (bg_i +
 * max(<a_i, x>, 0))).  NULL means no known material.  Read during the call
 * (the solvers keep a copy); must be finite and >= 0 (exact_solve, the
 * solver and the batch check it: -EINVAL).  The step-size rule keeps
 * Theorem 2's gamma for the unattenuated spectrum, which bounds every ray's
 * reparametrised one.
 */
typedef struct {
    int32_t n_energies;     /* K  */
    int32_t n_windows;      /* Wn */
    const double *mu;       /* [K]      */
    const double *weight;   /* [Wn][K]  */
    const float *background;/* [V][B] device, or NULL */
} exact_spectrum;

/* Stop rules for exact_solve.
 * NATURAL_RESIDUAL: stop after the first step t with
 *   rho_t = ||x_{t+1/2} - x_t|| / ||x_t|| <= tol (relative); returns x_{t+1}.
 * AVERAGED_ITERATE (the rule of the paper's experiments, Sec. 5, comparison
 *   of methods): with xbar_s the mean of the iterates x_j, j = floor(s/2)+1
 *   .. s (x_1 the starting point), stop after the first step t with
 *   ||xbar_{t+1} - xbar_t|| <= tol (absolute, as in the paper); returns
 *   xbar_{t+1}.  Keeps floor(J/2)+2 images of iterates, J =
 *   floor((max_iters+1)/2), plus a double running sum: bound max_iters
 *   accordingly.  exact_solve only; the solver and batch calls reject it. */
#define EXACT_STOP_NATURAL_RESIDUAL 0
#define EXACT_STOP_AVERAGED_ITERATE 1

typedef struct {
    double gamma;        /* step size; <= 0 selects gamma_scale / L (below)  */
    double gamma_scale;  /* c in gamma = c / (lambda_max(A^T A / n) *
                            sum_k J_k mu_k), J_k = sum_j weight[j][k];
                            Theorem 2 uses c = 1/4 (default)                */
    int32_t max_iters;   /* full extragradient steps (two F evaluations each) */
    double tol;          /* stop tolerance of the stop rule; 0 = run all     */
    int32_t stop_mode;   /* EXACT_STOP_NATURAL_RESIDUAL or _AVERAGED_ITERATE */
    int32_t check_every; /* steps between host reads of the device stop flag */
    int32_t power_iters; /* cap on power-iteration steps for lambda_max     */
    double lambda_hat;   /* lambda_max(A^T A / n) of the geometry when already
                            known (exact_step_size, or an earlier run's
                            info): > 0 makes the automatic step size use it
                            instead of running the power iteration; 0
                            (default) runs it.  Ignored when gamma > 0.      */
} exact_solve_opts;

typedef struct {
    int32_t iters;       /* steps taken                                      */
    double resid;        /* last rho_t = ||x_{t+1/2} - x_t|| / ||x_t|| (-1 if
                            undefined, i.e. x_t = 0); with the averaged rule
                            the last ||xbar_{t+1} - xbar_t||                 */
    double gamma;        /* step size used                                   */
    double lambda_hat;   /* lambda_max estimate used (0 if gamma was given) */
    double ms;           /* wall time of the call                            */
} exact_solve_info;

/* Fills opts with the defaults: gamma 0 (automatic), gamma_scale 0.25,
 * max_iters 500, tol 0, natural-residual stop, check_every 16,
 * power_iters 100, lambda_hat 0 (computed). */
void exact_solve_opts_default(exact_solve_opts *opts);

/*
 * Builds the per-view tables of the geometry above and uploads them to the
 * current HIP device.  n_pix, n_views, n_bins >= 1; n_pix <= 16384 and
 * n_views * (n_bins + 4) < 2^30 (the padded residual sinogram, n_views rows
 * of n_bins + 4 floats, is addressed with 32-bit byte offsets); half_turns
 * 1 (180 degrees) or 2 (360 degrees); pixel_cm, bin_cm > 0 and finite.
 * *out receives the handle.
 */
int exact_geometry_create(int32_t n_pix, int32_t n_views, int32_t n_bins,
                          int32_t half_turns, double pixel_cm, double bin_cm,
                          exact_geometry *out);

/* Releases the handle (synchronises the device first).  NULL is a no-op. */
int exact_geometry_destroy(exact_geometry g);

/*
 * Line integrals s = A x (the inner product <a_i, x> of paper Sec. 1.2,
 * eq. model-pre, for every ray).  x_dev [N*N], s_dev [V*B].
 */
int exact_forward(exact_geometry g, const float *x_dev, float *s_dev,
                  void *stream);

/*
 * Back-projection img = A^T r (the sum over rays of r_i a_i in the operator
 * of paper Sec. 1.2, eq. operator, without its 1/n).  The transpose of
 * exact_forward: the same float tent weights, formed per pixel (gather),
 * with no atomics, so results are bitwise reproducible; the path-length
 * factor multiplies r once per ray (into a stream-ordered scratch copy of
 * V*(B+4) floats) before the gather.  r_dev [V*B], img_dev [N*N].
 */
int exact_backproject(exact_geometry g, const float *r_dev, float *img_dev,
                      void *stream);

/*
 * The monotone operator of paper Sec. 1.2, eq. operator, summed over
 * windows:
 *     F(x) = (1/n) A^T r,   r_i = sum_j y[j][i] - sum_k J_k exp(-mu_k (Ax)_i+),
 * n = V*B (rays), J_k = sum_j weight[j][k].  y_dev [Wn*V*B], x_dev [N*N],
 * F_dev [N*N]; r_dev [V*B] receives r, or NULL.
 */
int exact_operator(exact_geometry g, const exact_spectrum *sp,
                   const float *y_dev, const float *x_dev, float *F_dev,
                   float *r_dev, void *stream);

/*
 * exact_operator for callers that cannot allocate device memory during the
 * call: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, results (bitwise) and stream ordering
 * as exact_operator, and no allocation of any kind on the device: the
 * call's scratch (the window sums of y, the padded image and its transpose,
 * the padded residual) lives in a static device array of
 * EXACT_NOALLOC_SCRATCH_MIB MiB, one per GPU the library runs on, held
 * until the process ends.  Needs 4 (V B + 2 (N (N + 8) + 64) + V (B + 4)) bytes
 * (each part rounded up to 256) of it, else -ENOSPC (1024^2 with 720 views
 * x 1448 bins needs 17 MB).  The geometry must belong to the current
 * device (-EINVAL).  Every call on a GPU shares that GPU's array, which
 * keeps the last call's contents (the call clears what must start at zero):
 * calls that overlap on one GPU (on different streams or threads) race, so
 * the caller serialises them.
 */
#define EXACT_NOALLOC_SCRATCH_MIB 32
int exact_operator_noalloc(exact_geometry g, const exact_spectrum *sp, const float *y_dev,
                           const float *x_dev, float *F_dev, float *r_dev, void *stream);

/*
 * lambda_max(Sigma), Sigma = A^T A / n (paper Sec. 1.3), by power iteration
 * from the constant vector with double-precision Rayleigh quotients (at
 * most max_iters steps, stopping when the quotient changes by less than
 * 1e-7 relative), and the step size gamma = gamma_scale / (lambda *
 * sum_k J_k mu_k) of Theorem 2 when sp is not NULL.  Blocks until done.
 * gamma_out may be NULL.
 */
int exact_step_size(exact_geometry g, const exact_spectrum *sp,
                    int32_t max_iters, double gamma_scale, double *lambda_out,
                    double *gamma_out, void *stream);

/*
 * Projected extragradient (paper Sec. 1.2, eq. extragrad-method) over
 * X = {x >= 0} (the orthant projection of Sec. 3.1):
 *     x_{t+1/2} = max(0, x_t - gamma F(x_t)),
 *     x_{t+1}   = max(0, x_t - gamma F(x_{t+1/2})),   t = 1, 2, ...
 * x_dev holds x_1 >= 0 on entry and, on return, the last iterate (or, with
 * EXACT_STOP_AVERAGED_ITERATE, the averaged iterate at the last index).
 * With tol > 0 the run stops after the first step t that meets the stop
 * rule (norms in double; see the stop rules above); otherwise it runs
 * max_iters steps.  Blocks until done; info (nullable) receives the
 * summary.  Returns EXACT_ENOTCONV if tol > 0 and max_iters steps did not
 * reach it (x_dev then holds the last iterate or average).  -ENOMEM if the
 * averaged rule's iterate ring does not fit.
 * Checks on the device that y is finite and >= 0 and x_1 finite and >= 0
 * (-EINVAL otherwise, x_dev unchanged).
 */
int exact_solve(exact_geometry g, const exact_spectrum *sp, const float *y_dev,
                float *x_dev, const exact_solve_opts *opts,
                exact_solve_info *info, void *stream);

/*
 * Constraint set of the paper's experiments (Sec. 5): X = {TV(x) <= tau}
 * intersected with the orthant, TV the isotropic total variation of the
 * N x N image with forward differences (nothing across the last row or
 * column).  The TV-ball projection is approximated as the paper does: the
 * TV-regularized point argmin ||x - v||^2 + lam TV(x) (eq.
 * TV-regularization) with lam found by binary search until |TV(xbar) -
 * tau| <= tv_tol; the regularized point is computed by prox_iters steps of
 * fast gradient projection on the dual of TV denoising (Beck and Teboulle
 * 2009) started from zero.  The binary search: if TV(v) <= tau the result
 * is v; else it brackets the weight, then halves the bracket.  The first
 * search of a projection call (or of a solve) starts cold: hi starts at 1
 * and doubles (at most 60 times) until TV(xbar(hi)) <= tau, lo being its
 * previous value (0 first).  Later searches of the same call start warm at
 * the weight lam0 of the previous one: xbar(lam0) first; if its TV is above
 * tau, lo = lam0 and hi grows by 5/4, then doubles, while TV(xbar(hi)) >
 * tau; otherwise hi = lam0 and lo shrinks by 4/5, then halves, while
 * TV(xbar(lo)) <= tau (at most 60 times each way); a point met on the way
 * within tv_tol of tau is the result.  Then up to max_bisect midpoints: the
 * first within tv_tol is the result, TV > tau moves lo up, TV <= tau moves
 * hi down; without a hit the result is xbar(hi).  (The paper leaves the
 * search's start open; the warm start is this library's reading, shared by
 * its test oracle.)  The intersection with the orthant is Dykstra's
 * algorithm (eq. projection-intersection), stopped once ||z_{k+1} - z_k||_2
 * <= dyk_tol or after max_outer rounds.  Defaults: the paper's tolerances (0.01, 1e-4),
 * prox_iters 100, max_bisect 40, max_outer 200.
 */
typedef struct {
    double tv_tol;
    int32_t prox_iters;
    int32_t max_bisect;
    double dyk_tol;
    int32_t max_outer;
} exact_tv_opts;

typedef struct {
    int32_t rounds;      /* Dykstra rounds of the (last) projection          */
    int32_t solves;      /* TV-regularized points computed (all projections) */
    double tv;           /* TV of the result                                 */
    double ms;           /* wall time of the call                            */
} exact_tv_info;

void exact_tv_opts_default(exact_tv_opts *opts);

/* TV(x) of an n_pix x n_pix image x_dev (device), in double; blocking. */
int exact_tv_norm(int32_t n_pix, const float *x_dev, double *tv_out, void *stream);

/* The TV-regularized point x = argmin ||x - b||^2 + lam TV(x) by `iters`
 * FGP steps from zero (lam <= 0: x = b).  Blocking. */
int exact_tv_prox(int32_t n_pix, const float *b_dev, double lam, int32_t iters, float *x_dev,
                  void *stream);

/* Projection of z_dev onto {TV <= tau} intersected with the orthant, into
 * out_dev (may equal z_dev).  tau > 0 and finite; opts nullable (defaults);
 * info nullable.  Blocking. */
int exact_project_tv(int32_t n_pix, const float *z_dev, double tau, const exact_tv_opts *opts,
                     float *out_dev, exact_tv_info *info, void *stream);

/*
 * exact_solve over X = {TV <= tau} intersected with the orthant: both
 * half-steps x_t - gamma F(.) are projected with exact_project_tv's
 * algorithm (the paper's experimental set-up, Sec. 5).  opts as for
 * exact_solve (stop_mode must be the natural residual); tv nullable;
 * tv_info (nullable) receives the projection counts summed over the run.
 * The known background of sp is honoured.  Blocking; far slower per step
 * than exact_solve, since every projection solves tens to thousands of
 * TV-regularized problems.
 */
int exact_solve_tv(exact_geometry g, const exact_spectrum *sp, const float *y_dev, float *x_dev,
                   const exact_solve_opts *opts, double tau, const exact_tv_opts *tv,
                   exact_solve_info *info, exact_tv_info *tv_info, void *stream);

/*
 * EXACT with an explicit measurement matrix (the Gaussian measurement model
 * of paper Sec. 2.2, Assumption Gaussian-assump, and its experiment in
 * Sec. 5): A is n x d, row-major float32 on the device (a_i its rows; any
 * real entries), the model and operator are those above,
 *     F(x) = (1/n) sum_i r_i a_i,  r_i = sum_j y[j][i] - sum_k J_k exp(-mu_k max(<a_i, x>, 0)),
 * with y [Wn][n] and the spectrum as in exact_spectrum (background must be
 * NULL).  1 <= d <= 4096.  Each evaluation of F reads A once.
 *
 * exact_dense_operator writes F(x) to F_dev [d] (blocking).
 * exact_dense_solve runs eq. extragrad-method over X = {||x||_2 <= radius}
 * (the bounded set of Assumption assump-X, centred at the origin; radius
 * <= 0 means the whole space), x_dev [d] in/out, x_1 finite.  opts as for
 * exact_solve (natural-residual stop only); gamma <= 0 selects
 * gamma_scale / (lambda_max(A^T A / n) sum_k J_k mu_k) with lambda_max by
 * power iteration.  Blocking; info nullable.
 */
int exact_dense_operator(int32_t n, int32_t d, const float *A_dev, const exact_spectrum *sp,
                         const float *y_dev, const float *x_dev, float *F_dev, void *stream);
int exact_dense_solve(int32_t n, int32_t d, const float *A_dev, const exact_spectrum *sp,
                      const float *y_dev, float *x_dev, const exact_solve_opts *opts,
                      double radius, exact_solve_info *info, void *stream);

/*
 * Resident solver: the same iteration as exact_solve, split so that a caller
 * can keep the run's state on the device and advance it in pieces.
 *
 * exact_solver_create validates the inputs (as exact_solve does), computes
 * the step size (power iteration when opts->gamma <= 0), allocates the run's
 * device state (about 16 N^2 + 8 V B bytes) and captures one full
 * extragradient step as a HIP graph.  y_dev is read during the call only;
 * x_dev is the iterate, updated in place by every step: it must stay valid
 * and must not be written by the caller until exact_solver_destroy.  Blocks
 * until set-up is done.
 *
 * exact_solver_step enqueues n_steps full steps on `stream` (asynchronous,
 * ordered after the stream's earlier work and before its later work).
 * Steps after the run has stopped (tolerance met or max_iters reached) are
 * no-ops on the device, so over-enqueueing is harmless.
 *
 * exact_solver_poll waits for the enqueued steps, fills info (nullable)
 * and returns 1 once the run has stopped, 0 while it is still running.
 *
 * exact_solver_destroy waits for the run's work and frees its state.
 *
 * exact_solver_profile (for measurement) runs n_steps (1..4096) further
 * steps launched one kernel at a time instead of through the captured
 * graph, each of the step's EXACT_STEP_PHASES phases its own kernel (in the
 * graph the reduction [4] runs inside the next step's first kernel), with
 * HIP events recorded on the solver's stream around each, and writes the
 * average milliseconds of each phase to phase_ms[EXACT_STEP_PHASES]:
 *   [0] forward projection + spectral residual at x_t,
 *   [1] back-projection + half-step update and residual partials,
 *   [2] forward projection + spectral residual at x_{t+1/2},
 *   [3] back-projection + full-step update,
 *   [4] reduction of rho_t and the stop test.
 * The steps advance the run exactly as exact_solver_step's would (after the
 * stop they are no-ops and time as such).  Ordered on `stream` like
 * exact_solver_step; blocks until the steps are done.
 */
typedef struct exact_solver_s *exact_solver;

#define EXACT_STEP_PHASES 5

int exact_solver_create(exact_geometry g, const exact_spectrum *sp, const float *y_dev,
                        float *x_dev, const exact_solve_opts *opts, exact_solver *out,
                        void *stream);
int exact_solver_step(exact_solver s, int32_t n_steps, void *stream);
int exact_solver_poll(exact_solver s, exact_solve_info *info);
int exact_solver_destroy(exact_solver s);
int exact_solver_profile(exact_solver s, int32_t n_steps, double *phase_ms, void *stream);

/*
 * exact_solver_time_kernels (for measurement) times each kernel of the
 * step's EXACT_STEP_PHASES phases (numbered as for exact_solver_profile) as
 * `reps` (1..4096) back-to-back launches between two HIP events on the
 * solver's stream, after an untimed pass of the same launches, and writes
 * the average milliseconds per launch to kernel_ms[EXACT_STEP_PHASES].  The run's state and iterate are left as
 * they were: the kernels read the run's current buffers, the full-step
 * update writes a scratch image instead of x, the reduction updates a
 * scratch copy of the state, and the other kernels rewrite buffers that the
 * next step writes again from the same inputs.  Works after the run has
 * stopped too.  Ordered on `stream`; blocks until done.
 */
int exact_solver_time_kernels(exact_solver s, int32_t reps, double *kernel_ms, void *stream);

/*
 * Exact number of positive entries of A (the tent weights that round to a
 * positive float), counted on the device with the projectors' own weight
 * expression.  Blocks until done.
 */
int exact_count_nonzeros(exact_geometry g, int64_t *nnz_out, void *stream);

/*
 * Batched and served extragradient (many independent reconstructions of
 * different shapes at once).  A batch holds runs in slots; every
 * exact_batch_step advances all running runs by whole extragradient steps
 * with one captured graph of five phase kernels, whose workgroups take
 * (run, tile) items from device lists, heaviest runs first.  The per-item
 * arithmetic is exact_solve's own, so each run's iterates are bitwise the
 * same alone and in any batch.  A run that has stopped costs nothing further
 * (its items return at once) until it is removed; runs may join or leave
 * between steps (the lists and the graph are then rebuilt).
 *
 * exact_run_footprint: device bytes one run allocates inside the library
 *   (the caller's x and y are extra; a run with a known background holds
 *   4 V B bytes more for its copy); 0 for invalid sizes.
 * exact_batch_create: hbm_budget_bytes caps the sum of the runs'
 *   footprints; capacity is the number of slots (1..65536).
 * exact_batch_add: validates and sets up one run as exact_solver_create
 *   does (blocking; ordered after `stream`), and returns its slot.  x_dev is
 *   the run's iterate, updated in place by every step: it must stay valid
 *   and unwritten by the caller until exact_batch_remove.  -ENOSPC when the
 *   budget or the slots are exhausted.
 * exact_batch_step: enqueues n_steps steps of every run on `stream`
 *   (asynchronous).
 * exact_batch_sync: waits for the enqueued steps and refreshes the host copy
 *   of every run's state; returns the number of runs still running.
 * exact_batch_poll: from the last sync: 0 running, 1 finished (tolerance
 *   met, or all max_iters steps run when tol = 0), 2 stopped at max_iters
 *   without meeting tol > 0; info (nullable) is filled.
 * exact_batch_remove: waits for the batch's work and frees the slot.
 * exact_batch_destroy: waits and frees everything.
 */
typedef struct exact_batch_s *exact_batch;

size_t exact_run_footprint(int32_t n_pix, int32_t n_views, int32_t n_bins);
int exact_batch_create(size_t hbm_budget_bytes, int32_t capacity, exact_batch *out);
int exact_batch_add(exact_batch b, exact_geometry g, const exact_spectrum *sp,
                    const float *y_dev, float *x_dev, const exact_solve_opts *opts,
                    int32_t *slot_out, void *stream);
int exact_batch_step(exact_batch b, int32_t n_steps, void *stream);
int exact_batch_sync(exact_batch b);
int exact_batch_poll(exact_batch b, int32_t slot, exact_solve_info *info);
int exact_batch_remove(exact_batch b, int32_t slot);
int exact_batch_destroy(exact_batch b);

/* Message for the last failure on the calling thread ("" if none). */
const char *exact_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EXACT_H */
