/*
 * Body of the EXACT CPU oracle, written once and instantiated for several
 * scalar types by exact_oracle.c (REAL = double, long double, float; FN()
 * appends the type suffix to every exported name).  Everything here is plain
 * loops in the order the definitions are stated; see exact_oracle.c for the
 * definitions and their sources in the paper.
 *
 * TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may call this code.  It is never part of the product path.
 */

/* ---------------------------------------------------------------- geometry */

/* theta_v = half_turns * pi * v / V (views evenly spaced, endpoint excluded). */
static REAL FN(view_angle)(const ora_geom *g, int v)
{
    return (REAL)g->half_turns * (REAL)ORA_PI * (REAL)v / (REAL)g->n_views;
}

/* Stepping axis, decided by an integer test so that 45 and 135 degrees are
 * row-stepping without any rounding dependence. */
static int FN(row_stepping)(const ora_geom *g, int v)
{
    long q = ((long)g->half_turns * (long)v) % (long)g->n_views;
    return 4 * q <= g->n_views || 4 * q >= 3L * g->n_views;
}

/* Per-view quantities of the definition. */
typedef struct {
    REAL ct, st;   /* cos theta, sin theta */
    REAL wstep;    /* pixel width / |cos| (row-stepping) or / |sin| (column)  */
    int row;       /* 1: one tap pair per image row; 0: per image column       */
} FN(view);

static FN(view) FN(make_view)(const ora_geom *g, int v)
{
    FN(view) w;
    REAL th = FN(view_angle)(g, v);
    w.ct = cos(th);
    w.st = sin(th);
    w.row = FN(row_stepping)(g, v);
    w.wstep = (REAL)g->pixel_cm / (w.row ? fabs(w.ct) : fabs(w.st));
    return w;
}

/* Detector coordinate of bin b: u_b = (b - (B-1)/2) * bin width. */
static REAL FN(bin_centre)(const ora_geom *g, int b)
{
    return ((REAL)b - (REAL)(g->n_bins - 1) / 2) * (REAL)g->bin_cm;
}

/* Fractional image coordinate where ray (view w, detector u) crosses the
 * centre line of row/column `k` (row index for row-stepping views, column
 * index otherwise), in pixel units with 0 at the first pixel centre. */
static REAL FN(crossing)(const ora_geom *g, const FN(view) *w, REAL u, int k)
{
    REAL c = (REAL)(g->n_pix - 1) / 2;
    REAL dpix = (REAL)g->pixel_cm;
    REAL along = ((REAL)k - c) * dpix;        /* eta_k (row) or xi_k (column) */
    if (w->row)
        return ((u - along * w->st) / w->ct) / dpix + c;
    return ((u - along * w->ct) / w->st) / dpix + c;
}

/* One matrix entry A[(v,b), (iy,ix)] straight from the definition:
 * wstep * max(0, 1 - |f - j|) where f is the crossing on the stepping line
 * through the pixel and j the pixel's index across that line. */
static REAL FN(entry)(const ora_geom *g, const FN(view) *w, int b, int iy, int ix)
{
    REAL u = FN(bin_centre)(g, b);
    REAL f = FN(crossing)(g, w, u, w->row ? iy : ix);
    REAL tent = 1 - fabs(f - (REAL)(w->row ? ix : iy));
    return tent > 0 ? w->wstep * tent : 0;
}

/* --------------------------------------------------------- linear operators */

/* s = A x.  For each ray, walk the stepping lines in increasing order; on
 * each line only the two pixels bracketing the crossing can have a positive
 * tent weight. */
static void FN(forward_rays)(const ora_geom *g, const REAL *x, int nsel,
                             const long *sel, REAL *s)
{
    int N = g->n_pix, B = g->n_bins;
    for (int q = 0; q < nsel; ++q) {
        long i = sel ? sel[q] : q;
        int v = (int)(i / B), b = (int)(i % B);
        FN(view) w = FN(make_view)(g, v);
        REAL u = FN(bin_centre)(g, b);
        REAL acc = 0;
        for (int k = 0; k < N; ++k) {
            REAL f = FN(crossing)(g, &w, u, k);
            REAL fl = floor(f);
            if (fl < -1 || fl > N - 1)
                continue;
            for (int j = (int)fl; j <= (int)fl + 1; ++j) {
                if (j < 0 || j >= N)
                    continue;
                REAL tent = 1 - fabs(f - (REAL)j);
                if (tent <= 0)
                    continue;
                long p = w.row ? (long)k * N + j : (long)j * N + k;
                acc += w.wstep * tent * x[p];
            }
        }
        s[q] = acc;
    }
}

/* img = A^T r in scatter form: every ray adds its weighted value into the
 * pixels it touches, in ray order. */
static void FN(back_scatter)(const ora_geom *g, const REAL *r, REAL *img)
{
    int N = g->n_pix, V = g->n_views, B = g->n_bins;
    for (long p = 0; p < (long)N * N; ++p)
        img[p] = 0;
    for (int v = 0; v < V; ++v) {
        FN(view) w = FN(make_view)(g, v);
        for (int b = 0; b < B; ++b) {
            REAL rv = r[(long)v * B + b];
            REAL u = FN(bin_centre)(g, b);
            for (int k = 0; k < N; ++k) {
                REAL f = FN(crossing)(g, &w, u, k);
                REAL fl = floor(f);
                if (fl < -1 || fl > N - 1)
                    continue;
                for (int j = (int)fl; j <= (int)fl + 1; ++j) {
                    if (j < 0 || j >= N)
                        continue;
                    REAL tent = 1 - fabs(f - (REAL)j);
                    if (tent <= 0)
                        continue;
                    long p = w.row ? (long)k * N + j : (long)j * N + k;
                    img[p] += w.wstep * tent * rv;
                }
            }
        }
    }
}

/* (A^T r)_p for selected pixels, one at a time: the sum over every ray of
 * entry(ray, p) * r_ray.  Slow (V*B entries per pixel) and used for sampled
 * checks at full problem sizes. */
static void FN(back_pixels)(const ora_geom *g, const REAL *r, int nsel,
                            const long *sel, REAL *out)
{
    int N = g->n_pix, V = g->n_views, B = g->n_bins;
    for (int q = 0; q < nsel; ++q) {
        int iy = (int)(sel[q] / N), ix = (int)(sel[q] % N);
        REAL acc = 0;
        for (int v = 0; v < V; ++v) {
            FN(view) w = FN(make_view)(g, v);
            for (int b = 0; b < B; ++b) {
                REAL a = FN(entry)(g, &w, b, iy, ix);
                if (a != 0)
                    acc += a * r[(long)v * B + b];
            }
        }
        out[q] = acc;
    }
}

/* ------------------------------------------------------- spectral model */

/* Literal per-window residual: r_i = sum_j y[j][i] - sum_j sum_k
 * Iwk[j][k] exp(-mu_k max(s_i, 0)).
 *
 * With bg (nullable, [n]) the other materials of the scan are known and bg_i
 * is their line integral on ray i.  The appendix's reparametrisation
 * (multi-material model with known materials) then gives ray i its own
 * window spectrum: per window j, Ibar'_ij = sum_k Iwk[j][k] exp(-mu_k bg_i)
 * and s'_ijk = Iwk[j][k] exp(-mu_k bg_i) / Ibar'_ij, and the model counts
 * are sum_j Ibar'_ij sum_k s'_ijk exp(-mu_k max(s_i, 0)). */
static void FN(residual)(long n, int K, int Wn, const REAL *mu, const REAL *Iwk,
                         const REAL *y, const REAL *s, const REAL *bg, REAL *r, REAL *model)
{
    for (long i = 0; i < n; ++i) {
        REAL sp = s[i] > 0 ? s[i] : 0;
        REAL ysum = 0, m = 0;
        for (int j = 0; j < Wn; ++j)
            ysum += y[(long)j * n + i];
        for (int j = 0; j < Wn; ++j) {
            if (!bg) {
                for (int k = 0; k < K; ++k)
                    m += Iwk[(long)j * K + k] * exp(-mu[k] * sp);
                continue;
            }
            REAL ibar = 0, win = 0;
            for (int k = 0; k < K; ++k)
                ibar += Iwk[(long)j * K + k] * exp(-mu[k] * bg[i]);
            if (ibar <= 0)
                continue;
            for (int k = 0; k < K; ++k) {
                REAL sk = Iwk[(long)j * K + k] * exp(-mu[k] * bg[i]) / ibar;
                win += sk * exp(-mu[k] * sp);
            }
            m += ibar * win;
        }
        r[i] = ysum - m;
        if (model)
            model[i] = m;
    }
}

typedef struct {
    int K, Wn;
    REAL *mu, *Iwk, *y, *bg;   /* [K], [Wn*K], [Wn*n], [n] or NULL */
} FN(spec);

/* F(x) = (1/n) A^T (Y - model(Ax)), n = number of rays. */
static void FN(apply_F)(const ora_geom *g, const FN(spec) *sp, const REAL *x,
                        REAL *F, REAL *s, REAL *r)
{
    long n = (long)g->n_views * g->n_bins, d = (long)g->n_pix * g->n_pix;
    FN(forward_rays)(g, x, (int)n, 0, s);
    FN(residual)(n, sp->K, sp->Wn, sp->mu, sp->Iwk, sp->y, s, sp->bg, r, 0);
    FN(back_scatter)(g, r, F);
    for (long p = 0; p < d; ++p)
        F[p] = F[p] / (REAL)n;
}

/* ------------------------------------------------------ helpers (copy in) */

static REAL *FN(to_real)(const double *a, long len)
{
    REAL *o = (REAL *)calloc((size_t)(len > 0 ? len : 1), sizeof(REAL));
    for (long i = 0; i < len; ++i)
        o[i] = (REAL)a[i];
    return o;
}

static void FN(to_double)(const REAL *a, long len, double *o)
{
    for (long i = 0; i < len; ++i)
        o[i] = (double)a[i];
}

static REAL FN(dot)(const REAL *a, const REAL *b, long len)
{
    REAL acc = 0;
    for (long i = 0; i < len; ++i)
        acc += a[i] * b[i];
    return acc;
}

static FN(spec) FN(load_spec)(const ora_geom *g, int K, int Wn, const double *mu,
                              const double *Iwk, const double *y, const double *bg)
{
    FN(spec) sp;
    long n = (long)g->n_views * g->n_bins;
    sp.K = K;
    sp.Wn = Wn;
    sp.mu = FN(to_real)(mu, K);
    sp.Iwk = FN(to_real)(Iwk, (long)Wn * K);
    sp.y = y ? FN(to_real)(y, (long)Wn * n) : 0;
    sp.bg = bg ? FN(to_real)(bg, n) : 0;
    return sp;
}

static void FN(free_spec)(FN(spec) *sp)
{
    free(sp->mu);
    free(sp->Iwk);
    free(sp->y);
    free(sp->bg);
}

/* ------------------------------------------------------------ exported API */

void FN(ora_forward)(const ora_geom *g, const double *x, double *s)
{
    long n = (long)g->n_views * g->n_bins, d = (long)g->n_pix * g->n_pix;
    REAL *xr = FN(to_real)(x, d);
    REAL *sr = (REAL *)malloc(sizeof(REAL) * (size_t)n);
    FN(forward_rays)(g, xr, (int)n, 0, sr);
    FN(to_double)(sr, n, s);
    free(xr);
    free(sr);
}

void FN(ora_forward_rays)(const ora_geom *g, const double *x, int nsel,
                          const long *sel, double *s)
{
    long d = (long)g->n_pix * g->n_pix;
    REAL *xr = FN(to_real)(x, d);
    REAL *sr = (REAL *)malloc(sizeof(REAL) * (size_t)(nsel > 0 ? nsel : 1));
    FN(forward_rays)(g, xr, nsel, sel, sr);
    FN(to_double)(sr, nsel, s);
    free(xr);
    free(sr);
}

void FN(ora_back)(const ora_geom *g, const double *r, double *img)
{
    long n = (long)g->n_views * g->n_bins, d = (long)g->n_pix * g->n_pix;
    REAL *rr = FN(to_real)(r, n);
    REAL *ir = (REAL *)malloc(sizeof(REAL) * (size_t)d);
    FN(back_scatter)(g, rr, ir);
    FN(to_double)(ir, d, img);
    free(rr);
    free(ir);
}

void FN(ora_back_pixels)(const ora_geom *g, const double *r, int nsel,
                         const long *sel, double *out)
{
    long n = (long)g->n_views * g->n_bins;
    REAL *rr = FN(to_real)(r, n);
    REAL *o = (REAL *)malloc(sizeof(REAL) * (size_t)(nsel > 0 ? nsel : 1));
    FN(back_pixels)(g, rr, nsel, sel, o);
    FN(to_double)(o, nsel, out);
    free(rr);
    free(o);
}

void FN(ora_residual)(long n, int K, int Wn, const double *mu, const double *Iwk,
                      const double *y, const double *s, const double *bg, double *r,
                      double *model)
{
    REAL *mur = FN(to_real)(mu, K), *Ir = FN(to_real)(Iwk, (long)Wn * K);
    REAL *yr = FN(to_real)(y, (long)Wn * n), *sr = FN(to_real)(s, n);
    REAL *br = bg ? FN(to_real)(bg, n) : 0;
    REAL *rr = (REAL *)malloc(sizeof(REAL) * (size_t)n);
    REAL *mr = (REAL *)malloc(sizeof(REAL) * (size_t)n);
    FN(residual)(n, K, Wn, mur, Ir, yr, sr, br, rr, mr);
    FN(to_double)(rr, n, r);
    if (model)
        FN(to_double)(mr, n, model);
    free(mur); free(Ir); free(yr); free(sr); free(br); free(rr); free(mr);
}

/* F(x); optionally also returns s = Ax and r (each may be NULL). */
void FN(ora_operator)(const ora_geom *g, int K, int Wn, const double *mu,
                      const double *Iwk, const double *y, const double *bg, const double *x,
                      double *F, double *s_out, double *r_out)
{
    long n = (long)g->n_views * g->n_bins, d = (long)g->n_pix * g->n_pix;
    FN(spec) sp = FN(load_spec)(g, K, Wn, mu, Iwk, y, bg);
    REAL *xr = FN(to_real)(x, d);
    REAL *Fr = (REAL *)malloc(sizeof(REAL) * (size_t)d);
    REAL *sr = (REAL *)malloc(sizeof(REAL) * (size_t)n);
    REAL *rr = (REAL *)malloc(sizeof(REAL) * (size_t)n);
    FN(apply_F)(g, &sp, xr, Fr, sr, rr);
    FN(to_double)(Fr, d, F);
    if (s_out)
        FN(to_double)(sr, n, s_out);
    if (r_out)
        FN(to_double)(rr, n, r_out);
    FN(free_spec)(&sp);
    free(xr); free(Fr); free(sr); free(rr);
}

/*
 * Projected extragradient, x in/out (x_1 on entry, last iterate on exit):
 *   x_{t+1/2} = max(0, x_t - gamma F(x_t))
 *   x_{t+1}   = max(0, x_t - gamma F(x_{t+1/2}))
 * for t = 1..max_iters.  If tol > 0, after step t the natural residual
 * rho_t = ||x_{t+1/2} - x_t|| / ||x_t|| (undefined, hence not tested, while
 * x_t = 0) is compared with tol and the loop stops with x_{t+1} once
 * rho_t <= tol.  rho_hist (nullable, length max_iters) receives rho_t
 * (-1 where undefined).  Returns the number of steps taken.
 */
int FN(ora_eg)(const ora_geom *g, int K, int Wn, const double *mu,
               const double *Iwk, const double *y, const double *bg, double *x, double gamma,
               int max_iters, double tol, double *rho_hist)
{
    long n = (long)g->n_views * g->n_bins, d = (long)g->n_pix * g->n_pix;
    FN(spec) sp = FN(load_spec)(g, K, Wn, mu, Iwk, y, bg);
    REAL *xt = FN(to_real)(x, d);
    REAL *xh = (REAL *)malloc(sizeof(REAL) * (size_t)d);
    REAL *F = (REAL *)malloc(sizeof(REAL) * (size_t)d);
    REAL *s = (REAL *)malloc(sizeof(REAL) * (size_t)n);
    REAL *r = (REAL *)malloc(sizeof(REAL) * (size_t)n);
    REAL gm = (REAL)gamma;
    int t;
    for (t = 1; t <= max_iters; ++t) {
        FN(apply_F)(g, &sp, xt, F, s, r);
        REAL num = 0, den = 0;
        for (long p = 0; p < d; ++p) {
            REAL z = xt[p] - gm * F[p];
            xh[p] = z > 0 ? z : 0;
            num += (xh[p] - xt[p]) * (xh[p] - xt[p]);
            den += xt[p] * xt[p];
        }
        double rho = den > 0 ? (double)sqrt(num / den) : -1.0;
        if (rho_hist)
            rho_hist[t - 1] = rho;
        FN(apply_F)(g, &sp, xh, F, s, r);
        for (long p = 0; p < d; ++p) {
            REAL z = xt[p] - gm * F[p];
            xt[p] = z > 0 ? z : 0;
        }
        if (tol > 0 && rho >= 0 && rho <= tol)
            break;
    }
    if (t > max_iters)
        t = max_iters;
    FN(to_double)(xt, d, x);
    FN(free_spec)(&sp);
    free(xt); free(xh); free(F); free(s); free(r);
    return t;
}

/*
 * Averaged iterate of the paper's experiments (Sec. 5, comparison of
 * methods): at index s the mean of the last half of the iterates,
 *   xbar_s = (1 / (s - floor(s/2))) * sum_{j = floor(s/2)+1}^{s} x_j,
 * taken here from traj, whose row j-1 holds x_j (x_1 the starting point).
 */
static void FN(window_mean)(const REAL *traj, long d, int s, REAL *out)
{
    int first = s / 2 + 1;
    for (long p = 0; p < d; ++p)
        out[p] = 0;
    for (int j = first; j <= s; ++j)
        for (long p = 0; p < d; ++p)
            out[p] += traj[(size_t)(j - 1) * (size_t)d + (size_t)p];
    for (long p = 0; p < d; ++p)
        out[p] /= (REAL)(s - first + 1);
}

/* window_mean on a caller-supplied trajectory (rows x_1 .. x_s). */
void FN(ora_window_mean)(const double *traj, long d, int s, double *out)
{
    REAL *tr = FN(to_real)(traj, (long)s * d);
    REAL *o = (REAL *)malloc(sizeof(REAL) * (size_t)d);
    FN(window_mean)(tr, d, s, o);
    FN(to_double)(o, d, out);
    free(tr); free(o);
}

/*
 * Projected extragradient with the paper's averaged-iterate stopping rule
 * (Sec. 5): the iterates are those of ora_eg; after step t the averaged
 * iterates at s = t+1 and s-1 = t are compared and the loop stops once
 * ||xbar_{t+1} - xbar_t||_2 <= tol (tol > 0; an absolute bound, as in the
 * paper).  On exit x holds xbar at the last index reached and x_last
 * (nullable) the last iterate x_{t+1}; crit_hist (nullable, length
 * max_iters) receives ||xbar_{t+1} - xbar_t||.  Keeps the whole trajectory
 * (max_iters + 1 images): small problems only.  Returns the steps taken.
 */
int FN(ora_eg_avg)(const ora_geom *g, int K, int Wn, const double *mu,
                   const double *Iwk, const double *y, const double *bg, double *x,
                   double gamma, int max_iters, double tol, double *crit_hist,
                   double *x_last)
{
    long n = (long)g->n_views * g->n_bins, d = (long)g->n_pix * g->n_pix;
    FN(spec) sp = FN(load_spec)(g, K, Wn, mu, Iwk, y, bg);
    REAL *traj = (REAL *)malloc(sizeof(REAL) * (size_t)(max_iters + 1) * (size_t)d);
    REAL *xh = (REAL *)malloc(sizeof(REAL) * (size_t)d);
    REAL *F = (REAL *)malloc(sizeof(REAL) * (size_t)d);
    REAL *s = (REAL *)malloc(sizeof(REAL) * (size_t)n);
    REAL *r = (REAL *)malloc(sizeof(REAL) * (size_t)n);
    REAL *prev = (REAL *)malloc(sizeof(REAL) * (size_t)d);
    REAL *cur = (REAL *)malloc(sizeof(REAL) * (size_t)d);
    REAL gm = (REAL)gamma;
    for (long p = 0; p < d; ++p)
        traj[p] = (REAL)x[p];
    FN(window_mean)(traj, d, 1, cur);
    int t;
    for (t = 1; t <= max_iters; ++t) {
        const REAL *xt = traj + (size_t)(t - 1) * (size_t)d;
        REAL *xn = traj + (size_t)t * (size_t)d;
        FN(apply_F)(g, &sp, xt, F, s, r);
        for (long p = 0; p < d; ++p) {
            REAL z = xt[p] - gm * F[p];
            xh[p] = z > 0 ? z : 0;
        }
        FN(apply_F)(g, &sp, xh, F, s, r);
        for (long p = 0; p < d; ++p) {
            REAL z = xt[p] - gm * F[p];
            xn[p] = z > 0 ? z : 0;
        }
        for (long p = 0; p < d; ++p)
            prev[p] = cur[p];
        FN(window_mean)(traj, d, t + 1, cur);
        REAL sq = 0;
        for (long p = 0; p < d; ++p)
            sq += (cur[p] - prev[p]) * (cur[p] - prev[p]);
        double crit = (double)sqrt(sq);
        if (crit_hist)
            crit_hist[t - 1] = crit;
        if (tol > 0 && crit <= tol)
            break;
    }
    if (t > max_iters)
        t = max_iters;
    FN(to_double)(cur, d, x);
    if (x_last)
        FN(to_double)(traj + (size_t)t * (size_t)d, d, x_last);
    FN(free_spec)(&sp);
    free(traj); free(xh); free(F); free(s); free(r); free(prev); free(cur);
    return t;
}

/* ------------------------------------------- TV ball and orthant (Sec. 5) */

/*
 * Isotropic total variation of an N x N image with forward differences and
 * nothing across the last row or column:
 *   TV(x) = sum_{iy,ix} sqrt(dx^2 + dy^2),
 *   dx = x[iy][ix+1] - x[iy][ix] (0 when ix = N-1), dy = x[iy+1][ix] - x[iy][ix]
 *   (0 when iy = N-1).
 */
static REAL FN(tv_norm)(int N, const REAL *x)
{
    REAL acc = 0;
    for (int iy = 0; iy < N; ++iy)
        for (int ix = 0; ix < N; ++ix) {
            REAL c = x[(long)iy * N + ix];
            REAL dx = ix + 1 < N ? x[(long)iy * N + ix + 1] - c : 0;
            REAL dy = iy + 1 < N ? x[(long)(iy + 1) * N + ix] - c : 0;
            acc += sqrt(dx * dx + dy * dy);
        }
    return acc;
}

/*
 * TV proximal point xbar = argmin_x ||x - b||^2 + lam TV(x) (Sec. 5, eq.
 * TV-regularization), by `iters` steps of the fast gradient projection
 * method on the dual of TV denoising (Beck and Teboulle, IEEE TIP 2009),
 * started from zero.  With l = lam / 2 the problem is min ||x - b||^2 +
 * 2 l TV(x); the dual variable is a pair of fields (p, q) with each
 * (p_ij, q_ij) in the unit disc, and
 *   L(p, q)_ij = p_ij + q_ij - p_{i-1,j} - q_{i,j-1},
 *   L^T(x)     = (x_ij - x_{i+1,j}, x_ij - x_{i,j+1})
 * (terms outside the image are zero; p on the last row and q on the last
 * column stay zero).  One step from (r, s) with momentum t:
 *   x = b - l L(r, s);  (p', q') = P_disc((r, s) + L^T(x) / (8 l));
 *   t' = (1 + sqrt(1 + 4 t^2)) / 2;  (r, s) = (p', q') + ((t - 1)/t') ((p', q') - (p, q)).
 * The result is b - l L(p, q).  lam <= 0 returns b.
 */
static void FN(tv_prox)(int N, const REAL *b, REAL lam, int iters, REAL *x)
{
    long d = (long)N * N;
    if (!(lam > 0)) {
        for (long i = 0; i < d; ++i)
            x[i] = b[i];
        return;
    }
    REAL l = lam / 2;
    REAL *p = (REAL *)calloc((size_t)d, sizeof(REAL)), *q = (REAL *)calloc((size_t)d, sizeof(REAL));
    REAL *r = (REAL *)calloc((size_t)d, sizeof(REAL)), *sv = (REAL *)calloc((size_t)d, sizeof(REAL));
    REAL *pn = (REAL *)calloc((size_t)d, sizeof(REAL)), *qn = (REAL *)calloc((size_t)d, sizeof(REAL));
    REAL t = 1;
    for (int k = 0; k < iters; ++k) {
        /* x = b - l L(r, s) */
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) {
                long c = (long)i * N + j;
                REAL Lv = r[c] + sv[c] - (i > 0 ? r[c - N] : 0) - (j > 0 ? sv[c - 1] : 0);
                x[c] = b[c] - l * Lv;
            }
        /* gradient step and projection onto the unit disc */
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) {
                long c = (long)i * N + j;
                REAL gp = i + 1 < N ? x[c] - x[c + N] : 0;
                REAL gq = j + 1 < N ? x[c] - x[c + 1] : 0;
                REAL a = r[c] + gp / (8 * l), bq = sv[c] + gq / (8 * l);
                if (i + 1 >= N)
                    a = 0;
                if (j + 1 >= N)
                    bq = 0;
                REAL nrm = sqrt(a * a + bq * bq);
                REAL den = nrm > 1 ? nrm : 1;
                pn[c] = a / den;
                qn[c] = bq / den;
            }
        REAL tn = (1 + sqrt(1 + 4 * t * t)) / 2;
        REAL w = (t - 1) / tn;
        for (long c = 0; c < d; ++c) {
            r[c] = pn[c] + w * (pn[c] - p[c]);
            sv[c] = qn[c] + w * (qn[c] - q[c]);
            p[c] = pn[c];
            q[c] = qn[c];
        }
        t = tn;
    }
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            long c = (long)i * N + j;
            REAL Lv = p[c] + q[c] - (i > 0 ? p[c - N] : 0) - (j > 0 ? q[c - 1] : 0);
            x[c] = b[c] - l * Lv;
        }
    free(p); free(q); free(r); free(sv); free(pn); free(qn);
}

/*
 * Approximate projection onto the TV ball {TV(x) <= tau} as in Sec. 5: the
 * TV-regularized point xbar(lam) for a lam found by binary search, until
 * |TV(xbar) - tau| <= tv_tol.  If TV(v) <= tau the result is v (lam 0).
 *
 * The search first brackets the weight, keeping hi the weight of the last
 * point found inside the ball (TV <= tau) and lo one whose point lies
 * outside (TV > tau), then halves [lo, hi].  The paper does not say where
 * the search starts; here:
 *   - cold (lam0 <= 0): hi starts at 1 and doubles (at most 60 times) while
 *     TV(xbar(hi)) > tau, lo being its previous value (0 first);
 *   - warm (lam0 > 0, the weight of a previous projection of the same run):
 *     the first point is xbar(lam0).  If its TV is above tau, lo = lam0 and
 *     hi grows by 5/4, then doubles (at most 60 times), while TV(xbar(hi))
 *     > tau (lo following hi); if it is at or below tau, hi = lam0 and lo
 *     shrinks by 4/5, then halves (at most 60 times), while TV(xbar(lo)) <=
 *     tau (hi following lo), lo = 0 if it never rises above tau.  A point
 *     met while bracketing with |TV - tau| <= tv_tol is the result.
 * Then up to max_bisect midpoints mid = (lo + hi)/2: the first with |TV -
 * tau| <= tv_tol is the result, TV > tau moves lo to mid and TV <= tau moves
 * hi to mid.  Without a hit the result is xbar(hi), the last point inside
 * the ball.  Returns the number of proximal solves; *lam_out receives the
 * lam of the result.
 */
static int FN(tv_ball)(int N, const REAL *v, REAL tau, REAL tv_tol, int iters, int max_bisect,
                       REAL lam0, REAL *out, REAL *lam_out)
{
    long d = (long)N * N;
    if (FN(tv_norm)(N, v) <= tau) {
        for (long i = 0; i < d; ++i)
            out[i] = v[i];
        *lam_out = 0;
        return 0;
    }
    REAL *x = (REAL *)malloc(sizeof(REAL) * (size_t)d);
    int solves = 0;
    REAL lo, hi, t;
    int hit = 0;
#define ORA_KEEP(L)                          \
    do {                                     \
        for (long i = 0; i < d; ++i)         \
            out[i] = x[i];                   \
        *lam_out = (L);                      \
    } while (0)
    if (lam0 <= 0) {
        lo = 0;
        hi = 1;
        FN(tv_prox)(N, v, hi, iters, x);
        ++solves;
        t = FN(tv_norm)(N, x);
        for (int grow = 0; t > tau && grow < 60; ++grow) {
            lo = hi;
            hi = 2 * hi;
            FN(tv_prox)(N, v, hi, iters, x);
            ++solves;
            t = FN(tv_norm)(N, x);
        }
        ORA_KEEP(hi);
    } else {
        FN(tv_prox)(N, v, lam0, iters, x);
        ++solves;
        t = FN(tv_norm)(N, x);
        if (fabs(t - tau) <= tv_tol) {
            ORA_KEEP(lam0);
            hit = 1;
        } else if (t > tau) {
            lo = lam0;
            hi = lam0 * 5 / 4;
            for (int grow = 0;; ++grow) {
                FN(tv_prox)(N, v, hi, iters, x);
                ++solves;
                t = FN(tv_norm)(N, x);
                if (fabs(t - tau) <= tv_tol) {
                    ORA_KEEP(hi);
                    hit = 1;
                    break;
                }
                if (t <= tau || grow + 1 >= 60)
                    break;
                lo = hi;
                hi = 2 * hi;
            }
            if (!hit)
                ORA_KEEP(hi);
        } else {
            hi = lam0;
            ORA_KEEP(hi);
            lo = lam0 * 4 / 5;
            for (int shrink = 0;; ++shrink) {
                FN(tv_prox)(N, v, lo, iters, x);
                ++solves;
                t = FN(tv_norm)(N, x);
                if (fabs(t - tau) <= tv_tol) {
                    ORA_KEEP(lo);
                    hit = 1;
                    break;
                }
                if (t > tau)
                    break;
                hi = lo;
                ORA_KEEP(hi);
                if (shrink + 1 >= 60) {
                    lo = 0;
                    break;
                }
                lo = lo / 2;
            }
        }
    }
    for (int it = 0; !hit && it < max_bisect; ++it) {
        REAL mid = (lo + hi) / 2;
        FN(tv_prox)(N, v, mid, iters, x);
        ++solves;
        t = FN(tv_norm)(N, x);
        if (fabs(t - tau) <= tv_tol) {
            ORA_KEEP(mid);
            break;
        }
        if (t > tau) {
            lo = mid;
        } else {
            hi = mid;
            ORA_KEEP(mid);
        }
    }
#undef ORA_KEEP
    free(x);
    return solves;
}

/*
 * Projection onto X = {TV(x) <= tau} intersected with the orthant by
 * Dykstra's algorithm (Sec. 5, eq. projection-intersection): z_0 = z,
 * p_0 = q_0 = 0; y_k = P_TV(z_k + p_k), p_{k+1} = z_k + p_k - y_k,
 * z_{k+1} = max(0, y_k + q_k), q_{k+1} = y_k + q_k - z_{k+1}; stops once
 * ||z_{k+1} - z_k||_2 <= tol or after max_outer rounds.  P_TV is tv_ball,
 * warm-started from *lam_carry (the weight of the last TV-ball point the
 * run found, 0 for none), which each round updates.
 */
static void FN(tv_dykstra)(int N, const REAL *z, REAL tau, REAL tv_tol, int iters,
                           int max_bisect, REAL tol, int max_outer, REAL *out, int *rounds,
                           int *solves, REAL *lam_carry)
{
    long d = (long)N * N;
    REAL *p = (REAL *)calloc((size_t)d, sizeof(REAL)), *q = (REAL *)calloc((size_t)d, sizeof(REAL));
    REAL *y = (REAL *)malloc(sizeof(REAL) * (size_t)d), *w = (REAL *)malloc(sizeof(REAL) * (size_t)d);
    for (long i = 0; i < d; ++i)
        out[i] = z[i];
    int k, ns = 0;
    for (k = 0; k < max_outer; ++k) {
        REAL lam;
        for (long i = 0; i < d; ++i)
            w[i] = out[i] + p[i];
        ns += FN(tv_ball)(N, w, tau, tv_tol, iters, max_bisect, *lam_carry, y, &lam);
        if (lam > 0)
            *lam_carry = lam;
        REAL sq = 0;
        for (long i = 0; i < d; ++i) {
            p[i] = w[i] - y[i];
            REAL zn = y[i] + q[i] > 0 ? y[i] + q[i] : 0;
            q[i] = y[i] + q[i] - zn;
            sq += (zn - out[i]) * (zn - out[i]);
            out[i] = zn;
        }
        if (sqrt(sq) <= tol) {
            ++k;
            break;
        }
    }
    if (rounds)
        *rounds = k;
    if (solves)
        *solves = ns;
    free(p); free(q); free(y); free(w);
}

double FN(ora_tv_norm)(int N, const double *x)
{
    REAL *xr = FN(to_real)(x, (long)N * N);
    REAL t = FN(tv_norm)(N, xr);
    free(xr);
    return (double)t;
}

void FN(ora_tv_prox)(int N, const double *b, double lam, int iters, double *x)
{
    long d = (long)N * N;
    REAL *br = FN(to_real)(b, d), *xr = (REAL *)malloc(sizeof(REAL) * (size_t)d);
    FN(tv_prox)(N, br, (REAL)lam, iters, xr);
    FN(to_double)(xr, d, x);
    free(br); free(xr);
}

int FN(ora_tv_ball)(int N, const double *v, double tau, double tv_tol, int iters,
                    int max_bisect, double lam0, double *out, double *lam_out)
{
    long d = (long)N * N;
    REAL *vr = FN(to_real)(v, d), *o = (REAL *)malloc(sizeof(REAL) * (size_t)d), lam = 0;
    int ns = FN(tv_ball)(N, vr, (REAL)tau, (REAL)tv_tol, iters, max_bisect, (REAL)lam0, o, &lam);
    FN(to_double)(o, d, out);
    if (lam_out)
        *lam_out = (double)lam;
    free(vr); free(o);
    return ns;
}

int FN(ora_project_tv)(int N, const double *z, double tau, double tv_tol, int iters,
                       int max_bisect, double tol, int max_outer, double *out, int *solves)
{
    long d = (long)N * N;
    REAL *zr = FN(to_real)(z, d), *o = (REAL *)malloc(sizeof(REAL) * (size_t)d);
    int rounds = 0;
    REAL lam_carry = 0;
    FN(tv_dykstra)(N, zr, (REAL)tau, (REAL)tv_tol, iters, max_bisect, (REAL)tol, max_outer, o,
                   &rounds, solves, &lam_carry);
    FN(to_double)(o, d, out);
    free(zr); free(o);
    return rounds;
}

/*
 * Projected extragradient over X = {TV(x) <= tau} intersected with the
 * orthant, the constraint set of the paper's experiments (Sec. 5): as
 * ora_eg, with both half-steps projected by tv_dykstra, each TV-ball search
 * warm-started from the weight of the run's previous one.  rho_hist as in
 * ora_eg; tol > 0 stops on the natural residual.  *solves_out (if not
 * NULL) receives the TV-regularized points computed over the run (the
 * search's decision path).  Returns the steps taken.
 */
int FN(ora_eg_tv)(const ora_geom *g, int K, int Wn, const double *mu, const double *Iwk,
                  const double *y, const double *bg, double *x, double gamma, int max_iters,
                  double tol, double tau, double tv_tol, int prox_iters, int max_bisect,
                  double dyk_tol, int max_outer, double *rho_hist, int *solves_out)
{
    int ns_total = 0, ns = 0;
    long n = (long)g->n_views * g->n_bins, d = (long)g->n_pix * g->n_pix;
    int N = g->n_pix;
    FN(spec) sp = FN(load_spec)(g, K, Wn, mu, Iwk, y, bg);
    REAL *xt = FN(to_real)(x, d);
    REAL *xh = (REAL *)malloc(sizeof(REAL) * (size_t)d);
    REAL *v = (REAL *)malloc(sizeof(REAL) * (size_t)d);
    REAL *F = (REAL *)malloc(sizeof(REAL) * (size_t)d);
    REAL *s = (REAL *)malloc(sizeof(REAL) * (size_t)n);
    REAL *r = (REAL *)malloc(sizeof(REAL) * (size_t)n);
    REAL gm = (REAL)gamma;
    REAL lam_carry = 0;
    int t;
    for (t = 1; t <= max_iters; ++t) {
        FN(apply_F)(g, &sp, xt, F, s, r);
        for (long p = 0; p < d; ++p)
            v[p] = xt[p] - gm * F[p];
        FN(tv_dykstra)(N, v, (REAL)tau, (REAL)tv_tol, prox_iters, max_bisect, (REAL)dyk_tol,
                       max_outer, xh, 0, &ns, &lam_carry);
        ns_total += ns;
        REAL num = 0, den = 0;
        for (long p = 0; p < d; ++p) {
            num += (xh[p] - xt[p]) * (xh[p] - xt[p]);
            den += xt[p] * xt[p];
        }
        double rho = den > 0 ? (double)sqrt(num / den) : -1.0;
        if (rho_hist)
            rho_hist[t - 1] = rho;
        FN(apply_F)(g, &sp, xh, F, s, r);
        for (long p = 0; p < d; ++p)
            v[p] = xt[p] - gm * F[p];
        FN(tv_dykstra)(N, v, (REAL)tau, (REAL)tv_tol, prox_iters, max_bisect, (REAL)dyk_tol,
                       max_outer, xt, 0, &ns, &lam_carry);
        ns_total += ns;
        if (tol > 0 && rho >= 0 && rho <= tol)
            break;
    }
    if (t > max_iters)
        t = max_iters;
    if (solves_out)
        *solves_out = ns_total;
    FN(to_double)(xt, d, x);
    FN(free_spec)(&sp);
    free(xt); free(xh); free(v); free(F); free(s); free(r);
    return t;
}

/* ------------------------------------- dense measurements (Sec. 2.2, Sec. 5) */

/*
 * The operator with an explicit measurement matrix A (n rows a_i, d
 * columns, row-major), as in the Gaussian measurement model: the same
 * single-index model and F(x) = (1/n) sum_i r_i a_i with
 * r_i = sum_j y[j][i] - sum_j sum_k I[j][k] exp(-mu_k max(<a_i, x>, 0)).
 */
static void FN(dense_F)(long n, long d, const REAL *A, const FN(spec) *sp, const REAL *x,
                        REAL *F, REAL *s, REAL *r)
{
    for (long i = 0; i < n; ++i) {
        REAL acc = 0;
        for (long j = 0; j < d; ++j)
            acc += A[i * d + j] * x[j];
        s[i] = acc;
    }
    FN(residual)(n, sp->K, sp->Wn, sp->mu, sp->Iwk, sp->y, s, 0, r, 0);
    for (long j = 0; j < d; ++j)
        F[j] = 0;
    for (long i = 0; i < n; ++i)
        for (long j = 0; j < d; ++j)
            F[j] += r[i] * A[i * d + j];
    for (long j = 0; j < d; ++j)
        F[j] = F[j] / (REAL)n;
}

/* Projection onto the ball {||x||_2 <= radius} (radius <= 0: no constraint). */
static void FN(ball)(long d, REAL radius, REAL *x)
{
    if (!(radius > 0))
        return;
    REAL nrm = sqrt(FN(dot)(x, x, d));
    if (nrm > radius)
        for (long j = 0; j < d; ++j)
            x[j] = x[j] * (radius / nrm);
}

static FN(spec) FN(load_dense_spec)(long n, int K, int Wn, const double *mu, const double *Iwk,
                                    const double *y)
{
    FN(spec) sp;
    sp.K = K;
    sp.Wn = Wn;
    sp.mu = FN(to_real)(mu, K);
    sp.Iwk = FN(to_real)(Iwk, (long)Wn * K);
    sp.y = FN(to_real)(y, (long)Wn * n);
    sp.bg = 0;
    return sp;
}

void FN(ora_dense_operator)(long n, long d, const double *A, int K, int Wn, const double *mu,
                            const double *Iwk, const double *y, const double *x, double *F)
{
    FN(spec) sp = FN(load_dense_spec)(n, K, Wn, mu, Iwk, y);
    REAL *Ar = FN(to_real)(A, n * d), *xr = FN(to_real)(x, d);
    REAL *Fr = (REAL *)malloc(sizeof(REAL) * (size_t)d);
    REAL *s = (REAL *)malloc(sizeof(REAL) * (size_t)n), *r = (REAL *)malloc(sizeof(REAL) * (size_t)n);
    FN(dense_F)(n, d, Ar, &sp, xr, Fr, s, r);
    FN(to_double)(Fr, d, F);
    FN(free_spec)(&sp);
    free(Ar); free(xr); free(Fr); free(s); free(r);
}

/*
 * Projected extragradient with a dense A over X = {||x|| <= radius} (the
 * bounded set of Assumption assump-X centred at the origin; radius <= 0 is
 * the whole space): both half-steps from x_t as in eq. extragrad-method.
 * rho_hist and tol as in ora_eg.  Returns the steps taken.
 */
int FN(ora_dense_eg)(long n, long d, const double *A, int K, int Wn, const double *mu,
                     const double *Iwk, const double *y, double *x, double gamma, double radius,
                     int max_iters, double tol, double *rho_hist)
{
    FN(spec) sp = FN(load_dense_spec)(n, K, Wn, mu, Iwk, y);
    REAL *Ar = FN(to_real)(A, n * d), *xt = FN(to_real)(x, d);
    REAL *xh = (REAL *)malloc(sizeof(REAL) * (size_t)d), *F = (REAL *)malloc(sizeof(REAL) * (size_t)d);
    REAL *s = (REAL *)malloc(sizeof(REAL) * (size_t)n), *r = (REAL *)malloc(sizeof(REAL) * (size_t)n);
    REAL gm = (REAL)gamma, R = (REAL)radius;
    int t;
    for (t = 1; t <= max_iters; ++t) {
        FN(dense_F)(n, d, Ar, &sp, xt, F, s, r);
        for (long j = 0; j < d; ++j)
            xh[j] = xt[j] - gm * F[j];
        FN(ball)(d, R, xh);
        REAL num = 0, den = 0;
        for (long j = 0; j < d; ++j) {
            num += (xh[j] - xt[j]) * (xh[j] - xt[j]);
            den += xt[j] * xt[j];
        }
        double rho = den > 0 ? (double)sqrt(num / den) : -1.0;
        if (rho_hist)
            rho_hist[t - 1] = rho;
        FN(dense_F)(n, d, Ar, &sp, xh, F, s, r);
        for (long j = 0; j < d; ++j)
            xt[j] = xt[j] - gm * F[j];
        FN(ball)(d, R, xt);
        if (tol > 0 && rho >= 0 && rho <= tol)
            break;
    }
    if (t > max_iters)
        t = max_iters;
    FN(to_double)(xt, d, x);
    FN(free_spec)(&sp);
    free(Ar); free(xt); free(xh); free(F); free(s); free(r);
    return t;
}

/*
 * Largest eigenvalue of Sigma = A^T A / n by power iteration from the
 * constant unit vector, with Rayleigh quotients; stops when the quotient
 * changes by less than rel_tol (relative) or after max_iters products.
 */
double FN(ora_power)(const ora_geom *g, int max_iters, double rel_tol, int *iters_out)
{
    long n = (long)g->n_views * g->n_bins, d = (long)g->n_pix * g->n_pix;
    REAL *v = (REAL *)malloc(sizeof(REAL) * (size_t)d);
    REAL *u = (REAL *)malloc(sizeof(REAL) * (size_t)d);
    REAL *s = (REAL *)malloc(sizeof(REAL) * (size_t)n);
    REAL lam = 0;
    int it;
    for (long p = 0; p < d; ++p)
        v[p] = 1 / sqrt((REAL)d);
    for (it = 1; it <= max_iters; ++it) {
        FN(forward_rays)(g, v, (int)n, 0, s);
        FN(back_scatter)(g, s, u);
        for (long p = 0; p < d; ++p)
            u[p] = u[p] / (REAL)n;
        REAL lam_new = FN(dot)(v, u, d) / FN(dot)(v, v, d);
        REAL nu = sqrt(FN(dot)(u, u, d));
        for (long p = 0; p < d; ++p)
            v[p] = u[p] / nu;
        int done = it > 1 && fabs(lam_new - lam) <= (REAL)rel_tol * fabs(lam_new);
        lam = lam_new;
        if (done)
            break;
    }
    if (iters_out)
        *iters_out = it > max_iters ? max_iters : it;
    free(v); free(u); free(s);
    return (double)lam;
}

/* Number of positive entries of A (exact count under the definition). */
long FN(ora_nnz)(const ora_geom *g)
{
    int N = g->n_pix, V = g->n_views, B = g->n_bins;
    long cnt = 0;
    for (int v = 0; v < V; ++v) {
        FN(view) w = FN(make_view)(g, v);
        for (int b = 0; b < B; ++b) {
            REAL u = FN(bin_centre)(g, b);
            for (int k = 0; k < N; ++k) {
                REAL f = FN(crossing)(g, &w, u, k);
                REAL fl = floor(f);
                if (fl < -1 || fl > N - 1)
                    continue;
                for (int j = (int)fl; j <= (int)fl + 1; ++j)
                    if (j >= 0 && j < N && 1 - fabs(f - (REAL)j) > 0)
                        ++cnt;
            }
        }
    }
    return cnt;
}
