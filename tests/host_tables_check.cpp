// CPU check of the forward projector's host tables against brute force
// (built and run by test_host_tables.py; host code only, no GPU call).
//
// block_lines: on random parallel-beam geometries (crossing parameters A,
// P, Q on the 2^-32 grid, as the geometry table holds them, including
// Q = 0 and |Q| = 1 views), every (ray, line) where the ray puts a positive
// tap weight on a pixel of the image must lie inside the line range of the
// ray's block.  A ray's taps on line k are columns floor(f) and floor(f) + 1
// with weights 1 - e and e, f = A + b P + k Q, e = f - floor(f); f is exact
// in long double here.
//
// balanced_order: for random weights, CU counts and slots per CU, the
// dispatch order is a permutation of the items.
#include "exact_tables.h"

#include <cstdio>
#include <random>

using exact::ViewGeom;

namespace {

long double on_grid(long double v) { return roundl(ldexpl(v, 32)) / 4294967296.0L; }

// One view with stepping-axis cosine cs and sine sn (|cs| >= |sn| by the
// caller's choice of axis), bins `ratio` pixels wide.
ViewGeom view(int N, int B, long double cs, long double sn, long double ratio)
{
    const long double c = (N - 1) / 2.0L, half = (B - 1) / 2.0L;
    ViewGeom G{};
    G.P = (double)on_grid(ratio / cs);
    G.Q = (double)on_grid(-sn / cs);
    G.A = (double)on_grid(c + c * sn / cs - half * ratio / cs);
    return G;
}

int check_lines(int N, int B, const std::vector<ViewGeom> &views, long *taps)
{
    const std::vector<int32_t> blk = exact::block_lines(views, N, B);
    const int R = exact::kFwdRays, nbb = (B + R - 1) / R;
    if (blk.size() != 2 * views.size() * (size_t)nbb)
        return 1;
    for (size_t s = 0; s < views.size(); ++s) {
        const ViewGeom &G = views[s];
        for (int b = 0; b < B; ++b) {
            const int32_t first = blk[2 * (s * nbb + b / R)], last = blk[2 * (s * nbb + b / R) + 1];
            for (int k = 0; k < N; ++k) {
                const long double f = (long double)G.A + (long double)b * G.P + (long double)k * G.Q;
                const long double c = floorl(f), e = f - c;
                const bool t0 = c >= 0 && c <= N - 1 && e < 1;
                const bool t1 = c + 1 >= 0 && c + 1 <= N - 1 && e > 0;
                if (!(t0 || t1))
                    continue;
                ++*taps;
                if (k < first || k > last) {
                    std::printf("MISS N=%d B=%d slot=%zu ray=%d line=%d range=[%d,%d] A=%.17g P=%.17g "
                                "Q=%.17g\n", N, B, s, b, k, first, last, G.A, G.P, G.Q);
                    return 1;
                }
            }
        }
    }
    return 0;
}

}  // namespace

int main()
{
    std::mt19937_64 rng(20260403);
    std::uniform_real_distribution<double> u01(0.0, 1.0);
    const long double pi = 3.14159265358979323846264338327950288L;
    long taps = 0;
    int geoms = 0;
    for (int trial = 0; trial < 400; ++trial) {
        const int N = trial < 8 ? 1 + trial : 1 + (int)(rng() % 96);
        const int B = 1 + (int)(rng() % 420);
        const long double ratio = 0.3L + 2.4L * (long double)u01(rng);
        const int V = 1 + (int)(rng() % 9);
        std::vector<ViewGeom> views;
        for (int v = 0; v < V; ++v) {
            long double th;
            const int kind = (int)(rng() % 6);
            if (kind == 0)
                th = 0.0L;                         // Q = 0
            else if (kind == 1)
                th = pi / 4;                       // |Q| = 1
            else
                th = pi * (long double)u01(rng);
            const long double ct = cosl(th), st = sinl(th);
            const bool row = fabsl(ct) >= fabsl(st);
            views.push_back(view(N, B, row ? ct : st, row ? st : ct, ratio));
        }
        if (check_lines(N, B, views, &taps))
            return 1;
        ++geoms;
    }
    // two workload-sized views
    {
        const int N = 512, B = 725;
        std::vector<ViewGeom> views = {view(N, B, cosl(0.3L), sinl(0.3L), 1.0L),
                                       view(N, B, cosl(pi / 4), sinl(pi / 4), 1.0L)};
        if (check_lines(N, B, views, &taps))
            return 1;
        ++geoms;
    }
    int orders = 0;
    for (int trial = 0; trial < 3000; ++trial) {
        const int n = (int)(rng() % 5000), cus = 1 + (int)(rng() % 300),
                  per = 1 + (int)(rng() % 9);
        std::vector<long> w((size_t)n);
        for (long &x : w)
            x = (long)(rng() % 700);
        const std::vector<int32_t> o = exact::balanced_order(w, cus, per);
        std::vector<char> seen((size_t)n, 0);
        if (o.size() != (size_t)n)
            return 1;
        for (int32_t i : o) {
            if (i < 0 || i >= n || seen[(size_t)i]++) {
                std::printf("NOT A PERMUTATION n=%d cus=%d per_cu=%d\n", n, cus, per);
                return 1;
            }
        }
        ++orders;
    }
    std::printf("OK %d geometries, %ld taps inside their block ranges; %d orders are permutations\n",
                geoms, taps, orders);
    return 0;
}
