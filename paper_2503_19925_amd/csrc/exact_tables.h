// Host-side tables of the forward projector: per (view slot, block of
// kFwdRays bins) the image lines its rays reach, and the dispatch order of
// its workgroups.  Host code only (no device code), included by the C-ABI
// implementation and by a CPU test harness.
#pragma once

#include "exact_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

namespace exact {

// First and last image line that any ray of each block of kFwdRays bins
// reaches, per table slot (the forward projector splits these lines among
// its waves).  Ray b of a view crosses line k at f = A + b P + k Q and has
// a tap inside the image iff floor(f) is in [-1, N - 1], i.e. f in [-1, N);
// the line interval of one ray is taken one line wider on each side.  The
// interval's ends are affine in b, so over a block they are extreme at its
// first or last ray; the union of the rays' intervals lies within the hull
// of those two.  A block no ray of which reaches a line gets first > last.
inline std::vector<int32_t> block_lines(const std::vector<ViewGeom> &views, int N, int B)
{
    const int R = exact::kFwdRays, nbb = (B + R - 1) / R;
    std::vector<int32_t> out(2 * views.size() * (size_t)nbb);
    for (size_t slot = 0; slot < views.size(); ++slot) {
        const ViewGeom &G = views[slot];
        for (int bb = 0; bb < nbb; ++bb) {
            const long double ends[2] = {(long double)R * bb,
                                         (long double)std::min(R * bb + R - 1, B - 1)};
            long double lo = 1e30L, hi = -1e30L;
            if (G.Q != 0.0) {
                for (long double b : ends) {
                    const long double base = (long double)G.A + b * (long double)G.P;
                    const long double ka = (-1.0L - base) / G.Q, kb = ((long double)N - base) / G.Q;
                    lo = std::min(lo, floorl(std::min(ka, kb)) - 1.0L);
                    hi = std::max(hi, ceill(std::max(ka, kb)) + 1.0L);
                }
            } else {
                // every line or none: some ray's f in [-1, N) (one pixel wider)
                const long double f0 = (long double)G.A + ends[0] * (long double)G.P;
                const long double f1 = (long double)G.A + ends[1] * (long double)G.P;
                if (std::max(f0, f1) >= -2.0L && std::min(f0, f1) < (long double)N + 1.0L) {
                    lo = 0.0L;
                    hi = N - 1;
                }
            }
            lo = std::max(lo, 0.0L);
            hi = std::min(hi, (long double)(N - 1));
            const size_t i = 2 * (slot * nbb + bb);
            out[i] = lo <= hi ? (int32_t)lo : N;
            out[i + 1] = lo <= hi ? (int32_t)hi : -1;
        }
    }
    return out;
}

// Lines a forward workgroup walks for block i (slot nbb + block) of a
// geometry's block table.
inline long block_weight(const std::vector<int32_t> &blk, size_t i)
{
    return std::max(0, blk[2 * i + 1] - blk[2 * i] + 1);
}

// Dispatch order of the forward projector's workgroups, one per item of
// weight w[i] (the lines it walks).  The hardware hands workgroups to the
// XCDs in turn and fills each CU with `per_cu` of them at once, so
// workgroups i and i + cus * k share a CU in the first round.  Longest
// items first; the first min(n, cus * per_cu) go to the CUs' slots greedily
// (each to the CU with the fewest lines so far among those with a free
// slot: slot k of CU c is workgroup c + cus * k, which must exist), so that
// every CU's first round holds about the same number of lines; the rest
// follow, longest first, into slots as they free.  Returns the item of each
// workgroup.  The order changes which workgroup projects which rays, never
// the arithmetic.
inline std::vector<int32_t> balanced_order(const std::vector<long> &w, int cus, int per_cu)
{
    const int n = (int)w.size();
    std::vector<int32_t> idx((size_t)n), order((size_t)n);
    for (int i = 0; i < n; ++i)
        idx[(size_t)i] = i;
    std::stable_sort(idx.begin(), idx.end(),
                     [&](int32_t a, int32_t b) { return w[(size_t)a] > w[(size_t)b]; });
    if (cus < 1 || per_cu < 1)
        return idx;
    const long first = std::min((long)cus * per_cu, (long)n);
    std::vector<long> load((size_t)cus, 0);
    std::vector<int> used((size_t)cus, 0);
    for (long r = 0; r < first; ++r) {
        int best = -1;
        for (int c = 0; c < cus; ++c)
            if (c + (long)cus * used[(size_t)c] < first &&
                (best < 0 || load[(size_t)c] < load[(size_t)best]))
                best = c;
        order[(size_t)best + (size_t)cus * used[(size_t)best]] = idx[(size_t)r];
        load[(size_t)best] += w[(size_t)idx[(size_t)r]];
        ++used[(size_t)best];
    }
    for (long r = first; r < n; ++r)
        order[(size_t)r] = idx[(size_t)r];
    return order;
}

}  // namespace exact
