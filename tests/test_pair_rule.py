"""The back-projector's bin-pair rule reproduces the forward projector's
float weights exactly (CPU emulation of the device arithmetic).

The GPU gather takes, for pixel j of line k and a view with |P| >= 1, the
bins b_f = trunc(-T / P) (clamped to the padded row) and b_f + 1, where
T = f(0, k) - j in padded-bin units, with weights (float)(1 - |d|) and
(float)(|d| + 1 - |P|), d = f(b_f, k) - j.  The forward projector puts
(float)(1 - e0) on pixel floor(f) and (float)e0 on pixel floor(f) + 1 of
each line crossing f = A + b P + k Q.  With A, P, Q multiples of 2^-32
(as the geometry rounds them) both sides' double arithmetic is exact, so
the two sets of (bin, line, pixel, weight) must be identical.  numpy's
float64 operations and float32 conversion round as the device's do.
Geometries: square pixels, bins of 1 to 2 pixels, 180 and 360 degrees,
detectors narrower and wider than the image, |P| = 1 views.
"""
import math

import numpy as np
import pytest

PAD_B = 2


def fx(v):
    return round(v * 2.0 ** 32) / 2.0 ** 32


def views(N, V, B, half_turns, ratio):
    c = (N - 1) / 2.0
    half = (B - 1) / 2.0
    out = []
    for v in range(V):
        q = (half_turns * v) % V
        row = 4 * q <= V or 4 * q >= 3 * V
        th = half_turns * math.pi * v / V
        ct, st = math.cos(th), math.sin(th)
        cs, sn = (ct, st) if row else (st, ct)
        out.append((fx(c + c * sn / cs - half * ratio / cs), fx(ratio / cs), fx(-sn / cs)))
    return out


def forward_weights(N, B, A, P, Q):
    w = {}
    b = np.arange(B, dtype=np.float64)
    for k in range(N):
        f = A + b * P + k * Q                       # exact
        e0 = f - np.floor(f)
        j0 = np.floor(f).astype(np.int64)
        w0 = (1.0 - e0).astype(np.float32)
        w1 = e0.astype(np.float32)
        for bb in range(B):
            if 0 <= j0[bb] < N and w0[bb] > 0:
                w[(bb, k, int(j0[bb]))] = w0[bb]
            if 0 <= j0[bb] + 1 < N and w1[bb] > 0:
                w[(bb, k, int(j0[bb]) + 1)] = w1[bb]
    return w


def pair_rule_weights(N, B, A, P, Q):
    w = {}
    Ab = A - PAD_B * P
    inv_p = 1.0 / P
    om_p = 1.0 - abs(P)
    k, j = np.meshgrid(np.arange(N, dtype=np.float64), np.arange(N, dtype=np.float64),
                       indexing="ij")
    T = (Ab - j) + k * Q                            # exact
    t = -T * inv_p
    bf = np.clip(np.clip(np.trunc(t), -2.0 ** 31, 2.0 ** 31 - 1).astype(np.int64), 0,
                 B + 2 * PAD_B - 2)
    d = bf * P + T                                  # exact
    u0 = np.clip((1.0 - np.abs(d)).astype(np.float32), 0, 1)
    u1 = np.clip((np.abs(d) + om_p).astype(np.float32), 0, 1)
    for kk in range(N):
        for jj in range(N):
            b0 = int(bf[kk, jj]) - PAD_B
            if 0 <= b0 < B and u0[kk, jj] > 0:
                w[(b0, kk, jj)] = u0[kk, jj]
            if 0 <= b0 + 1 < B and u1[kk, jj] > 0:
                w[(b0 + 1, kk, jj)] = u1[kk, jj]
    return w


@pytest.mark.parametrize("N,V,B,half_turns,ratio", [
    (16, 12, 24, 1, 1.0),       # detector wider than the image diagonal
    (33, 17, 47, 1, 1.0),       # ragged sizes
    (20, 9, 31, 2, 1.3),        # 360 degrees, wide bins
    (24, 10, 20, 1, 1.0),       # detector narrower than the image
    (31, 7, 11, 1, 2.0),        # bins of two pixels, very narrow detector
    (40, 36, 57, 1, 1.0),       # many views, |P| = 1 at 0 and 90 degrees
])
def test_pair_rule_matches_forward_weights(N, V, B, half_turns, ratio):
    total = 0
    for (A, P, Q) in views(N, V, B, half_turns, ratio):
        wf = forward_weights(N, B, A, P, Q)
        wb = pair_rule_weights(N, B, A, P, Q)
        assert wf.keys() == wb.keys(), (P, len(set(wf) ^ set(wb)))
        assert all(wf[key] == wb[key] for key in wf), P
        total += len(wf)
    assert total > 0


def test_round_to_nearest_in_place_of_truncation_fails():
    """The check has teeth: rounding t to nearest (a plausible slip) loses or
    misplaces weights on some view."""
    N, V, B = 40, 36, 57

    def rint_rule(A, P, Q):
        w = {}
        Ab, inv_p, om_p = A - PAD_B * P, 1.0 / P, 1.0 - abs(P)
        k, j = np.meshgrid(np.arange(N, dtype=np.float64), np.arange(N, dtype=np.float64),
                           indexing="ij")
        T = (Ab - j) + k * Q
        bf = np.clip(np.rint(-T * inv_p).astype(np.int64), 0, B + 2 * PAD_B - 2)
        d = bf * P + T
        u0 = np.clip((1.0 - np.abs(d)).astype(np.float32), 0, 1)
        u1 = np.clip((np.abs(d) + om_p).astype(np.float32), 0, 1)
        for kk in range(N):
            for jj in range(N):
                b0 = int(bf[kk, jj]) - PAD_B
                if 0 <= b0 < B and u0[kk, jj] > 0:
                    w[(b0, kk, jj)] = u0[kk, jj]
                if 0 <= b0 + 1 < B and u1[kk, jj] > 0:
                    w[(b0 + 1, kk, jj)] = u1[kk, jj]
        return w

    bad = sum(forward_weights(N, B, A, P, Q) != rint_rule(A, P, Q)
              for (A, P, Q) in views(N, V, B, 1, 1.0))
    assert bad > 0


def covers(N, B, vs):
    """The geometry's coverage test: t at the image's corners within
    [-1/2, B + 2 PAD_B - 3/2] for every view."""
    for (A, P, Q) in vs:
        Ab = A - PAD_B * P
        for j in (0, N - 1):
            for k in (0, N - 1):
                t = -((Ab - j) + k * Q) / P
                if not (-0.5 <= t <= B + 2 * PAD_B - 1.5):
                    return False
    return True


@pytest.mark.parametrize("N,V,B,half_turns,ratio,expect", [
    (16, 12, 24, 1, 1.0, True),
    (64, 45, 91, 1, 1.0, True),        # bins_for(64): the test workloads' detector
    (512, 180, 725, 1, 1.0, True),     # the benchmark geometry
    (24, 10, 20, 1, 1.0, False),       # detector narrower than the image
    (31, 7, 11, 1, 2.0, False),
])
def test_clamp_free_pairs_stay_in_the_row(N, V, B, half_turns, ratio, expect):
    """Where the coverage test passes, every pixel's first bin trunc(t) and
    its neighbour lie in the padded row without clamping, so the gather may
    skip the clamp."""
    vs = views(N, V, B, half_turns, ratio)
    assert covers(N, B, vs) == expect
    if not expect:
        return
    k, j = np.meshgrid(np.arange(N, dtype=np.float64), np.arange(N, dtype=np.float64),
                       indexing="ij")
    for (A, P, Q) in vs:
        T = ((A - PAD_B * P) - j) + k * Q
        bf = np.trunc(-T * (1.0 / P))
        assert bf.min() >= 0 and bf.max() + 1 <= B + 2 * PAD_B - 1


def test_forward_lower_weight_from_the_32_bit_negate():
    """The forward projector forms the lower tap's weight times 2^32, the
    float of 2^32 - w for the crossing's low word w, as the 32-bit negate -w
    converted once (and 2^32 itself for w = 0).  For w > 0 the negate is the
    exact value, so its correctly rounded conversion is the weight: checked
    here against the definition (the exact value in double, rounded once) on
    the ends of the range, on every low word whose value sits at or next to
    a float rounding tie, and on random words."""
    rng = np.random.default_rng(5)
    edge = [0, 1, 2, 3, 2 ** 24 - 1, 2 ** 24, 2 ** 24 + 1, 2 ** 31 - 1, 2 ** 31, 2 ** 31 + 1,
            2 ** 32 - 2, 2 ** 32 - 1]
    ties = []
    for e in range(24, 33):                 # 2^32 - w in [2^(e-1), 2^e): ulp 2^(e-24)
        ulp = 2 ** (e - 24)
        m = rng.integers(2 ** 23, 2 ** 24, size=2000, dtype=np.int64)
        for off in (-1, 0, 1):
            v = m * ulp + ulp // 2 + off    # at and next to a tie
            v = v[(v >= 1) & (v <= 2 ** 32)]
            ties.append(2 ** 32 - v)
    w = np.concatenate([np.array(edge, dtype=np.int64)] + ties +
                       [rng.integers(0, 2 ** 32, size=1 << 20, dtype=np.int64)]).astype(np.uint32)
    want = (4294967296.0 - w.astype(np.float64)).astype(np.float32)
    neg = (np.uint32(0) - w).astype(np.uint32)
    got = np.where(w > 0, neg.astype(np.float32), np.float32(4294967296.0))
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    # a plausible slip, rounding the low word before subtracting, is caught
    slip = np.float32(4294967296.0) - w.astype(np.float32)
    assert not np.array_equal(slip.view(np.uint32), want.view(np.uint32))
