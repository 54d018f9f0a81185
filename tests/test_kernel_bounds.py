"""Host checks of the rules three kernel shortcuts rest on, with IEEE FP32
arithmetic emulated in numpy where it matters (float32 operations round to
nearest even as the GPU's do; a fused multiply-add is formed exactly in
float64 and rounded once).  No test runs GPU code: they check that the
derivations in the kernel sources accept no wrong result, on random and on
adversarial inputs (values placed next to the rounding boundaries, many
equal values).

1. The nearest-pixel shortcut of the voxel pass: with tq = fl(a r) for an
   approximate reciprocal r of z, yq = fl(tq + c), the convention's
   coordinate floor(fl(fl(fl(a / z) + c) + 1/2)) equals rint(yq) whenever
   |yq - rint(yq)| < fma(|tq|, -2^-20, kin), kin = fl(1/2 - (2 + |c|) 2^-21).
2. The RGBA8 channel shortcut of the voxel pass's update: the FP32 estimate
   y' = fl(fl(c swq + fl(C Wq)) fl(1/M)) rounded to the nearest integer is
   the exact round-half-even of (C Wq + c swq) / M, clamped to [0, 255],
   whenever |y' - rint(y')| + fma(|y'|, 2^-22, E0) <= 1/2,
   E0 = fma(fl(Wq fl(1/M)), 255 2^-22, 2^-22).
3. The colour median's per-observation test: the observation whose
   strictly-before weight is below half the total and reaches half with its
   own is the one lower weighted median.
"""
import numpy as np

F32 = np.float32


def f32(x):
    return np.asarray(x, dtype=np.float64).astype(F32)


def fma32(a, b, c):
    """fl32(a b + c) with one rounding (exact in float64 for these sizes)."""
    return f32(np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64))


def _pixel_case(a, z, c, rulp):
    """Accepted lanes of the rint test and whether each equals the
    convention; r is the correctly rounded reciprocal moved by rulp ulps."""
    r = F32(1.0) / z
    if rulp:
        r = np.nextafter(r, np.where(rulp > 0, np.inf, -np.inf).astype(F32)).astype(F32)
    tq = a * r
    yq = tq + c
    fl = np.rint(yq)
    kin = f32(0.5 - (2.0 + np.abs(c.astype(np.float64))) * 2.0 ** -21)
    inner = fma32(np.abs(tq), -(2.0 ** -20), kin)
    acc = np.abs(yq - fl) < inner
    t = a / z  # IEEE single division: correctly rounded
    conv = np.floor((t + c) + F32(0.5))
    return acc, fl == conv


def test_pixel_rint_test_accepts_no_wrong_coordinate():
    rng = np.random.default_rng(11)
    n = 400_000
    for c0 in (319.5, 159.5, 0.0, 711.25):
        z = f32(rng.uniform(0.05, 20.0, n))
        c = np.full(n, F32(c0))
        # random coordinates, then coordinates placed near a half-integer
        # (the rounding boundary of the convention): within 4e-3 px, about
        # the test's margin, and within 2e-5 px, far inside it
        half = np.floor(rng.uniform(-20.0, 700.0, n)) + 0.5
        targets = [rng.uniform(-50.0, 700.0, n), half + rng.uniform(-4e-3, 4e-3, n),
                   half + rng.uniform(-2e-5, 2e-5, n)]
        for ti, tgt in enumerate(targets):
            a = f32((tgt - c0) * z.astype(np.float64))
            for rulp in (0, 1, -1):
                acc, good = _pixel_case(a, z, c, rulp)
                assert good[acc].all(), f"c={c0} rulp={rulp}: accepted wrong coordinate"
                if ti < 2:
                    assert acc.any()
        # random data: the shortcut decides almost every lane
        acc, _ = _pixel_case(f32((targets[0] - c0) * z.astype(np.float64)), z, c, 1)
        assert acc.mean() > 0.99


def _exact_channel(C, c, Wq, swq):
    """Round half to even of (C Wq + c swq) / M, clamped to [0, 255]."""
    N = C * Wq + c * swq
    M = Wq + swq
    q = np.floor_divide(N, M)
    rem = N - q * M
    up = (2 * rem > M) | ((2 * rem == M) & (q % 2 == 1))
    return np.clip(q + up, 0, 255)


def _fast_channel(C, c, Wq, swq):
    """(accepted, value) of the FP32 estimate with its error test."""
    M = (Wq + swq).astype(np.float64)
    rMf = f32(1.0 / M)
    Wq32, swq32 = f32(Wq), f32(swq)
    E0 = fma32(Wq32 * rMf, 255.0 * 2.0 ** -22, 2.0 ** -22)
    P1 = f32(C) * Wq32
    Nf = fma32(f32(c), swq32, P1)
    y = Nf * rMf
    q = np.rint(y)
    ok = (np.abs(y - q) + fma32(np.abs(y), 2.0 ** -22, E0)) <= F32(0.5)
    return ok, np.clip(q, 0, 255).astype(np.int64)


def _weights(rng, n, lo_exp, hi_exp):
    """Multiples of 2^-10 spread over [2^lo, 2^hi) (as integers Wq)."""
    e = rng.uniform(lo_exp, hi_exp, n)
    return np.maximum(np.floor(2.0 ** e * 1024.0), 1).astype(np.int64)


def test_colour_estimate_accepts_no_wrong_byte():
    rng = np.random.default_rng(5)
    n = 400_000
    lim = 16384 * 1024
    cases = []
    # integration: W in [0, 2^14), w > 0, W + w < 2^14
    W = _weights(rng, n, -10, 13.9)
    w = _weights(rng, n, -10, 13.9)
    keep = W + w < lim
    cases.append((W[keep], w[keep]))
    # de-integration that removes most of the weight (large C Wq / M)
    W = _weights(rng, n, 0, 13.9)
    frac = rng.uniform(0.0, 1.0, n) ** 8
    w = np.maximum(np.floor(W * (1.0 - frac)), 1).astype(np.int64)
    keep = W - w > 0
    cases.append((W[keep], -w[keep]))
    # equal weights: every odd C + c is an exact tie
    W = _weights(rng, n, -10, 12.9)
    cases.append((W, W.copy()))
    for Wq, swq in cases:
        C = rng.integers(0, 256, len(Wq)).astype(np.int64)
        c = rng.integers(0, 256, len(Wq)).astype(np.int64)
        exact = _exact_channel(C, c, Wq, swq)
        ok, fast = _fast_channel(C, c, Wq, swq)
        assert (fast[ok] == exact[ok]).all(), "the estimate accepted a wrong byte"
    # ties are never accepted; random integrations almost always are
    Wq, swq = cases[2]
    C = rng.integers(0, 128, len(Wq)).astype(np.int64) * 2
    c = C + 1
    ok, _ = _fast_channel(C, c, Wq, swq)
    assert not ok.any()
    Wq, swq = cases[0]
    C = rng.integers(0, 256, len(Wq)).astype(np.int64)
    c = rng.integers(0, 256, len(Wq)).astype(np.int64)
    ok, _ = _fast_channel(C, c, Wq, swq)
    assert ok.mean() > 0.99


def test_median_rule_picks_exactly_the_lower_weighted_median():
    """The colour median's per-observation rule: with the valid observations
    ordered by (value, frame), observation j passes when the weight ordered
    strictly before it is below half the total and that weight plus its own
    reaches half.  Exactly one passes, and it is the lower weighted median
    (the first in that order whose cumulative weight reaches half), on random
    cases with many equal values, missing frames (weight 0) and weights on
    the 2^-20 grid up to 2^31."""
    rng = np.random.default_rng(17)
    for trial in range(20000):
        m = int(rng.integers(1, 65))
        c = rng.integers(0, 4 if trial % 2 else 65281, m).astype(np.float64)
        w = rng.integers(1, 2 ** (int(rng.integers(1, 32))), m, dtype=np.int64)
        w[rng.random(m) < 0.2] = 0
        if not (w > 0).any():
            continue
        total = int(w.sum())
        idx = [j for j in range(m) if w[j] > 0]
        # brute force: sorted by (value, frame), first cumulative >= half
        srt = sorted(idx, key=lambda j: (c[j], j))
        cum, brute = 0, None
        for j in srt:
            cum += int(w[j])
            if 2 * cum >= total:
                brute = c[j]
                break
        passed = []
        for j in idx:
            below = sum(int(w[l]) for l in idx if c[l] < c[j] or (c[l] == c[j] and l < j))
            if 2 * below < total <= 2 * (below + int(w[j])):
                passed.append(j)
        assert len(passed) == 1, (trial, passed)
        assert c[passed[0]] == brute
