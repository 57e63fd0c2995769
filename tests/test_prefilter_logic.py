"""The candidate prefilter's decision rule, emulated in FP64 on the CPU and
checked against the exact box test on adversarial inputs.

The search kernel stores each master box bound x as the largest level q with
B(q) = qo + q qu <= x (qu a power of two, q < 2^21) and decides a candidate
test from the levels when they separate the values, running the exact FP64
test otherwise.  This module restates that rule in numpy (the same FP64
operations: a product by a power of two is exact, one rounded addition) and
asserts, for every axis and every decision, that a decided test agrees with
the exact comparison -- with bounds placed exactly on levels, one ulp to
either side, between levels, far outside the grid and non-finite.  The GPU
parity tests check the kernel's candidate lists against the oracle; this
checks the rule itself where those workloads rarely go."""

import math

import numpy as np

QBITS = 21
QMAX = (1 << QBITS) - 1


def level(qo, qu, q):
    return qo + float(q) * qu


def q_max_le_bisect(qo, qu, x, strict):
    """max{q in [0, QMAX + 1] : B(q) <= x (< x when strict)}, -1 if none,
    by bisection alone (B is non-decreasing in q)."""
    ok = (lambda b: b < x) if strict else (lambda b: b <= x)
    lo, hi = -1, QMAX + 2
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if ok(level(qo, qu, mid)):
            lo = mid
        else:
            hi = mid
    return lo


def q_max_le(qo, qu, x, strict):
    """The same maximum the way the kernel finds it: a guess from one
    division, up to four unit steps, bisection if those do not settle."""
    ok = (lambda q: level(qo, qu, q) < x) if strict else (lambda q: level(qo, qu, q) <= x)
    f = math.floor((x - qo) / qu)
    q = int(min(max(f, -1.0), float(QMAX + 1)))
    for _ in range(4):
        if q >= 0 and not ok(q):
            q -= 1
        elif q <= QMAX and ok(q + 1):
            q += 1
        else:
            return q
    return q_max_le_bisect(qo, qu, x, strict)


def grid_levels(lo, length):
    e = math.frexp(2.0 * length / QMAX)[1]
    return lo, math.ldexp(1.0, e)


def master_record(qo, qu, mlo, mhi):
    """(ql, qh, exact_only) as the kernel stores them."""
    exact = False
    out = []
    for x in (mlo, mhi):
        q = q_max_le(qo, qu, x, False) if math.isfinite(x) else -1
        if q < 0 or q > QMAX:
            exact, q = True, 0
        out.append(q)
    return out[0], out[1], exact


def slave_thresholds(qo, qu, slo, shi, delta):
    a, c = slo - delta, shi + delta
    if math.isfinite(a) and math.isfinite(c):
        la = q_max_le(qo, qu, a, True)
        ea = q_max_le(qo, qu, a, False)
        ec = q_max_le(qo, qu, c, False)
        return la, ea, ec, ec
    return QMAX + 1, -1, -1, QMAX + 1


def decide(th, rec):
    """'fail', 'pass' or None (exact test) for one axis."""
    la, ea, ecp, ecf = th
    ql, qh, exact = rec
    if exact:
        return None
    if qh < ea or ql > ecf:
        return "fail"
    if qh > la and ql < ecp:
        return "pass"
    return None


def exact_axis(slo, shi, mlo, mhi, delta):
    return (slo - delta) <= mhi and mlo <= (shi + delta)


def adversarial_values(qo, qu, rng, n):
    """Values on levels, one ulp around them, between levels, outside."""
    qs = rng.integers(0, QMAX + 1, n)
    base = np.array([level(qo, qu, int(q)) for q in qs])
    kind = rng.integers(0, 5, n)
    vals = base.copy()
    vals[kind == 1] = np.nextafter(base[kind == 1], np.inf)
    vals[kind == 2] = np.nextafter(base[kind == 2], -np.inf)
    vals[kind == 3] = base[kind == 3] + rng.uniform(0, qu, (kind == 3).sum())
    vals[kind == 4] = qo + rng.uniform(-0.5, 2.5, (kind == 4).sum()) * QMAX * qu
    return vals


def run_axis_checks(qo, qu, delta, seed, n=4000):
    rng = np.random.default_rng(seed)
    lo_s = adversarial_values(qo, qu, rng, n)
    hi_s = lo_s + rng.choice([0.0, qu, 17.3 * qu, rng.uniform(0, 500 * qu)], n)
    lo_m = adversarial_values(qo, qu, rng, n)
    hi_m = lo_m + rng.choice([0.0, qu, 3 * qu, rng.uniform(0, 500 * qu)], n)
    decided = undecided = 0
    for k in range(n):
        a, c = lo_s[k] - delta, hi_s[k] + delta
        # also master bounds at the slave's enlarged bounds and one ulp past them
        for mlo, mhi in ((lo_m[k], hi_m[k]), (c, c + qu), (a - qu, a),
                         (np.nextafter(c, np.inf), c + qu), (a - qu, np.nextafter(a, -np.inf))):
            th = slave_thresholds(qo, qu, lo_s[k], hi_s[k], delta)
            rec = master_record(qo, qu, mlo, mhi)
            d = decide(th, rec)
            ex = exact_axis(lo_s[k], hi_s[k], mlo, mhi, delta)
            if d is None:
                undecided += 1
            else:
                decided += 1
                assert (d == "pass") == ex, (qo, qu, lo_s[k], hi_s[k], mlo, mhi, delta, d)
    return decided, undecided


def test_levels_are_monotone_and_exact_products():
    qo, qu = grid_levels(-0.3751, 1.8)
    prev = -math.inf
    for q in list(range(0, 50)) + list(range(QMAX - 50, QMAX + 2)):
        b = level(qo, qu, q)
        assert b >= prev
        prev = b
        assert float(q) * qu == math.ldexp(float(q), math.frexp(qu)[1] - 1)  # exact product
    assert level(qo, qu, QMAX) >= qo + 2 * 1.8


def test_master_bounds_bracketed_by_levels():
    qo, qu = grid_levels(0.0, 1.0)
    rng = np.random.default_rng(1)
    for x in adversarial_values(qo, qu, rng, 2000):
        if not (qo <= x <= qo + 1.0):
            continue
        q = q_max_le(qo, qu, x, False)
        assert 0 <= q <= QMAX
        assert level(qo, qu, q) <= x < level(qo, qu, q + 1)


def test_guess_and_steps_equal_bisection():
    for lo, length in ((0.0, 1.0), (1.0e6 + 0.37, 3.0), (-2.5e-4, 7e-4)):
        qo, qu = grid_levels(lo, length)
        rng = np.random.default_rng(7)
        for x in adversarial_values(qo, qu, rng, 1500):
            for strict in (False, True):
                assert q_max_le(qo, qu, x, strict) == q_max_le_bisect(qo, qu, x, strict), (lo, x, strict)


def test_decisions_agree_with_the_exact_test_unit_grid():
    decided, undecided = run_axis_checks(*grid_levels(0.0, 1.0), delta=1.25e-3, seed=2)
    assert decided > 0 and undecided > 0  # both branches exercised


def test_levels_decide_plain_boxes():
    # boxes at element scale on a grid a few hundred elements wide: the
    # levels (2^21 per axis) decide nearly every test without the exact one
    qo, qu = grid_levels(-0.05, 1.1)
    rng = np.random.default_rng(8)
    decided = 0
    n = 3000
    for _ in range(n):
        c_s, c_m = rng.uniform(0.0, 1.0, 2)
        h_s, h_m = rng.uniform(1e-3, 4e-3, 2)
        th = slave_thresholds(qo, qu, c_s - h_s, c_s + h_s, 1e-4)
        rec = master_record(qo, qu, c_m - h_m, c_m + h_m)
        d = decide(th, rec)
        if d is not None:
            decided += 1
            assert (d == "pass") == exact_axis(c_s - h_s, c_s + h_s, c_m - h_m, c_m + h_m, 1e-4)
    assert decided >= 0.999 * n


def test_decisions_agree_with_the_exact_test_offset_grids():
    # a grid far from the origin (levels not exactly representable sums),
    # a tiny grid, and zero delta
    for (lo, length, delta, seed) in ((1.0e6 + 0.37, 3.0, 1e-4, 3), (-2.5e-4, 7e-4, 1e-9, 4), (5.0, 2.0, 0.0, 5)):
        run_axis_checks(*grid_levels(lo, length), delta=delta, seed=seed, n=1500)


def test_three_axis_record_rule():
    """The whole-record rule: fail if any axis fails, pass if every axis
    passes and the record is not flagged exact, otherwise the exact test;
    checked against the exact three-axis box test."""
    qo, qu = grid_levels(0.0, 1.0)
    rng = np.random.default_rng(9)
    delta = 2e-3
    for _ in range(3000):
        slo = adversarial_values(qo, qu, rng, 3)
        shi = slo + rng.uniform(0, 40 * qu, 3)
        mlo = np.where(rng.random(3) < 0.5, adversarial_values(qo, qu, rng, 3), shi + delta)
        mhi = mlo + rng.uniform(0, 40 * qu, 3)
        if rng.random() < 0.05:
            mhi[rng.integers(0, 3)] = math.inf
        recs = [master_record(qo, qu, mlo[d], mhi[d]) for d in range(3)]
        flagged = any(r[2] for r in recs)
        ths = [slave_thresholds(qo, qu, slo[d], shi[d], delta) for d in range(3)]
        fail = pass_ = False
        if not flagged:
            ds = [decide(ths[d], recs[d]) for d in range(3)]
            fail = any(d == "fail" for d in ds)
            pass_ = all(d == "pass" for d in ds)
        exact = all(exact_axis(slo[d], shi[d], mlo[d], mhi[d], delta) for d in range(3))
        if fail:
            assert not exact
        elif pass_:
            assert exact


def test_non_finite_values_go_to_the_exact_test():
    qo, qu = grid_levels(0.0, 1.0)
    for slo, shi in ((math.nan, 0.5), (0.1, math.inf), (-math.inf, 0.2)):
        th = slave_thresholds(qo, qu, slo, shi, 1e-3)
        assert decide(th, master_record(qo, qu, 0.2, 0.3)) is None
    for mlo, mhi in ((math.nan, 0.3), (0.2, math.inf)):
        th = slave_thresholds(qo, qu, 0.1, 0.4, 1e-3)
        assert decide(th, master_record(qo, qu, mlo, mhi)) is None
