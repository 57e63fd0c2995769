"""Pins of the oracle's contact search (brute force and binning, Alg. 2)."""

from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth


def rational_interval_overlaps(ns, nm):
    # closed-interval overlaps of [i/ns, (i+1)/ns] and [j/nm, (j+1)/nm]
    c = 0
    for i in range(ns):
        for j in range(nm):
            if Fraction(i, ns) <= Fraction(j + 1, nm) and Fraction(j, nm) <= Fraction(i + 1, ns):
                c += 1
    return c


def test_unjittered_flat_count_closed_form():
    itf = synth.flat_tied(8, 7, jitter=0.0)
    cs, cm = oracle.search(itf.slave, itf.master, 0.0, "brute")
    k = rational_interval_overlaps(8, 7)
    assert k == 8 + 7 - 1
    assert cs.size == k * k
    # and every candidate of this grid has a positive-area overlap
    r = oracle.evaluate(itf)
    assert r["pair_s"].size == (8 + 7 - 1) ** 2


def random_surface_mesh(rng, n, shift, warp):
    s, t, conn, _ = synth.tensor_grid(n, n)
    X = np.stack([s, t, warp * np.sin(3 * s + 2 * t)], 1)
    X[:, :2] += rng.uniform(-0.15 / n, 0.15 / n, (X.shape[0], 2))
    X += shift
    return synth.Mesh(X, conn)


@pytest.mark.parametrize("seed", range(6))
def test_binned_equals_brute(seed):
    rng = np.random.default_rng(seed)
    ns, nm = rng.integers(3, 13, 2)
    S = random_surface_mesh(rng, int(ns), 0.0, 0.05)
    M = random_surface_mesh(rng, int(nm), rng.uniform(-0.2, 0.2, 3) * [1, 1, 0.01], 0.05)
    delta = float(rng.choice([0.0, 1e-3, 0.05]))
    a = oracle.search(S, M, delta, "brute")
    b = oracle.search(S, M, delta, "binned")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    # sorted by (s, m)
    key = a[0].astype(np.int64) * (M.n_el + 1) + a[1]
    assert np.all(np.diff(key) > 0)


def test_brute_force_matches_independent_loop():
    rng = np.random.default_rng(11)
    S = random_surface_mesh(rng, 4, 0.0, 0.1)
    M = random_surface_mesh(rng, 5, np.array([0.1, -0.05, 0.02]), 0.1)
    delta = 0.01
    got = set(zip(*oracle.search(S, M, delta, "brute")))
    exp = set()
    for s in range(S.n_el):
        xs = S.X[S.conn[s]]
        for m in range(M.n_el):
            xm = M.X[M.conn[m]]
            ok = all(xs[:, d].min() - delta <= xm[:, d].max() and xm[:, d].min() <= xs[:, d].max() + delta
                     for d in range(3))
            if ok:
                exp.add((s, m))
    assert got == exp


@pytest.mark.parametrize("seed", range(3))
def test_search_misses_no_overlapping_pair(seed):
    # Every (slave, master) pair with a positive-area clip, found by clipping
    # all pairs, is a candidate of the search.
    rng = np.random.default_rng(100 + seed)
    S = random_surface_mesh(rng, 5, 0.0, 0.0)
    M = random_surface_mesh(rng, 6, np.array([0.05, 0.02, 5e-4]), 0.0)
    delta = 1e-3
    alls = np.repeat(np.arange(S.n_el, dtype=np.int32), M.n_el)
    allm = np.tile(np.arange(M.n_el, dtype=np.int32), S.n_el)
    nv, _, _ = oracle.eval_candidates(S, M, oracle.params(delta=delta), alls, allm, integrate=False)
    overlapping = set(zip(alls[nv >= 3], allm[nv >= 3]))
    cands = set(zip(*oracle.search(S, M, delta, "binned")))
    assert overlapping and overlapping <= cands


def test_cylinder_reduced_binned_equals_brute():
    itf = synth.cylinder(24, 19, seed=7)
    a = oracle.search(itf.slave, itf.master, itf.delta, "brute")
    b = oracle.search(itf.slave, itf.master, itf.delta, "binned")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
