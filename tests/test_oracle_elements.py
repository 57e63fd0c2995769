"""Pins of the oracle's element-based integration (the alternative to the
segments of Alg. 1: a Gauss product rule on the whole slave element, each
point assigned to the master element it projects into).

Pinned against: the Gauss-Legendre rule's closed forms and numpy's
independent rule; coincident meshes (where every point lies inside one
master and the element-based values are exact, so they equal the pinned
segment-based values); the exact slave area under full coverage; the
partition of unity of the master shape functions (row sums of M equal those
of D per pair); a constant normal offset (gap = offset x row sums of D); the
biorthogonality of the dual basis; and convergence to the segment-based
values as the rule grows.
"""

import copy

import numpy as np
import pytest

import oracle
import synth


def rel(a, b):
    a = np.asarray(a.todense() if hasattr(a, "todense") else a).ravel()
    b = np.asarray(b.todense() if hasattr(b, "todense") else b).ravel()
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_gauss_legendre_closed_forms_and_library_rule():
    x, w = oracle.gauss_legendre(1)
    assert x[0] == 0.0 and w[0] == 2.0
    x, w = oracle.gauss_legendre(2)
    np.testing.assert_allclose(x, [-1 / np.sqrt(3), 1 / np.sqrt(3)], rtol=0, atol=3e-16)
    np.testing.assert_allclose(w, [1.0, 1.0], rtol=0, atol=1e-15)
    x, w = oracle.gauss_legendre(3)
    np.testing.assert_allclose(x, [-np.sqrt(0.6), 0.0, np.sqrt(0.6)], rtol=0, atol=3e-16)
    np.testing.assert_allclose(w, [5 / 9, 8 / 9, 5 / 9], rtol=0, atol=1e-15)
    for n in range(1, 9):
        x, w = oracle.gauss_legendre(n)
        xr, wr = np.polynomial.legendre.leggauss(n)
        np.testing.assert_allclose(x, xr, rtol=0, atol=3e-16)
        np.testing.assert_allclose(w, wr, rtol=0, atol=2e-15)
        for k in range(2 * n):
            exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
            assert abs(np.sum(w * x ** k) - exact) <= 1e-14


def coincident(n, jitter=0.0, dz=0.0, seed=1000):
    itf = synth.flat_tied(n, n, seed=seed, jitter=jitter)
    itf.master = copy.deepcopy(itf.slave)
    itf.master.X[:, 2] += dz
    return itf


@pytest.mark.parametrize("ng", [2, 3, 5])
def test_coincident_meshes_equal_segment_based(ng):
    # every Gauss point lies strictly inside the coincident master, and on
    # rectangles the integrands are polynomials the rules integrate exactly
    itf = coincident(6)
    prm = oracle.params(delta=itf.delta)
    seg = oracle.evaluate(itf, prm)
    assert np.array_equal(seg["pair_s"], seg["pair_m"])  # only coincident pairs
    el = oracle.evaluate_elements(itf, ng, prm, pairs=(seg["pair_s"], seg["pair_m"]))
    assert rel(el["D"], seg["D"]) <= 1e-14
    assert rel(el["M"], seg["M"]) <= 1e-14
    assert rel(el["M"], el["D"]) <= 1e-14
    assert np.abs(el["g"]).max() == 0.0


@pytest.mark.parametrize("ng", [1, 2, 4, 8])
def test_full_coverage_area_and_partition_of_unity(ng):
    itf = synth.interface_config(0)
    prm = oracle.params(delta=itf.delta)
    el = oracle.evaluate_elements(itf, ng, prm)
    # the Jacobian determinant of a bilinear map is linear in xi: any rule
    # gives the exact area, and all points are owned (the master covers the
    # slave), so sum(D) is the area of the unit square
    assert abs(el["D"].sum() - 1.0) <= 1e-14
    B = el["blocks"]
    rs_D = B[:, :16].reshape(-1, 4, 4).sum(axis=2)
    rs_M = B[:, 16:32].reshape(-1, 4, 4).sum(axis=2)
    np.testing.assert_allclose(rs_M, rs_D, rtol=0, atol=1e-15)
    # tied flat: zero gap
    assert np.abs(el["g"]).max() <= 1e-17


@pytest.mark.parametrize("ng", [2, 5])
def test_constant_normal_offset_gap(ng):
    d = 3e-3
    itf = synth.interface_config(0)
    itf.master.X[:, 2] += d
    prm = oracle.params(delta=0.01)
    el = oracle.evaluate_elements(itf, ng, prm)
    rs = np.asarray(el["D"].sum(axis=1)).ravel()
    np.testing.assert_allclose(el["g"], d * rs, rtol=1e-12, atol=1e-18)


def test_curved_partition_of_unity_and_convergence():
    itf = synth.interface_config(1, scale=20)
    prm = oracle.params(delta=itf.delta)
    seg = oracle.evaluate(itf, prm)
    pairs = (seg["pair_s"], seg["pair_m"])
    errs = []
    for ng in (2, 4, 8):
        el = oracle.evaluate_elements(itf, ng, prm, pairs=pairs)
        assert (el["status"] == 0).all()
        B = el["blocks"]
        rs_D = B[:, :16].reshape(-1, 4, 4).sum(axis=2)
        rs_M = B[:, 16:32].reshape(-1, 4, 4).sum(axis=2)
        np.testing.assert_allclose(rs_M, rs_D, rtol=0, atol=1e-15)
        errs.append((rel(el["M"], seg["M"]), rel(el["g"], seg["g"])))
    # points near the uncovered rim and near master edges converge slowly,
    # but they converge
    assert errs[0][0] > errs[1][0] > errs[2][0] and errs[2][0] < 0.01
    assert errs[0][1] > errs[1][1] > errs[2][1] and errs[2][1] < 0.05


@pytest.mark.parametrize("ng", [2, 4])
def test_dual_basis_biorthogonal_under_full_coverage(ng):
    itf = synth.interface_config(0)
    prm = oracle.params(delta=itf.delta, dual=True)
    el = oracle.evaluate_elements(itf, ng, prm)
    D = el["D"].toarray()
    off = D - np.diag(np.diag(D))
    assert np.abs(off).max() <= 1e-15
    std = oracle.evaluate_elements(itf, ng, oracle.params(delta=itf.delta))
    # diag of the dual D = row sums of the standard D (int Phi_j = int N_j)
    np.testing.assert_allclose(np.diag(D), np.asarray(std["D"].sum(axis=1)).ravel(), rtol=1e-13)


def test_converges_to_segment_based():
    itf = synth.interface_config(0)
    prm = oracle.params(delta=itf.delta)
    seg = oracle.evaluate(itf, prm)
    pairs = (seg["pair_s"], seg["pair_m"])
    errs = [rel(oracle.evaluate_elements(itf, ng, prm, pairs=pairs)["M"], seg["M"]) for ng in (2, 4, 8)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.3 * errs[0]


def test_rule_out_of_range():
    itf = synth.interface_config(0)
    prm = oracle.params(delta=itf.delta)
    with pytest.raises(ValueError):
        oracle.evaluate_elements(itf, 9, prm)
