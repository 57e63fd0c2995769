"""GPU parity of the forward path (search, clip, integrate, assemble) with the
oracle, through the C ABI: candidates, pairs, clip vertex counts and CSR
patterns bit-exact; D, M and gap within a relative Frobenius error of 1e-10."""

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import assert_forward_parity, gpu_run, oracle_params

pytestmark = pytest.mark.gpu


def test_flat_tied_config():
    itf = synth.interface_config(0)
    g = gpu_run(itf)
    o = oracle.evaluate(itf, oracle_params(itf))
    assert_forward_parity(g, o)
    # tied flat: full coverage and momentum conservation on the GPU values
    assert abs(g["D"].sum() - 1.0) < 1e-13
    np.testing.assert_allclose(np.asarray(g["M"].sum(1)).ravel(), np.asarray(g["D"].sum(1)).ravel(), atol=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_flat_tied_other_seeds_and_unjittered(seed):
    itf = synth.flat_tied(8, 7, seed=seed, jitter=0.0 if seed == 3 else 0.1)
    assert_forward_parity(gpu_run(itf), oracle.evaluate(itf, oracle_params(itf)))


@pytest.mark.parametrize("k,scale", [(1, 37), (2, 53), (1, 90), (2, 130)])
def test_reduced_curved_configs(k, scale):
    # several tiles of 64 pairs with ragged tails
    itf = synth.interface_config(k, scale=scale)
    assert_forward_parity(gpu_run(itf), oracle.evaluate(itf, oracle_params(itf)))


def test_dual_basis_and_three_point_rule():
    itf = synth.interface_config(1, scale=40)
    for dual, rule in ((True, 7), (False, 3), (True, 3)):
        g = gpu_run(itf, dual=dual, rule=rule)
        o = oracle.evaluate(itf, oracle_params(itf, dual=dual, rule=rule))
        assert_forward_parity(g, o)


def test_dual_basis_diagonal_D_unjittered_flat():
    itf = synth.flat_tied(16, 13, jitter=0.0)
    g = gpu_run(itf, dual=True)
    Dd = g["D"].toarray()
    assert abs(Dd - np.diag(np.diag(Dd))).max() < 1e-15
    np.testing.assert_allclose(np.diag(Dd), np.asarray(g["M"].sum(1)).ravel(), atol=1e-15)


def test_full_cylinder_config():
    itf = synth.interface_config(1)
    g = gpu_run(itf)
    o = oracle.evaluate(itf, oracle_params(itf))
    assert_forward_parity(g, o)
    assert g["stats"]["n_pairs"] == o["pair_s"].size
    print("cylinder pairs", o["pair_s"].size, "candidates", o["cand_s"].size)


def test_full_wavy_config():
    itf = synth.interface_config(2)
    g = gpu_run(itf)
    o = oracle.evaluate(itf, oracle_params(itf))
    assert_forward_parity(g, o)
    print("wavy pairs", o["pair_s"].size, "candidates", o["cand_s"].size)


def test_empty_and_single_element_interfaces():
    # master far away: no candidate, no pair, empty pattern, zero gap
    itf = synth.flat_tied(5, 4, seed=9)
    itf.master.X = itf.master.X + np.array([5.0, 0.0, 0.0])
    g = gpu_run(itf)
    assert g["cand_s"].size == 0 and g["pair_s"].size == 0
    assert g["D"].nnz == 0 and g["M"].nnz == 0
    assert np.all(g["g"] == 0.0)
    # one element on each side
    one = synth.flat_tied(1, 1, jitter=0.0)
    g = gpu_run(one)
    o = oracle.evaluate(one, oracle_params(one))
    assert_forward_parity(g, o)
    c = one.slave.conn[0]
    np.testing.assert_allclose(g["D"].toarray()[np.ix_(c, c)], np.array([[4, 2, 1, 2], [2, 4, 2, 1], [1, 2, 4, 2],
                                                                         [2, 1, 2, 4]]) / 36.0, atol=1e-15)


def test_bitwise_deterministic():
    itf = synth.interface_config(2, scale=96)
    a = gpu_run(itf)
    b = gpu_run(itf)
    assert np.array_equal(a["D"].data, b["D"].data)
    assert np.array_equal(a["M"].data, b["M"].data)
    assert np.array_equal(a["g"], b["g"])


@pytest.mark.parametrize("ns,nm", [(4, 20), (3, 20)])
def test_many_candidates_per_slave(ns, nm):
    # coarse slave on a fine master: 33-42 (ns=4) and 49-64 (ns=3)
    # candidates per slave element, beyond what the count pass keeps
    itf = synth.flat_tied(ns, nm, seed=5)
    g = gpu_run(itf)
    o = oracle.evaluate(itf, oracle_params(itf))
    assert_forward_parity(g, o)
    assert np.bincount(o["cand_s"]).min() > 32


def test_mixed_candidate_counts():
    # one interface whose slave elements have from a few to several dozen
    # candidates, so every fill path runs in the same launch
    itf = synth.graded_flat(6, 40, 3.0)
    g = gpu_run(itf)
    o = oracle.evaluate(itf, oracle_params(itf))
    assert_forward_parity(g, o)
    c = np.bincount(o["cand_s"], minlength=itf.slave.n_el)
    assert (c <= 32).any() and ((c > 32) & (c <= 48)).any() and (c > 48).any()


def test_rows_longer_than_the_accumulator():
    # master finer than slave (ratio 1.3): many rows of D and M together hold
    # more than 32 entries (each part fits), and every assembly form of a row
    # must give the oracle's values; the gradient sums run over the same rows
    itf = synth.flat_tied(16, 21, seed=4)
    g = gpu_run(itf, backward_seed=31)
    o = oracle.evaluate(itf, oracle_params(itf))
    assert_forward_parity(g, o)
    nd, nm = np.diff(o["D"].indptr), np.diff(o["M"].indptr)
    assert ((nd + nm > 32) & (nm <= 32)).sum() > 0
