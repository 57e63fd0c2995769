"""The sampled-node oracle helpers of the GPU tests give the full oracle's
rows and gradients at the sampled nodes (CPU only)."""

import numpy as np

import oracle
import synth
from tests.gpu_util import oracle_params, sampled_oracle, weight_fns, window_oracle


def test_sampled_oracle_equals_full_rows_and_gradients():
    itf = synth.interface_config(1, scale=20)
    prm = oracle_params(itf)
    full = oracle.evaluate(itf, prm)
    rng = np.random.default_rng(1)
    sn = rng.choice(itf.slave.n_nodes, 30, replace=False)
    mn = rng.choice(itf.master.n_nodes, 30, replace=False)
    o = sampled_oracle(itf, prm, sn, mn, seed=77)
    assert np.array_equal(o["pair_s"], full["pair_s"]) and np.array_equal(o["pair_m"], full["pair_m"])
    for key in ("D", "M"):
        A, B = o[key][sn], full[key][sn]
        assert np.array_equal(A.indptr, B.indptr) and np.array_equal(A.indices, B.indices)
        assert np.array_equal(A.data, B.data)
    assert np.array_equal(o["g"][sn], full["g"][sn])
    w = oracle.pair_weights(itf.slave, itf.master, full["pair_s"], full["pair_m"], *weight_fns(77))
    g24, _ = oracle.pair_grads(itf.slave, itf.master, prm, full["pair_s"], full["pair_m"], w)
    gs, gm = oracle.scatter_grads(itf.slave, itf.master, full["pair_s"], full["pair_m"], g24)
    np.testing.assert_allclose(o["gXs"][sn], gs[sn], rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(o["gXm"][mn], gm[mn], rtol=1e-14, atol=1e-16)


def test_window_oracle_complete_rows():
    itf = synth.interface_config(2, scale=24)
    prm = oracle_params(itf)
    full = oracle.evaluate(itf, prm)
    els = np.arange(5 * 24, 12 * 24)
    o, nodes = window_oracle(itf, els, prm)
    assert nodes.size > 0
    for key in ("D", "M"):
        A, B = o[key][nodes], full[key][nodes]
        assert np.array_equal(A.indices, B.indices) and np.array_equal(A.data, B.data)
    assert np.array_equal(o["g"][nodes], full["g"][nodes])
