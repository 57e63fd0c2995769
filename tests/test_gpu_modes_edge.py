"""Degenerate inputs in every mode of the HIP path (dual basis, continuous
normal field, element-based integration), through the C ABI: an interface
with no pair gives empty patterns, zero gap and zero gradients; a single
element pair and a ragged reduced interface match the oracle."""

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import TOL, gpu_run, oracle_params, rel_err, weight_fns

pytestmark = pytest.mark.gpu

MODES = [dict(dual=True), dict(nodal=True), dict(nodal=True, dual=True), dict(element_rule=3),
         dict(element_rule=2, nodal=True)]


def oracle_for(itf, mode):
    prm = oracle_params(itf, dual=mode.get("dual", False), nodal=mode.get("nodal", False))
    if mode.get("element_rule"):
        return oracle.evaluate_elements(itf, mode["element_rule"], prm), prm
    return oracle.evaluate(itf, prm), prm


@pytest.mark.parametrize("mode", MODES, ids=lambda m: "-".join(f"{k}{v}" for k, v in m.items()))
def test_empty_interface(mode):
    itf = synth.flat_tied(5, 4, seed=9)
    itf.master.X = itf.master.X + np.array([5.0, 0.0, 0.0])
    seed = None if mode.get("element_rule") else 77
    g = gpu_run(itf, backward_seed=seed, **mode)
    assert g["pair_s"].size == 0 and g["D"].nnz == 0 and g["M"].nnz == 0
    assert np.all(g["g"] == 0.0)
    if seed is not None:
        assert np.all(g["gXs"] == 0.0) and np.all(g["gXm"] == 0.0)


@pytest.mark.parametrize("mode", MODES, ids=lambda m: "-".join(f"{k}{v}" for k, v in m.items()))
def test_single_pair_and_ragged_interface(mode):
    for itf in (synth.flat_tied(1, 1, jitter=0.0), synth.interface_config(2, scale=29)):
        g = gpu_run(itf, **mode)
        o, prm = oracle_for(itf, mode)
        assert np.array_equal(g["pair_s"], o["pair_s"]) and np.array_equal(g["pair_m"], o["pair_m"])
        assert rel_err(g["D"].data, o["D"].data) <= TOL
        assert rel_err(g["M"].data, o["M"].data) <= TOL
        if np.linalg.norm(o["g"]) > 0:
            assert rel_err(g["g"], o["g"]) <= TOL
        else:
            assert np.abs(g["g"]).max() <= 1e-17


@pytest.mark.parametrize("mode", [m for m in MODES if not m.get("element_rule")],
                         ids=lambda m: "-".join(f"{k}{v}" for k, v in m.items()))
def test_ragged_gradients(mode):
    itf = synth.interface_config(2, scale=29)
    g = gpu_run(itf, backward_seed=78, **mode)
    o, prm = oracle_for(itf, mode)
    ps, pm = o["pair_s"], o["pair_m"]
    w = oracle.pair_weights(itf.slave, itf.master, ps, pm, *weight_fns(78))
    g24, gn0, st = oracle.pair_grads(itf.slave, itf.master, prm, ps, pm, w, with_n0=True)
    gs, gm = oracle.scatter_grads(itf.slave, itf.master, ps, pm, g24)
    if mode.get("nodal"):
        ge = np.zeros((itf.slave.n_el, 3))
        np.add.at(ge, ps, gn0)
        gs = gs + oracle.normal_chain(itf.slave, ge)
    assert rel_err(g["gXs"], gs) <= TOL and rel_err(g["gXm"], gm) <= TOL


@pytest.mark.parametrize("fan", [(6, 7), (16, 18)], ids=["valence6", "valence16"])
@pytest.mark.parametrize("mode", MODES, ids=lambda m: "-".join(f"{k}{v}" for k, v in m.items()))
def test_nodes_with_more_than_four_elements(mode, fan):
    # fans of kites: the slave centre has 6 (16) incident elements, the master
    # centre 7 (18), so the row gathers take their general loops; with 16 the
    # centre's D and M rows (33 and 37 columns) outgrow the per-thread
    # segments of the pattern and assembly kernels
    itf = synth.kite_fan(*fan)
    seed = None if mode.get("element_rule") else 79
    g = gpu_run(itf, backward_seed=seed, **mode)
    o, prm = oracle_for(itf, mode)
    assert np.array_equal(g["pair_s"], o["pair_s"]) and np.array_equal(g["pair_m"], o["pair_m"])
    for key in ("D", "M"):
        assert rel_err(g[key].data, o[key].data) <= TOL
    assert rel_err(g["g"], o["g"]) <= TOL
    if seed is None:
        return
    ps, pm = o["pair_s"], o["pair_m"]
    w = oracle.pair_weights(itf.slave, itf.master, ps, pm, *weight_fns(seed))
    g24, gn0, st = oracle.pair_grads(itf.slave, itf.master, prm, ps, pm, w, with_n0=True)
    gs, gm = oracle.scatter_grads(itf.slave, itf.master, ps, pm, g24)
    if mode.get("nodal"):
        ge = np.zeros((itf.slave.n_el, 3))
        np.add.at(ge, ps, gn0)
        gs = gs + oracle.normal_chain(itf.slave, ge)
    assert abs(gs[0]).max() > 0 and abs(gm[0]).max() > 0
    assert rel_err(g["gXs"], gs) <= TOL and rel_err(g["gXm"], gm) <= TOL
