"""GPU parity on interfaces whose master normals oppose the slave normals,
the contact setting (Alg. 1 projects master elements onto the slave side;
their projections then run clockwise and are clipped as (M0, M3, M2, M1)).
The master connectivity of configurations 0-2 is reversed, (0,1,2,3) ->
(0,3,2,1): topology bit-exact against the oracle, D, M, gap and gradients
within 1e-10, finite differences, and the batched launch."""

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import TOL, assert_forward_parity, gpu_run, oracle_params, rel_err, weight_fns

pytestmark = pytest.mark.gpu


def oracle_grad(itf, prm, ps, pm, seed):
    w = oracle.pair_weights(itf.slave, itf.master, ps, pm, *weight_fns(seed))
    g24, st = oracle.pair_grads(itf.slave, itf.master, prm, ps, pm, w)
    return oracle.scatter_grads(itf.slave, itf.master, ps, pm, g24)


@pytest.mark.parametrize("k,scale", [(0, None), (1, 37), (2, 53), (2, 130)])
def test_forward_parity_opposing(k, scale):
    itf = synth.interface_config(k, scale, opposing_normals=True)
    g = gpu_run(itf)
    assert_forward_parity(g, oracle.evaluate(itf, oracle_params(itf)))
    # the same surfaces as the original interface: equal to its results
    h = gpu_run(synth.interface_config(k, scale))
    assert np.array_equal(g["cand_nv"], h["cand_nv"])
    assert rel_err(g["M"].data, h["M"].data) <= 1e-13 and rel_err(g["D"].data, h["D"].data) <= 1e-13


@pytest.mark.parametrize("k", [1, 2])
def test_full_size_forward_opposing(k):
    itf = synth.interface_config(k, opposing_normals=True)
    g = gpu_run(itf)
    assert_forward_parity(g, oracle.evaluate(itf, oracle_params(itf)))
    assert g["stats"]["n_degenerate_master"] == 0


@pytest.mark.parametrize("k,scale,dual", [(2, 41, False), (1, 37, False), (2, 90, False), (2, 41, True),
                                          (1, 37, True)])
def test_gradient_parity_opposing(k, scale, dual):
    itf = synth.interface_config(k, scale, opposing_normals=True)
    prm = oracle_params(itf, dual=dual)
    g = gpu_run(itf, dual=dual, backward_seed=3000)
    o = oracle.evaluate(itf, prm)
    assert_forward_parity(g, o)
    gs, gm = oracle_grad(itf, prm, o["pair_s"], o["pair_m"], 3000)
    es, em = rel_err(g["gXs"], gs), rel_err(g["gXm"], gm)
    print(f"opposing grad rel err slave {es:.2e} master {em:.2e}")
    assert es <= TOL and em <= TOL


def test_nodal_normals_opposing():
    itf = synth.interface_config(2, 41, opposing_normals=True)
    prm = oracle_params(itf, nodal=True)
    g = gpu_run(itf, nodal=True, backward_seed=3300)
    o = oracle.evaluate(itf, prm)
    assert_forward_parity(g, o)
    w = oracle.pair_weights(itf.slave, itf.master, o["pair_s"], o["pair_m"], *weight_fns(3300))
    g24, gn0, _ = oracle.pair_grads(itf.slave, itf.master, prm, o["pair_s"], o["pair_m"], w, with_n0=True)
    gs, gm = oracle.scatter_grads(itf.slave, itf.master, o["pair_s"], o["pair_m"], g24)
    gn0_el = np.zeros((itf.slave.n_el, 3))
    np.add.at(gn0_el, o["pair_s"], gn0)
    gs = gs + oracle.normal_chain(itf.slave, gn0_el)
    assert rel_err(g["gXs"], gs) <= TOL and rel_err(g["gXm"], gm) <= TOL


@pytest.mark.parametrize("k", [1, 2])
def test_full_size_gradient_opposing_sampled(k):
    itf = synth.interface_config(k, opposing_normals=True)
    prm = oracle_params(itf)
    g = gpu_run(itf, backward_seed=3000)
    o = oracle.evaluate(itf, prm)
    assert_forward_parity(g, o)
    rng = np.random.default_rng(3004)
    sn = rng.choice(itf.slave.n_nodes, 200, replace=False)
    mn = rng.choice(itf.master.n_nodes, 200, replace=False)
    ps, pm = o["pair_s"], o["pair_m"]
    sel = np.isin(itf.slave.conn[ps], sn).any(1) | np.isin(itf.master.conn[pm], mn).any(1)
    gs, gm = oracle_grad(itf, prm, ps[sel], pm[sel], 3000)
    es, em = rel_err(g["gXs"][sn], gs[sn]), rel_err(g["gXm"][mn], gm[mn])
    print(f"opposing sampled grad rel err slave {es:.2e} master {em:.2e} over {sel.sum()} pairs")
    assert es <= TOL and em <= TOL


def test_finite_differences_opposing_cylinder():
    from tests.test_gpu_backward import _fd_check
    _fd_check(synth.interface_config(1, opposing_normals=True), n_coords=60, interior=0.6)


def test_batch_opposing_bitwise_and_oracle():
    from tests.test_gpu_batch import run_batch_checks
    instances = [synth.opposing(i) for i in synth.batched_instances(n_inst=9, max_side=40)]
    ifaces, outs, grads = run_batch_checks(instances, autotune=False)
    for itf, it, (D, M, gv), (gs, gm) in zip(instances, ifaces, outs, grads):
        prm = oracle_params(itf)
        o = oracle.evaluate(itf, prm)
        assert np.array_equal(it.M_col.cpu().numpy(), o["M"].indices)
        assert rel_err(D.cpu().numpy(), o["D"].data) <= TOL
        assert rel_err(M.cpu().numpy(), o["M"].data) <= TOL
        if itf.meta["geometry"] == "flat":
            continue  # tied flat boundaries: not differentiable
        w = oracle.pair_weights(itf.slave, itf.master, o["pair_s"], o["pair_m"],
                                *weight_fns(4000 + itf.meta["instance"]))
        g24, _ = oracle.pair_grads(itf.slave, itf.master, prm, o["pair_s"], o["pair_m"], w)
        ogs, ogm = oracle.scatter_grads(itf.slave, itf.master, o["pair_s"], o["pair_m"], g24)
        assert rel_err(gs.cpu().numpy().T, ogs) <= TOL and rel_err(gm.cpu().numpy().T, ogm) <= TOL
