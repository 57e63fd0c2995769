"""GPU parity of element-based integration (an n x n Gauss rule on each
slave element, each point taken by the first master that contains it) with
the oracle, through the C ABI: D, M and gap within a relative Frobenius error
of 1e-10, on the pair list and CSR pattern of the segment-based search."""

import numpy as np
import pytest

import oracle
import synth
from synth.meshes import Interface, Mesh
from tests.gpu_util import TOL, assert_same_pattern, gpu_run, oracle_params, rel_err

pytestmark = pytest.mark.gpu


def check(g, o):
    assert np.array_equal(g["pair_s"], o["pair_s"]) and np.array_equal(g["pair_m"], o["pair_m"])
    assert_same_pattern(g["D"], o["D"])
    assert_same_pattern(g["M"], o["M"])
    eD, eM = rel_err(g["D"].data, o["D"].data), rel_err(g["M"].data, o["M"].data)
    assert eD <= TOL and eM <= TOL, (eD, eM)
    if np.linalg.norm(o["g"]) == 0.0:
        assert np.abs(g["g"]).max() <= 1e-17
    else:
        assert rel_err(g["g"], o["g"]) <= TOL
    assert g["stats"]["n_noconv"] == 0


@pytest.mark.parametrize("ng", [1, 2, 5, 8])
def test_flat_tied(ng):
    itf = synth.interface_config(0)
    prm = oracle_params(itf)
    g = gpu_run(itf, element_rule=ng)
    o = oracle.evaluate_elements(itf, ng, prm)
    check(g, o)
    assert abs(g["D"].sum() - 1.0) <= 1e-14


@pytest.mark.parametrize("k,scale,ng,dual", [(1, 37, 3, False), (2, 53, 8, False), (1, 44, 4, True),
                                             (2, 41, 6, True), (2, 130, 4, False)])
def test_reduced_curved(k, scale, ng, dual):
    itf = synth.interface_config(k, scale=scale)
    prm = oracle_params(itf, dual=dual)
    g = gpu_run(itf, dual=dual, element_rule=ng)
    o = oracle.evaluate_elements(itf, ng, prm)
    check(g, o)


def test_full_wavy_sampled_rows():
    # the oracle on a window of slave elements (rows 300..331 of the slave
    # grid) against the whole master side: a slave node whose incident
    # elements all lie in the window has its complete row
    itf = synth.interface_config(2)
    ng = 4
    g = gpu_run(itf, element_rule=ng)
    n = 1024
    rows = np.arange(300, 332)
    els = (rows[:, None] * n + np.arange(n)[None, :]).ravel()
    sub = Interface(Mesh(itf.slave.X, itf.slave.conn[els]), itf.master, itf.delta)
    prm = oracle_params(itf)
    o = oracle.evaluate_elements(sub, ng, prm)
    ps_global = els[o["pair_s"]]
    sel = np.isin(g["pair_s"], els)
    assert np.array_equal(g["pair_s"][sel], ps_global) and np.array_equal(g["pair_m"][sel], o["pair_m"])
    cnt = np.bincount(itf.slave.conn.ravel(), minlength=itf.slave.n_nodes)
    cnt_w = np.bincount(itf.slave.conn[els].ravel(), minlength=itf.slave.n_nodes)
    nodes = np.nonzero((cnt_w == cnt) & (cnt > 0))[0]
    assert nodes.size > 20000
    for key in ("D", "M"):
        A, B = g[key][nodes], o[key][nodes]
        assert_same_pattern(A, B)
        assert rel_err(A.data, B.data) <= TOL, key
    assert rel_err(g["g"][nodes], o["g"][nodes]) <= TOL
    print(f"element-based wavy: {nodes.size} complete rows compared")


def test_element_rule_errors():
    import torch
    from paper_2202_03933_amd import MortarBatch, MortarError, MortarInterface, default_params
    from paper_2202_03933_amd import _capi as C
    itf = synth.interface_config(0)
    dev = torch.device("cuda", 0)
    args = (torch.from_numpy(itf.slave.X), torch.from_numpy(itf.slave.conn), torch.from_numpy(itf.master.X),
            torch.from_numpy(itf.master.conn))
    with pytest.raises(MortarError) as e:
        MortarInterface(*args, params=default_params(element_rule=9), device=dev)
    assert e.value.code == C.MT_EINVAL
    it = MortarInterface(*args, params=default_params(element_rule=3), device=dev).setup()
    it.integrate()
    z = torch.zeros(max(it.nnz_D, it.nnz_M, it.n_slave_nodes), dtype=torch.float64, device=dev)
    with pytest.raises(MortarError) as e:
        it.backward(z[:it.nnz_D], z[:it.nnz_M], z[:it.n_slave_nodes])
    assert e.value.code == C.MT_EUNSUPPORTED
    with pytest.raises(MortarError) as e:
        MortarBatch([it])
    assert e.value.code == C.MT_EUNSUPPORTED
