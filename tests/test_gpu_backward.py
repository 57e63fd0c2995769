"""GPU parity of the backward pass (hand-written reverse mode) with the
oracle's forward-mode dual-number gradients, central finite differences of
the GPU's own forward pass, and the torch.autograd.Function wrapper."""

import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import (TOL, assert_forward_parity, assert_rows_parity, gpu_run, oracle_params, rel_err,
                            sampled_oracle, weight_fns)

pytestmark = pytest.mark.gpu


def oracle_grad(itf, prm, ps, pm, seed):
    w = oracle.pair_weights(itf.slave, itf.master, ps, pm, *weight_fns(seed))
    g24, st = oracle.pair_grads(itf.slave, itf.master, prm, ps, pm, w)
    return oracle.scatter_grads(itf.slave, itf.master, ps, pm, g24)


# The tied flat configuration is left out of gradient parity: there slave and
# master boundary edges are exactly collinear, a clip crossing of two collinear
# edges can sit anywhere on the common line, and the loss is not
# differentiable (the oracle's chain rule through the crossing parameter
# returns values of order 1e14 there).  It is checked by finite differences
# on interior coordinates instead (test_finite_differences_flat_interior).
@pytest.mark.parametrize("k,scale", [(2, 41), (1, 37), (2, 90), (1, 64)])
def test_gradient_parity_reduced(k, scale):
    itf = synth.interface_config(k, scale=scale)
    prm = oracle_params(itf)
    g = gpu_run(itf, backward_seed=3000)
    o = oracle.evaluate(itf, prm)
    assert np.array_equal(g["pair_s"], o["pair_s"]) and np.array_equal(g["pair_m"], o["pair_m"])
    gs, gm = oracle_grad(itf, prm, o["pair_s"], o["pair_m"], 3000)
    es, em = rel_err(g["gXs"], gs), rel_err(g["gXm"], gm)
    print(f"grad rel err slave {es:.2e} master {em:.2e}")
    assert es <= TOL and em <= TOL


# A master mesh much coarser than the slave mesh (mortar methods put the finer
# mesh on the slave side): each master element meets ~190, ~2,300 or ~4,300
# slave elements, so the master-node gradient sums run over long per-element
# pair lists (sorted by a workgroup in LDS runs of 2,048, merged beyond one
# run).  Parity with the oracle, and the same bits from a second run.
@pytest.mark.parametrize("ns,nm", [(64, 5), (96, 2), (128, 2)])
def test_gradient_parity_coarse_master(ns, nm):
    itf = synth.cylinder(ns, nm)
    prm = oracle_params(itf)
    g = gpu_run(itf, backward_seed=3200)
    o = oracle.evaluate(itf, prm)
    assert np.array_equal(g["pair_s"], o["pair_s"]) and np.array_equal(g["pair_m"], o["pair_m"])
    per_master = np.bincount(o["pair_m"], minlength=itf.master.n_el)
    print(f"pairs per master element {per_master.min()}..{per_master.max()}")
    gs, gm = oracle_grad(itf, prm, o["pair_s"], o["pair_m"], 3200)
    es, em = rel_err(g["gXs"], gs), rel_err(g["gXm"], gm)
    print(f"coarse-master grad rel err slave {es:.2e} master {em:.2e}")
    assert es <= TOL and em <= TOL
    g2 = gpu_run(itf, backward_seed=3200)
    assert np.array_equal(g2["gXm"], g["gXm"]) and np.array_equal(g2["gXs"], g["gXs"])


# Dual basis (Sec. 2): the gradient also runs through A_e = D_e M_e^-1 of
# every slave element.
@pytest.mark.parametrize("k,scale,rule", [(2, 41, 7), (1, 37, 7), (2, 52, 3)])
def test_dual_gradient_parity_reduced(k, scale, rule):
    itf = synth.interface_config(k, scale=scale)
    prm = oracle_params(itf, dual=True, rule=rule)
    g = gpu_run(itf, dual=True, rule=rule, backward_seed=3100)
    o = oracle.evaluate(itf, prm)
    assert np.array_equal(g["pair_s"], o["pair_s"]) and np.array_equal(g["pair_m"], o["pair_m"])
    gs, gm = oracle_grad(itf, prm, o["pair_s"], o["pair_m"], 3100)
    es, em = rel_err(g["gXs"], gs), rel_err(g["gXm"], gm)
    print(f"dual grad rel err slave {es:.2e} master {em:.2e}")
    assert es <= TOL and em <= TOL


def test_dual_gradient_parity_full_wavy_sampled():
    itf = synth.interface_config(2)
    prm = oracle_params(itf, dual=True)
    g = gpu_run(itf, dual=True, backward_seed=3100)
    o = oracle.evaluate(itf, prm)
    # full-size dual forward values, then the sampled gradients
    eD, eM, eg = assert_forward_parity(g, o)
    print(f"full wavy dual forward rel err D {eD:.2e} M {eM:.2e} g {eg:.2e}")
    rng = np.random.default_rng(3102)
    sn = rng.choice(itf.slave.n_nodes, 200, replace=False)
    mn = rng.choice(itf.master.n_nodes, 200, replace=False)
    ps, pm = o["pair_s"], o["pair_m"]
    sel = np.isin(itf.slave.conn[ps], sn).any(1) | np.isin(itf.master.conn[pm], mn).any(1)
    gs, gm = oracle_grad(itf, prm, ps[sel], pm[sel], 3100)
    es, em = rel_err(g["gXs"][sn], gs[sn]), rel_err(g["gXm"][mn], gm[mn])
    print(f"sampled dual grad rel err slave {es:.2e} master {em:.2e} over {sel.sum()} pairs")
    assert es <= TOL and em <= TOL


def test_gradient_parity_full_wavy_sampled():
    itf = synth.interface_config(2)
    prm = oracle_params(itf)
    g = gpu_run(itf, backward_seed=3000)
    o = oracle.evaluate(itf, prm)
    assert np.array_equal(g["pair_s"], o["pair_s"]) and np.array_equal(g["pair_m"], o["pair_m"])
    rng = np.random.default_rng(3002)
    sn = rng.choice(itf.slave.n_nodes, 300, replace=False)
    mn = rng.choice(itf.master.n_nodes, 300, replace=False)
    ps, pm = o["pair_s"], o["pair_m"]
    sel = np.isin(itf.slave.conn[ps], sn).any(1) | np.isin(itf.master.conn[pm], mn).any(1)
    gs, gm = oracle_grad(itf, prm, ps[sel], pm[sel], 3000)
    es, em = rel_err(g["gXs"][sn], gs[sn]), rel_err(g["gXm"][mn], gm[mn])
    print(f"sampled grad rel err slave {es:.2e} master {em:.2e} over {sel.sum()} pairs")
    assert es <= TOL and em <= TOL


def test_gradient_parity_full_cylinder_sampled():
    itf = synth.interface_config(1)
    prm = oracle_params(itf)
    g = gpu_run(itf, backward_seed=3000)
    rng = np.random.default_rng(3003)
    sn = rng.choice(itf.slave.n_nodes, 300, replace=False)
    mn = rng.choice(itf.master.n_nodes, 300, replace=False)
    o = sampled_oracle(itf, prm, sn, mn, seed=3000)
    assert np.array_equal(g["pair_s"], o["pair_s"]) and np.array_equal(g["pair_m"], o["pair_m"])
    assert_rows_parity(g["D"], g["M"], g["g"], o, sn)
    es, em = rel_err(g["gXs"][sn], o["gXs"][sn]), rel_err(g["gXm"][mn], o["gXm"][mn])
    print(f"sampled cylinder grad rel err slave {es:.2e} master {em:.2e}")
    assert es <= TOL and em <= TOL


def _fd_check(itf, seed=3000, n_coords=200, interior=0.35, dual=False):
    from paper_2202_03933_amd import MortarInterface
    from tests.gpu_util import csr_weights, gpu_params
    dev = torch.device("cuda", 0)
    Xs = torch.from_numpy(itf.slave.X).to(dev)
    Xm = torch.from_numpy(itf.master.X).to(dev)
    iface = MortarInterface(Xs, torch.from_numpy(itf.slave.conn), Xm, torch.from_numpy(itf.master.conn),
                            params=gpu_params(itf, dual=dual), device=dev).setup()
    import scipy.sparse as sp
    D, M, gp = iface.integrate()
    Dc = sp.csr_matrix((D.cpu().numpy(), iface.D_col.cpu().numpy(), iface.D_rowptr.cpu().numpy()),
                       shape=(itf.slave.n_nodes,) * 2)
    Mc = sp.csr_matrix((M.cpu().numpy(), iface.M_col.cpu().numpy(), iface.M_rowptr.cpu().numpy()),
                       shape=(itf.slave.n_nodes, itf.master.n_nodes))
    wD, wM, wg = (torch.from_numpy(a).to(dev) for a in csr_weights(Dc, Mc, itf.slave.n_nodes, seed))
    gXs, gXm = iface.backward(wD, wM, wg)
    gXs, gXm = gXs.cpu().numpy(), gXm.cpu().numpy()

    def dL(side, node, d, h):
        out = []
        for sgn in (1.0, -1.0):
            A, B = Xs.clone(), Xm.clone()
            (A if side == 0 else B)[node, d] += sgn * h
            iface.set_coordinates(A, B)
            out.append(iface.integrate())
        diff = sum(torch.dot(w, p - q).item() for w, p, q in zip((wD, wM, wg), out[0], out[1]))
        return diff / (2 * h)

    rng = np.random.default_rng(3001)
    checked = refined = 0
    while checked < n_coords:
        side = int(rng.integers(0, 2))
        mesh = itf.slave if side == 0 else itf.master
        node = int(rng.integers(0, mesh.n_nodes))
        d = int(rng.integers(0, 3))
        if np.any(np.abs(mesh.X[node, :2] - 0.5) > interior):
            continue
        an = (gXs if side == 0 else gXm)[d, node]
        fd = dL(side, node, d, 1e-6)
        checked += 1
        if checked % 25 == 0:
            print(f"FD {itf.name}: {checked} coordinates", flush=True)
        if abs(fd - an) > 1e-4 * abs(an) + 1e-10:
            refined += 1
            fd = dL(side, node, d, 1e-7)
            assert abs(fd - an) <= 1e-4 * abs(an) + 1e-9, (side, node, d, fd, an)
    iface.set_coordinates(Xs, Xm)
    print(f"FD: {checked} coordinates, {refined} re-checked with h=1e-7")
    assert refined <= 0.1 * checked


def test_finite_differences_flat_interior():
    _fd_check(synth.interface_config(0), n_coords=40, interior=0.3)


def test_finite_differences_full_wavy():
    _fd_check(synth.interface_config(2))


def test_finite_differences_cylinder():
    _fd_check(synth.interface_config(1), n_coords=60, interior=0.6)


def test_finite_differences_dual_cylinder():
    _fd_check(synth.interface_config(1, scale=48), n_coords=60, interior=0.6, dual=True)


def test_autograd_function_matches_backward():
    from paper_2202_03933_amd import MortarFunction, MortarInterface
    from tests.gpu_util import gpu_params
    itf = synth.interface_config(2, scale=64)
    dev = torch.device("cuda", 0)
    Xs = torch.from_numpy(itf.slave.X).to(dev).requires_grad_(True)
    Xm = torch.from_numpy(itf.master.X).to(dev).requires_grad_(True)
    iface = MortarInterface(Xs.detach(), torch.from_numpy(itf.slave.conn), Xm.detach(),
                            torch.from_numpy(itf.master.conn), params=gpu_params(itf), device=dev).setup()
    D, M, g = MortarFunction.apply(Xs, Xm, iface)
    gen = torch.Generator(device="cpu").manual_seed(5)
    wD = torch.randn(D.shape, generator=gen, dtype=torch.float64).to(dev)
    wM = torch.randn(M.shape, generator=gen, dtype=torch.float64).to(dev)
    wg = torch.randn(g.shape, generator=gen, dtype=torch.float64).to(dev)
    L = (wD * D).sum() + (wM * M).sum() + (wg * g).sum()
    L.backward()
    gs, gm = iface.backward(wD, wM, wg)
    assert torch.equal(Xs.grad, gs.t()) and torch.equal(Xm.grad, gm.t())


def test_autograd_two_forwards_before_backward():
    # a second forward at other coordinates (a line-search trial point) runs
    # before the first loss's backward: that gradient is still the one at the
    # first forward's coordinates, bitwise equal to a fresh interface there
    from paper_2202_03933_amd import MortarFunction, MortarInterface
    from tests.gpu_util import gpu_params
    itf = synth.interface_config(2, scale=48)
    dev = torch.device("cuda", 0)
    cs, cm = torch.from_numpy(itf.slave.conn), torch.from_numpy(itf.master.conn)
    X1s = torch.from_numpy(itf.slave.X).to(dev).requires_grad_(True)
    X1m = torch.from_numpy(itf.master.X).to(dev).requires_grad_(True)
    iface = MortarInterface(X1s.detach(), cs, X1m.detach(), cm, params=gpu_params(itf), device=dev).setup()
    D1, M1, g1 = MortarFunction.apply(X1s, X1m, iface)
    shift = torch.tensor([2e-4, -1e-4, 0.0], dtype=torch.float64, device=dev)
    X2s = X1s.detach().clone().requires_grad_(True)
    X2m = (X1m.detach() + shift).requires_grad_(True)
    D2, M2, g2 = MortarFunction.apply(X2s, X2m, iface)
    assert not torch.equal(M1, M2)
    gen = torch.Generator(device="cpu").manual_seed(11)
    wD = torch.randn(D1.shape, generator=gen, dtype=torch.float64).to(dev)
    wM = torch.randn(M1.shape, generator=gen, dtype=torch.float64).to(dev)
    wg = torch.randn(g1.shape, generator=gen, dtype=torch.float64).to(dev)
    ((wD * D1).sum() + (wM * M1).sum() + (wg * g1).sum()).backward()
    ref = MortarInterface(X1s.detach(), cs, X1m.detach(), cm, params=gpu_params(itf), device=dev).setup()
    assert ref.n_pairs == iface.n_pairs and ref.nnz_M == iface.nnz_M
    gs, gm = ref.backward(wD, wM, wg)
    torch.cuda.synchronize()
    assert torch.equal(X1s.grad, gs.t()) and torch.equal(X1m.grad, gm.t())


def _fused_vs_sequential(itf, dual=False, nodal=False, seed=3300):
    from paper_2202_03933_amd import MortarInterface
    from tests.gpu_util import csr_weights, gpu_params
    import scipy.sparse as sp
    dev = torch.device("cuda", 0)

    def make(single_stream=0):
        p = gpu_params(itf, dual=dual, nodal=nodal)
        p.single_stream = single_stream
        return MortarInterface(torch.from_numpy(itf.slave.X), torch.from_numpy(itf.slave.conn),
                               torch.from_numpy(itf.master.X), torch.from_numpy(itf.master.conn),
                               params=p, device=dev).setup()
    a, b, c = make(), make(), make(single_stream=1)
    ns, nm = a.n_slave_nodes, a.n_master_nodes
    D = sp.csr_matrix((np.zeros(a.nnz_D), a.D_col.cpu().numpy(), a.D_rowptr.cpu().numpy()), shape=(ns, ns))
    M = sp.csr_matrix((np.zeros(a.nnz_M), a.M_col.cpu().numpy(), a.M_rowptr.cpu().numpy()), shape=(ns, nm))
    W = tuple(torch.from_numpy(x).to(dev) for x in csr_weights(D, M, ns, seed))
    rng = np.random.default_rng(seed)
    for step in range(2):
        if step == 1:  # moved in place: polygons and blocks recomputed inside the calls
            Xs = itf.slave.X + rng.uniform(-1e-5, 1e-5, itf.slave.X.shape)
            a.move_coordinates(Xs, itf.master.X)
            b.move_coordinates(Xs, itf.master.X)
            c.move_coordinates(Xs, itf.master.X)
        f_seq = tuple(t.clone() for t in a.integrate())
        g_seq = tuple(t.clone() for t in a.backward(*W))
        f_fus, g_fus = b.integrate_backward(*W)
        # every kernel on the caller's stream: the same values
        f_one, g_one = c.integrate_backward(*W)
        torch.cuda.synchronize()
        assert all(torch.equal(x, y) for x, y in zip(f_seq, f_fus)), step
        assert all(torch.equal(x, y) for x, y in zip(g_seq, g_fus)), step
        assert all(torch.equal(x, y) for x, y in zip(f_seq, f_one)), step
        assert all(torch.equal(x, y) for x, y in zip(g_seq, g_one)), step


# mt_integrate_backward (assembly beside the reverse sweep) equals
# mt_integrate followed by mt_backward bit for bit, and so does a context
# that runs every kernel on the caller's stream: standard and dual basis,
# the continuous normal field, before and after an in-place coordinate move.
@pytest.mark.parametrize("dual,nodal", [(False, False), (True, False), (False, True), (True, True)])
def test_integrate_backward_equals_sequential(dual, nodal):
    _fused_vs_sequential(synth.interface_config(1, scale=56), dual=dual, nodal=nodal)


def test_integrate_backward_equals_sequential_full_wavy():
    _fused_vs_sequential(synth.interface_config(2))


def test_backward_bitwise_deterministic():
    itf = synth.interface_config(1, scale=80)
    a = gpu_run(itf, backward_seed=7)
    b = gpu_run(itf, backward_seed=7)
    assert np.array_equal(a["gXs"], b["gXs"]) and np.array_equal(a["gXm"], b["gXm"])


def test_error_codes():
    from paper_2202_03933_amd import MortarError, MortarInterface, default_params
    from paper_2202_03933_amd import _capi as C
    itf = synth.interface_config(0)
    dev = torch.device("cuda", 0)
    iface = MortarInterface(torch.from_numpy(itf.slave.X), torch.from_numpy(itf.slave.conn),
                            torch.from_numpy(itf.master.X), torch.from_numpy(itf.master.conn),
                            params=default_params(dual=True), device=dev)
    # integrate before any build: the library reports the state (the binding
    # checks the gap buffer's length, which it knows, and not D and M, whose
    # lengths no build has counted yet); a short gap buffer never reaches it
    one = torch.empty(1, dtype=torch.float64, device=dev)
    with pytest.raises(MortarError) as e:
        iface.integrate(out=(one, one, torch.empty(itf.slave.n_nodes, dtype=torch.float64, device=dev)))
    assert e.value.code == C.MT_ESTATE
    with pytest.raises(ValueError):
        iface.integrate(out=(one, one, one))
    p = default_params()
    p.single_stream = 2
    assert C.lib().mt_set_params(iface.h, ctypes.byref(p)) == C.MT_EINVAL
    iface.setup()
    # connectivity out of range is reported by the upload, not read
    bad = itf.slave.conn.copy()
    bad[3, 2] = itf.slave.n_nodes + 5
    with pytest.raises(MortarError) as e:
        MortarInterface(torch.from_numpy(itf.slave.X), torch.from_numpy(bad), torch.from_numpy(itf.master.X),
                        torch.from_numpy(itf.master.conn), device=dev)
    assert e.value.code == C.MT_EINVAL


# Meshes numbered in random order (nodes and elements of both sides): the
# forward matches the oracle on the renumbered meshes, and the gradients, with
# each upstream weight attached to the same pair of original nodes, are those
# of the original numbering up to the order of summation.  The rows a
# workgroup of the CSR-position pass needs are then far apart, so it searches
# them in global memory instead of a staged span.
def test_renumbered_meshes_forward_and_gradients():
    from synth.weights import keyed_normal, TAG_D, TAG_M, TAG_G
    base = synth.interface_config(2, scale=53)
    itf = synth.renumbered(base, seed=11)
    g_new = gpu_run(itf)
    assert_forward_parity(g_new, oracle.evaluate(itf, oracle_params(itf)))
    g_old = gpu_run(base)
    ps, pm = itf.meta["new_of_old"]
    ident_s, ident_m = np.arange(base.slave.n_nodes), np.arange(base.master.n_nodes)
    old_s, old_m = np.argsort(ps), np.argsort(pm)  # original index of each new node
    dev = torch.device("cuda", 0)

    def grads(run, os_, om_):
        D, M = run["D"], run["M"]
        Dr = np.repeat(np.arange(D.shape[0]), np.diff(D.indptr))
        Mr = np.repeat(np.arange(M.shape[0]), np.diff(M.indptr))
        idx = np.arange(D.shape[0])
        W = (keyed_normal(5, TAG_D, os_[Dr], os_[D.indices]), keyed_normal(5, TAG_M, os_[Mr], om_[M.indices]),
             keyed_normal(5, TAG_G, os_[idx], 0 * idx))
        gs, gm = run["iface"].backward(*(torch.from_numpy(w).to(dev) for w in W))
        torch.cuda.synchronize()
        return gs.cpu().numpy(), gm.cpu().numpy()

    gs_old, gm_old = grads(g_old, ident_s, ident_m)
    gs_new, gm_new = grads(g_new, old_s, old_m)
    assert np.abs(gs_new[:, ps] - gs_old).max() <= 1e-12 * np.abs(gs_old).max()
    assert np.abs(gm_new[:, pm] - gm_old).max() <= 1e-12 * np.abs(gm_old).max()
    # the values themselves, renumbered back
    Dn, Mn = g_new["D"][ps][:, ps], g_new["M"][ps][:, pm]
    assert abs(Dn - g_old["D"]).max() <= 1e-13 * abs(g_old["D"]).max()
    assert abs(Mn - g_old["M"]).max() <= 1e-13 * abs(g_old["M"]).max()
    np.testing.assert_allclose(g_new["g"][ps], g_old["g"], rtol=0, atol=1e-13 * np.abs(g_old["g"]).max())
