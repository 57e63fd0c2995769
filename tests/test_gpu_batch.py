"""Batched evaluation of many interfaces (persistent launches, HIP graphs,
autotuned tiles): bitwise equal to one call per interface, and through it to
the oracle."""

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import (TOL, assert_rows_parity, csr_weights, gpu_params, oracle_params, rel_err, sampled_oracle,
                            weight_fns)

pytestmark = pytest.mark.gpu


def make_ifaces(instances, dual=False):
    from paper_2202_03933_amd import MortarInterface
    dev = torch.device("cuda", 0)
    out = []
    for itf in instances:
        it = MortarInterface(torch.from_numpy(itf.slave.X), torch.from_numpy(itf.slave.conn),
                             torch.from_numpy(itf.master.X), torch.from_numpy(itf.master.conn),
                             params=gpu_params(itf, dual=dual), device=dev).setup()
        out.append(it)
    return out


def weights_for(it, seed):
    import scipy.sparse as sp
    ns, nm = it.n_slave_nodes, it.n_master_nodes
    D = sp.csr_matrix((np.zeros(it.nnz_D), it.D_col.cpu().numpy(), it.D_rowptr.cpu().numpy()), shape=(ns, ns))
    M = sp.csr_matrix((np.zeros(it.nnz_M), it.M_col.cpu().numpy(), it.M_rowptr.cpu().numpy()), shape=(ns, nm))
    return tuple(torch.from_numpy(a).to(it.device) for a in csr_weights(D, M, ns, seed))


def equal_outs(a, b):
    return all(torch.equal(x, y) for x, y in zip(a, b))


def run_batch_checks(instances, autotune=True, dual=False):
    from paper_2202_03933_amd import MortarBatch
    ifaces = make_ifaces(instances, dual=dual)
    print(f"[gpu] batch of {len(ifaces)} interfaces, {sum(i.n_pairs for i in ifaces)} pairs", flush=True)
    ref = [tuple(t.clone() for t in it.integrate()) for it in ifaces]
    W = [weights_for(it, 4000 + k) for k, it in enumerate(ifaces)]
    ref_g = [tuple(t.clone() for t in it.backward(*w)) for it, w in zip(ifaces, W)]
    b = MortarBatch(ifaces)
    outs = b.forward()
    torch.cuda.synchronize()
    assert all(equal_outs(o, r) for o, r in zip(outs, ref))
    # graph replays, with eager work of the program between them
    outs2 = b.alloc_outputs()
    for rep in range(3):
        for o in outs2:
            for t in o:
                t.fill_(float("nan"))
        b.forward(outs2, use_graph=True)
        torch.cuda.synchronize()
        ifaces[rep % len(ifaces)].integrate()
        torch.cuda.synchronize()
        assert all(equal_outs(o, r) for o, r in zip(outs2, ref)), rep
    g = b.backward(W)
    torch.cuda.synchronize()
    assert all(equal_outs(x, r) for x, r in zip(g, ref_g))
    g2 = [(torch.empty_like(a), torch.empty_like(c)) for a, c in ref_g]
    for rep in range(3):
        b.backward(W, outs=g2, use_graph=True)
        torch.cuda.synchronize()
        ifaces[0].backward(*W[0])
        torch.cuda.synchronize()
        assert all(equal_outs(x, r) for x, r in zip(g2, ref_g)), rep
    if autotune:
        choice = b.autotune()
        print("autotuned", choice)
        assert choice["block"] in (64, 128, 256) and choice["blocks_per_cu"] >= 1 and choice["bucket"] >= 1
        outs3 = b.forward(use_graph=True)
        torch.cuda.synchronize()
        assert all(equal_outs(o, r) for o, r in zip(outs3, ref))
        g3 = b.backward(W, use_graph=True)
        torch.cuda.synchronize()
        assert all(equal_outs(x, r) for x, r in zip(g3, ref_g))
    return ifaces, outs, g


def test_batch_small_instances_bitwise_and_oracle():
    instances = synth.batched_instances(n_inst=9, max_side=40)
    ifaces, outs, grads = run_batch_checks(instances)
    # oracle parity of every instance through the batched outputs
    for itf, it, (D, M, gv), (gs, gm) in zip(instances, ifaces, outs, grads):
        prm = oracle_params(itf)
        o = oracle.evaluate(itf, prm)
        assert np.array_equal(it.D_col.cpu().numpy(), o["D"].indices)
        assert np.array_equal(it.M_col.cpu().numpy(), o["M"].indices)
        assert rel_err(D.cpu().numpy(), o["D"].data) <= TOL
        assert rel_err(M.cpu().numpy(), o["M"].data) <= TOL
        if np.linalg.norm(o["g"]) > 0:
            assert rel_err(gv.cpu().numpy(), o["g"]) <= TOL
        if itf.meta["geometry"] == "flat":
            continue  # tied flat boundaries: not differentiable (see test_gpu_backward)
        w = oracle.pair_weights(itf.slave, itf.master, o["pair_s"], o["pair_m"],
                                *weight_fns(4000 + itf.meta["instance"]))
        g24, _ = oracle.pair_grads(itf.slave, itf.master, prm, o["pair_s"], o["pair_m"], w)
        ogs, ogm = oracle.scatter_grads(itf.slave, itf.master, o["pair_s"], o["pair_m"], g24)
        assert rel_err(gs.cpu().numpy().T, ogs) <= TOL and rel_err(gm.cpu().numpy().T, ogm) <= TOL


def test_batch_dual_basis_bitwise_and_oracle():
    # dual basis: the batched backward recomputes the dual blocks and takes
    # the dual-coefficient adjoint; bitwise equal to one call per interface
    instances = synth.batched_instances(n_inst=9, max_side=40)
    ifaces, outs, grads = run_batch_checks(instances, autotune=False, dual=True)
    for itf, it, (gs, gm) in zip(instances, ifaces, grads):
        if itf.meta["geometry"] == "flat":
            continue
        prm = oracle_params(itf, dual=True)
        o = oracle.evaluate(itf, prm)
        w = oracle.pair_weights(itf.slave, itf.master, o["pair_s"], o["pair_m"],
                                *weight_fns(4000 + itf.meta["instance"]))
        g24, _ = oracle.pair_grads(itf.slave, itf.master, prm, o["pair_s"], o["pair_m"], w)
        ogs, ogm = oracle.scatter_grads(itf.slave, itf.master, o["pair_s"], o["pair_m"], g24)
        assert rel_err(gs.cpu().numpy().T, ogs) <= TOL and rel_err(gm.cpu().numpy().T, ogm) <= TOL


def test_batch_full_64_instances_bitwise():
    import scipy.sparse as sp
    instances = synth.batched_instances(n_inst=64)
    ifaces, outs, grads = run_batch_checks(instances, autotune=False)
    # the three largest instances against the oracle at sampled nodes
    big = sorted(range(len(instances)), key=lambda i: -instances[i].slave.n_el)[:3]
    for i in big:
        itf, it, (D, M, gv), (gs, gm) = instances[i], ifaces[i], outs[i], grads[i]
        print(f"[gpu] batch instance {i}: {itf.name}, {it.n_pairs} pairs", flush=True)
        prm = oracle_params(itf)
        rng = np.random.default_rng(5000 + i)
        sn = rng.choice(itf.slave.n_nodes, 150, replace=False)
        mn = rng.choice(itf.master.n_nodes, 150, replace=False)
        flat = itf.meta["geometry"] == "flat"
        o = sampled_oracle(itf, prm, sn, mn, seed=None if flat else 4000 + i)
        ns, nm = itf.slave.n_nodes, itf.master.n_nodes
        Dc = sp.csr_matrix((D.cpu().numpy(), it.D_col.cpu().numpy(), it.D_rowptr.cpu().numpy()), shape=(ns, ns))
        Mc = sp.csr_matrix((M.cpu().numpy(), it.M_col.cpu().numpy(), it.M_rowptr.cpu().numpy()), shape=(ns, nm))
        assert_rows_parity(Dc, Mc, gv.cpu().numpy(), o, sn)
        if not flat:  # tied flat boundaries: not differentiable
            assert rel_err(gs.cpu().numpy().T[sn], o["gXs"][sn]) <= TOL
            assert rel_err(gm.cpu().numpy().T[mn], o["gXm"][mn]) <= TOL


def test_batch_rejects_mixed_rules_and_graph_on_default_stream():
    from paper_2202_03933_amd import MortarBatch, MortarError, MortarInterface, default_params
    from paper_2202_03933_amd import _capi as C
    import ctypes
    dev = torch.device("cuda", 0)
    a, b = synth.flat_tied(4, 3, seed=1), synth.flat_tied(5, 4, seed=2)
    ia = make_ifaces([a])[0]
    ib = MortarInterface(torch.from_numpy(b.slave.X), torch.from_numpy(b.slave.conn), torch.from_numpy(b.master.X),
                         torch.from_numpy(b.master.conn), params=default_params(rule=3), device=dev).setup()
    with pytest.raises(MortarError) as e:
        MortarBatch([ia, ib])
    assert e.value.code == C.MT_EINVAL
    bt = MortarBatch([ia])
    outs = bt.alloc_outputs()
    from paper_2202_03933_amd.batch import _ptr_table
    tabs = [_ptr_table([o[k] for o in outs]) for k in range(3)]
    rc = C.lib().mt_batch_forward(bt.h, *tabs, 1, ctypes.c_void_p(0))
    assert rc == C.MT_EINVAL


def _moved(itf, step):
    """The instance with its master slid tangentially by 0.37 (step + 1) of
    a master element (along the cylinder axis, else along x): the pair lists
    change from step to step."""
    from synth.meshes import Interface, Mesh
    Xm = itf.master.X.copy()
    c = itf.master.conn
    h = float(np.linalg.norm(Xm[c[:, 1]] - Xm[c[:, 0]], axis=1).mean())
    d = 2 if itf.meta["geometry"] == "cylinder" else 0
    Xm[:, d] += 0.37 * h * (step + 1)
    return Interface(itf.slave, Mesh(Xm, c), itf.delta, name=itf.name + f", moved {step}", meta=itf.meta)


# The search of all instances in one call (Alg. 1 and 2 per instance, then
# the pattern) while the instances move, eagerly and as a HIP graph captured
# at the first step and replayed at the next two: candidates, pairs, patterns
# and the batched forward and backward after it bitwise equal to fresh
# per-interface builds at the moved coordinates.
@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_search_moving_instances(use_graph):
    from paper_2202_03933_amd import MortarBatch
    instances = synth.batched_instances(n_inst=12, max_side=48)
    ifaces = make_ifaces(instances)
    b = MortarBatch(ifaces)
    for step in range(3):
        moved = [_moved(itf, step) for itf in instances]
        print(f"[gpu] batched search, graph={use_graph}, step {step}", flush=True)
        for it, itf in zip(ifaces, moved):
            it.move_coordinates(itf.slave.X, itf.master.X)
        b.search(use_graph=use_graph)
        refs = make_ifaces(moved)
        for it, ref in zip(ifaces, refs):
            assert (it.n_cand, it.n_pairs, it.nnz_D, it.nnz_M) == (ref.n_cand, ref.n_pairs, ref.nnz_D, ref.nnz_M)
            for x, y in zip(it.candidates() + it.pairs(), ref.candidates() + ref.pairs()):
                assert torch.equal(x, y)
            for x, y in zip((it.D_rowptr, it.D_col, it.M_rowptr, it.M_col),
                            (ref.D_rowptr, ref.D_col, ref.M_rowptr, ref.M_col)):
                assert torch.equal(x, y)
        outs = b.forward(use_graph=use_graph)
        ref_out = [tuple(t.clone() for t in r.integrate()) for r in refs]
        W = [weights_for(r, 4100 + k) for k, r in enumerate(refs)]
        g = b.backward(W, use_graph=use_graph)
        ref_g = [tuple(t.clone() for t in r.backward(*w)) for r, w in zip(refs, W)]
        torch.cuda.synchronize()
        assert all(equal_outs(o, r) for o, r in zip(outs, ref_out)), step
        assert all(equal_outs(x, r) for x, r in zip(g, ref_g)), step


def _assert_same_search(ifaces, refs):
    for it, ref in zip(ifaces, refs):
        assert (it.n_cand, it.n_pairs, it.nnz_D, it.nnz_M) == (ref.n_cand, ref.n_pairs, ref.nnz_D, ref.nnz_M)
        for x, y in zip(it.candidates() + it.pairs(), ref.candidates() + ref.pairs()):
            assert torch.equal(x, y)
        for x, y in zip((it.D_rowptr, it.D_col, it.M_rowptr, it.M_col),
                        (ref.D_rowptr, ref.D_col, ref.M_rowptr, ref.M_col)):
            assert torch.equal(x, y)


# The captured search is replayed only while what it was captured from holds:
# an instance bound to other capacities (a new workspace layout) makes the
# next graph search capture again, with the same results as fresh builds;
# the eager search in between leaves the graph alone.
def test_batch_search_graph_recaptured_after_rebind():
    from paper_2202_03933_amd import MortarBatch
    instances = synth.batched_instances(n_inst=6, max_side=40)
    ifaces = make_ifaces(instances)
    b = MortarBatch(ifaces)
    b.search(use_graph=True)
    _assert_same_search(ifaces, make_ifaces(instances))
    it0 = ifaces[0]
    it0.set_capacity(pairs=it0.capacity.pairs + 4096)
    it0.build_pairs()
    for step in range(3):  # graph (captured again), eager, graph (replayed)
        moved = [_moved(itf, step) for itf in instances]
        print(f"[gpu] graph search after a rebind, step {step}", flush=True)
        for it, itf in zip(ifaces, moved):
            it.move_coordinates(itf.slave.X, itf.master.X)
        b.search(use_graph=step != 1)
        refs = make_ifaces(moved)
        _assert_same_search(ifaces, refs)
        outs = b.forward()
        ref_out = [tuple(t.clone() for t in r.integrate()) for r in refs]
        torch.cuda.synchronize()
        assert all(equal_outs(o, r) for o, r in zip(outs, ref_out)), step
        # an instance's own calls after the batched search: its host state
        # (pair list, pattern, generations) is that of a search call
        W = weights_for(refs[1], 4200 + step)
        own = tuple(t.clone() for t in ifaces[1].integrate()) + tuple(t.clone() for t in ifaces[1].backward(*W))
        ref = tuple(t.clone() for t in refs[1].integrate()) + tuple(t.clone() for t in refs[1].backward(*W))
        torch.cuda.synchronize()
        assert equal_outs(own, ref), step


# Instances that run every kernel on the caller's stream (single_stream) in
# a batch: the batched search (eager, then captured and replayed), forward
# and backward equal fresh builds with the internal streams bit for bit.
def test_batch_single_stream_instances():
    from paper_2202_03933_amd import MortarBatch, MortarInterface
    dev = torch.device("cuda", 0)
    instances = synth.batched_instances(n_inst=6, max_side=40)
    ifaces = []
    for itf in instances:
        p = gpu_params(itf)
        p.single_stream = 1
        ifaces.append(MortarInterface(torch.from_numpy(itf.slave.X), torch.from_numpy(itf.slave.conn),
                                      torch.from_numpy(itf.master.X), torch.from_numpy(itf.master.conn),
                                      params=p, device=dev).setup())
    b = MortarBatch(ifaces)
    for step in range(3):  # eager, graph (captured), graph (replayed)
        moved = [_moved(itf, step) for itf in instances]
        print(f"[gpu] batch of single-stream instances, step {step}", flush=True)
        for it, itf in zip(ifaces, moved):
            it.move_coordinates(itf.slave.X, itf.master.X)
        b.search(use_graph=step > 0)
        refs = make_ifaces(moved)
        _assert_same_search(ifaces, refs)
        outs = b.forward(use_graph=step > 0)
        ref_out = [tuple(t.clone() for t in r.integrate()) for r in refs]
        W = [weights_for(r, 4400 + k) for k, r in enumerate(refs)]
        g = b.backward(W, use_graph=step > 0)
        ref_g = [tuple(t.clone() for t in r.backward(*w)) for r, w in zip(refs, W)]
        torch.cuda.synchronize()
        assert all(equal_outs(o, r) for o, r in zip(outs, ref_out)), step
        assert all(equal_outs(x, r) for x, r in zip(g, ref_g)), step
    b.close()
