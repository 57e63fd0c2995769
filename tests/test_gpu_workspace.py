"""The boundary's memory and synchronisation contract, through the C ABI:
the library allocates nothing (a torch workspace sized by
mt_workspace_size), capacities exceeded are reported (MT_ECAPACITY with the
counts needed) and a rebuild with them equals a fresh search bit for bit,
the chain build -> pattern -> integrate -> backward runs without host waits
and equals the synchronous one bitwise, and the whole step on the large wavy
interface runs as one captured HIP graph replayed from torch-allocated
memory, also after the coordinates move in place."""

import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import csr_weights, gpu_params, oracle_params

pytestmark = pytest.mark.gpu


def _iface(itf, Xs=None, Xm=None):
    from paper_2202_03933_amd import MortarInterface
    dev = torch.device("cuda", 0)
    Xs = itf.slave.X if Xs is None else Xs
    Xm = itf.master.X if Xm is None else Xm
    print(f"[gpu] {itf.name}", flush=True)
    return MortarInterface(torch.as_tensor(Xs), torch.from_numpy(itf.slave.conn), torch.as_tensor(Xm),
                           torch.from_numpy(itf.master.conn), params=gpu_params(itf), device=dev)


def _weights(it, seed):
    import scipy.sparse as sp
    ns, nm = it.n_slave_nodes, it.n_master_nodes
    D = sp.csr_matrix((np.zeros(it.nnz_D), it.D_col.cpu().numpy(), it.D_rowptr.cpu().numpy()), shape=(ns, ns))
    M = sp.csr_matrix((np.zeros(it.nnz_M), it.M_col.cpu().numpy(), it.M_rowptr.cpu().numpy()), shape=(ns, nm))
    return tuple(torch.from_numpy(a).to(it.device) for a in csr_weights(D, M, ns, seed))


def test_capacity_exceeded_is_reported():
    from paper_2202_03933_amd import _capi as C
    L = C.lib()
    itf = synth.interface_config(2, scale=40)
    o = oracle.evaluate(itf, oracle_params(itf))
    it = _iface(itf)
    small = C.mt_capacity(1000, 100, 100, 1 << 12)
    n = ctypes.c_size_t()
    assert L.mt_workspace_size(it.h, ctypes.byref(small), ctypes.byref(n)) == C.MT_OK
    from paper_2202_03933_amd.interface import workspace
    ws, ptr = workspace(n.value, it.device)
    nc, npairs = ctypes.c_int64(), ctypes.c_int64()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # a workspace one byte short is refused before any launch
    assert L.mt_build_pairs(it.h, ctypes.byref(small), ctypes.c_void_p(ptr), n.value - 1, None, None,
                            s) == C.MT_ECAPACITY
    assert L.mt_build_pairs(it.h, ctypes.byref(small), ctypes.c_void_p(ptr + 8), n.value, None, None,
                            s) == C.MT_EINVAL
    rc = L.mt_build_pairs(it.h, ctypes.byref(small), ctypes.c_void_p(ptr), n.value, ctypes.byref(nc),
                          ctypes.byref(npairs), s)
    assert rc == C.MT_ECAPACITY
    need = C.mt_capacity()
    assert L.mt_required_capacity(it.h, ctypes.byref(need)) == C.MT_OK
    assert need.candidates == o["cand_s"].size
    # with the candidates fitting, the next build learns the screened and
    # pair counts; the wrapper's retry loop does exactly this
    it.set_capacity(candidates=need.candidates, screened=100, pairs=100, cells=1 << 12)
    it.setup()
    assert it.n_cand == o["cand_s"].size and it.n_pairs == o["pair_s"].size
    assert it.capacity.pairs == o["pair_s"].size  # enlarged to exactly what was needed
    ps, pm, pnv = (t.cpu().numpy() for t in it.pairs())
    assert np.array_equal(ps, o["pair_s"]) and np.array_equal(pm, o["pair_m"])
    assert np.array_equal(pnv, o["nverts"])
    it.check()


def test_async_chain_equals_sync():
    itf = synth.interface_config(1, scale=90)
    a = _iface(itf).setup()
    W = _weights(a, 5)
    fa = tuple(t.clone() for t in a.integrate())
    ga = tuple(t.clone() for t in a.backward(*W))
    b = _iface(itf)
    b.set_capacity(a.capacity)
    b.build_pairs(sync=False)
    b.csr_pattern(sync=False)
    out = tuple(torch.full_like(t, float("nan")) for t in fa)
    gout = tuple(torch.full_like(t, float("nan")) for t in ga)
    b.integrate(out=out)
    b.backward(*W, out=gout)
    torch.cuda.synchronize()
    b.check()
    assert all(torch.equal(x, y) for x, y in zip(out + gout, fa + ga))
    assert b.stats()["n_pairs"] == a.n_pairs


def _step(it, W, out, gout):
    it.build_pairs(sync=False)
    it.csr_pattern(sync=False)
    it.integrate(out=out)
    it.backward(*W, out=gout)


def _step_fused(it, W, out, gout):
    it.build_pairs(sync=False)
    it.csr_pattern(sync=False)
    it.integrate_backward(*W, out=out, grad_out=gout)


# The whole step captured into one HIP graph, with mt_integrate +
# mt_backward or with mt_integrate_backward (the assembly beside the reverse
# sweep on the library's internal stream, joined into the capture).
@pytest.mark.parametrize("fused", [False, True])
def test_graph_captured_whole_step_wavy1024(fused):
    step = _step_fused if fused else _step
    itf = synth.interface_config(2)
    dev = torch.device("cuda", 0)
    Xs = torch.from_numpy(itf.slave.X).to(dev)
    Xm = torch.from_numpy(itf.master.X).to(dev)
    it = _iface(itf, Xs, Xm).setup()
    W = _weights(it, 3000)
    ref = tuple(t.clone() for t in it.integrate()) + tuple(t.clone() for t in it.backward(*W))
    torch.cuda.synchronize()
    out = tuple(torch.empty_like(t) for t in ref[:3])
    gout = tuple(torch.empty_like(t) for t in ref[3:])
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step(it, W, out, gout)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        step(it, W, out, gout)
    print(f"[gpu] captured (fused={fused}); replaying", flush=True)
    for rep in range(3):
        for t in out + gout:
            t.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        it.check()
        assert all(torch.equal(x, y) for x, y in zip(out + gout, ref)), rep
        # eager work of the program between replays
        torch.cuda.synchronize()
        _ = (it.Xs * 2.0).sum().item()
    # Newton-like use: the coordinates move in place and the same graph
    # computes the new pair list and operators (fixed capacities); a move
    # small enough to keep the pattern, so that the same weights apply
    rng = np.random.default_rng(7)
    moved_m = itf.master.X + 1e-8 * rng.standard_normal(itf.master.X.shape)
    # the arrays the library reads: the interface's registered (3, n) copy
    it.Xm.copy_(torch.from_numpy(moved_m).t())
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    it.check()
    fresh = _iface(itf, itf.slave.X, moved_m)
    fresh.set_capacity(it.capacity)
    fresh.setup()
    assert (fresh.nnz_D, fresh.nnz_M) == (it.nnz_D, it.nnz_M)
    for x, y in zip((fresh.D_rowptr, fresh.D_col, fresh.M_rowptr, fresh.M_col),
                    (it.D_rowptr, it.D_col, it.M_rowptr, it.M_col)):
        assert torch.equal(x, y)
    f = tuple(t.clone() for t in fresh.integrate())
    gg = tuple(t.clone() for t in fresh.backward(*W))
    torch.cuda.synchronize()
    assert not torch.equal(out[1], ref[1])  # the replay did see the move
    assert all(torch.equal(x, y) for x, y in zip(out + gout, f + gg))
