"""The build that allocates nothing (mt_build_pairs_static: the workspace is
the library's static device array) through the C ABI, against the build in
a caller workspace: same candidates, pairs, pattern, D, M, gap and
gradients bit for bit, on two builds in a row, the second with a smaller
interface; a context whose static build was superseded is refused; a
workspace beyond the array is refused before any launch."""

import ctypes

import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import csr_weights, gpu_params

pytestmark = pytest.mark.gpu


def _iface(itf):
    from paper_2202_03933_amd import MortarInterface
    dev = torch.device("cuda", 0)
    return MortarInterface(torch.from_numpy(itf.slave.X), torch.from_numpy(itf.slave.conn),
                           torch.from_numpy(itf.master.X), torch.from_numpy(itf.master.conn),
                           params=gpu_params(itf), device=dev)


def _outputs(it):
    import scipy.sparse as sp
    ns, nm = it.n_slave_nodes, it.n_master_nodes
    D = sp.csr_matrix((np.zeros(it.nnz_D), it.D_col.cpu().numpy(), it.D_rowptr.cpu().numpy()), shape=(ns, ns))
    M = sp.csr_matrix((np.zeros(it.nnz_M), it.M_col.cpu().numpy(), it.M_rowptr.cpu().numpy()), shape=(ns, nm))
    W = tuple(torch.from_numpy(a).to(it.device) for a in csr_weights(D, M, ns, 77))
    f = tuple(t.clone() for t in it.integrate())
    g = tuple(t.clone() for t in it.backward(*W))
    torch.cuda.synchronize()
    return (it.D_rowptr, it.D_col, it.M_rowptr, it.M_col) + f + g


def _static_build(it):
    from paper_2202_03933_amd import _capi as C
    nc, npairs = ctypes.c_int64(), ctypes.c_int64()
    rc = C.lib().mt_build_pairs_static(it.h, None, ctypes.byref(nc), ctypes.byref(npairs),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    C.check(rc)
    it.n_cand, it.n_pairs = nc.value, npairs.value
    it.csr_pattern()
    return it


def test_static_build_matches_workspace_build():
    from paper_2202_03933_amd import MortarError
    from paper_2202_03933_amd import _capi as C
    first = None
    for scale in (96, 40):  # the second call with a smaller interface
        itf = synth.interface_config(2, scale)
        print(f"[gpu] static scratch build: {itf.name}", flush=True)
        ref = _iface(itf).setup()
        it = _static_build(_iface(itf))
        assert (it.n_cand, it.n_pairs, it.nnz_D, it.nnz_M) == (ref.n_cand, ref.n_pairs, ref.nnz_D, ref.nnz_M)
        for x, y in zip(it.candidates() + it.pairs(), ref.candidates() + ref.pairs()):
            assert torch.equal(x, y)
        a, b = _outputs(it), _outputs(ref)
        assert all(torch.equal(x, y) for x, y in zip(a, b))
        it.check()
        if first is None:
            first = it
    # the first context's build was superseded by the second's
    with pytest.raises(MortarError) as e:
        first.integrate()
    assert e.value.code == C.MT_ESTATE


def test_static_build_refuses_more_than_the_array():
    from paper_2202_03933_amd import _capi as C
    it = _iface(synth.interface_config(2))
    nc, npairs = ctypes.c_int64(), ctypes.c_int64()
    rc = C.lib().mt_build_pairs_static(it.h, None, ctypes.byref(nc), ctypes.byref(npairs),
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == C.MT_ECAPACITY
    assert b"static scratch" in C.lib().mt_last_error()
