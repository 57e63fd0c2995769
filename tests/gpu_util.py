"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
on a synthetic interface and compare with the oracle."""

import numpy as np
import scipy.sparse as sp
import torch

import oracle
from synth.weights import keyed_normal, TAG_D, TAG_M, TAG_G

TOL = 1e-10  # relative Frobenius error bar for D, M, gap and gradients


def gpu_params(itf, dual=False, rule=7, element_rule=0, nodal=False):
    from paper_2202_03933_amd import default_params
    return default_params(delta=float(itf.delta), dual=dual, rule=rule, element_rule=element_rule,
                          nodal_normals=nodal)


def oracle_params(itf, dual=False, rule=7, nodal=False):
    return oracle.params(delta=itf.delta, dual=dual, rule=rule, nodal_normals=nodal)


def gpu_run(itf, dual=False, rule=7, backward_seed=None, element_rule=0, nodal=False):
    """Full HIP path; returns numpy results."""
    from paper_2202_03933_amd import MortarInterface
    print(f"[gpu] {itf.name} dual={dual} rule={rule} element_rule={element_rule} nodal={nodal}", flush=True)
    dev = torch.device("cuda", 0)
    iface = MortarInterface(torch.from_numpy(itf.slave.X), torch.from_numpy(itf.slave.conn),
                            torch.from_numpy(itf.master.X), torch.from_numpy(itf.master.conn),
                            params=gpu_params(itf, dual, rule, element_rule, nodal), device=dev)
    iface.build_pairs()
    cs, cm, cnv = (t.cpu().numpy() for t in iface.candidates())
    ps, pm, pnv = (t.cpu().numpy() for t in iface.pairs())
    iface.csr_pattern()
    D, M, g = iface.integrate()
    torch.cuda.synchronize()
    ns, nmn = itf.slave.n_nodes, itf.master.n_nodes
    Dc = sp.csr_matrix((D.cpu().numpy(), iface.D_col.cpu().numpy(), iface.D_rowptr.cpu().numpy()), shape=(ns, ns))
    Mc = sp.csr_matrix((M.cpu().numpy(), iface.M_col.cpu().numpy(), iface.M_rowptr.cpu().numpy()), shape=(ns, nmn))
    out = {"iface": iface, "cand_s": cs, "cand_m": cm, "cand_nv": cnv, "pair_s": ps, "pair_m": pm, "nverts": pnv,
           "D": Dc, "M": Mc, "g": g.cpu().numpy(), "stats": iface.stats()}
    if backward_seed is not None:
        wD, wM, wg = csr_weights(Dc, Mc, ns, backward_seed)
        gs, gm = iface.backward(torch.from_numpy(wD).to(dev), torch.from_numpy(wM).to(dev),
                                torch.from_numpy(wg).to(dev))
        torch.cuda.synchronize()
        out["gXs"] = gs.cpu().numpy().T.copy()
        out["gXm"] = gm.cpu().numpy().T.copy()
    return out


def csr_weights(D, M, n_slave_nodes, seed):
    """Keyed N(0,1) weights on the nonzeros of D, M (CSR order) and on nodes."""
    Dr = np.repeat(np.arange(D.shape[0]), np.diff(D.indptr))
    Mr = np.repeat(np.arange(M.shape[0]), np.diff(M.indptr))
    wD = keyed_normal(seed, TAG_D, Dr, D.indices)
    wM = keyed_normal(seed, TAG_M, Mr, M.indices)
    idx = np.arange(n_slave_nodes)
    wg = keyed_normal(seed, TAG_G, idx, np.zeros_like(idx))
    return wD, wM, wg


def weight_fns(seed):
    return (lambda r, c: keyed_normal(seed, TAG_D, r, c),
            lambda r, c: keyed_normal(seed, TAG_M, r, c),
            lambda r: keyed_normal(seed, TAG_G, r, np.zeros_like(r)))


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    d = np.linalg.norm(a - b)
    if nb == 0.0:
        return d
    return d / nb


def assert_same_pattern(A, B):
    assert A.shape == B.shape
    assert np.array_equal(A.indptr, B.indptr), "row pointers differ"
    assert np.array_equal(A.indices, B.indices), "column indices differ"


def assert_forward_parity(g, o):
    """Bit-exact candidates / pairs / vertex counts / pattern; values within TOL."""
    assert np.array_equal(g["cand_s"], o["cand_s"]) and np.array_equal(g["cand_m"], o["cand_m"]), "candidates"
    assert np.array_equal(g["cand_nv"], o["cand_nverts"]), "clip vertex counts"
    assert np.array_equal(g["pair_s"], o["pair_s"]) and np.array_equal(g["pair_m"], o["pair_m"]), "pairs"
    assert np.array_equal(g["nverts"], o["nverts"])
    hist = np.bincount(o["cand_nverts"].astype(np.int64), minlength=17)
    assert list(hist) == list(g["stats"]["nverts_hist"]), "vertex-count histogram"
    assert_same_pattern(g["D"], o["D"])
    assert_same_pattern(g["M"], o["M"])
    eD = rel_err(g["D"].data, o["D"].data)
    eM = rel_err(g["M"].data, o["M"].data)
    eg = rel_err(g["g"], o["g"])
    assert eD <= TOL and eM <= TOL, (eD, eM)
    if np.linalg.norm(o["g"]) == 0.0:
        assert np.abs(g["g"]).max() <= 1e-15 * max(1.0, np.abs(o["D"].data).max())
    else:
        assert eg <= TOL, eg
    return eD, eM, eg


def window_oracle(itf, els, prm, elements=None):
    """Oracle on the slave elements `els` only (against the whole master
    side): returns the oracle results with global slave element indices in
    'pair_s' and the slave nodes whose rows it computes completely (every
    incident slave element lies in the window)."""
    from synth.meshes import Interface, Mesh
    els = np.asarray(els)
    sub = Interface(Mesh(itf.slave.X, itf.slave.conn[els]), itf.master, itf.delta)
    o = oracle.evaluate(sub, prm) if elements is None else oracle.evaluate_elements(sub, elements, prm)
    o["pair_s"] = els[o["pair_s"]]
    cnt = np.bincount(itf.slave.conn.ravel(), minlength=itf.slave.n_nodes)
    cnt_w = np.bincount(itf.slave.conn[els].ravel(), minlength=itf.slave.n_nodes)
    nodes = np.nonzero((cnt_w == cnt) & (cnt > 0))[0]
    return o, nodes


def assert_rows_parity(D, M, g, o, nodes):
    """Rows `nodes` of GPU CSR D, M and gap against the oracle's: same
    pattern, values within TOL."""
    for A, B in ((D, o["D"]), (M, o["M"])):
        A, B = A[nodes], B[nodes]
        assert_same_pattern(A, B)
        assert rel_err(A.data, B.data) <= TOL
    if np.linalg.norm(o["g"][nodes]) > 0:
        assert rel_err(g[nodes], o["g"][nodes]) <= TOL


def sampled_oracle(itf, prm, sn, mn, seed=None):
    """Oracle values at sampled nodes without evaluating every pair: the pair
    list of the whole interface (search + clip only), then the blocks of the
    pairs whose slave element holds a node of `sn` (complete rows of D, M and
    gap for those nodes) and, with `seed`, the keyed-weight gradient of the
    pairs touching `sn` or `mn` (complete for those nodes)."""
    cs, cm = oracle.search(itf.slave, itf.master, prm.delta)
    nv, _, _ = oracle.eval_candidates(itf.slave, itf.master, prm, cs, cm, integrate=False)
    keep = nv >= 3
    ps, pm = cs[keep], cm[keep]
    out = {"pair_s": ps, "pair_m": pm}
    rows = np.isin(itf.slave.conn[ps], sn).any(1)
    _, blocks, st = oracle.eval_candidates(itf.slave, itf.master, prm, ps[rows], pm[rows])
    out["D"], out["M"], out["g"] = oracle.assemble(itf.slave, itf.master, ps[rows], pm[rows], blocks)
    if seed is not None:
        sel = rows | np.isin(itf.master.conn[pm], mn).any(1)
        w = oracle.pair_weights(itf.slave, itf.master, ps[sel], pm[sel], *weight_fns(seed))
        g24, _ = oracle.pair_grads(itf.slave, itf.master, prm, ps[sel], pm[sel], w)
        out["gXs"], out["gXm"] = oracle.scatter_grads(itf.slave, itf.master, ps[sel], pm[sel], g24)
    return out
