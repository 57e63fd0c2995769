"""CPU oracle of the mortar coupling path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding)
never does.  The arithmetic lives in `mortar_oracle.cpp`, a plain serial FP64
implementation written from the paper (see its header); this module builds
it with g++, binds it with ctypes and assembles the per-pair blocks into
sparse matrices with scipy (coordinate format summed into CSR).

Parity status: every function here is pinned by tests under `tests/`
(worked example of Fig. 1, hand-worked pairs, exact rational integration,
brute-force search, invariants, closed forms and finite differences).
"""

import ctypes
import os
import subprocess

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mortar_oracle.cpp")
_SO = os.path.join(_HERE, "_mortar_oracle.so")

_lib_handle = None


def build(force=True):
    """Compile the oracle with g++ (FP64, no fused multiply-add, no fast-math)."""
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-o", _SO + ".tmp", _SRC]
    subprocess.check_call(cmd)
    os.replace(_SO + ".tmp", _SO)


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        i64, i32, dbl, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
        lib.or_search.argtypes = [ctypes.c_int, i64, vp, i64, vp, i64, vp, i64, vp, dbl, i64, vp, vp, vp]
        lib.or_eval_candidates.argtypes = [i64, vp, i64, vp, i64, vp, i64, vp, vp, i64, vp, vp, vp, vp, vp]
        lib.or_pair_grads.argtypes = [i64, vp, i64, vp, i64, vp, i64, vp, vp, i64, vp, vp, vp, vp, vp, vp]
        lib.or_normal_chain.argtypes = [i64, vp, i64, vp, vp, vp]
        lib.or_nodal_normals.argtypes = [i64, vp, i64, vp, vp, vp]
        lib.or_nodal_normals.restype = None
        lib.or_count_flops.argtypes = [i64, vp, i64, vp, i64, vp, i64, vp, vp, i64, vp, vp, vp]
        lib.or_count_flops.restype = None
        lib.or_pair_polygon.argtypes = [vp, vp, vp, vp, vp, vp]
        lib.or_clip2d.argtypes = [ctypes.c_int, vp, vp, ctypes.c_int, vp, vp, dbl, vp, vp, vp, vp, vp]
        lib.or_fan_points.argtypes = [ctypes.c_int, vp, vp, ctypes.c_int, vp, vp, vp]
        lib.or_rule.argtypes = [ctypes.c_int, vp, vp]
        lib.or_inverse_bilinear.argtypes = [vp, vp, dbl, dbl, vp, vp, vp]
        lib.or_dual_matrix.argtypes = [vp, vp]
        lib.or_dual_matrix.restype = None
        lib.or_gauss_legendre.argtypes = [ctypes.c_int, vp, vp]
        lib.or_gauss_legendre.restype = None
        lib.or_eval_elements.argtypes = [i64, vp, i64, vp, i64, vp, i64, vp, vp, ctypes.c_int, i64, vp, vp, vp, vp]
        lib.or_count_flops_elements.argtypes = [i64, vp, i64, vp, i64, vp, i64, vp, vp, ctypes.c_int, i64, vp, vp]
        lib.or_count_flops_elements.restype = ctypes.c_uint64
        _lib_handle = lib
    return _lib_handle


class OrParams(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_double), ("dual", ctypes.c_int32), ("rule", ctypes.c_int32),
                ("eps_d", ctypes.c_double), ("eps_a", ctypes.c_double),
                ("newton_tol", ctypes.c_double), ("newton_maxit", ctypes.c_int32),
                ("normals", ctypes.c_int32)]


def params(delta=0.0, dual=False, rule=7, eps_d=1e-12, eps_a=1e-12, newton_tol=1e-14,
           newton_maxit=30, nodal_normals=False):
    """nodal_normals: auxiliary planes from the averaged nodal normal field
    instead of each element's own normal."""
    return OrParams(float(delta), int(bool(dual)), int(rule), float(eps_d), float(eps_a),
                    float(newton_tol), int(newton_maxit), int(bool(nodal_normals)))


ST_NOCONV, ST_OVERFLOW, ST_DEGEN_SLAVE, ST_DEGEN_MASTER = 1, 2, 4, 8


def capacity():
    """Size of the vertex buffers the polygon helpers below pass (the
    oracle's own clip polygons are growable)."""
    return int(_lib().or_capacity())


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _mesh_args(slave, master):
    Xs = np.ascontiguousarray(slave.X, dtype=np.float64)
    Cs = np.ascontiguousarray(slave.conn, dtype=np.int32)
    Xm = np.ascontiguousarray(master.X, dtype=np.float64)
    Cm = np.ascontiguousarray(master.conn, dtype=np.int32)
    keep = (Xs, Cs, Xm, Cm)
    args = [Xs.shape[0], _p(Xs), Cs.shape[0], _p(Cs), Xm.shape[0], _p(Xm), Cm.shape[0], _p(Cm)]
    return args, keep


def search(slave, master, delta, method="binned"):
    """Candidate pairs (slave element, master element), sorted by (s, m)."""
    args, keep = _mesh_args(slave, master)
    cap = max(1024, 64 * (slave.n_el + master.n_el))
    while True:
        cs = np.empty(cap, np.int32)
        cm = np.empty(cap, np.int32)
        n = ctypes.c_int64(0)
        rc = _lib().or_search(0 if method == "brute" else 1, *args, float(delta), cap, _p(cs), _p(cm),
                              ctypes.byref(n))
        if rc == 0:
            return cs[: n.value].copy(), cm[: n.value].copy()
        cap = int(n.value)


def eval_candidates(slave, master, prm, cs, cm, integrate=True):
    """Vertex counts, local blocks (n, 36) and status bits per candidate."""
    args, keep = _mesh_args(slave, master)
    cs = np.ascontiguousarray(cs, np.int32)
    cm = np.ascontiguousarray(cm, np.int32)
    n = cs.size
    nv = np.zeros(n, np.uint8)
    st = np.zeros(n, np.int32)
    blocks = np.zeros((n, 36), np.float64) if integrate else None
    _lib().or_eval_candidates(*args, ctypes.byref(prm), n, _p(cs), _p(cm), _p(nv),
                              _p(blocks) if integrate else None, _p(st))
    return nv, blocks, st


def assemble(slave, master, ps, pm, blocks):
    """Sum local blocks of the pairs (ps, pm) into CSR D, M and the gap.

    The sparsity pattern is the union of the 4x4 blocks of all pairs
    (structural zeros kept), columns sorted.
    """
    Cs = slave.conn[ps]  # (n, 4)
    Cm = master.conn[pm]
    n = ps.size
    rD = np.repeat(Cs, 4, axis=1).reshape(-1)
    cD = np.tile(Cs, (1, 4)).reshape(-1)
    rM = np.repeat(Cs, 4, axis=1).reshape(-1)
    cM = np.tile(Cm, (1, 4)).reshape(-1)
    D = sp.coo_matrix((blocks[:, :16].reshape(-1), (rD, cD)),
                      shape=(slave.n_nodes, slave.n_nodes)).tocsr()
    M = sp.coo_matrix((blocks[:, 16:32].reshape(-1), (rM, cM)),
                      shape=(slave.n_nodes, master.n_nodes)).tocsr()
    D.sort_indices()
    M.sort_indices()
    g = np.zeros(slave.n_nodes)
    np.add.at(g, Cs.reshape(-1), blocks[:, 32:36].reshape(-1))
    assert n == 0 or D.nnz > 0
    return D, M, g


def evaluate(itf, prm=None, method="binned"):
    """Whole path on one interface: search, per-pair evaluation, assembly."""
    if prm is None:
        prm = params(delta=itf.delta)
    cs, cm = search(itf.slave, itf.master, prm.delta, method)
    nv, blocks, st = eval_candidates(itf.slave, itf.master, prm, cs, cm, integrate=True)
    keep = nv >= 3
    ps, pm = cs[keep], cm[keep]
    D, M, g = assemble(itf.slave, itf.master, ps, pm, blocks[keep])
    return {"cand_s": cs, "cand_m": cm, "cand_nverts": nv, "pair_s": ps, "pair_m": pm,
            "nverts": nv[keep], "blocks": blocks[keep], "status": st, "D": D, "M": M, "g": g}


def gauss_legendre(n):
    """Gauss-Legendre points and weights on [-1, 1] (ascending)."""
    x = np.zeros(n)
    w = np.zeros(n)
    _lib().or_gauss_legendre(int(n), _p(x), _p(w))
    return x, w


def eval_elements(slave, master, prm, ps, pm, ng):
    """Element-based integration: local blocks (n, 36) of the pairs (ps, pm),
    sorted by slave element, with an ng x ng Gauss rule per slave element;
    and the status bits per pair (those of its slave element)."""
    args, keep = _mesh_args(slave, master)
    ps = np.ascontiguousarray(ps, np.int32)
    pm = np.ascontiguousarray(pm, np.int32)
    assert np.all(np.diff(ps) >= 0)
    blocks = np.zeros((ps.size, 36))
    st = np.zeros(ps.size, np.int32)
    rc = _lib().or_eval_elements(*args, ctypes.byref(prm), int(ng), ps.size, _p(ps), _p(pm), _p(blocks), _p(st))
    if rc < 0:
        raise ValueError(f"element rule {ng} out of range 1..8")
    return blocks, st


def evaluate_elements(itf, ng, prm=None, pairs=None):
    """Element-based D, M and gap on the pair list of the segment-based
    search (the pairs whose clip polygon is a segment)."""
    if prm is None:
        prm = params(delta=itf.delta)
    if pairs is None:
        r = evaluate(itf, prm)
        pairs = (r["pair_s"], r["pair_m"])
    ps, pm = pairs
    blocks, st = eval_elements(itf.slave, itf.master, prm, ps, pm, ng)
    D, M, g = assemble(itf.slave, itf.master, ps, pm, blocks)
    return {"pair_s": ps, "pair_m": pm, "blocks": blocks, "status": st, "D": D, "M": M, "g": g}


def count_flops_elements(slave, master, prm, ps, pm, ng):
    """Counted flops of the element-based integration of the pairs (ps, pm)."""
    args, keep = _mesh_args(slave, master)
    ps = np.ascontiguousarray(ps, np.int32)
    pm = np.ascontiguousarray(pm, np.int32)
    return int(_lib().or_count_flops_elements(*args, ctypes.byref(prm), int(ng), ps.size, _p(ps), _p(pm)))


def pair_grads(slave, master, prm, ps, pm, w36, with_n0=False):
    """d(<w, blocks>)/d(24 nodal coordinates) per pair, forward-mode exact;
    with_n0 also returns d/d(element normal n0) per pair (n, 3), the input
    the nodal normal field adds (params(nodal_normals=True))."""
    args, keep = _mesh_args(slave, master)
    ps = np.ascontiguousarray(ps, np.int32)
    pm = np.ascontiguousarray(pm, np.int32)
    w36 = np.ascontiguousarray(w36, np.float64)
    n = ps.size
    out = np.zeros((n, 24))
    gn0 = np.zeros((n, 3))
    st = np.zeros(n, np.int32)
    _lib().or_pair_grads(*args, ctypes.byref(prm), n, _p(ps), _p(pm), _p(w36), _p(out), _p(gn0), _p(st))
    if with_n0:
        return out, gn0, st
    return out, st


def nodal_normals(slave):
    """(nodal normals (n_nodes, 3), element normals (n_el, 3)) of the slave side."""
    X = np.ascontiguousarray(slave.X, np.float64)
    C = np.ascontiguousarray(slave.conn, np.int32)
    nn = np.zeros((X.shape[0], 3))
    ne = np.zeros((C.shape[0], 3))
    _lib().or_nodal_normals(X.shape[0], _p(X), C.shape[0], _p(C), _p(nn), _p(ne))
    return nn, ne


def normal_chain(slave, gn0_el):
    """Gradient (n_nodes, 3) of sum_e <gn0_el[e], n0_e> with respect to the
    slave coordinates through the nodal normal field."""
    X = np.ascontiguousarray(slave.X, np.float64)
    C = np.ascontiguousarray(slave.conn, np.int32)
    g = np.ascontiguousarray(gn0_el, np.float64)
    out = np.zeros((X.shape[0], 3))
    if _lib().or_normal_chain(X.shape[0], _p(X), C.shape[0], _p(C), _p(g), _p(out)) != 0:
        raise RuntimeError("normal_chain: element patch larger than 48 nodes")
    return out


def pair_weights(slave, master, ps, pm, wD_fn, wM_fn, wg_fn):
    """Per-pair weights (n, 36) from functions of (row, col) / (row)."""
    Cs = slave.conn[ps]
    Cm = master.conn[pm]
    rD = np.repeat(Cs, 4, axis=1)
    cD = np.tile(Cs, (1, 4))
    cM = np.tile(Cm, (1, 4))
    w = np.empty((ps.size, 36))
    w[:, :16] = wD_fn(rD, cD)
    w[:, 16:32] = wM_fn(rD, cM)
    w[:, 32:] = wg_fn(Cs)
    return w


def scatter_grads(slave, master, ps, pm, g24):
    """Sum per-pair gradients onto nodes: (dL/dXs (n_s,3), dL/dXm (n_m,3))."""
    gs = np.zeros((slave.n_nodes, 3))
    gm = np.zeros((master.n_nodes, 3))
    g24 = g24.reshape(-1, 8, 3)
    np.add.at(gs, slave.conn[ps].reshape(-1), g24[:, :4, :].reshape(-1, 3))
    np.add.at(gm, master.conn[pm].reshape(-1), g24[:, 4:, :].reshape(-1, 3))
    return gs, gm


def count_flops(slave, master, prm, cs, cm, detail=False):
    """(flops of the candidate pass over all candidates, flops of the full
    evaluation over the candidates that are pairs).  With detail=True also
    (reverse-mode adjoint flops of those pairs outside the inverse maps,
    number of inverse maps evaluated, reverse-mode adjoint flops of the
    candidate pass of those pairs)."""
    args, keep = _mesh_args(slave, master)
    cs = np.ascontiguousarray(cs, np.int32)
    cm = np.ascontiguousarray(cm, np.int32)
    out = np.zeros(5, np.uint64)
    _lib().or_count_flops(*args, ctypes.byref(prm), cs.size, _p(cs), _p(cm), _p(out))
    if detail:
        return tuple(int(x) for x in out)
    return int(out[0]), int(out[1])


def pair_polygon(xs4, xm4, prm):
    xs4 = np.ascontiguousarray(xs4, np.float64)
    xm4 = np.ascontiguousarray(xm4, np.float64)
    pu = np.zeros(capacity())
    pv = np.zeros(capacity())
    st = ctypes.c_int32(0)
    n = _lib().or_pair_polygon(_p(xs4), _p(xm4), ctypes.byref(prm), _p(pu), _p(pv), ctypes.byref(st))
    if n < 0:
        raise RuntimeError("pair_polygon: more vertices than the output buffer holds")
    return np.stack([pu[:n], pv[:n]], axis=1), st.value


def clip2d(subject, clipper, tol=0.0):
    """(raw Sutherland-Hodgman polygon, cleaned polygon) of two 2-D polygons."""
    s = np.ascontiguousarray(subject, np.float64)
    c = np.ascontiguousarray(clipper, np.float64)
    su, sv = s[:, 0].copy(), s[:, 1].copy()
    cu, cv = c[:, 0].copy(), c[:, 1].copy()
    cap = capacity()
    ru, rv, ou, ov = (np.zeros(cap) for _ in range(4))
    nraw = ctypes.c_int32(0)
    n = _lib().or_clip2d(len(su), _p(su), _p(sv), len(cu), _p(cu), _p(cv), float(tol), _p(ru), _p(rv),
                         ctypes.byref(nraw), _p(ou), _p(ov))
    if n < 0:
        raise RuntimeError(f"clip2d failed ({n})")
    k = nraw.value
    return np.stack([ru[:k], rv[:k]], 1), np.stack([ou[:n], ov[:n]], 1)


def fan_points(poly, rule=3):
    p = np.ascontiguousarray(poly, np.float64)
    pu, pv = p[:, 0].copy(), p[:, 1].copy()
    m = max(1, (len(pu) - 2) * 7)
    qu, qv, qw = np.zeros(m), np.zeros(m), np.zeros(m)
    c = _lib().or_fan_points(len(pu), _p(pu), _p(pv), int(rule), _p(qu), _p(qv), _p(qw))
    return np.stack([qu[:c], qv[:c]], 1), qw[:c]


def rule(which):
    l = np.zeros(21)
    w = np.zeros(7)
    n = _lib().or_rule(int(which), _p(l), _p(w))
    return l[: 3 * n].reshape(n, 3), w[:n]


def inverse_bilinear(quad, p, prm=None):
    if prm is None:
        prm = params()
    q = np.ascontiguousarray(quad, np.float64)
    qu, qv = q[:, 0].copy(), q[:, 1].copy()
    x1, x2 = ctypes.c_double(0), ctypes.c_double(0)
    st = _lib().or_inverse_bilinear(_p(qu), _p(qv), float(p[0]), float(p[1]), ctypes.byref(prm),
                                    ctypes.byref(x1), ctypes.byref(x2))
    return np.array([x1.value, x2.value]), st


def dual_matrix(xs4):
    xs4 = np.ascontiguousarray(xs4, np.float64)
    A = np.zeros(16)
    _lib().or_dual_matrix(_p(xs4), _p(A))
    return A.reshape(4, 4)
