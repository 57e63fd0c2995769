"""Pins of the oracle's continuous normal field (averaged nodal normals) and
of the evaluation with auxiliary planes built from it.

Pinned against: flat surfaces (every normal is e_z and the evaluation equals
the element-normal one bit for bit); the unjittered cylinder, whose interior
nodal normals are exactly radial by symmetry and whose element normals equal
the geometric ones (so both evaluations agree to rounding); second-order
convergence to the analytic normal of the wavy surface; invariance of the
values under a rigid motion; and central finite differences of the whole
loss, through the normal field, at slave nodes outside a pair's own element.
"""

import math

import numpy as np
import pytest

import oracle
import synth
from synth.meshes import Interface, Mesh, tensor_grid
from synth.weights import keyed_normal, TAG_D, TAG_M, TAG_G


def rel(a, b):
    a = np.asarray(a.todense() if hasattr(a, "todense") else a).ravel()
    b = np.asarray(b.todense() if hasattr(b, "todense") else b).ravel()
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_flat_normals_and_identical_evaluation():
    itf = synth.interface_config(0)
    nn, ne = oracle.nodal_normals(itf.slave)
    assert np.array_equal(nn, np.tile([0.0, 0.0, 1.0], (itf.slave.n_nodes, 1)))
    assert np.array_equal(ne, np.tile([0.0, 0.0, 1.0], (itf.slave.n_el, 1)))
    a = oracle.evaluate(itf, oracle.params(delta=itf.delta))
    b = oracle.evaluate(itf, oracle.params(delta=itf.delta, nodal_normals=True))
    assert np.array_equal(a["pair_s"], b["pair_s"]) and np.array_equal(a["cand_nverts"], b["cand_nverts"])
    assert np.array_equal(a["blocks"], b["blocks"])


def test_cylinder_radial_normals_and_equal_evaluation():
    itf = synth.cylinder(24, 19, seed=5)
    nn, ne = oracle.nodal_normals(itf.slave)
    n = 24
    th = np.arange(n + 1) * (math.pi / 2) / n
    I, J = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    interior = ((I > 0) & (I < n)).ravel()  # away from the straight edges theta = 0, pi/2
    radial = np.stack([np.cos(th[I.ravel()]), np.sin(th[I.ravel()]), 0 * th[I.ravel()]], 1)
    assert np.abs(nn[interior] - radial[interior]).max() <= 1e-15
    ei = np.arange(itf.slave.n_el) % n
    mid = (ei > 0) & (ei < n - 1)
    thc = (ei + 0.5) * (math.pi / 2) / n
    rc = np.stack([np.cos(thc), np.sin(thc), 0 * thc], 1)
    assert np.abs(ne[mid] - rc[mid]).max() <= 1e-15
    # on the interior columns the geometric and the nodal frame coincide
    prm_e = oracle.params(delta=itf.delta)
    prm_n = oracle.params(delta=itf.delta, nodal_normals=True)
    a = oracle.evaluate(itf, prm_e)
    cs, cm = a["pair_s"], a["pair_m"]
    sel = mid[cs]
    _, be, _ = oracle.eval_candidates(itf.slave, itf.master, prm_e, cs[sel], cm[sel])
    _, bn, _ = oracle.eval_candidates(itf.slave, itf.master, prm_n, cs[sel], cm[sel])
    assert rel(bn, be) <= 1e-13


def wavy_slave(n, amp=0.05):
    s, t, conn, _ = tensor_grid(n, n)
    X = np.stack([s, t, amp * np.sin(2 * math.pi * s) * np.sin(2 * math.pi * t)], 1)
    return Mesh(X, conn), s, t


def test_nodal_normals_converge_to_the_surface_normal():
    errs = []
    for n in (16, 32, 64):
        mesh, s, t = wavy_slave(n)
        nn, _ = oracle.nodal_normals(mesh)
        a = 0.05 * 2 * math.pi
        zx = a * np.cos(2 * math.pi * s) * np.sin(2 * math.pi * t)
        zy = a * np.sin(2 * math.pi * s) * np.cos(2 * math.pi * t)
        ex = np.stack([-zx, -zy, np.ones_like(zx)], 1)
        ex /= np.linalg.norm(ex, axis=1)[:, None]
        inner = (s > 0) & (s < 1) & (t > 0) & (t < 1)
        errs.append(np.abs(nn[inner] - ex[inner]).max())
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs


def test_rigid_motion_invariance():
    itf = synth.wavy(12, 9, seed=3, amp=0.05, normal_offset=2e-3, delta=3e-3)
    prm = oracle.params(delta=itf.delta, nodal_normals=True)
    a = oracle.evaluate(itf, prm)
    c, s_ = math.cos(0.7), math.sin(0.7)
    Q = np.array([[c, -s_, 0.0], [s_, c, 0.0], [0.0, 0.0, 1.0]]) @ np.array(
        [[1.0, 0.0, 0.0], [0.0, math.cos(0.3), -math.sin(0.3)], [0.0, math.sin(0.3), math.cos(0.3)]])
    rot = Interface(Mesh(itf.slave.X @ Q.T + 0.3, itf.slave.conn), Mesh(itf.master.X @ Q.T + 0.3, itf.master.conn),
                    itf.delta)
    _, b, st = oracle.eval_candidates(rot.slave, rot.master, prm, a["pair_s"], a["pair_m"])
    assert np.all(st == 0)
    assert rel(b[:, :16], a["blocks"][:, :16]) <= 1e-12
    assert rel(b[:, 16:32], a["blocks"][:, 16:32]) <= 1e-12
    assert rel(b[:, 32:], a["blocks"][:, 32:]) <= 1e-10


def weights(itf, ps, pm, seed):
    return oracle.pair_weights(itf.slave, itf.master, ps, pm,
                               lambda r, c: keyed_normal(seed, TAG_D, r, c),
                               lambda r, c: keyed_normal(seed, TAG_M, r, c),
                               lambda r: keyed_normal(seed, TAG_G, r, np.zeros_like(r)))


def total_grad(itf, prm, ps, pm, w):
    g24, gn0, st = oracle.pair_grads(itf.slave, itf.master, prm, ps, pm, w, with_n0=True)
    assert np.all(st == 0)
    gs, gm = oracle.scatter_grads(itf.slave, itf.master, ps, pm, g24)
    ge = np.zeros((itf.slave.n_el, 3))
    np.add.at(ge, ps, gn0)
    return gs + oracle.normal_chain(itf.slave, ge), gm


def loss(itf, prm, ps, pm, w):
    nv, b, st = oracle.eval_candidates(itf.slave, itf.master, prm, ps, pm)
    assert np.all(nv >= 3)
    return np.sum(w * b)


@pytest.mark.parametrize("dual", [False, True])
def test_finite_differences_through_the_normal_field(dual):
    itf = synth.wavy(9, 7, seed=11, amp=0.08, normal_offset=2e-3, delta=3e-3)
    prm = oracle.params(delta=itf.delta, dual=dual, nodal_normals=True)
    r = oracle.evaluate(itf, prm)
    ps, pm = r["pair_s"], r["pair_m"]
    w = weights(itf, ps, pm, 17)
    gs, gm = total_grad(itf, prm, ps, pm, w)
    rng = np.random.default_rng(2)
    checked = refined = 0
    for side, node in [(0, int(k)) for k in rng.choice(itf.slave.n_nodes, 14, replace=False)] + \
                      [(1, int(k)) for k in rng.choice(itf.master.n_nodes, 6, replace=False)]:
        mesh = itf.slave if side == 0 else itf.master
        for d in range(3):
            def fd(h):
                vals = []
                for sg in (1, -1):
                    x0 = mesh.X[node, d]
                    mesh.X[node, d] = x0 + sg * h
                    vals.append(loss(itf, prm, ps, pm, w))
                    mesh.X[node, d] = x0
                return (vals[0] - vals[1]) / (2 * h)
            an = (gs if side == 0 else gm)[node, d]
            v = fd(1e-6)
            if abs(v - an) > 1e-6 * max(1.0, abs(an)):
                # a clip sliver narrower than ~100 h: the loss is smooth only
                # on a finer scale there
                refined += 1
                v = fd(1e-7)
            assert abs(v - an) <= 1e-6 * max(1.0, abs(an)), (side, node, d, v, an)
            checked += 1
    assert checked == 60 and refined <= 12
    # the normal field reaches beyond a pair's own element: a slave node whose
    # elements have no pair can still carry gradient
    assert np.abs(gs).max() > 0


def test_normal_chain_reaches_neighbour_nodes():
    # n0_e depends on the corner normals at e's four nodes in the 3 x 3
    # elements around e; a corner normal involves its node and the two edge
    # neighbours, so the 4 x 4 node patch minus its 4 outer corners: 12 nodes
    itf = synth.wavy(6, 5, seed=1, amp=0.08, normal_offset=2e-3, delta=3e-3)
    g = np.zeros((itf.slave.n_el, 3))
    e = 2 * 6 + 2  # element (2, 2) of the 6 x 6 grid, nodes 16, 17, 24, 23
    g[e] = [0.3, -0.2, 0.5]
    out = oracle.normal_chain(itf.slave, g)
    touched = set(np.nonzero(np.abs(out).sum(1) > 0)[0].tolist())
    patch = {j * 7 + i for j in range(1, 5) for i in range(1, 5)}
    corners = {1 * 7 + 1, 1 * 7 + 4, 4 * 7 + 1, 4 * 7 + 4}
    assert touched == patch - corners
