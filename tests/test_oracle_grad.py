"""Pins of the oracle's gradients (forward-mode dual numbers).

Checked against central finite differences of the oracle's own values and
against exact identities of the loss L = <W_D, D> + <W_M, M> + <w_g, g>:
invariance under translation and rotation of both meshes, and homogeneity
under uniform scaling (D, M scale with area, the gap with area x length).
"""

import numpy as np
import pytest

import oracle
import synth
from synth.weights import keyed_normal, TAG_D, TAG_M, TAG_G


def weight_fns(seed):
    return (lambda r, c: keyed_normal(seed, TAG_D, r, c),
            lambda r, c: keyed_normal(seed, TAG_M, r, c),
            lambda r: keyed_normal(seed, TAG_G, r, np.zeros_like(r)))


def loss_parts(itf, prm, ps, pm, seed):
    nv, blocks, st = oracle.eval_candidates(itf.slave, itf.master, prm, ps, pm)
    assert np.all(nv >= 3)
    w = oracle.pair_weights(itf.slave, itf.master, ps, pm, *weight_fns(seed))
    return (np.sum(w[:, :16] * blocks[:, :16]), np.sum(w[:, 16:32] * blocks[:, 16:32]),
            np.sum(w[:, 32:] * blocks[:, 32:]))


def grad_total(itf, prm, ps, pm, seed, parts=(1, 1, 1)):
    w = oracle.pair_weights(itf.slave, itf.master, ps, pm, *weight_fns(seed))
    w[:, :16] *= parts[0]
    w[:, 16:32] *= parts[1]
    w[:, 32:] *= parts[2]
    g24, st = oracle.pair_grads(itf.slave, itf.master, prm, ps, pm, w)
    assert np.all(st == 0)
    return oracle.scatter_grads(itf.slave, itf.master, ps, pm, g24)


def small_curved(seed=4):
    itf = synth.wavy(11, 8, seed=seed, amp=0.05, normal_offset=2e-3, delta=3e-3)
    return itf


def local_fd(itf, prm, ps, pm, side, node, d, h, seed):
    mesh = itf.slave if side == 0 else itf.master
    conn = mesh.conn[ps] if side == 0 else mesh.conn[pm]
    sel = np.any(conn == node, axis=1)
    vals = []
    for sgn in (1, -1):
        x0 = mesh.X[node, d]
        mesh.X[node, d] = x0 + sgn * h
        vals.append(sum(loss_parts(itf, prm, ps[sel], pm[sel], seed)))
        mesh.X[node, d] = x0
    return (vals[0] - vals[1]) / (2 * h), sel.any()


def test_fd_central_differences():
    # Central differences with h = 1e-6 on random coordinates.  Where a clip
    # polygon has a feature narrower than about 100 h (a sliver between
    # nearly coincident edges), the step straddles a change of the polygon's
    # topology and the difference quotient is not a derivative there; such a
    # coordinate is re-checked with h = 1e-7, and at most a few may need it.
    # Nodes near the domain boundary are skipped: there the two meshes'
    # boundary lines coincide and master nodes whose surface normal is
    # vertical sit exactly on a slave edge, a tie at which the loss has a kink.
    itf = small_curved()
    prm = oracle.params(delta=itf.delta)
    r = oracle.evaluate(itf, prm)
    ps, pm = r["pair_s"], r["pair_m"]
    gs, gm = grad_total(itf, prm, ps, pm, 3000)
    rng = np.random.default_rng(3001)
    checked = refined = 0
    for _ in range(150):
        side = int(rng.integers(0, 2))
        mesh = itf.slave if side == 0 else itf.master
        node = int(rng.integers(0, mesh.n_nodes))
        d = int(rng.integers(0, 3))
        if np.any(np.abs(mesh.X[node, :2] - 0.5) > 0.35):
            continue
        fd, touched = local_fd(itf, prm, ps, pm, side, node, d, 1e-6, 3000)
        if not touched:
            continue
        an = (gs if side == 0 else gm)[node, d]
        checked += 1
        if abs(fd - an) > 2e-6 * max(1.0, abs(an)):
            refined += 1
            fd, _ = local_fd(itf, prm, ps, pm, side, node, d, 1e-7, 3000)
            assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (side, node, d, fd, an)
    assert checked >= 30 and refined <= 0.1 * checked


def test_translation_and_rotation_invariance():
    itf = small_curved(5)
    prm = oracle.params(delta=itf.delta)
    r = oracle.evaluate(itf, prm)
    ps, pm = r["pair_s"], r["pair_m"]
    gs, gm = grad_total(itf, prm, ps, pm, 7)
    G = np.concatenate([gs, gm])
    X = np.concatenate([itf.slave.X, itf.master.X])
    scale = np.abs(G).max()
    np.testing.assert_allclose(G.sum(0), 0.0, atol=1e-12 * scale * len(G))
    np.testing.assert_allclose(np.cross(X, G).sum(0), 0.0, atol=1e-12 * scale * len(G))


def test_scaling_homogeneity():
    itf = small_curved(6)
    prm = oracle.params(delta=itf.delta)
    r = oracle.evaluate(itf, prm)
    ps, pm = r["pair_s"], r["pair_m"]
    LD, LM, Lg = loss_parts(itf, prm, ps, pm, 9)
    X = np.concatenate([itf.slave.X, itf.master.X])
    for parts, L, deg in (((1, 0, 0), LD, 2), ((0, 1, 0), LM, 2), ((0, 0, 1), Lg, 3)):
        gs, gm = grad_total(itf, prm, ps, pm, 9, parts)
        G = np.concatenate([gs, gm])
        euler = np.sum(X * G)
        assert abs(euler - deg * L) <= 1e-11 * max(1.0, abs(L)), (parts, euler, deg * L)


def test_dual_basis_gradient_fd():
    # the oracle differentiates the dual basis too (through A_e)
    itf = small_curved(8)
    prm = oracle.params(delta=itf.delta, dual=True)
    r = oracle.evaluate(itf, prm)
    ps, pm = r["pair_s"][:60], r["pair_m"][:60]
    gs, gm = grad_total(itf, prm, ps, pm, 21)
    h = 1e-6
    node = int(itf.slave.conn[ps[10], 2])
    for d in range(3):
        vals = []
        for sgn in (1, -1):
            x0 = itf.slave.X[node, d]
            itf.slave.X[node, d] = x0 + sgn * h
            vals.append(sum(loss_parts(itf, prm, ps, pm, 21)))
            itf.slave.X[node, d] = x0
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - gs[node, d]) <= 2e-6 * max(1.0, abs(fd))
