"""Pins of the oracle's clockwise-master branch (opposing normals).

In contact the master surface faces the slave, so its elements, projected
onto a slave element's auxiliary plane, run clockwise (Alg. 1 projects the
master side onto the slave side).  The oracle then clips with the master
polygon walked as (M0, M3, M2, M1) while its shape functions keep the node
order.  Reversing a master element's node order, (0, 1, 2, 3) ->
(0, 3, 2, 1), leaves its bilinear surface unchanged and only swaps its two
parameter axes, so:
  * the clip polygon, D and the gap are those of the original order, and
    the local M block has its columns permuted by that reversal;
  * the assembled D, M (columns are global master nodes) and gap, and the
    gradient of any loss on them, are those of the original interface up to
    rounding.
The exact rational tables of the axis-aligned pairs (test_oracle_blocks)
and finite differences pin it independently.
"""

from fractions import Fraction as F

import numpy as np

import oracle
import synth
from test_oracle_blocks import flat_rect, rect_pair_exact, tofloat
from test_oracle_grad import grad_total, loss_parts

REV = [0, 3, 2, 1]  # reversed node order; also the column permutation of M


def one_pair(xs, xm, prm, conn_m=(0, 1, 2, 3)):
    S = synth.Mesh(xs, np.array([[0, 1, 2, 3]], np.int32))
    M = synth.Mesh(xm, np.array([conn_m], np.int32))
    nv, blocks, st = oracle.eval_candidates(S, M, prm, np.array([0], np.int32), np.array([0], np.int32))
    return nv[0], blocks[0, :16].reshape(4, 4), blocks[0, 16:32].reshape(4, 4), blocks[0, 32:], st[0]


def test_clockwise_shifted_half_pair_exact():
    half = F(1, 2)
    Dx, Mx, _ = rect_pair_exact((F(0), F(1)), (F(0), F(1)), (half, half + 1), (half, half + 1))
    xs = flat_rect((0, 1), (0, 1))
    xm = flat_rect((0.5, 1.5), (0.5, 1.5))
    nv, D, M, g, st = one_pair(xs, xm, oracle.params(), conn_m=REV)
    assert nv == 4 and st == 0
    np.testing.assert_allclose(D, tofloat(Dx), atol=1e-15)
    # local master node l is original node REV[l]
    np.testing.assert_allclose(M, tofloat(Mx)[:, REV], atol=1e-15)
    np.testing.assert_allclose(D * 2304, [[4, 8, 16, 8], [8, 28, 56, 16], [16, 56, 196, 56], [8, 16, 56, 28]],
                               atol=1e-11)
    np.testing.assert_allclose(M * 2304, [[25, 5, 1, 5], [65, 13, 5, 25], [169, 65, 25, 65], [65, 25, 5, 13]],
                               atol=1e-11)
    np.testing.assert_allclose(g, 0.0, atol=0)
    # row sums of M equal those of D (partition of unity on the master side)
    np.testing.assert_allclose(M.sum(1), D.sum(1), atol=1e-16)


def test_clockwise_master_polygon_is_the_counter_clockwise_one():
    # the clip walks the clockwise master as (M0, M3, M2, M1): the original
    # counter-clockwise order, so polygon and vertex order are unchanged
    rng = np.random.default_rng(12)
    prm = oracle.params()
    for _ in range(50):
        xs = flat_rect((0, 1), (0, 1)) + np.c_[rng.uniform(-0.2, 0.2, (4, 2)), np.zeros(4)]
        xm = flat_rect((0.3, 1.2), (-0.1, 0.8)) + np.c_[rng.uniform(-0.2, 0.2, (4, 2)), np.zeros(4)]
        p0, s0 = oracle.pair_polygon(xs, xm, prm)
        p1, s1 = oracle.pair_polygon(xs, xm[REV], prm)
        assert s0 == s1 == 0
        np.testing.assert_array_equal(p0, p1)


def test_clockwise_tilted_master_gap_exact():
    c0, c1 = F(1, 4), F(1, 2)
    sx, sy = (F(0), F(1, 2)), (F(1, 4), F(3, 4))
    mx, my = (F(-1, 4), F(3, 4)), (F(0), F(1))
    Dx, Mx, gx = rect_pair_exact(sx, sy, mx, my, gap_line=(c0, c1))
    xs = flat_rect((0, 0.5), (0.25, 0.75))
    xm = flat_rect((-0.25, 0.75), (0.0, 1.0), z=lambda x: 0.25 + 0.5 * x)
    nv, D, M, g, st = one_pair(xs, xm, oracle.params(), conn_m=REV)
    assert nv == 4 and st == 0
    np.testing.assert_allclose(D, tofloat(Dx), atol=1e-15)
    # master is tilted: eta differs from the flat projection only by rounding
    np.testing.assert_allclose(M, tofloat(Mx)[:, REV], atol=1e-15)
    np.testing.assert_allclose(g, tofloat(gx), atol=1e-15)


def _pair_loss_and_grad(xs, xm, conn_m, w):
    S = synth.Mesh(xs, np.array([[0, 1, 2, 3]], np.int32))
    M = synth.Mesh(xm, np.array([conn_m], np.int32))
    prm = oracle.params()
    z = np.array([0], np.int32)
    nv, blocks, st = oracle.eval_candidates(S, M, prm, z, z)
    g24, st2 = oracle.pair_grads(S, M, prm, z, z, w[None, :])
    return nv[0], float(np.sum(w * blocks[0])), g24[0], st[0] | st2[0]


def test_clockwise_pair_gradient_fd_and_invariance():
    # a generic warped pair in 3-D with a clockwise master: central
    # differences of the oracle's own values, plus the exact identities of
    # a loss that depends on relative positions only
    rng = np.random.default_rng(31)
    xs = np.array([[0, 0, 0], [1, 0.05, 0.02], [1.1, 0.95, -0.03], [-0.05, 1, 0.01]], float)
    xm = np.array([[0.4, 0.3, 0.01], [1.3, 0.35, 0.02], [1.25, 1.2, 0.0], [0.35, 1.15, -0.01]], float)
    w = rng.standard_normal(36)
    nv, L, g24, st = _pair_loss_and_grad(xs, xm, REV, w)
    assert nv >= 3 and st == 0
    # gradient slots are per local node: master local node k is xm[REV[k]]
    # (REV is its own inverse), so global order is slaves, then xm[0..3]
    G = np.concatenate([g24[:12].reshape(4, 3), g24[12:].reshape(4, 3)[REV]])
    h = 1e-6
    X = np.concatenate([xs, xm])
    for i in range(8):
        for d in range(3):
            Xp, Xn = X.copy(), X.copy()
            Xp[i, d] += h
            Xn[i, d] -= h
            Lp = _pair_loss_and_grad(Xp[:4], Xp[4:], REV, w)[1]
            Ln = _pair_loss_and_grad(Xn[:4], Xn[4:], REV, w)[1]
            fd = (Lp - Ln) / (2 * h)
            assert abs(fd - G[i, d]) <= 1e-7 * max(1.0, abs(fd)), (i, d, fd, G[i, d])
    scale = np.abs(G).max()
    np.testing.assert_allclose(G.sum(0), 0.0, atol=1e-13 * scale)
    np.testing.assert_allclose(np.cross(X, G).sum(0), 0.0, atol=1e-13 * scale)


def test_clockwise_pair_gradient_is_the_counter_clockwise_one():
    # the reversed master is the same surface: the gradient of a loss whose
    # M weights follow the nodes (columns permuted with them) is unchanged
    rng = np.random.default_rng(32)
    xs = np.array([[0, 0, 0], [1, 0.05, 0.02], [1.1, 0.95, -0.03], [-0.05, 1, 0.01]], float)
    xm = np.array([[0.4, 0.3, 0.01], [1.3, 0.35, 0.02], [1.25, 1.2, 0.0], [0.35, 1.15, -0.01]], float)
    w = rng.standard_normal(36)
    wr = w.copy()
    wr[16:32] = w[16:32].reshape(4, 4)[:, REV].reshape(-1)
    _, L0, g0, _ = _pair_loss_and_grad(xs, xm, (0, 1, 2, 3), w)
    _, L1, g1, _ = _pair_loss_and_grad(xs, xm, REV, wr)
    assert abs(L1 - L0) <= 1e-14 * abs(L0)
    g1 = np.concatenate([g1[:12], g1[12:].reshape(4, 3)[REV].reshape(-1)])  # to global node order
    np.testing.assert_allclose(g1, g0, rtol=0, atol=1e-12 * np.abs(g0).max())


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def test_opposing_interfaces_equal_the_original():
    for k, scale in ((0, None), (1, 24), (2, 24)):
        itf = synth.interface_config(k, scale)
        opp = synth.opposing(itf)
        prm = oracle.params(delta=itf.delta)
        a = oracle.evaluate(itf, prm)
        b = oracle.evaluate(opp, prm)
        np.testing.assert_array_equal(a["cand_nverts"], b["cand_nverts"])
        np.testing.assert_array_equal(a["pair_s"], b["pair_s"])
        np.testing.assert_array_equal(a["pair_m"], b["pair_m"])
        for key in ("D", "M"):
            assert (a[key] != b[key]).nnz == 0 or _rel(b[key].data, a[key].data) <= 1e-13, (k, key)
            np.testing.assert_array_equal(a[key].indices, b[key].indices)
        assert _rel(b["g"], a["g"]) <= 1e-13 or np.abs(a["g"]).max() == 0.0
        # gradients of the same keyed loss
        ps, pm = a["pair_s"], a["pair_m"]
        gs0, gm0 = grad_total(itf, prm, ps, pm, 3000)
        gs1, gm1 = grad_total(opp, prm, ps, pm, 3000)
        if k == 0:
            continue  # tied flat meshes: the loss has kinks at the coinciding boundary lines
        assert _rel(gs1, gs0) <= 1e-12 and _rel(gm1, gm0) <= 1e-12, k
        assert abs(sum(loss_parts(opp, prm, ps, pm, 5)) - sum(loss_parts(itf, prm, ps, pm, 5))) <= 1e-12
