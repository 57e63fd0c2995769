"""GPU parity with the oracle on randomly drawn interfaces: wavy surfaces of
random amplitude and resolution ratio (slave finer or coarser than master),
master nodes moved off the surface, master orientation reversed at random,
and the whole interface in a random position and orientation in space; in
the default mode and with the dual basis, the continuous normal field and
the 3-point rule.
Candidates, pairs, vertex counts and patterns bit-exact; D, M and gap within
TOL; the gradients within TOL, or within ten times the oracle's own change
under a translation where a draw is that sensitive to rounding."""

import math

import numpy as np
import pytest

import oracle
import synth
from synth.meshes import Interface, Mesh
from tests.gpu_util import TOL, assert_forward_parity, gpu_run, oracle_params, rel_err, weight_fns

pytestmark = pytest.mark.gpu


def random_interface(seed):
    rng = np.random.default_rng(9000 + seed)
    # resolutions at least 10% apart and without a common factor: grid lines
    # of both sides at the same parameter put slave and master edges almost
    # on one line in the projection, where a clip crossing, and with it the
    # gradient, is ill-conditioned (per-pair gradients up to 1e3 that cancel
    # in the sums), as for the tied configuration
    ns = int(rng.integers(6, 41))
    nm = int(rng.integers(5, 41))
    while abs(ns / nm - 1.0) < 0.1 or math.gcd(ns, nm) != 1:
        nm = int(rng.integers(5, 41))
    amp = float(rng.uniform(0.0, 0.08))
    itf = synth.wavy(ns, nm, seed=9100 + seed, amp=amp)
    if rng.random() < 0.5:
        itf = synth.opposing(itf)
    # a rigid motion: rotation from the QR factor of a Gaussian matrix
    # (determinant +1), translation U[-2, 2]^3
    Q, R = np.linalg.qr(rng.standard_normal((3, 3)))
    Q = Q * np.sign(np.diag(R))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    t = rng.uniform(-2.0, 2.0, 3)
    move = lambda X: X @ Q.T + t  # noqa: E731
    return Interface(Mesh(move(itf.slave.X), itf.slave.conn), Mesh(move(itf.master.X), itf.master.conn), itf.delta,
                     name=f"random {seed}: {itf.name}, amp {amp:.3f}", meta=itf.meta)


def oracle_gradients(itf, prm, o, seed):
    """The oracle's gradient, with the chain through the nodal normal field
    (element normal gradients to the slave coordinates) when it is on."""
    ps, pm = o["pair_s"], o["pair_m"]
    w = oracle.pair_weights(itf.slave, itf.master, ps, pm, *weight_fns(seed))
    g24, gn0, _ = oracle.pair_grads(itf.slave, itf.master, prm, ps, pm, w, with_n0=True)
    gs, gm = oracle.scatter_grads(itf.slave, itf.master, ps, pm, g24)
    if prm.normals:
        ge = np.zeros((itf.slave.n_el, 3))
        np.add.at(ge, ps, gn0)
        gs = gs + oracle.normal_chain(itf.slave, ge)
    return gs, gm


# seeds 0-5 in the default mode; 6-11 with the dual basis, the continuous
# normal field, the 3-point rule, or both of the first two
MODES = [dict()] * 6 + [dict(dual=True), dict(nodal=True), dict(dual=True, nodal=True), dict(rule=3),
                        dict(dual=True), dict(nodal=True)]


@pytest.mark.parametrize("seed", range(len(MODES)))
def test_random_interface_forward_and_gradients(seed):
    itf = random_interface(seed)
    mode = MODES[seed]
    print(f"[gpu] {itf.name} {mode}", flush=True)
    prm = oracle_params(itf, **mode)
    g = gpu_run(itf, backward_seed=3300 + seed, **mode)
    o = oracle.evaluate(itf, prm)
    assert_forward_parity(g, o)
    gs, gm = oracle_gradients(itf, prm, o, 3300 + seed)
    # The gradient is invariant under a translation; how much the oracle's
    # own gradient moves under one measures the rounding sensitivity of this
    # draw (slivers between nearly coincident grid lines raise it), and no
    # agreement can be asked beyond it.
    sh = np.array([0.37, -0.21, 0.13])
    moved = Interface(Mesh(itf.slave.X + sh, itf.slave.conn), Mesh(itf.master.X + sh, itf.master.conn), itf.delta)
    o2 = oracle.evaluate(moved, prm)
    assert np.array_equal(o2["pair_s"], o["pair_s"]) and np.array_equal(o2["pair_m"], o["pair_m"])
    gs2, gm2 = oracle_gradients(moved, prm, o2, 3300 + seed)
    tol = max(TOL, 10 * rel_err(gs2, gs), 10 * rel_err(gm2, gm))
    es, em = rel_err(g["gXs"], gs), rel_err(g["gXm"], gm)
    print(f"pairs {o['pair_s'].size}, grad rel err slave {es:.2e} master {em:.2e}, tolerance {tol:.1e}", flush=True)
    assert es <= tol and em <= tol


# Element-based integration (an n x n rule on each whole slave element) on
# random interfaces, with both bases.
@pytest.mark.parametrize("seed,ng,dual", [(0, 2, False), (3, 3, True), (6, 5, False), (9, 8, True)])
def test_random_interface_element_based(seed, ng, dual):
    itf = random_interface(seed)
    print(f"[gpu] {itf.name} element rule {ng} dual={dual}", flush=True)
    prm = oracle_params(itf, dual=dual)
    g = gpu_run(itf, dual=dual, element_rule=ng)
    o = oracle.evaluate_elements(itf, ng, prm)
    assert np.array_equal(g["pair_s"], o["pair_s"]) and np.array_equal(g["pair_m"], o["pair_m"])
    eD, eM, eg = rel_err(g["D"].data, o["D"].data), rel_err(g["M"].data, o["M"].data), rel_err(g["g"], o["g"])
    print(f"pairs {o['pair_s'].size}, rel err D {eD:.1e} M {eM:.1e} g {eg:.1e}", flush=True)
    assert np.array_equal(g["D"].indices, o["D"].indices) and np.array_equal(g["M"].indices, o["M"].indices)
    assert eD <= TOL and eM <= TOL and eg <= TOL
    assert g["stats"]["n_noconv"] == 0
