"""GPU parity with the oracle on randomly drawn interfaces: wavy surfaces of
random amplitude and resolution ratio (slave finer or coarser than master),
master nodes moved off the surface, master orientation reversed at random,
and the whole interface in a random position and orientation in space.
Candidates, pairs, vertex counts and patterns bit-exact; D, M, gap and the
gradients within TOL."""

import numpy as np
import pytest

import oracle
import synth
from synth.meshes import Interface, Mesh
from tests.gpu_util import TOL, assert_forward_parity, gpu_run, oracle_params, rel_err, weight_fns

pytestmark = pytest.mark.gpu


def random_interface(seed):
    rng = np.random.default_rng(9000 + seed)
    ns = int(rng.integers(6, 41))
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


@pytest.mark.parametrize("seed", range(6))
def test_random_interface_forward_and_gradients(seed):
    itf = random_interface(seed)
    print(f"[gpu] {itf.name}", flush=True)
    prm = oracle_params(itf)
    g = gpu_run(itf, backward_seed=3300 + seed)
    o = oracle.evaluate(itf, prm)
    assert_forward_parity(g, o)
    w = oracle.pair_weights(itf.slave, itf.master, o["pair_s"], o["pair_m"], *weight_fns(3300 + seed))
    g24, _ = oracle.pair_grads(itf.slave, itf.master, prm, o["pair_s"], o["pair_m"], w)
    gs, gm = oracle.scatter_grads(itf.slave, itf.master, o["pair_s"], o["pair_m"], g24)
    es, em = rel_err(g["gXs"], gs), rel_err(g["gXm"], gm)
    print(f"pairs {o['pair_s'].size}, grad rel err slave {es:.2e} master {em:.2e}", flush=True)
    assert es <= TOL and em <= TOL
