"""Oracle status bits on degenerate inputs (CPU): a collapsed (zero-area)
slave element, a master element perpendicular to the slave plane, and inverse
maps cut off before convergence.  The GPU error-path tests compare the HIP
path's counts with these."""

import numpy as np

import oracle
import synth


def test_collapsed_slave_element_is_degenerate():
    itf = synth.collapsed_slave()
    r = oracle.evaluate(itf)
    bad = itf.slave.n_el - 1
    deg = (r["status"] & oracle.ST_DEGEN_SLAVE) != 0
    assert deg.sum() >= 1 and np.all(r["cand_s"][deg] == bad) and np.all(deg[r["cand_s"] == bad])
    assert not np.any(r["pair_s"] == bad)
    # the other six unit squares under one master: D sums to their area
    assert abs(r["D"].sum() - 6.0) < 1e-13


def test_perpendicular_master_is_degenerate():
    itf = synth.perpendicular_master()
    r = oracle.evaluate(itf)
    deg = (r["status"] & oracle.ST_DEGEN_MASTER) != 0
    assert np.all(r["cand_m"][deg] == 0) and np.all(deg[r["cand_m"] == 0]) and deg.sum() == 4
    # the flat master element is one pair, fully inside slave element 0
    assert list(r["pair_s"]) == [0] and list(r["pair_m"]) == [1]
    assert abs(r["D"].sum() - 0.64) < 1e-14


def test_one_newton_iteration_does_not_converge():
    itf = synth.interface_config(1, scale=20)
    r1 = oracle.evaluate(itf, oracle.params(delta=itf.delta, newton_maxit=1))
    r30 = oracle.evaluate(itf, oracle.params(delta=itf.delta))
    pairs1 = r1["cand_nverts"] >= 3
    assert np.all(r1["status"][pairs1] & oracle.ST_NOCONV)
    assert not np.any(r30["status"] & oracle.ST_NOCONV)
    # the cut-off only concerns the quadrature: the pair list is the same
    assert np.array_equal(r1["cand_nverts"], r30["cand_nverts"])
