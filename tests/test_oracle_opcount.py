"""The oracle's op-counting build (oracle/opcount.cpp): it computes exactly what
the plain oracle computes, its per-pair counts are additive over pairs, and
the stored per-pair counts (tests/golden/pair_opcounts.json, which the
benchmark's flop rates use) are the ones it produces now."""
import json

import numpy as np
import pytest

from oracle import opcount
from oracle import oracle as O
from paper_1906_01211_amd import synth

S = synth.AMOEBA_SETTINGS


@pytest.fixture(scope="module")
def water():
    w = synth.make("water216")
    rp, cp = O.nblist(w.xyz, w.box, S["rc_ewald"] + S["skin"])
    rp9, cp9 = O.nblist(w.xyz, w.box, S["rc_vdw"] + S["skin"])
    return w, rp, cp, rp9, cp9


def _both(fn):
    """fn(O) on the plain oracle and on the counting build."""
    plain = fn(O)
    with opcount.counting() as Oc:
        counted = fn(Oc)
    return plain, counted


def _flat(x):
    if isinstance(x, tuple):
        return np.concatenate([_flat(v) for v in x])
    return np.atleast_1d(np.asarray(x, dtype=np.float64)).ravel()


@pytest.mark.parametrize("term", ["tmatvec", "empole", "efield", "hal", "epolar"])
def test_counting_build_computes_the_same_values(water, term):
    w, rp, cp, rp9, cp9 = water
    mu = np.random.default_rng(3).normal(0.0, 0.05, (w.n, 3))
    b, rc = S["beta"], S["rc_ewald"]
    calls = {
        "tmatvec": lambda M: M.tmatvec(w.xyz, w.box, rp, cp, w.polarity, w.thole, b, rc, mu, 0),
        "empole": lambda M: M.empole_real(w.xyz, w.box, w.molid, rp, cp, w.mpole, b, rc),
        "efield": lambda M: M.efield_direct(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity,
                                            w.thole, b, rc),
        "hal": lambda M: M.evdw(w.xyz, w.box, w.molid, rp9, cp9, M.VDW_HAL, w.vdw_rad, w.vdw_eps,
                                S["rc_vdw"]),
        "epolar": lambda M: M.epolar_real(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity,
                                          w.thole, mu, b, rc),
    }
    plain, counted = _both(calls[term])
    assert np.array_equal(_flat(plain), _flat(counted))


def test_counts_add_over_pairs():
    """Four atoms: two listed pairs inside the cutoff cost exactly twice one."""
    u = np.array([0.48, -0.36, 0.8]) / np.linalg.norm([0.48, -0.36, 0.8])
    xyz = np.array([[1.0, 1.0, 1.0], [1.0, 1.0, 1.0], [15.0, 1.0, 1.0], [15.0, 1.0, 1.0]])
    xyz[1] += 3.1 * u
    xyz[3] += 4.2 * u
    pol, th = np.full(4, 0.8), np.full(4, 0.39)
    mu = np.random.default_rng(4).normal(0.0, 0.05, (4, 3))
    res = []
    for rows, cols in (([0, 1, 1, 2, 2], [1, 3]), ([0, 1, 1, 1, 1], [1]), ([0, 0, 0, 0, 0], [])):
        with opcount.counting() as Oc:
            opcount.reset()
            Oc.tmatvec(xyz, 30.0, np.array(rows, np.int32), np.array(cols, np.int32), pol, th,
                       S["beta"], S["rc_ewald"], mu, 0)
            res.append(opcount.ops())
    two = opcount._diff(res[0], res[2])
    one = opcount._diff(res[1], res[2])
    assert all(two[k] == 2 * one[k] for k in opcount.KINDS)
    assert opcount.flops(one) > 0


def test_stored_counts_are_current():
    with open(opcount.GOLDEN) as f:
        stored = json.load(f)["counts"]
    assert stored == json.loads(json.dumps(opcount.pair_counts()))
    # the mat-vec evaluated on the fly takes erfc and exponentials; the 14-7
    # term takes none of them
    assert stored["tmatvec"]["evaluated_pair"]["erfc"] == 1
    assert stored["evdw_hal"]["evaluated_pair"]["erfc"] == 0
