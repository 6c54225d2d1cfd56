"""Pins of the oracle's neighbour list (integer, exact): the cell list equals the
O(N^2) definition, and both agree with an independent periodic k-d tree away
from the quantisation band at the cutoff."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import oracle as O
from paper_1906_01211_amd import synth


def _pairs(row_ptr, col):
    n = len(row_ptr) - 1
    i = np.repeat(np.arange(n), np.diff(row_ptr))
    return i, col


@pytest.mark.parametrize("n,box,rc", [(40, 10.0, 4.9), (300, 12.0, 3.0), (200, 9.0, 4.5),
                                      (500, 20.0, 6.0), (120, 7.0, 2.2)])
def test_cell_equals_brute(n, box, rc):
    rng = np.random.default_rng(n)
    xyz = rng.uniform(-box, 2 * box, size=(n, 3))      # outside the box too: wrapped
    rb, cb = O.nblist(xyz, box, rc, method="brute")
    rcl, ccl = O.nblist(xyz, box, rc, method="cell")
    assert np.array_equal(rb, rcl) and np.array_equal(cb, ccl)
    for i in range(n):                                 # rows ascending, j > i
        row = cb[rb[i]:rb[i + 1]]
        assert np.all(np.diff(row) > 0) and np.all(row > i)


@pytest.mark.parametrize("name,rc", [("water216", 7.001), ("water216", 9.001)])
def test_water216_lists(name, rc):
    w = synth.make(name)
    rb, cb = O.nblist(w.xyz, w.box, rc, method="brute")
    rcl, ccl = O.nblist(w.xyz, w.box, rc, method="cell")
    assert np.array_equal(rb, rcl) and np.array_equal(cb, ccl)
    # pair count near (2 pi / 3) rc^3 rho N
    est = 2 * np.pi / 3 * rc ** 3 * (w.n / w.box ** 3) * w.n
    assert abs(len(cb) / est - 1) < 0.05


@pytest.mark.parametrize("n,box,rc", [(400, 15.0, 5.0), (648, 18.64, 7.001)])
def test_against_periodic_kdtree(n, box, rc):
    rng = np.random.default_rng(7)
    xyz = rng.uniform(0, box, size=(n, 3))
    rp, cp = O.nblist(xyz, box, rc)
    got = set(zip(*[a.tolist() for a in _pairs(rp, cp)]))
    tree = cKDTree(xyz, boxsize=box)
    inner = tree.query_pairs(rc - 1e-6)
    outer = tree.query_pairs(rc + 1e-6)
    assert inner <= got <= outer


def test_quantisation_edges():
    box = 10.0
    xyz = np.array([[0.0, 0.0, 0.0], [10.0, -1e-300, -10.0], [-1e-18, 5.0, 9.999999999999998]])
    u = O.quantize(xyz, box)
    assert u[0].tolist() == [0, 0, 0]
    assert u[1, 0] == 0 and u[1, 2] == 0       # exactly on the box edge wraps to 0
    assert u[1, 1] == 0                        # -tiny rounds up to 1.0 -> 0
    assert u[2, 1] == 2 ** 31
    assert O.cutoff_quantum(5.0, 10.0) == 2 ** 31
    with pytest.raises(O.OracleError):
        O.quantize(np.array([[np.nan, 0, 0]]), box)


def test_cutoff_and_capacity_errors():
    xyz = np.random.default_rng(1).uniform(0, 10, size=(50, 3))
    with pytest.raises(O.OracleError) as e:
        O.nblist(xyz, 10.0, 5.1)
    assert e.value.status == O.E_CUTOFF
    # capacity overflow reports the required size
    full_r, full_c = O.nblist(xyz, 10.0, 4.0)
    import ctypes
    row_ptr = np.zeros(51, dtype=np.int32)
    col = np.zeros(5, dtype=np.int32)
    npairs = ctypes.c_int64(0)
    st = O.lib().or_nblist_cell(50, np.ascontiguousarray(xyz), 10.0, 4.0, row_ptr, col, 5,
                                ctypes.byref(npairs))
    assert st == O.E_CAPACITY and npairs.value == len(full_c)


def test_empty_and_single():
    r, c = O.nblist(np.zeros((0, 3)), 10.0, 3.0)
    assert r.tolist() == [0] and len(c) == 0
    r, c = O.nblist(np.array([[1.0, 2.0, 3.0]]), 10.0, 3.0)
    assert r.tolist() == [0, 0] and len(c) == 0


def test_pair_exactly_at_the_quantised_cutoff_is_inside():
    box, rc = 16.0, 4.0                         # rq = 2^30 exactly
    q = box / 2 ** 32
    assert O.cutoff_quantum(rc, box) == 2 ** 30
    xyz = np.array([[1.0, 1.0, 1.0], [1.0 + 2 ** 30 * q, 1.0, 1.0],
                    [1.0, 1.0 + (2 ** 30 + 1) * q, 1.0], [9.0, 9.0, 9.0],
                    [9.0 + 2 ** 29 * q, 9.0 + 2 ** 29 * q, 9.0 + 2 ** 29 * q]])
    u = O.quantize(xyz, box)
    assert int(u[1, 0]) - int(u[0, 0]) == 2 ** 30
    r, c = O.nblist(xyz, box, rc, method="brute")
    assert set(c[r[0]:r[1]].tolist()) == {1, 4} or set(c[r[0]:r[1]].tolist()) == {1}
    assert 1 in c[r[0]:r[1]].tolist()           # D^2 == rq^2 counts as inside
    assert 2 not in c[r[0]:r[1]].tolist()       # one quantum further is outside
    assert 4 in c[r[3]:r[4]].tolist()           # 3 * (2^29)^2 < 2^60
    rc2, cc2 = O.nblist(xyz, box, rc, method="cell")
    assert np.array_equal(r, rc2) and np.array_equal(c, cc2)
