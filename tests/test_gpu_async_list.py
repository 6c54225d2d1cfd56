"""GPU: the stream-ordered list build (tk_nblist_build_async).

The list it queues must be the oracle's list bit for bit, and its plan must
drive the pair terms and the solver exactly as the synchronous build's plan
does (same cells, same unit order, same pair codes: results equal bitwise).
A bound below what the build needs must come back as TK_E_CAPACITY in the
device status word, with the measured sizes in the report, and every call
that then takes the list must skip its work (the solve returns the error).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1906_01211_amd import synth

pytestmark = pytest.mark.gpu

S = synth.AMOEBA_SETTINGS
E_CAPACITY = -3
R7 = S["rc_ewald"] + S["skin"]
R9 = S["rc_vdw"] + S["skin"]


@pytest.fixture(scope="module")
def tk():
    import torch
    from paper_1906_01211_amd import tk as _tk
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _tk.load()
    return _tk


@pytest.fixture(scope="module")
def ctx(tk):
    c = tk.Context(0)
    yield c
    c.close()


_cache = {}


def water(name):
    if name not in _cache:
        _cache[name] = synth.make(name)
    return _cache[name]


def oracle_list(name, rc):
    key = (name, rc)
    if key not in _cache:
        w = water(name)
        _cache[key] = O.nblist(w.xyz, w.box, rc)
    return _cache[key]


def np_(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("name,rc", [("water216", R7), ("water216", R9), ("water7853", R7),
                                     ("water7853", R9)])
def test_async_list_bit_exact(ctx, name, rc):
    w = water(name)
    sysr = ctx.system(w.xyz, w.box, w.molid)
    sync = ctx.nblist(sysr, rc, plan_slot=0)
    exact = ctx.nblist_bounds(0, headroom=0.0)
    assert exact.npairs == sync.npairs
    al = ctx.nblist_async(sysr, rc, plan_slot=1, bounds=ctx.nblist_bounds(0, headroom=0.1))
    assert al.npairs == -1
    assert al.status() == 0
    rp, cp = oracle_list(name, rc)
    r = al.resolved()
    assert r.npairs == len(cp)
    assert np.array_equal(np_(r.row_ptr), rp)
    assert np.array_equal(np_(r.col), cp)
    # the measured sizes are the synchronous build's
    assert al.report() == exact.as_dict()


def test_async_list_drives_the_terms(ctx, tk):
    w = water("water7853")
    sysr = ctx.system(w.xyz, w.box, w.molid)
    s7, s9 = ctx.nblists(sysr, [R7, R9], [0, 2])
    a7 = ctx.nblist_async(sysr, R7, plan_slot=1, bounds=ctx.nblist_bounds(0, 0.1))
    a9 = ctx.nblist_async(sysr, R9, plan_slot=3, bounds=ctx.nblist_bounds(2, 0.1))
    assert a7.status() == 0 and a9.status() == 0
    import torch
    T = lambda a: torch.as_tensor(a, device=ctx.device)
    mp, pol, th = T(w.mpole), T(w.polarity), T(w.thole)
    for prec in (tk.FP64, tk.MIXED):
        res = []
        for lst in (s7, a7):
            (e, f, v), (mu, info) = ctx.empole_polarize(sysr, lst, mp, pol, th, S["beta"],
                                                         S["rc_ewald"], tol_debye=S["tol_debye"],
                                                         maxiter=S["maxiter"], prec=prec)
            res.append((np_(e), np_(f), np_(v), np_(mu), info["iters"]))
        for x, y in zip(res[0], res[1]):
            assert np.array_equal(x, y)
    rad, eps = T(w.vdw_rad), T(w.vdw_eps)
    out = [ctx.evdw(sysr, lst, tk.VDW_HAL, rad, eps, S["rc_vdw"], S["taper_frac"], S["dhal"],
                    S["ghal"]) for lst in (s9, a9)]
    assert float(out[0][0]) == float(out[1][0])
    assert np.array_equal(np_(out[0][1]), np_(out[1][1]))


def test_async_lists_on_two_streams(ctx):
    import torch
    w = water("water216")
    sysr = ctx.system(w.xyz, w.box, w.molid)
    ctx.nblists(sysr, [R7, R9], [0, 2])
    b7, b9 = ctx.nblist_bounds(0, 0.2), ctx.nblist_bounds(2, 0.2)
    side = torch.cuda.Stream(device=ctx.device)
    main = torch.cuda.current_stream(ctx.device)
    side.wait_stream(main)
    a7 = ctx.nblist_async(sysr, R7, plan_slot=1, bounds=b7, stream=main)
    a9 = ctx.nblist_async(sysr, R9, plan_slot=3, bounds=b9, stream=side)
    main.wait_stream(side)
    torch.cuda.synchronize()
    for lst, rc in ((a7, R7), (a9, R9)):
        assert lst.status() == 0
        rp, cp = oracle_list("water216", rc)
        r = lst.resolved()
        assert np.array_equal(np_(r.row_ptr), rp)
        assert np.array_equal(np_(r.col), cp)


@pytest.mark.parametrize("short", ["max_occ", "max_row", "max_nbhd", "windows", "cap"])
def test_async_list_reports_a_short_bound(ctx, tk, short):
    w = water("water216")
    sysr = ctx.system(w.xyz, w.box, w.molid)
    sync = ctx.nblist(sysr, R7, plan_slot=0)
    exact = ctx.nblist_bounds(0, headroom=0.0)
    b = ctx.nblist_bounds(0, headroom=0.0)
    cap = int(exact.npairs)
    if short == "cap":
        cap -= 1
    else:
        setattr(b, short, getattr(b, short) - 1)
    al = ctx.nblist_async(sysr, R7, plan_slot=1, bounds=b, cap=cap)
    assert al.status() == E_CAPACITY
    rep = al.report()
    assert rep["max_occ"] == exact.max_occ
    assert rep["max_nbhd"] == exact.max_nbhd
    assert rep["windows"] == exact.windows
    if short == "max_occ":   # the enumeration itself did not fit: no count
        assert rep["npairs"] == -1 and al.count() == -1
    else:
        assert rep["npairs"] == sync.npairs and al.count() == sync.npairs
        assert rep["max_row"] == exact.max_row
    # the calls that take the failed list skip their work: the solve says so
    import torch
    T = lambda a: torch.as_tensor(a, device=ctx.device)
    with pytest.raises(tk.TkError) as err:
        ctx.polarize_pcg(sysr, al, T(w.mpole), T(w.polarity), T(w.thole), S["beta"],
                         S["rc_ewald"], tol_debye=S["tol_debye"], maxiter=S["maxiter"])
    assert err.value.status == E_CAPACITY
    torch.cuda.synchronize()
    # the slot recovers with bounds that fit
    ok = ctx.nblist_async(sysr, R7, plan_slot=1, bounds=ctx.nblist_bounds(0, 0.1))
    assert ok.status() == 0
    rp, cp = oracle_list("water216", R7)
    assert np.array_equal(np_(ok.resolved().col), cp)


def test_async_list_argument_errors(ctx, tk):
    w = water("water216")
    sysr = ctx.system(w.xyz, w.box, w.molid)
    ctx.nblist(sysr, R7, plan_slot=0)
    b = ctx.nblist_bounds(0, 0.1)
    for field in ("max_occ", "max_row", "max_nbhd", "windows"):
        bad = ctx.nblist_bounds(0, 0.1)
        setattr(bad, field, 0)
        with pytest.raises(tk.TkError) as err:
            ctx.nblist_async(sysr, R7, plan_slot=1, bounds=bad)
        assert err.value.status == -1
    with pytest.raises(tk.TkError):
        ctx.nblist_bounds(7, 0.1)   # an empty slot
    with pytest.raises(tk.TkError):
        ctx.nblist_bounds(0, -1.0)
    with pytest.raises(tk.TkError):
        ctx.nblist_async(sysr, R7, plan_slot=1, bounds=b, cap=-1)


def test_async_plan_only_and_empty(ctx, tk):
    import torch
    w = water("water216")
    sysr = ctx.system(w.xyz, w.box, w.molid)
    s9 = ctx.nblist(sysr, R9, plan_slot=2)
    b = ctx.nblist_bounds(2, 0.1)
    # the plan alone (no CSR): the pair count still bounded by cap
    a9 = ctx.nblist_async(sysr, R9, plan_slot=3, bounds=b, want_csr=False)
    assert a9.status() == 0 and a9.count() == s9.npairs
    T = lambda a: torch.as_tensor(a, device=ctx.device)
    rad, eps = T(w.vdw_rad), T(w.vdw_eps)
    out = [ctx.evdw(sysr, lst, tk.VDW_HAL, rad, eps, S["rc_vdw"], S["taper_frac"], S["dhal"],
                    S["ghal"]) for lst in (s9, a9)]
    assert float(out[0][0]) == float(out[1][0])
    assert np.array_equal(np_(out[0][1]), np_(out[1][1]))
    # a system with no atoms
    e = ctx.system(np.zeros((0, 3)), w.box, np.zeros(0, dtype=np.int32))
    a0 = ctx.nblist_async(e, R9, plan_slot=4, bounds=b)
    assert a0.status() == 0 and a0.count() == 0
    assert np_(a0.row_ptr).tolist() == [0]


@pytest.mark.parametrize("n,box,rc,seed", [(1, 10.0, 3.0, 0), (2, 10.0, 5.0, 1), (37, 7.0, 3.4, 2),
                                           (300, 12.0, 3.0, 3), (500, 20.0, 9.9, 4),
                                           (1000, 17.0, 2.0, 5)])
def test_async_list_random_boxes(ctx, n, box, rc, seed):
    # small grids (one or two cells per edge: repeated neighbour cells) and
    # sparse ones; bounds from the synchronous build of the same atoms
    rng = np.random.default_rng(seed)
    xyz = rng.uniform(-box, 2 * box, size=(n, 3))
    sysr = ctx.system(xyz, box, np.arange(n) // 3)
    ctx.nblist(sysr, rc, plan_slot=5)
    al = ctx.nblist_async(sysr, rc, plan_slot=6, bounds=ctx.nblist_bounds(5, 0.0))
    assert al.status() == 0
    rp, cp = O.nblist(xyz, box, rc)
    r = al.resolved()
    assert np.array_equal(np_(r.row_ptr), rp)
    assert np.array_equal(np_(r.col), cp)


def test_async_list_clustered(ctx, tk):
    # cells far denser than the mean (the synchronous build reruns its
    # enumeration there; the stream-ordered one takes the measured bound)
    import torch
    rng = np.random.default_rng(7)
    box = 30.0
    xyz = np.concatenate([rng.uniform(11.0, 16.0, size=(300, 3)),
                          rng.uniform(0.0, box, size=(60, 3))])
    sysr = ctx.system(xyz, box, np.arange(len(xyz)) // 3)
    s = ctx.nblist(sysr, 7.001, plan_slot=5)
    al = ctx.nblist_async(sysr, 7.001, plan_slot=6, bounds=ctx.nblist_bounds(5, 0.05))
    assert al.status() == 0
    rp, cp = O.nblist(xyz, box, 7.001)
    assert np.array_equal(np_(al.resolved().col), cp)
    # and its plan drives a pair term as the synchronous plan does
    mp = np.zeros((len(xyz), 10))
    mp[:, 0] = rng.normal(0.0, 0.3, len(xyz))
    out = [ctx.empole_real(sysr, lst, mp, 0.4, 7.0) for lst in (s, al)]
    for x, y in zip(out[0], out[1]):
        assert np.array_equal(np_(x), np_(y))
