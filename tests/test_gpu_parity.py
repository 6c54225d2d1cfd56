"""GPU parity: the HIP path (through the C-ABI) against the FP64 CPU oracle on
the same seeded inputs.

Tolerances (FP64 path): neighbour lists bit-exact; each energy component
relative 1e-10; forces and fields max |diff| <= 1e-8 * RMS of the oracle's;
solver iterates at a fixed iteration count relative 1e-10.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1906_01211_amd import synth

pytestmark = pytest.mark.gpu

C, DEBYE = O.constants()
S = synth.AMOEBA_SETTINGS


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


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def fmax_rel(got, ref):
    got = np.asarray(got)
    ref = np.asarray(ref)
    return np.abs(got - ref).max() / np.sqrt(np.mean(ref ** 2))


def np_(t):
    return t.detach().cpu().numpy()


def assert_list_equal(lst, row_ptr, col):
    assert lst.npairs == len(col)
    assert np.array_equal(np_(lst.row_ptr), row_ptr)
    assert np.array_equal(np_(lst.col), col)


_cache = {}


def water(name):
    if name not in _cache:
        _cache[name] = synth.make(name)
    return _cache[name]


def oracle_list(w, rc):
    key = ("list", w.params.get("name", id(w)), w.n, rc)
    if key not in _cache:
        _cache[key] = O.nblist(w.xyz, w.box, rc)
    return _cache[key]


# ----------------------------------------------------------------------------
@pytest.mark.parametrize("name,rc", [("water216", 7.001), ("water216", 9.001),
                                     ("water7853", 7.001), ("water7853", 9.001)])
def test_nblist_bit_exact(ctx, name, rc):
    w = water(name)
    sysr = ctx.system(w.xyz, w.box, w.molid)
    lst = ctx.nblist(sysr, rc, plan_slot=0)
    rp, cp = oracle_list(w, rc)
    assert_list_equal(lst, rp, cp)


@pytest.mark.parametrize("n,box,rc,seed", [(1, 10.0, 3.0, 0), (2, 10.0, 5.0, 1), (37, 7.0, 3.4, 2),
                                           (300, 12.0, 3.0, 3), (500, 20.0, 9.9, 4),
                                           (1000, 17.0, 2.0, 5)])
def test_nblist_random_boxes(ctx, n, box, rc, seed):
    rng = np.random.default_rng(seed)
    xyz = rng.uniform(-box, 2 * box, size=(n, 3))
    sysr = ctx.system(xyz, box, np.arange(n) // 3)
    lst = ctx.nblist(sysr, rc, plan_slot=1)
    rp, cp = O.nblist(xyz, box, rc)
    assert_list_equal(lst, rp, cp)


@pytest.mark.parametrize("seed", [5, 6])
def test_nblist_clustered(ctx, seed):
    # most atoms in one small region: cells far denser than the mean, which
    # exceeds the enumeration's first staging bound and makes the build rerun
    rng = np.random.default_rng(seed)
    box = 30.0
    xyz = np.concatenate([rng.uniform(11.0, 16.0, size=(300, 3)),
                          rng.uniform(0.0, box, size=(60, 3))])
    sysr = ctx.system(xyz, box, np.arange(len(xyz)) // 3)
    lst = ctx.nblist(sysr, 7.001, plan_slot=1)
    rp, cp = O.nblist(xyz, box, 7.001)
    assert_list_equal(lst, rp, cp)
    # the plan left by the rerun drives the pair kernels correctly
    mp = np.zeros((len(xyz), 10))
    mp[:, 0] = rng.normal(0.0, 0.3, len(xyz))
    mp[:, 1:4] = rng.normal(0.0, 0.05, (len(xyz), 3))
    e, f, _ = ctx.empole_real(sysr, lst, mp, S["beta"], 7.0)
    eo, fo, _ = O.empole_real(xyz, box, np.arange(len(xyz)) // 3, rp, cp, mp, S["beta"], 7.0)
    assert rel(np_(e)[0], eo[0]) < 1e-10
    assert fmax_rel(np_(f), fo) < 1e-8


@pytest.mark.parametrize("two_streams", [False, True])
def test_nblist_multi(ctx, tk, two_streams):
    # the Ewald and vdW lists of a step in one call (one or two streams): each
    # equals the oracle's, and each plan drives its pair term
    import torch
    w = water("water7853")
    sysr = ctx.system(w.xyz, w.box, w.molid)
    main = torch.cuda.current_stream(ctx.device)
    side = torch.cuda.Stream(device=ctx.device)
    side.wait_stream(main)
    l7, l9 = ctx.nblists(sysr, [7.001, 9.001], [0, 1],
                         streams=[main, side] if two_streams else None)
    main.wait_stream(side)
    for lst, rc in ((l7, 7.001), (l9, 9.001)):
        rp, cp = oracle_list(w, rc)
        assert_list_equal(lst, rp, cp)
    e7, _, _ = ctx.empole_real(sysr, l7, w.mpole, S["beta"], S["rc_ewald"])
    e9, _, _ = ctx.evdw(sysr, l9, tk.VDW_HAL, w.vdw_rad, w.vdw_eps, S["rc_vdw"], S["taper_frac"],
                        S["dhal"], S["ghal"])
    rp7, cp7 = oracle_list(w, 7.001)
    rp9, cp9 = oracle_list(w, 9.001)
    eo, _, _ = O.empole_real(w.xyz, w.box, w.molid, rp7, cp7, w.mpole, S["beta"], S["rc_ewald"])
    ev, _, _ = O.evdw(w.xyz, w.box, w.molid, rp9, cp9, 0, w.vdw_rad, w.vdw_eps, S["rc_vdw"])
    assert rel(np_(e7)[0], eo[0]) < 1e-10
    assert rel(float(np_(e9).ravel()[0]), ev) < 1e-10
    # the same slot twice is rejected before anything is queued
    with pytest.raises(tk.TkError) as e:
        ctx.nblists(sysr, [7.001, 9.001], [2, 2])
    assert e.value.status == tk.E_ARG


def test_nblist_multi_four_and_empty(ctx, tk):
    # four lists on two streams (two per stream), then an empty system
    import torch
    rng = np.random.default_rng(11)
    box, n = 21.0, 900
    xyz = rng.uniform(0.0, box, size=(n, 3))
    sysr = ctx.system(xyz, box, np.arange(n) // 3)
    main = torch.cuda.current_stream(ctx.device)
    side = torch.cuda.Stream(device=ctx.device)
    side.wait_stream(main)
    cuts = [2.5, 4.0, 6.0, 10.4]
    lists = ctx.nblists(sysr, cuts, [4, 5, 6, 7], streams=[main, side, main, side])
    main.wait_stream(side)
    for lst, rc in zip(lists, cuts):
        rp, cp = O.nblist(xyz, box, rc)
        assert_list_equal(lst, rp, cp)
    empty = ctx.system(np.zeros((0, 3)), box, np.zeros(0, dtype=np.int32))
    l0, l1 = ctx.nblists(empty, [3.0, 5.0], [4, 5])
    assert l0.npairs == 0 and l1.npairs == 0
    assert np.array_equal(np_(l0.row_ptr), [0]) and np.array_equal(np_(l1.row_ptr), [0])


def test_pair_terms_on_streams(ctx, tk):
    # multipoles and HAL of one context on two streams at once (each stream has
    # its own scratch) give bitwise what they give one after the other
    import torch
    w = water("water7853")
    sysr = ctx.system(w.xyz, w.box, w.molid)
    l7, l9 = ctx.nblists(sysr, [7.001, 9.001], [0, 1])

    def run():
        em = ctx.empole_real(sysr, l7, w.mpole, S["beta"], S["rc_ewald"])
        ev = ctx.evdw(sysr, l9, tk.VDW_HAL, w.vdw_rad, w.vdw_eps, S["rc_vdw"], S["taper_frac"],
                      S["dhal"], S["ghal"])
        return em, ev

    em0, ev0 = run()
    main = torch.cuda.current_stream(ctx.device)
    s1, s2 = torch.cuda.Stream(device=ctx.device), torch.cuda.Stream(device=ctx.device)
    s1.wait_stream(main)
    s2.wait_stream(main)
    for _ in range(3):
        with torch.cuda.stream(s1):
            em = ctx.empole_real(sysr, l7, w.mpole, S["beta"], S["rc_ewald"])
        with torch.cuda.stream(s2):
            ev = ctx.evdw(sysr, l9, tk.VDW_HAL, w.vdw_rad, w.vdw_eps, S["rc_vdw"],
                          S["taper_frac"], S["dhal"], S["ghal"])
        main.wait_stream(s1)
        main.wait_stream(s2)
        for a, b in zip(em + ev, em0 + ev0):
            assert np.array_equal(np_(a), np_(b))


def test_nblist_errors(ctx, tk):
    xyz = np.random.default_rng(0).uniform(0, 10, size=(20, 3))
    sysr = ctx.system(xyz, 10.0, np.arange(20))
    with pytest.raises(tk.TkError) as e:
        ctx.nblist(sysr, 5.5)
    assert e.value.status == tk.E_CUTOFF
    bad = xyz.copy()
    bad[3, 1] = np.nan
    with pytest.raises(tk.TkError) as e:
        ctx.nblist(ctx.system(bad, 10.0, np.arange(20)), 4.0)
    assert e.value.status == tk.E_ARG
    # too small a capacity reports the required size (binding then retries)
    lst = ctx.nblist(sysr, 4.0, cap=3)
    rp, cp = O.nblist(xyz, 10.0, 4.0)
    assert_list_equal(lst, rp, cp)


# ----------------------------------------------------------------------------
def setup_amoeba(ctx, name, rc_list, slot):
    w = water(name)
    sysr = ctx.system(w.xyz, w.box, w.molid)
    lst = ctx.nblist(sysr, rc_list, plan_slot=slot)
    rp, cp = oracle_list(w, rc_list)
    return w, sysr, lst, rp, cp


@pytest.mark.parametrize("name", ["water216", "water7853"])
def test_empole_fp64(ctx, name):
    w, sysr, lst, rp, cp = setup_amoeba(ctx, name, 7.001, 2)
    e, f, vir = ctx.empole_real(sysr, lst, w.mpole, S["beta"], 7.0)
    eo, fo, vo = O.empole_real(w.xyz, w.box, w.molid, rp, cp, w.mpole, S["beta"], 7.0)
    e = np_(e)
    for k in range(3):
        assert rel(e[k], eo[k]) < 1e-10, (k, e[k], eo[k])
    assert fmax_rel(np_(f), fo) < 1e-8
    assert np.abs(np_(vir) - vo).max() < 1e-10 * np.abs(vo).max()


@pytest.mark.parametrize("name", ["water216", "water7853"])
def test_efield_and_tmatvec_fp64(ctx, name):
    w, sysr, lst, rp, cp = setup_amoeba(ctx, name, 7.001, 2)
    fld = ctx.efield_direct(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0)
    fo = O.efield_direct(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole, S["beta"],
                         7.0)
    assert fmax_rel(np_(fld), fo) < 1e-8
    mu = np.random.default_rng(7).normal(0, 0.05, size=(w.n, 3))
    for diag in (0, 1):
        out = ctx.tmatvec(sysr, lst, w.polarity, w.thole, S["beta"], 7.0, mu, include_diag=diag)
        oo = O.tmatvec(w.xyz, w.box, rp, cp, w.polarity, w.thole, S["beta"], 7.0, mu, diag)
        assert fmax_rel(np_(out), oo) < 1e-8


@pytest.mark.parametrize("k", [0, 1, 3, 6])
def test_pcg_iterates_fp64(ctx, k):
    w, sysr, lst, rp, cp = setup_amoeba(ctx, "water216", 7.001, 2)
    mu, info = ctx.polarize_pcg(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0,
                                tol_debye=0.0, maxiter=k)
    mo, io = O.polarize_pcg(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole,
                            S["beta"], 7.0, tol_debye=0.0, maxiter=k)
    assert info["iters"] == io["iters"] == k
    assert info["status"] == io["status"]
    assert np.abs(np_(mu) - mo).max() <= 1e-10 * np.abs(mo).max()
    assert rel(info["rms_debye"], io["rms_debye"]) < 1e-8
    assert rel(info["epol"], io["epol"]) < 1e-10


@pytest.mark.parametrize("name", ["water216", "water7853"])
def test_pcg_converged_fp64(ctx, name):
    w, sysr, lst, rp, cp = setup_amoeba(ctx, name, 7.001, 2)
    mu, info = ctx.polarize_pcg(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0,
                                tol_debye=S["tol_debye"])
    mo, io = O.polarize_pcg(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole,
                            S["beta"], 7.0, tol_debye=S["tol_debye"])
    assert info["converged"] == io["converged"] == 1
    assert info["iters"] == io["iters"]
    assert np.abs(np_(mu) - mo).max() <= 1e-10 * np.abs(mo).max()
    assert rel(info["epol"], io["epol"]) < 1e-10
    assert rel(info["rms_true_debye"], io["rms_true_debye"]) < 1e-6


@pytest.mark.parametrize("name", ["water216", "water7853"])
@pytest.mark.parametrize("form", [0, 1])
def test_evdw_fp64(ctx, name, form):
    w, sysr, lst, rp, cp = setup_amoeba(ctx, name, 9.001, 3)
    rad = w.vdw_rad if form == 0 else np.where(np.arange(w.n) % 3 == 0, 3.15, 1.2)
    e, f, vir = ctx.evdw(sysr, lst, form, rad, w.vdw_eps, 9.0)
    eo, fo, vo = O.evdw(w.xyz, w.box, w.molid, rp, cp, form, rad, w.vdw_eps, 9.0)
    assert rel(float(e), eo) < 1e-10
    assert fmax_rel(np_(f), fo) < 1e-8
    assert np.abs(np_(vir) - vo).max() < 1e-10 * np.abs(vo).max()


def test_echarge_fp64_small(ctx):
    w = synth.charge_lj_water_box(1000, 31.0, 77)
    sysr = ctx.system(w.xyz, w.box, w.molid)
    lst = ctx.nblist(sysr, 12.001, plan_slot=4)
    rp, cp = O.nblist(w.xyz, w.box, 12.001)
    assert_list_equal(lst, rp, cp)
    e, f, vir = ctx.echarge_real(sysr, lst, w.charges, 0.34, 12.0)
    eo, fo, vo = O.echarge_real(w.xyz, w.box, w.molid, rp, cp, w.charges, 0.34, 12.0)
    for k in range(3):
        assert rel(np_(e)[k], eo[k]) < 1e-10
    assert fmax_rel(np_(f), fo) < 1e-8
    # the multipole kernel with mu = Theta = 0 gives the same result
    e2, f2, _ = ctx.empole_real(sysr, lst, w.mpole, 0.34, 12.0)
    assert rel(np_(e2)[0], eo[0]) < 1e-10
    e3, f3, _ = ctx.evdw(sysr, lst, 1, w.vdw_rad, w.vdw_eps, 12.0)
    eo3, fo3, _ = O.evdw(w.xyz, w.box, w.molid, rp, cp, 1, w.vdw_rad, w.vdw_eps, 12.0)
    assert rel(float(e3), eo3) < 1e-10
    assert fmax_rel(np_(f3), fo3) < 1e-8


def test_charge_lj_full_size(ctx, tk):
    # the 96,000-atom charge + LJ box at its full size, as bench.py runs it:
    # the 12 A list bit-exact, FP64 within 1e-10 / 1e-8, the mixed form within
    # 1e-6 relative in energy and 1e-4 kcal/mol/A RMS in force
    print("charge_lj water32000 full size", flush=True)
    w = _cache.setdefault("water32000_charge_lj", synth.make("water32000_charge_lj"))
    sysr = ctx.system(w.xyz, w.box, w.molid)
    lst = ctx.nblist(sysr, 12.001, plan_slot=4)
    rp, cp = O.nblist(w.xyz, w.box, 12.001)
    assert_list_equal(lst, rp, cp)
    eo, fo, vo = O.echarge_real(w.xyz, w.box, w.molid, rp, cp, w.charges, 0.34, 12.0)
    elj, flj, _ = O.evdw(w.xyz, w.box, w.molid, rp, cp, 1, w.vdw_rad, w.vdw_eps, 12.0)
    e, f, vir = ctx.echarge_real(sysr, lst, w.charges, 0.34, 12.0)
    for k in range(3):
        assert rel(np_(e)[k], eo[k]) < 1e-10, k
    assert fmax_rel(np_(f), fo) < 1e-8
    assert np.abs(np_(vir) - vo).max() < 1e-10 * np.abs(vo).max()
    e2, f2, _ = ctx.evdw(sysr, lst, 1, w.vdw_rad, w.vdw_eps, 12.0)
    assert rel(float(e2), elj) < 1e-10
    assert fmax_rel(np_(f2), flj) < 1e-8
    rms = lambda a, b: float(np.sqrt(np.mean(np.sum((a - b) ** 2, axis=1))))
    em, fm, _ = ctx.echarge_real(sysr, lst, w.charges, 0.34, 12.0, prec=tk.MIXED)
    for k in range(3):
        assert rel(np_(em)[k], eo[k]) < 1e-6, k
    assert rms(np_(fm), fo) <= 1e-4
    em2, fm2, _ = ctx.evdw(sysr, lst, 1, w.vdw_rad, w.vdw_eps, 12.0, prec=tk.MIXED)
    assert rel(float(em2), elj) < 1e-6
    assert rms(np_(fm2), flj) <= 1e-4


def test_deterministic_repeat(ctx):
    w, sysr, lst, rp, cp = setup_amoeba(ctx, "water7853", 7.001, 2)
    e1, f1, _ = ctx.empole_real(sysr, lst, w.mpole, S["beta"], 7.0)
    e2, f2, _ = ctx.empole_real(sysr, lst, w.mpole, S["beta"], 7.0)
    assert np.array_equal(np_(e1), np_(e2)) and np.array_equal(np_(f1), np_(f2))
    m1, _ = ctx.polarize_pcg(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0)
    m2, _ = ctx.polarize_pcg(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0)
    assert np.array_equal(np_(m1), np_(m2))


def test_plan_mismatch_is_rejected(ctx, tk):
    w, sysr, lst, rp, cp = setup_amoeba(ctx, "water216", 7.001, 2)
    other = ctx.system(w.xyz[:30], w.box, w.molid[:30])
    with pytest.raises(tk.TkError) as e:
        ctx.empole_real(other, lst, w.mpole[:30], S["beta"], 7.0)
    assert e.value.status == tk.E_PLAN
    with pytest.raises(tk.TkError) as e:
        ctx.empole_real(sysr, lst, w.mpole, S["beta"], 7.5)   # kernel cutoff beyond the list
    assert e.value.status == tk.E_ARG
