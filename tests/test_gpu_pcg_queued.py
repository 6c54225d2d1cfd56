"""GPU: the queued polarization solve (tk_polarize_pcg_queued).

The same PCG as tk_polarize_pcg with no host synchronisation: given at least
the iterations the synchronous solve takes, its dipoles and every outcome
field must equal that solve's bitwise (steps queued after convergence change
nothing); at a fixed iteration count it must match the oracle's iterate; its
outcome lives in device memory and is written in stream order, so chained
solves need no synchronisation between them.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1906_01211_amd import synth

pytestmark = pytest.mark.gpu

S = synth.AMOEBA_SETTINGS
E_ARG, E_CAPACITY, E_NOCONV = -1, -3, -4
R7 = S["rc_ewald"] + S["skin"]


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


def np_(t):
    return t.detach().cpu().numpy()


def setup(ctx, name, slot=0):
    import torch
    w = water(name)
    sysr = ctx.system(w.xyz, w.box, w.molid)
    lst = ctx.nblist(sysr, R7, plan_slot=slot)
    T = lambda a: torch.as_tensor(a, device=ctx.device)
    return w, sysr, lst, T(w.mpole), T(w.polarity), T(w.thole)


@pytest.mark.parametrize("name", ["water216", "water7853"])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("extra", [0, 7])
def test_queued_equals_sync(ctx, tk, name, prec, extra):
    w, sysr, lst, mp, pol, th = setup(ctx, name)
    mu, info = ctx.polarize_pcg(sysr, lst, mp, pol, th, S["beta"], S["rc_ewald"],
                                tol_debye=S["tol_debye"], maxiter=S["maxiter"], prec=prec)
    assert info["status"] == 0
    if prec == tk.MIXED and info["refinements"]:
        pytest.skip("the synchronous mixed solve refined (the queued one does not)")
    mq, idev = ctx.polarize_pcg_queued(sysr, lst, mp, pol, th, S["beta"], S["rc_ewald"],
                                       info["iters"] + extra, tol_debye=S["tol_debye"],
                                       prec=prec)
    iq = ctx.pcg_info(idev)
    assert np.array_equal(np_(mq), np_(mu))
    assert iq == info


@pytest.mark.parametrize("k", [1, 3, 6])
def test_queued_fixed_iterations_against_oracle(ctx, k):
    w, sysr, lst, mp, pol, th = setup(ctx, "water216")
    rp, cp = O.nblist(w.xyz, w.box, R7)
    mq, idev = ctx.polarize_pcg_queued(sysr, lst, mp, pol, th, S["beta"], S["rc_ewald"], k,
                                       tol_debye=0.0)
    iq = ctx.pcg_info(idev)
    mo, io = O.polarize_pcg(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole,
                            S["beta"], S["rc_ewald"], tol_debye=0.0, maxiter=k)
    assert iq["iters"] == io["iters"] == k
    assert iq["status"] == io["status"] == E_NOCONV and iq["converged"] == 0
    assert np.abs(np_(mq) - mo).max() <= 1e-10 * np.abs(mo).max()
    assert abs(iq["rms_debye"] - io["rms_debye"]) <= 1e-8 * io["rms_debye"]
    assert abs(iq["epol"] - io["epol"]) <= 1e-10 * abs(io["epol"])


def test_queued_chain_without_sync(ctx):
    # two solves back to back on a side stream, the second starting from the
    # first's dipoles, and nothing read in between: the same as the
    # synchronous pair
    import torch
    w, sysr, lst, mp, pol, th = setup(ctx, "water7853")
    m1, i1 = ctx.polarize_pcg(sysr, lst, mp, pol, th, S["beta"], S["rc_ewald"],
                              tol_debye=S["tol_debye"], maxiter=S["maxiter"])
    m2, i2 = ctx.polarize_pcg(sysr, lst, mp, pol, th, S["beta"], S["rc_ewald"],
                              tol_debye=S["tol_debye"] * 0.1, maxiter=S["maxiter"], mu_guess=m1)
    side = torch.cuda.Stream(device=ctx.device)
    side.wait_stream(torch.cuda.current_stream(ctx.device))
    with torch.cuda.stream(side):
        q1, d1 = ctx.polarize_pcg_queued(sysr, lst, mp, pol, th, S["beta"], S["rc_ewald"],
                                         S["maxiter"], tol_debye=S["tol_debye"])
        q2, d2 = ctx.polarize_pcg_queued(sysr, lst, mp, pol, th, S["beta"], S["rc_ewald"],
                                         S["maxiter"], tol_debye=S["tol_debye"] * 0.1,
                                         mu_guess=q1)
    torch.cuda.current_stream(ctx.device).wait_stream(side)
    torch.cuda.synchronize()
    assert np.array_equal(np_(q1), np_(m1)) and ctx.pcg_info(d1) == i1
    assert np.array_equal(np_(q2), np_(m2)) and ctx.pcg_info(d2) == i2


def test_queued_failed_list(ctx, tk):
    # a stream-ordered list whose build went past a bound: the queued solve
    # reports TK_E_CAPACITY on the device
    import torch
    w, sysr, lst, mp, pol, th = setup(ctx, "water216")
    b = ctx.nblist_bounds(0, headroom=0.0)
    b.max_row -= 1
    al = ctx.nblist_async(sysr, R7, plan_slot=1, bounds=b)
    assert al.status() == E_CAPACITY
    info_dev = torch.full((40,), 0xAB, dtype=torch.uint8, device=ctx.device)
    mq, idev = ctx.polarize_pcg_queued(sysr, al, mp, pol, th, S["beta"], S["rc_ewald"], 20,
                                       tol_debye=S["tol_debye"], info_dev=info_dev)
    iq = ctx.pcg_info(idev)
    assert iq["status"] == E_CAPACITY and iq["converged"] == 0
    # a good list in the same slot solves again
    ok = ctx.nblist_async(sysr, R7, plan_slot=1, bounds=ctx.nblist_bounds(0, 0.1))
    mu, info = ctx.polarize_pcg(sysr, lst, mp, pol, th, S["beta"], S["rc_ewald"],
                                tol_debye=S["tol_debye"], maxiter=S["maxiter"])
    mq, idev = ctx.polarize_pcg_queued(sysr, ok, mp, pol, th, S["beta"], S["rc_ewald"],
                                       S["maxiter"], tol_debye=S["tol_debye"])
    assert np.array_equal(np_(mq), np_(mu)) and ctx.pcg_info(idev) == info


def test_queued_arguments_and_empty(ctx, tk):
    import torch
    w, sysr, lst, mp, pol, th = setup(ctx, "water216")
    for it in (0, -1, 10001):
        with pytest.raises(tk.TkError) as err:
            ctx.polarize_pcg_queued(sysr, lst, mp, pol, th, S["beta"], S["rc_ewald"], it)
        assert err.value.status == E_ARG
    with pytest.raises(tk.TkError) as err:
        ctx.polarize_pcg_queued(sysr, lst, mp, pol, th, S["beta"], S["rc_ewald"], 5, prec=7)
    assert err.value.status == E_ARG
    e = ctx.system(np.zeros((0, 3)), w.box, np.zeros(0, dtype=np.int32))
    le = ctx.nblist(e, R7, plan_slot=4)
    z = torch.zeros((0, 10), dtype=torch.float64, device=ctx.device)
    z1 = torch.zeros(0, dtype=torch.float64, device=ctx.device)
    mq, idev = ctx.polarize_pcg_queued(e, le, z, z1, z1, S["beta"], S["rc_ewald"], 5)
    iq = ctx.pcg_info(idev)
    assert mq.shape == (0, 3)
    assert iq["status"] == 0 and iq["converged"] == 1 and iq["iters"] == 0


@pytest.mark.parametrize("name", ["water216", "water7853"])
@pytest.mark.parametrize("prec", [0, 1])
def test_fused_queued_equals_sync(ctx, tk, name, prec):
    # tk_empole_polarize_queued: multipole terms and dipoles bitwise those of
    # tk_empole_polarize
    w, sysr, lst, mp, pol, th = setup(ctx, name)
    (e, f, v), (mu, info) = ctx.empole_polarize(sysr, lst, mp, pol, th, S["beta"], S["rc_ewald"],
                                                tol_debye=S["tol_debye"], maxiter=S["maxiter"],
                                                prec=prec)
    assert info["status"] == 0
    if prec == tk.MIXED and info["refinements"]:
        pytest.skip("the synchronous mixed solve refined (the queued one does not)")
    (eq, fq, vq), (mq, idev) = ctx.empole_polarize_queued(sysr, lst, mp, pol, th, S["beta"],
                                                          S["rc_ewald"], info["iters"] + 2,
                                                          tol_debye=S["tol_debye"], prec=prec)
    for x, y in ((eq, e), (fq, f), (vq, v), (mq, mu)):
        assert np.array_equal(np_(x), np_(y))
    assert ctx.pcg_info(idev) == info


def test_fused_queued_empty(ctx, tk):
    import torch
    w = water("water216")
    e = ctx.system(np.zeros((0, 3)), w.box, np.zeros(0, dtype=np.int32))
    le = ctx.nblist(e, R7, plan_slot=4)
    z = torch.zeros((0, 10), dtype=torch.float64, device=ctx.device)
    z1 = torch.zeros(0, dtype=torch.float64, device=ctx.device)
    (en, f, v), (mq, idev) = ctx.empole_polarize_queued(e, le, z, z1, z1, S["beta"],
                                                        S["rc_ewald"], 3)
    assert np_(en).tolist() == [0.0] * 3 and np_(v).tolist() == [0.0] * 9
    iq = ctx.pcg_info(idev)
    assert iq["status"] == 0 and iq["converged"] == 1


def test_queued_mixed_outcome_is_the_fp64_check(ctx, tk):
    # a tolerance below what the FP32 operator resolves: the synchronous mixed
    # solve refines in FP64; the queued one does not refine, so it must report
    # the failed FP64 check (not the FP32 recurrence's test)
    w, sysr, lst, mp, pol, th = setup(ctx, "water216")
    _, info = ctx.polarize_pcg(sysr, lst, mp, pol, th, S["beta"], S["rc_ewald"],
                               tol_debye=1e-10, maxiter=100, prec=tk.MIXED)
    assert info["refinements"] >= 1
    _, idev = ctx.polarize_pcg_queued(sysr, lst, mp, pol, th, S["beta"], S["rc_ewald"], 100,
                                      tol_debye=1e-10, prec=tk.MIXED)
    iq = ctx.pcg_info(idev)
    assert iq["rms_true_debye"] > 1e-10
    assert iq["status"] == E_NOCONV and iq["converged"] == 0 and iq["refinements"] == 0
    # at the usual tolerance the same queued solve meets its FP64 check
    _, idev = ctx.polarize_pcg_queued(sysr, lst, mp, pol, th, S["beta"], S["rc_ewald"], 100,
                                      tol_debye=S["tol_debye"], prec=tk.MIXED)
    iq = ctx.pcg_info(idev)
    assert iq["status"] == 0 and iq["converged"] == 1
    assert iq["rms_true_debye"] <= S["tol_debye"]
