"""GPU: the multi-system batch step and the serving runtime, through the C-ABI.

- A system stepped inside a batch gives bitwise the same results as the same
  system stepped alone (every per-system sum runs in a fixed order over that
  system's own units and cells).
- Every system of a batch matches the FP64 oracle at the parity tolerances
  (energies 1e-10 relative, forces 1e-8 of the RMS, converged dipoles with
  the same iteration count), including a box small enough that its vdW
  cutoff is clamped to box/2 - skin.
- The server returns what the batch step returns, keeps its lanes' measured
  device memory within its budget, rejects requests larger than the budget,
  takes a request that arrives while another batch is on the GPU at once on
  another lane (bitwise the same results as alone), and starts a session's
  solve from its previous dipoles.
"""
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_1906_01211_amd import synth

pytestmark = pytest.mark.gpu
S = synth.AMOEBA_SETTINGS
DENSITY = 0.03335   # waters per A^3, as in the serving request stream


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


def box_of(n_w):
    return (n_w / DENSITY) ** (1.0 / 3.0)


@pytest.fixture(scope="module")
def systems():
    # 300 atoms (vdW cutoff clamped), 648 atoms, 1,500 atoms, 3,000 atoms
    return [synth.amoeba_water_box(100, box_of(100), 31),
            synth.make("water216"),
            synth.amoeba_water_box(500, box_of(500), 32),
            synth.amoeba_water_box(1000, box_of(1000), 33)]


def np_(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def fmax_rel(got, ref):
    return np.abs(np.asarray(got) - ref).max() / np.sqrt(np.mean(ref ** 2))


def same_result(a, b):
    assert a["e_mpole"] == b["e_mpole"] and a["w_mpole"] == b["w_mpole"]
    assert a["e_vdw"] == b["e_vdw"] and a["w_vdw"] == b["w_vdw"]
    assert a["pcg"] == b["pcg"] and a["rc_vdw"] == b["rc_vdw"]


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_equals_alone(tk, ctx, systems, prec):
    prm = tk.step_params(S, prec)
    res, fm, mu, fv = ctx.batch_step(systems, prm)
    for k, w in enumerate(systems):
        r1, fm1, mu1, fv1 = ctx.batch_step([w], prm)
        same_result(res[k], r1[0])
        assert np.array_equal(np_(fm[k]), np_(fm1[0]))
        assert np.array_equal(np_(mu[k]), np_(mu1[0]))
        assert np.array_equal(np_(fv[k]), np_(fv1[0]))
    # a different batch order changes nothing either
    rr, fmr, mur, fvr = ctx.batch_step(systems[::-1], prm)
    for k in range(len(systems)):
        same_result(res[k], rr[len(systems) - 1 - k])
        assert np.array_equal(np_(mu[k]), np_(mur[len(systems) - 1 - k]))


def test_batch_matches_oracle(tk, ctx, systems):
    prm = tk.step_params(S, 0)
    res, fm, mu, fv = ctx.batch_step(systems, prm)
    for k, w in enumerate(systems):
        rv = min(S["rc_vdw"], 0.5 * w.box - S["skin"])
        assert res[k]["rc_vdw"] == rv
        if k == 0:
            assert rv < S["rc_vdw"]   # the small box clamps its vdW cutoff
        rp7, cp7 = O.nblist(w.xyz, w.box, S["rc_ewald"] + S["skin"])
        rp9, cp9 = O.nblist(w.xyz, w.box, rv + S["skin"])
        e, f, vir = O.empole_real(w.xyz, w.box, w.molid, rp7, cp7, w.mpole, S["beta"], S["rc_ewald"])
        for j in range(3):
            assert rel(res[k]["e_mpole"][j], e[j]) < 1e-10
        assert fmax_rel(np_(fm[k]), f) < 1e-8
        assert np.abs(np.array(res[k]["w_mpole"]) - vir.ravel()).max() < 1e-10 * np.abs(vir).max()
        mo, io = O.polarize_pcg(w.xyz, w.box, w.molid, rp7, cp7, w.mpole, w.polarity, w.thole,
                                S["beta"], S["rc_ewald"], tol_debye=S["tol_debye"])
        assert res[k]["pcg"]["iters"] == io["iters"] and res[k]["pcg"]["converged"] == 1
        assert np.abs(np_(mu[k]) - mo).max() <= 1e-10 * np.abs(mo).max()
        assert rel(res[k]["pcg"]["epol"], io["epol"]) < 1e-10
        ev, fvo, vvo = O.evdw(w.xyz, w.box, w.molid, rp9, cp9, 0, w.vdw_rad, w.vdw_eps, rv)
        assert rel(res[k]["e_vdw"], ev) < 1e-10
        assert fmax_rel(np_(fv[k]), fvo) < 1e-8


def test_batch_mixed_within_budget(tk, ctx, systems):
    r64, fm64, mu64, fv64 = ctx.batch_step(systems, tk.step_params(S, 0))
    rmx, fmmx, mumx, fvmx = ctx.batch_step(systems, tk.step_params(S, 1))
    for k in range(len(systems)):
        assert rel(rmx[k]["e_mpole"][0], r64[k]["e_mpole"][0]) < 1e-6
        assert rel(rmx[k]["e_vdw"], r64[k]["e_vdw"]) < 1e-6
        assert np.sqrt(np.mean(np.sum((np_(fmmx[k]) - np_(fm64[k])) ** 2, axis=1))) < 1e-4
        assert np.sqrt(np.mean(np.sum((np_(fvmx[k]) - np_(fv64[k])) ** 2, axis=1))) < 1e-4
        # dipoles: both solves stop at 1e-5 D; their difference is at that level
        d = 4.80320 * np.sqrt(np.mean(np.sum((np_(mumx[k]) - np_(mu64[k])) ** 2, axis=1)))
        assert d < 2e-5
        assert rmx[k]["pcg"]["rms_true_debye"] <= S["tol_debye"]


def test_mixed_step_first_on_a_fresh_context(tk, ctx, systems):
    """A mixed-form batch step as the first call of a new context (its
    per-stream pair-term buffers still at the sizes the 14-7 pass gave them;
    the multipole pass inside the solve grows them) returns bitwise what the
    same step returns on a context that has run other work before.
    Regression: the solver used to take the shared accumulator buffer before
    the multipole pass reallocated it."""
    prm = tk.step_params(S, 1)
    batch = systems[::-1]
    ref = ctx.batch_step(batch, prm)
    fresh = tk.Context(0)
    try:
        got = fresh.batch_step(batch, prm)
        for k in range(len(batch)):
            same_result(got[0][k], ref[0][k])
            for j in (1, 2, 3):
                assert np.array_equal(np_(got[j][k]), np_(ref[j][k]))
    finally:
        fresh.close()


def test_batch_guess_per_system(tk, ctx, systems):
    prm = tk.step_params(S, 0)
    res, fm, mu, fv = ctx.batch_step(systems, prm)
    import torch
    guess = torch.cat(mu)
    use = [1, 0, 1, 0]
    rg, _, mug, _ = ctx.batch_step(systems, prm, mu_guess=guess, use_guess=use)
    for k in range(len(systems)):
        if use[k]:   # started from the converged dipoles: (almost) converged at once
            assert rg[k]["pcg"]["iters"] <= 1 and rg[k]["pcg"]["converged"] == 1
        else:        # not using the guess: identical to the plain step
            same_result(rg[k], res[k])


def test_batch_errors(tk, ctx, systems):
    prm = tk.step_params(dict(S, rc_ewald=7.3), 0)   # 7.3 + skin > 14.42/2
    with pytest.raises(tk.TkError) as e:
        ctx.batch_step(systems, prm)
    assert e.value.status == tk.E_CUTOFF
    bad = tk.step_params(dict(S, tol_debye=-1.0), 0)
    with pytest.raises(tk.TkError) as e:
        ctx.batch_step(systems, bad)
    assert e.value.status == tk.E_ARG


def wait(srv, rid, limit=60.0):
    t0 = time.time()
    while True:
        out = srv.poll(rid)
        if out is not None:
            return out
        assert time.time() - t0 < limit, "request did not complete"
        time.sleep(0.001)


@pytest.mark.parametrize("prec", [0, 1])
def test_server_matches_batch_and_budget(tk, ctx, systems, prec):
    prm = tk.step_params(S, prec)
    ref = [ctx.batch_step([w], prm) for w in systems]
    # the largest system alone, on a fresh context, to size the budget: room
    # for about two lanes' worth, so admission binds and several batches form
    big = tk.Context(0)
    try:
        big.batch_step([systems[3]], prm)
        one = big.arena_bytes()
    finally:
        big.close()
    budget = 2 * one + (24 << 20)
    srv = tk.Server(prm, budget, max_batch=8)
    try:
        ids = [srv.submit(w) for w in systems + systems]
        outs = [wait(srv, i) for i in ids]
        for j, out in enumerate(outs):
            r, t, fm, mu, fv = out
            k = j % len(systems)
            same_result(r, ref[k][0][0])
            assert np.array_equal(fm, np_(ref[k][1][0]))
            assert np.array_equal(mu, np_(ref[k][2][0]))
            assert np.array_equal(fv, np_(ref[k][3][0]))
            assert t["t_submit"] <= t["t_start"] <= t["t_done"]
            assert 0 <= t["lane"] < 3
        assert len({out[1]["batch_index"] for out in outs}) >= 2
        st = srv.stats()
        # measured (not estimated) device bytes of the lanes stayed in the budget
        assert 0 < st["peak_device_bytes"] <= budget
        for i in ids:
            srv.release(i)
        with pytest.raises(tk.TkError) as e:
            srv.submit(synth.amoeba_water_box(40000, box_of(40000), 34))
        assert e.value.status == tk.E_CAPACITY
    finally:
        srv.close()


def test_server_admits_while_a_batch_runs(tk, ctx, systems):
    """A request submitted while a large one is on the GPU is taken by another
    lane at once (it starts before the large one ends), and its results are
    bitwise those of the same system stepped alone."""
    prm = tk.step_params(S, 0)
    large = synth.amoeba_water_box(10000, box_of(10000), 35)   # 30,000 atoms
    small = systems[1]
    alone = ctx.batch_step([small], prm)
    srv = tk.Server(prm, 16 << 30, max_batch=8)
    try:
        for rep in range(2):   # first on fresh lanes (the large step is long), then warm
            a = srv.submit(large)
            time.sleep(0.001)   # a lane has taken the large request
            b = srv.submit(small)
            ob = wait(srv, b)
            oa = wait(srv, a)
            ra, ta = oa[0], oa[1]
            rb, tb = ob[0], ob[1]
            if rep == 0:
                assert tb["batch_index"] != ta["batch_index"] and tb["lane"] != ta["lane"]
                assert tb["t_start"] < ta["t_done"], "the small request waited for the large one"
                assert tb["t_done"] < ta["t_done"]
            same_result(rb, alone[0][0])
            assert np.array_equal(ob[2], np_(alone[1][0]))
            assert np.array_equal(ob[3], np_(alone[2][0]))
            assert np.array_equal(ob[4], np_(alone[3][0]))
            assert ra["pcg"]["converged"] == 1
    finally:
        srv.close()


def test_server_one_lane(tk, ctx, systems):
    """One lane and batches of one: every request runs alone, in arrival order,
    on lane 0, with the results of the same system stepped alone; a lane
    count outside 1-3 is rejected."""
    import ctypes as C
    prm = tk.step_params(S, 0)
    ref = [ctx.batch_step([w], prm) for w in systems[:2]]
    srv = tk.Server(prm, 1 << 30, max_batch=1, lanes=1)
    try:
        ids = [srv.submit(w) for w in systems[:2]]
        outs = [wait(srv, i) for i in ids]
        for k, out in enumerate(outs):
            same_result(out[0], ref[k][0][0])
            assert np.array_equal(out[3], np_(ref[k][2][0]))
            assert out[1]["lane"] == 0 and out[1]["batch_size"] == 1
        assert outs[0][1]["t_done"] <= outs[1][1]["t_start"]
        assert srv.stats()["lanes"] == 1
    finally:
        srv.close()
    h = C.c_void_p()
    for bad in (0, 4):
        st = tk.load().tk_server_create_lanes(0, C.byref(prm), 1 << 30, 8, bad, C.byref(h))
        assert st == tk.E_ARG


def test_server_session_guess(tk, systems):
    prm = tk.step_params(S, 0)
    srv = tk.Server(prm, 1 << 30)
    try:
        w = systems[2]
        a = wait(srv, srv.submit(w, session=7))
        b = wait(srv, srv.submit(w, session=7))   # starts from a's dipoles
        c = wait(srv, srv.submit(w))               # no session: from alpha * E_perm
        assert b[0]["pcg"]["iters"] <= 1 and b[0]["pcg"]["converged"] == 1
        assert c[0]["pcg"]["iters"] == a[0]["pcg"]["iters"] > 0
        assert np.array_equal(c[3], a[3])
    finally:
        srv.close()
