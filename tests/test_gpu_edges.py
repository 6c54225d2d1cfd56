"""Degenerate cases of the solver and the pair terms against the FP64 CPU
oracle: no polarizable atoms, polarizable oxygens only, a zero iteration
limit, and systems of one and two atoms."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1906_01211_amd import synth

pytestmark = pytest.mark.gpu

S = synth.AMOEBA_SETTINGS
_cache = {}


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


def np_(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def water216(ctx):
    w = _cache.setdefault("w", synth.make("water216"))
    sysr = ctx.system(w.xyz, w.box, w.molid)
    lst = ctx.nblist(sysr, 7.001, plan_slot=2)
    if "list" not in _cache:
        _cache["list"] = O.nblist(w.xyz, w.box, 7.001)
    return w, sysr, lst, _cache["list"]


@pytest.mark.parametrize("which", ["none", "oxygens"])
def test_pcg_with_unpolarizable_atoms(ctx, which):
    w, sysr, lst, (rp, cp) = water216(ctx)
    pol = np.zeros(w.n) if which == "none" else np.where(np.arange(w.n) % 3 == 0, w.polarity, 0.0)
    print(f"pcg polarizable {which}", flush=True)
    mu, info = ctx.polarize_pcg(sysr, lst, w.mpole, pol, w.thole, S["beta"], 7.0)
    mo, io = O.polarize_pcg(w.xyz, w.box, w.molid, rp, cp, w.mpole, pol, w.thole, S["beta"], 7.0)
    assert info["iters"] == io["iters"] and info["converged"] == io["converged"] == 1
    m = np_(mu)
    assert np.all(m[pol == 0.0] == 0.0)   # unpolarizable atoms carry no dipole
    if which == "none":
        assert info["iters"] == 0 and info["epol"] == 0.0 and np.all(m == 0.0)
    else:
        assert np.abs(m - mo).max() <= 1e-10 * np.abs(mo).max()
        assert rel(info["epol"], io["epol"]) < 1e-10
    mu2, info2 = ctx.polarize_pcg2(sysr, lst, w.mpole, pol, w.thole, S["beta"], 7.0, 0.5)
    mo2, io2 = O.polarize_pcg2(w.xyz, w.box, w.molid, rp, cp, w.mpole, pol, w.thole, S["beta"],
                               7.0, 0.5)
    for v in range(2):
        assert info2[v]["iters"] == io2[v]["iters"]
        if which == "oxygens":
            assert np.abs(np_(mu2)[v] - mo2[v]).max() <= 1e-10 * np.abs(mo2[v]).max()
        else:
            assert np.all(np_(mu2)[v] == 0.0)


def test_pcg_zero_iteration_limit(ctx, tk):
    w, sysr, lst, (rp, cp) = water216(ctx)
    mu, info = ctx.polarize_pcg(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0,
                                maxiter=0)
    mo, io = O.polarize_pcg(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole,
                            S["beta"], 7.0, maxiter=0)
    assert info["status"] == io["status"] == tk.E_NOCONV
    assert info["iters"] == io["iters"] == 0 and info["converged"] == 0
    # the returned dipoles are the direct guess alpha E
    assert np.abs(np_(mu) - mo).max() <= 1e-12 * np.abs(mo).max()
    assert rel(info["rms_debye"], io["rms_debye"]) < 1e-10


@pytest.mark.parametrize("n", [1, 2])
def test_one_and_two_atoms(ctx, tk, n):
    box = 20.0
    xyz = np.array([[3.0, 4.0, 5.0], [5.1, 4.6, 6.2]])[:n]
    molid = np.arange(n, dtype=np.int32)
    rng = np.random.default_rng(n)
    mpole = rng.normal(0, 0.1, (n, 10))
    mpole[:, 9] = -(mpole[:, 4] + mpole[:, 7])
    pol = np.full(n, 0.837)
    th = np.full(n, 0.39)
    print(f"{n} atoms", flush=True)
    sysr = ctx.system(xyz, box, molid)
    lst = ctx.nblist(sysr, 7.001, plan_slot=6)
    rp, cp = O.nblist(xyz, box, 7.001)
    assert lst.npairs == len(cp) == n - 1
    e, f, _ = ctx.empole_real(sysr, lst, mpole, S["beta"], 7.0)
    eo, fo, _ = O.empole_real(xyz, box, molid, rp, cp, mpole, S["beta"], 7.0)
    assert np.allclose(np_(e), eo, rtol=1e-12, atol=0)
    assert np.abs(np_(f) - fo).max() <= 1e-12 * max(np.abs(fo).max(), 1e-300)
    mu, info = ctx.polarize_pcg(sysr, lst, mpole, pol, th, S["beta"], 7.0)
    mo, io = O.polarize_pcg(xyz, box, molid, rp, cp, mpole, pol, th, S["beta"], 7.0)
    assert info["iters"] == io["iters"] and info["converged"] == 1
    assert np.abs(np_(mu) - mo).max() <= 1e-12 * np.abs(mo).max()
    ev, fv, _ = ctx.evdw(sysr, lst, tk.VDW_HAL, np.full(n, 3.4), np.full(n, 0.11), 7.0)
    evo, fvo, _ = O.evdw(xyz, box, molid, rp, cp, 0, np.full(n, 3.4), np.full(n, 0.11), 7.0)
    assert rel(float(ev), evo) < 1e-12 if n == 2 else float(ev) == 0.0


def test_arena_budget_refuses_then_recovers(tk):
    """A context with a device budget too small for a list build returns
    TK_E_NOMEM without touching what it holds; with the budget raised the same
    calls succeed and match the oracle.  A solve that needs buffers beyond a
    budget pinned at the current holdings is refused the same way."""
    c = tk.Context(0)
    try:
        w = synth.make("water216")
        print("arena budget: water216", flush=True)
        sysr = c.system(w.xyz, w.box, w.molid)
        c.set_arena_budget(64 << 10)
        with pytest.raises(tk.TkError) as ei:
            c.nblist(sysr, 7.001, plan_slot=0)
        assert ei.value.status == tk.E_NOMEM
        assert c.arena_bytes() <= 64 << 10
        c.set_arena_budget(0)
        lst = c.nblist(sysr, 7.001, plan_slot=0)
        rp, cp = O.nblist(w.xyz, w.box, 7.001)
        assert np.array_equal(np_(lst.col), cp)
        # nothing beyond what the context now holds: the solver's scratch is refused
        c.set_arena_budget(c.arena_bytes())
        with pytest.raises(tk.TkError) as ei:
            c.polarize_pcg(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0)
        assert ei.value.status == tk.E_NOMEM
        c.set_arena_budget(0)
        mu, info = c.polarize_pcg(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0)
        mo, io = O.polarize_pcg(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole,
                                S["beta"], 7.0)
        assert info["converged"] == 1 and info["iters"] == io["iters"]
        assert np.abs(np_(mu) - mo).max() <= 1e-10 * np.abs(mo).max()
    finally:
        c.close()
