"""One-step truncated conjugate gradient (tk_polarize_tcg1) against the FP64
CPU oracle: dipoles within 1e-10 of their largest component, energy within
1e-10 relative, forces (the total derivative) within 1e-8 of their RMS."""
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


def fmax_rel(got, ref):
    return np.abs(np.asarray(got) - ref).max() / np.sqrt(np.mean(ref ** 2))


@pytest.mark.parametrize("name", ["water216", "water7853"])
def test_tcg1_fp64(ctx, name):
    w = _cache.setdefault(name, synth.make(name))
    sysr = ctx.system(w.xyz, w.box, w.molid)
    lst = ctx.nblist(sysr, 7.001, plan_slot=2)
    rp, cp = O.nblist(w.xyz, w.box, 7.001)
    print(f"tcg1 {name}", flush=True)
    mu, e, f = ctx.polarize_tcg1(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0)
    mo, eo, fo = O.polarize_tcg1(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole,
                                 S["beta"], 7.0)
    assert np.abs(np_(mu) - mo).max() <= 1e-10 * np.abs(mo).max()
    assert abs(np_(e)[0] - eo) <= 1e-10 * abs(eo)
    assert fmax_rel(np_(f), fo) < 1e-8
    # the same dipoles as the first iterate of the device solver
    m1, info = ctx.polarize_pcg(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0,
                                tol_debye=0.0, maxiter=1)
    assert np.abs(np_(m1) - np_(mu)).max() <= 1e-12 * np.abs(mo).max()


def test_tcg1_without_forces_and_without_polarizability(ctx):
    w = _cache.setdefault("water216", synth.make("water216"))
    sysr = ctx.system(w.xyz, w.box, w.molid)
    lst = ctx.nblist(sysr, 7.001, plan_slot=2)
    mu, e, f = ctx.polarize_tcg1(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0,
                                 forces=False)
    assert f is None and np.isfinite(np_(e)[0])
    mu0, e0, f0 = ctx.polarize_tcg1(sysr, lst, w.mpole, np.zeros(w.n), w.thole, S["beta"], 7.0)
    assert not np.any(np_(mu0)) and np_(e0)[0] == 0.0 and not np.any(np_(f0))
    empty = ctx.system(np.zeros((0, 3)), 20.0, np.zeros(0, np.int32))
    l0 = ctx.nblist(empty, 7.001, plan_slot=6)
    mu, e, f = ctx.polarize_tcg1(empty, l0, np.zeros((0, 10)), np.zeros(0), np.zeros(0),
                                 S["beta"], 7.0)
    assert np_(e)[0] == 0.0


@pytest.mark.parametrize("seed", [41, 42])
def test_tcg1_random_boxes(ctx, seed):
    # random water counts (not cubes) at the water density and random cutoffs
    rng = np.random.default_rng(seed)
    n_w = int(rng.integers(60, 400))
    box = (n_w / 0.03335) ** (1.0 / 3.0)
    rc = float(min(rng.uniform(4.0, 7.0), 0.5 * box - 0.01))
    w = synth.amoeba_water_box(n_w, box, 6000 + seed)
    print(f"tcg1 random seed={seed} n_w={n_w} box={box:.2f} rc={rc:.2f}", flush=True)
    sysr = ctx.system(w.xyz, w.box, w.molid)
    lst = ctx.nblist(sysr, rc + 0.001, plan_slot=7)
    rp, cp = O.nblist(w.xyz, w.box, rc + 0.001)
    mu, e, f = ctx.polarize_tcg1(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], rc)
    mo, eo, fo = O.polarize_tcg1(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole,
                                 S["beta"], rc)
    assert np.abs(np_(mu) - mo).max() <= 1e-10 * np.abs(mo).max()
    assert abs(np_(e)[0] - eo) <= 1e-10 * abs(eo)
    assert fmax_rel(np_(f), fo) < 1e-8
