"""Local-frame multipoles (tk_rotate_mpole, tk_empole_frames, tk_epolar_frames)
against the FP64 CPU oracle, on the water frames and on a topology using all
five frame types: rotated multipoles to rounding, energies within 1e-10
relative, forces (torques included) within 1e-8 of their RMS; invalid frames
and empty systems."""
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


def case(ctx, name, frames="water"):
    w = _cache.setdefault(name, synth.make(name))
    n_w = w.n // 3
    ft, fa = (synth.water_frames if frames == "water" else synth.mixed_frames)(n_w)
    loc = synth.water_local_multipoles(n_w, 7)
    sysr = ctx.system(w.xyz, w.box, w.molid)
    lst = ctx.nblist(sysr, 7.001, plan_slot=2)
    key = (name, "list")
    if key not in _cache:
        _cache[key] = O.nblist(w.xyz, w.box, 7.001)
    rp, cp = _cache[key]
    return w, ft, fa, loc, sysr, lst, rp, cp


@pytest.mark.parametrize("frames", ["water", "mixed"])
@pytest.mark.parametrize("name", ["water216", "water7853"])
def test_frames_fp64(ctx, name, frames):
    w, ft, fa, loc, sysr, lst, rp, cp = case(ctx, name, frames)
    print(f"frames {name} {frames}", flush=True)
    g = ctx.rotate_mpole(sysr, ft, fa, loc)
    go = O.rotate_mpole(w.xyz, w.box, ft, fa, loc)
    assert np.abs(np_(g) - go).max() <= 1e-13 * np.abs(go).max()
    e, f, mg, vir = ctx.empole_frames(sysr, lst, ft, fa, loc, S["beta"], 7.0)
    eo, fo, vo = O.empole_frames(w.xyz, w.box, w.molid, rp, cp, ft, fa, loc, S["beta"], 7.0)
    e = np_(e)
    for k in range(3):
        assert abs(e[k] - eo[k]) <= 1e-10 * abs(eo[k]), (k, e[k], eo[k])
    assert fmax_rel(np_(f), fo) < 1e-8
    assert np.abs(np_(vir) - vo).max() <= 1e-10 * np.abs(vo).max()
    assert np.abs(np_(mg) - go).max() <= 1e-13 * np.abs(go).max()
    # the frame part matters: forces at fixed lab-frame multipoles differ
    _, f_lab, _ = O.empole_real(w.xyz, w.box, w.molid, rp, cp, go, S["beta"], 7.0)
    assert fmax_rel(f_lab, fo) > 1e-3


def test_frames_mixed_types_and_reproducible(ctx):
    w, ft, fa, loc, sysr, lst, rp, cp = case(ctx, "water216")
    ft2 = ft.copy()
    ft2[::5] = 0                     # some sites without a frame
    e, f, _, _ = ctx.empole_frames(sysr, lst, ft2, fa, loc, S["beta"], 7.0)
    eo, fo, vo = O.empole_frames(w.xyz, w.box, w.molid, rp, cp, ft2, fa, loc, S["beta"], 7.0)
    assert abs(np_(e)[0] - eo[0]) <= 1e-10 * abs(eo[0])
    assert fmax_rel(np_(f), fo) < 1e-8
    e2, f2, _, _ = ctx.empole_frames(sysr, lst, ft2, fa, loc, S["beta"], 7.0)
    assert np.array_equal(np_(e), np_(e2))   # energies: fixed-order sums
    assert np.abs(np_(f2) - np_(f)).max() <= 1e-12 * np.abs(fo).max()   # forces: atomics


def test_frames_invalid_and_empty(ctx, tk):
    w, ft, fa, loc, sysr, lst, rp, cp = case(ctx, "water216")
    bad = fa.copy()
    bad[3, 0] = 3                    # the site itself
    e, _, _, _ = ctx.empole_frames(sysr, lst, ft, bad, loc, S["beta"], 7.0)
    assert np.all(np.isnan(np_(e)))
    out = ctx.rotate_mpole(sysr, ft, bad, loc)
    assert np.array_equal(np_(out)[3], loc[3])   # an invalid frame copies the site
    e, f, _, _ = ctx.empole_frames(sysr, lst, ft, fa, loc, S["beta"], 7.0)   # clean again
    assert np.all(np.isfinite(np_(e)))
    # a type that takes a y atom refuses a missing or repeated one
    mt, ma = synth.mixed_frames(w.n // 3)
    k = int(np.nonzero(mt == synth.FRAME_3FOLD)[0][0])
    for y in (-1, ma[k, 1]):
        bad = ma.copy()
        bad[k, 2] = y
        e, _, _, w = ctx.empole_frames(sysr, lst, mt, bad, loc, S["beta"], 7.0)
        assert np.all(np.isnan(np_(e))) and np.all(np.isnan(np_(w)))
    with pytest.raises(ValueError):   # frame atoms are [n, 3]
        ctx.rotate_mpole(sysr, ft, fa[:, :2], loc)
    empty = ctx.system(np.zeros((0, 3)), 20.0, np.zeros(0, np.int32))
    l0 = ctx.nblist(empty, 7.001, plan_slot=6)
    e, f, _, _ = ctx.empole_frames(empty, l0, np.zeros(0, np.int32), np.zeros((0, 3), np.int32),
                                np.zeros((0, 10)), S["beta"], 7.0)
    assert np.all(np_(e) == 0.0) and f.shape == (0, 3)


@pytest.mark.parametrize("name", ["water216", "water7853"])
def test_vdw_reduction_chain(ctx, name):
    # sites -> list on the sites -> HAL on the sites -> forces on the atoms
    w = _cache.setdefault(name, synth.make(name))
    parent, red = synth.water_vdw_reduction(w.n // 3)
    sysr = ctx.system(w.xyz, w.box, w.molid)
    sites = ctx.vdw_sites(sysr, parent, red)
    so = O.vdw_sites(w.xyz, w.box, parent, red)
    assert np.abs(np_(sites) - so).max() <= 1e-13 * w.box
    ssys = ctx.system(sites, w.box, w.molid)
    lst = ctx.nblist(ssys, 9.001, plan_slot=3)
    e, fs, _ = ctx.evdw(ssys, lst, 0, w.vdw_rad, w.vdw_eps, 9.0)
    f = ctx.vdw_site_forces(parent, red, fs)
    rp, cp = O.nblist(so, w.box, 9.001)
    eo, fso, _ = O.evdw(so, w.box, w.molid, rp, cp, 0, w.vdw_rad, w.vdw_eps, 9.0)
    fo = O.vdw_forces_to_atoms(parent, red, fso)
    assert abs(float(e) - eo) <= 1e-10 * abs(eo)
    assert fmax_rel(np_(f), fo) < 1e-8


def test_vdw_reduction_invalid_parent(ctx):
    w = _cache.setdefault("water216", synth.make("water216"))
    parent, red = synth.water_vdw_reduction(w.n // 3)
    parent[4] = 4
    sites = np_(ctx.vdw_sites(ctx.system(w.xyz, w.box, w.molid), parent, red))
    assert np.all(np.isnan(sites[4])) and np.all(np.isfinite(np.delete(sites, 4, axis=0)))


@pytest.mark.parametrize("frames", ["water", "mixed"])
@pytest.mark.parametrize("name", ["water216", "water7853"])
def test_epolar_frames_fp64(ctx, name, frames):
    w, ft, fa, loc, sysr, lst, rp, cp = case(ctx, name, frames)
    mu = np.random.default_rng(9).normal(0, 0.03, (w.n, 3))
    e, f, vir = ctx.epolar_frames(sysr, lst, ft, fa, loc, w.polarity, w.thole, mu, S["beta"], 7.0)
    eo, fo, vo = O.epolar_frames(w.xyz, w.box, w.molid, rp, cp, ft, fa, loc, w.polarity, w.thole, mu,
                             S["beta"], 7.0)
    e = np_(e)
    for k in range(3):
        assert abs(e[k] - eo[k]) <= 1e-10 * abs(eo[k]), (k, e[k], eo[k])
    assert fmax_rel(np_(f), fo) < 1e-8
    assert np.abs(np_(vir) - vo).max() <= 1e-10 * np.abs(vo).max()


@pytest.mark.parametrize("seed", [51, 52])
def test_frames_random_boxes(ctx, seed):
    # every frame type on random water counts (not cubes) and random cutoffs
    rng = np.random.default_rng(seed)
    n_w = int(rng.integers(60, 400))
    box = (n_w / 0.03335) ** (1.0 / 3.0)
    rc = float(min(rng.uniform(4.0, 7.0), 0.5 * box - 0.01))
    w = synth.amoeba_water_box(n_w, box, 7000 + seed)
    ft, fa = synth.mixed_frames(n_w)
    loc = synth.water_local_multipoles(n_w, seed)
    print(f"frames random seed={seed} n_w={n_w} box={box:.2f} rc={rc:.2f}", flush=True)
    sysr = ctx.system(w.xyz, w.box, w.molid)
    lst = ctx.nblist(sysr, rc + 0.001, plan_slot=7)
    rp, cp = O.nblist(w.xyz, w.box, rc + 0.001)
    e, f, _, vir = ctx.empole_frames(sysr, lst, ft, fa, loc, S["beta"], rc)
    eo, fo, vo = O.empole_frames(w.xyz, w.box, w.molid, rp, cp, ft, fa, loc, S["beta"], rc)
    e = np_(e)
    for k in range(3):
        assert abs(e[k] - eo[k]) <= 1e-10 * abs(eo[k]), k
    assert fmax_rel(np_(f), fo) < 1e-8
    assert np.abs(np_(vir) - vo).max() <= 1e-10 * np.abs(vo).max()
    mu = rng.normal(0, 0.03, (w.n, 3))
    e, f, vir = ctx.epolar_frames(sysr, lst, ft, fa, loc, w.polarity, w.thole, mu, S["beta"], rc)
    eo, fo, vo = O.epolar_frames(w.xyz, w.box, w.molid, rp, cp, ft, fa, loc, w.polarity, w.thole,
                                 mu, S["beta"], rc)
    assert abs(np_(e)[0] - eo[0]) <= 1e-10 * abs(eo[0])
    assert fmax_rel(np_(f), fo) < 1e-8
    assert np.abs(np_(vir) - vo).max() <= 1e-10 * np.abs(vo).max()
