"""The two-dipole-set solve (tk_polarize_pcg2) against the FP64 CPU oracle: the
same iteration counts, iterates within 1e-10 of their largest entry, energies
within 1e-10 relative; a fixed iteration count; the one-right-hand-side solve
at pscale = 0; guesses; a set that stops before the other; empty systems; and
the polarization forces with both sets (tk_epolar2_real), energies within 1e-10
relative and forces within 1e-8 of their RMS."""
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
    return abs(a - b) / abs(b)


def case(ctx, name):
    w = _cache.setdefault(name, synth.make(name))
    sysr = ctx.system(w.xyz, w.box, w.molid)
    lst = ctx.nblist(sysr, 7.001, plan_slot=2)
    key = (name, "list")
    if key not in _cache:
        _cache[key] = O.nblist(w.xyz, w.box, 7.001)
    rp, cp = _cache[key]
    return w, sysr, lst, rp, cp


def oracle2(w, rp, cp, pscale, **kw):
    return O.polarize_pcg2(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole,
                           S["beta"], 7.0, pscale, **kw)


def check(mu, info, mo, io):
    for v in range(2):
        assert info[v]["iters"] == io[v]["iters"], (v, info[v]["iters"], io[v]["iters"])
        assert info[v]["status"] == io[v]["status"] and info[v]["converged"] == io[v]["converged"]
        assert np.abs(np_(mu)[v] - mo[v]).max() <= 1e-10 * np.abs(mo[v]).max(), v
        assert rel(info[v]["epol"], io[v]["epol"]) < 1e-10, v


@pytest.mark.parametrize("name", ["water216", "water7853"])
def test_pcg2_converged_fp64(ctx, name):
    w, sysr, lst, rp, cp = case(ctx, name)
    print(f"pcg2 {name}", flush=True)
    mu, info = ctx.polarize_pcg2(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0, 0.5,
                                 tol_debye=S["tol_debye"])
    mo, io = oracle2(w, rp, cp, 0.5, tol_debye=S["tol_debye"])
    check(mu, info, mo, io)
    for v in range(2):
        assert info[v]["converged"] == 1
        assert rel(info[v]["rms_true_debye"], io[v]["rms_true_debye"]) < 1e-6
    assert np.abs(mo[0] - mo[1]).max() > 1e-3 * np.abs(mo[0]).max()   # the sets differ


@pytest.mark.parametrize("k", [1, 3])
def test_pcg2_fixed_iterations(ctx, k):
    w, sysr, lst, rp, cp = case(ctx, "water216")
    mu, info = ctx.polarize_pcg2(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0, 0.7,
                                 tol_debye=0.0, maxiter=k)
    mo, io = oracle2(w, rp, cp, 0.7, tol_debye=0.0, maxiter=k)
    check(mu, info, mo, io)
    assert all(i["iters"] == k for i in info)
    for v in range(2):
        assert rel(info[v]["rms_debye"], io[v]["rms_debye"]) < 1e-8


def test_pcg2_at_pscale_zero_is_the_one_rhs_solve(ctx):
    w, sysr, lst, rp, cp = case(ctx, "water216")
    mu, info = ctx.polarize_pcg2(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0, 0.0)
    m1, i1 = ctx.polarize_pcg(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0)
    for v in range(2):
        assert np.array_equal(np_(mu)[v], np_(m1)), v   # same sums in the same order
        assert info[v]["iters"] == i1["iters"] and info[v]["epol"] == i1["epol"]


def test_pcg2_one_set_stops_first(ctx):
    # mu_p starts from its converged value (0 iterations), mu_d from alpha E_d
    w, sysr, lst, rp, cp = case(ctx, "water216")
    mo, io = oracle2(w, rp, cp, 0.5, tol_debye=1e-8)
    guess = mo.copy()
    guess[0] = 0.0   # zero guess: mu_d starts from zero (alpha = 0 rows stay zero)
    mu, info = ctx.polarize_pcg2(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0, 0.5,
                                 tol_debye=1e-5, mu_guess=guess)
    mo2, io2 = oracle2(w, rp, cp, 0.5, tol_debye=1e-5, mu_guess=guess)
    check(mu, info, mo2, io2)
    assert info[1]["iters"] == 0 and info[0]["iters"] > 3


def test_pcg2_arguments_and_empty(ctx, tk):
    w, sysr, lst, rp, cp = case(ctx, "water216")
    for bad in (-0.5, 2.0, float("nan")):
        with pytest.raises(tk.TkError) as e:
            ctx.polarize_pcg2(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0, bad)
        assert e.value.status == tk.E_ARG
    empty = ctx.system(np.zeros((0, 3)), 20.0, np.zeros(0, np.int32))
    l0 = ctx.nblist(empty, 7.001, plan_slot=6)
    mu, info = ctx.polarize_pcg2(empty, l0, np.zeros((0, 10)), np.zeros(0), np.zeros(0),
                                 S["beta"], 7.0, 0.5)
    assert mu.shape == (2, 0, 3) and all(i["converged"] == 1 for i in info)
    # the one-rhs solve still works after the two-rhs one (shared scratch)
    m1, i1 = ctx.polarize_pcg(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0)
    mo1, io1 = O.polarize_pcg(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole,
                              S["beta"], 7.0)
    assert i1["iters"] == io1["iters"]
    assert np.abs(np_(m1) - mo1).max() <= 1e-10 * np.abs(mo1).max()


def fmax_rel(got, ref):
    return np.abs(np.asarray(got) - ref).max() / np.sqrt(np.mean(ref ** 2))


@pytest.mark.parametrize("name", ["water216", "water7853"])
def test_epolar2_fp64(ctx, name):
    w, sysr, lst, rp, cp = case(ctx, name)
    print(f"epolar2 {name}", flush=True)
    mu2 = np.random.default_rng(11).normal(0, 0.03, (2, w.n, 3))
    e, f, vir = ctx.epolar2_real(sysr, lst, w.mpole, w.polarity, w.thole, mu2, S["beta"], 7.0, 0.5)
    eo, fo, vo = O.epolar2_real(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole, mu2,
                                S["beta"], 7.0, 0.5)
    e = np_(e)
    for k in range(3):
        assert rel(e[k], eo[k]) < 1e-10, (k, e[k], eo[k])
    assert fmax_rel(np_(f), fo) < 1e-8
    assert np.abs(np_(vir) - vo).max() <= 1e-10 * np.abs(vo).max()


def test_epolar2_at_solved_sets_and_one_set_limit(ctx, tk):
    w, sysr, lst, rp, cp = case(ctx, "water216")
    mu2, _ = ctx.polarize_pcg2(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0, 0.7)
    m = np_(mu2)
    e, f, _ = ctx.epolar2_real(sysr, lst, w.mpole, w.polarity, w.thole, mu2, S["beta"], 7.0, 0.7)
    eo, fo, _ = O.epolar2_real(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole, m,
                               S["beta"], 7.0, 0.7)
    assert rel(np_(e)[0], eo[0]) < 1e-10 and fmax_rel(np_(f), fo) < 1e-8
    # equal sets, pscale 0: the one-set forces
    mu = m[0]
    e2, f2, v2 = ctx.epolar2_real(sysr, lst, w.mpole, w.polarity, w.thole, np.stack([mu, mu]),
                                  S["beta"], 7.0, 0.0)
    e1, f1, v1 = ctx.epolar_real(sysr, lst, w.mpole, w.polarity, w.thole, mu, S["beta"], 7.0)
    assert np.allclose(np_(e2), np_(e1), rtol=1e-12, atol=0)
    assert fmax_rel(np_(f2), np_(f1)) < 1e-12
    assert np.abs(np_(v2) - np_(v1)).max() <= 1e-12 * np.abs(np_(v1)).max()
    with pytest.raises(tk.TkError):
        ctx.epolar2_real(sysr, lst, w.mpole, w.polarity, w.thole, np.stack([mu, mu]), S["beta"],
                         7.0, 1.5)


@pytest.mark.parametrize("name,K", [("water216", 32), ("water7853", 64)])
def test_pcg2_ewald_converged(ctx, name, K):
    w, sysr, lst, rp, cp = case(ctx, name)
    print(f"pcg2 ewald {name} K={K}", flush=True)
    mu, info = ctx.polarize_pcg2_ewald(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0,
                                       K, 0.5, tol_debye=S["tol_debye"])
    mo, io = O.polarize_pcg2_ewald(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole,
                                   S["beta"], 7.0, K, 0.5, tol_debye=S["tol_debye"])
    check(mu, info, mo, io)
    for v in range(2):
        assert info[v]["converged"] == 1
        # the reciprocal field passes through the 2^-40 fixed-point mesh
        assert rel(info[v]["rms_true_debye"], io[v]["rms_true_debye"]) < 1e-5


def test_pcg2_ewald_fixed_iterations(ctx):
    w, sysr, lst, rp, cp = case(ctx, "water216")
    mu, info = ctx.polarize_pcg2_ewald(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0,
                                       32, 0.7, tol_debye=0.0, maxiter=3)
    mo, io = O.polarize_pcg2_ewald(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole,
                                   S["beta"], 7.0, 32, 0.7, tol_debye=0.0, maxiter=3)
    check(mu, info, mo, io)
    for v in range(2):
        assert info[v]["iters"] == 3
        assert rel(info[v]["rms_debye"], io[v]["rms_debye"]) < 1e-7


def test_two_set_full_ewald_forces_composed(ctx):
    # the two-set full-Ewald force as its composition of GPU calls:
    # tk_epolar2_real + 1/2 [F(M + x + y) - F(M) - F(x) - F(y)] of tk_pme_mpole
    w, sysr, lst, rp, cp = case(ctx, "water216")
    K = 32
    mu2, _ = ctx.polarize_pcg2_ewald(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0, K,
                                     0.5)
    m = np_(mu2)

    def dip(v):
        d = np.zeros((w.n, 10))
        d[:, 1:4] = v
        return d
    mxy = w.mpole.copy()
    mxy[:, 1:4] += m[0] + m[1]
    parts = (mxy, w.mpole, dip(m[0]), dip(m[1]))
    _, f, _ = ctx.epolar2_real(sysr, lst, w.mpole, w.polarity, w.thole, m, S["beta"], 7.0, 0.5)
    fg = np_(f) + 0.5 * sum(sg * np_(ctx.pme_mpole(sysr, q, S["beta"], K, 5, want_field=False)[1])
                            for sg, q in zip((1, -1, -1, -1), parts))
    _, fo, _ = O.epolar2_real(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole, m,
                              S["beta"], 7.0, 0.5)
    fo = fo + 0.5 * sum(sg * O.pme_mpole(w.xyz, w.box, q, S["beta"], K, 5)[1]
                        for sg, q in zip((1, -1, -1, -1), parts))
    assert fmax_rel(fg, fo) < 1e-8


@pytest.mark.parametrize("seed", [31, 32, 33])
def test_pcg2_and_forces_random_boxes(ctx, seed):
    # random water counts (not cubes) at the water density, random scale
    rng = np.random.default_rng(seed)
    n_w = int(rng.integers(60, 400))
    box = (n_w / 0.03335) ** (1.0 / 3.0)
    rc = min(7.0, 0.5 * box - 0.01)
    ps = float(rng.uniform(0.1, 1.0))
    w = synth.amoeba_water_box(n_w, box, 5000 + seed)
    print(f"pcg2 random seed={seed} n_w={n_w} box={box:.2f} rc={rc:.2f} pscale={ps:.3f}", flush=True)
    sysr = ctx.system(w.xyz, w.box, w.molid)
    lst = ctx.nblist(sysr, rc + 0.001, plan_slot=7)
    rp, cp = O.nblist(w.xyz, w.box, rc + 0.001)
    mu, info = ctx.polarize_pcg2(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], rc, ps)
    mo, io = O.polarize_pcg2(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole,
                             S["beta"], rc, ps)
    check(mu, info, mo, io)
    e, f, vir = ctx.epolar2_real(sysr, lst, w.mpole, w.polarity, w.thole, mo, S["beta"], rc, ps)
    eo, fo, vo = O.epolar2_real(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole, mo,
                                S["beta"], rc, ps)
    assert rel(np_(e)[0], eo[0]) < 1e-10
    assert fmax_rel(np_(f), fo) < 1e-8
    assert np.abs(np_(vir) - vo).max() <= 1e-10 * np.abs(vo).max()


def test_pcg2_ewald_sets_stop_apart(ctx):
    # Set 0 starts from the oracle's tightly converged dipoles and stops before
    # its first iteration; set 1 starts from zero and iterates alone.  The two
    # sets share each packed complex FFT, so this checks that the stopped
    # set's half of the mesh no longer feeds the running set's field.
    w, sysr, lst, rp, cp = case(ctx, "water216")
    K = 32
    tight, _ = O.polarize_pcg2_ewald(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole,
                                     S["beta"], 7.0, K, 0.5, tol_debye=1e-9, maxiter=200)
    guess = np.stack([tight[0], np.zeros((w.n, 3))])
    print("pcg2 ewald sets apart water216", flush=True)
    mu, info = ctx.polarize_pcg2_ewald(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0,
                                       K, 0.5, tol_debye=S["tol_debye"], mu_guess=guess)
    mo, io = O.polarize_pcg2_ewald(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole,
                                   S["beta"], 7.0, K, 0.5, tol_debye=S["tol_debye"],
                                   mu_guess=guess)
    assert io[0]["iters"] == 0 and io[1]["iters"] >= 5
    check(mu, info, mo, io)
    # the same with the roles swapped
    guess = np.stack([np.zeros((w.n, 3)), tight[1]])
    mu, info = ctx.polarize_pcg2_ewald(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0,
                                       K, 0.5, tol_debye=S["tol_debye"], mu_guess=guess)
    mo, io = O.polarize_pcg2_ewald(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole,
                                   S["beta"], 7.0, K, 0.5, tol_debye=S["tol_debye"],
                                   mu_guess=guess)
    assert io[1]["iters"] == 0 and io[0]["iters"] >= 5
    check(mu, info, mo, io)
