"""Reciprocal-space PME (tk_pme_mpole) against the FP64 CPU oracle's smooth
PME on the same grid and spline order: energy within 1e-10 relative, forces
and field within 1e-8 of their RMS; determinism, edge cases and errors."""
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


def check(ctx, xyz, box, mpole, beta, K, p):
    sysr = ctx.system(xyz, box, np.zeros(len(xyz), np.int32))
    print(f"pme n={len(xyz)} K={K} p={p}", flush=True)
    e, f, fld = ctx.pme_mpole(sysr, mpole, beta, K, p)
    eo, fo, fldo = O.pme_mpole(xyz, box, mpole, beta, K, p)
    assert abs(np_(e)[0] - eo) <= 1e-10 * abs(eo), (np_(e)[0], eo)
    assert fmax_rel(np_(f), fo) < 1e-8
    assert fmax_rel(np_(fld), fldo) < 1e-8
    return e, f, fld


@pytest.mark.parametrize("K,p", [(16, 5), (32, 5), (32, 8), (16, 6), (16, 7)])
def test_pme_water216(ctx, K, p):
    w = _cache.setdefault("water216", synth.make("water216"))
    check(ctx, w.xyz, w.box, w.mpole, S["beta"], K, p)


def test_pme_water7853_grid64(ctx):
    w = _cache.setdefault("water7853", synth.make("water7853"))
    check(ctx, w.xyz, w.box, w.mpole, S["beta"], 64, 5)


@pytest.mark.parametrize("n,box,seed", [(1, 12.0, 0), (7, 10.0, 1), (300, 20.0, 2)])
def test_pme_random_sites(ctx, n, box, seed):
    # sites anywhere (negative coordinates and several boxes away included)
    rng = np.random.default_rng(seed)
    xyz = rng.uniform(-2 * box, 3 * box, size=(n, 3))
    m = rng.normal(0, 0.3, size=(n, 10))
    m[:, 9] = -(m[:, 4] + m[:, 7])
    check(ctx, xyz, box, m, 0.45, 32, 5)


def test_pme_grid128(ctx):
    w = _cache.setdefault("water216", synth.make("water216"))
    rng = np.random.default_rng(4)
    idx = rng.choice(w.n, 60, replace=False)
    check(ctx, w.xyz[idx], w.box, w.mpole[idx], S["beta"], 128, 5)


def test_pme_deterministic_and_no_field(ctx):
    w = _cache.setdefault("water7853", synth.make("water7853"))
    sysr = ctx.system(w.xyz, w.box, w.molid)
    e1, f1, fl1 = ctx.pme_mpole(sysr, w.mpole, S["beta"], 64, 5)
    e2, f2, fl2 = ctx.pme_mpole(sysr, w.mpole, S["beta"], 64, 5, want_field=False)
    assert fl2 is None
    assert np.array_equal(np_(e1), np_(e2)) and np.array_equal(np_(f1), np_(f2))


def test_pme_edge_cases_and_errors(ctx, tk):
    empty = ctx.system(np.zeros((0, 3)), 20.0, np.zeros(0, np.int32))
    e, f, _ = ctx.pme_mpole(empty, np.zeros((0, 10)), S["beta"], 16, 5)
    assert np_(e)[0] == 0.0 and f.shape == (0, 3)
    w = _cache.setdefault("water216", synth.make("water216"))
    sysr = ctx.system(w.xyz, w.box, w.molid)
    for K, p, beta in ((48, 5, S["beta"]), (16, 4, S["beta"]), (16, 9, S["beta"]),
                       (8, 5, S["beta"]), (16, 5, 0.0)):
        with pytest.raises(tk.TkError):
            ctx.pme_mpole(sysr, w.mpole, beta, K, p)
    # a contribution outside the fixed-point range gives a NaN energy, not a wrong number
    big = w.mpole.copy()
    big[5, 0] = 1e6
    e, _, _ = ctx.pme_mpole(sysr, big, S["beta"], 16, 5)
    assert np.isnan(np_(e)[0])
    # a non-finite coordinate: NaN energy as well
    bad = w.xyz.copy()
    bad[7, 0] = np.nan
    e, _, _ = ctx.pme_mpole(ctx.system(bad, w.box, w.molid), w.mpole, S["beta"], 16, 5)
    assert np.isnan(np_(e)[0])
    # and the next call with ordinary input is clean again
    check(ctx, w.xyz, w.box, w.mpole, S["beta"], 16, 5)


# ---------------------------------------------------------------- full-Ewald solve
def _ewald_case(ctx, name, K, p):
    w = _cache.setdefault(name, synth.make(name))
    sysr = ctx.system(w.xyz, w.box, w.molid)
    lst = ctx.nblist(sysr, 7.001, plan_slot=2)
    key = (name, "list")
    if key not in _cache:
        _cache[key] = O.nblist(w.xyz, w.box, 7.001)
    rp, cp = _cache[key]
    return w, sysr, lst, rp, cp


@pytest.mark.parametrize("k", [0, 1, 4])
def test_pcg_ewald_iterates(ctx, k):
    # fixed iteration counts: every iterate equals the oracle's
    w, sysr, lst, rp, cp = _ewald_case(ctx, "water216", 32, 5)
    print(f"pcg ewald water216 k={k}", flush=True)
    mu, info = ctx.polarize_pcg_ewald(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0, 32,
                                      5, tol_debye=0.0, maxiter=k)
    mo, io = O.polarize_pcg_ewald(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole,
                                  S["beta"], 7.0, 32, 5, tol_debye=0.0, maxiter=k)
    assert info["iters"] == io["iters"] == k and info["status"] == io["status"]
    assert np.abs(np_(mu) - mo).max() <= 1e-10 * np.abs(mo).max()
    assert abs(info["epol"] - io["epol"]) <= 1e-10 * abs(io["epol"])
    # the reciprocal field passes through the 2^-40 fixed-point mesh (absolute
    # ~1e-12 e/A^2), small against these residual norms but not at 1e-8
    assert abs(info["rms_debye"] - io["rms_debye"]) <= 1e-7 * io["rms_debye"]


@pytest.mark.parametrize("name,K,p", [("water216", 32, 5), ("water216", 16, 8),
                                      ("water7853", 64, 5)])
def test_pcg_ewald_converged(ctx, name, K, p):
    w, sysr, lst, rp, cp = _ewald_case(ctx, name, K, p)
    print(f"pcg ewald {name} K={K} p={p}", flush=True)
    mu, info = ctx.polarize_pcg_ewald(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0, K,
                                      p, tol_debye=S["tol_debye"])
    mo, io = O.polarize_pcg_ewald(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole,
                                  S["beta"], 7.0, K, p, tol_debye=S["tol_debye"])
    assert info["converged"] == io["converged"] == 1 and info["iters"] == io["iters"]
    assert np.abs(np_(mu) - mo).max() <= 1e-10 * np.abs(mo).max()
    assert abs(info["epol"] - io["epol"]) <= 1e-10 * abs(io["epol"])
    # a converged true residual (~3e-6 D) against the mesh's fixed-point
    # rounding of the reciprocal field (~1e-11 D)
    assert abs(info["rms_true_debye"] - io["rms_true_debye"]) <= 1e-5 * io["rms_true_debye"]
    # the plain real-space solve on the same context is unaffected afterwards
    m2, i2 = ctx.polarize_pcg(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0,
                              tol_debye=S["tol_debye"])
    m3, i3 = O.polarize_pcg(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole,
                            S["beta"], 7.0, tol_debye=S["tol_debye"])
    assert i2["iters"] == i3["iters"]
    assert np.abs(np_(m2) - m3).max() <= 1e-10 * np.abs(m3).max()


def test_pcg_ewald_guess_zero_polarizability_and_errors(ctx, tk):
    w, sysr, lst, rp, cp = _ewald_case(ctx, "water216", 16, 5)
    mo, io = O.polarize_pcg_ewald(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole,
                                  S["beta"], 7.0, 16, 5, tol_debye=1e-9, maxiter=100)
    # converged dipoles as the guess: zero or one iteration, same answer
    mu, info = ctx.polarize_pcg_ewald(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0, 16,
                                      5, tol_debye=1e-5, mu_guess=mo)
    assert info["converged"] == 1 and info["iters"] <= 1
    assert np.abs(np_(mu) - mo).max() <= 1e-6 * np.abs(mo).max()
    # no polarizable atom: zero dipoles at once
    mu0, info0 = ctx.polarize_pcg_ewald(sysr, lst, w.mpole, np.zeros(w.n), w.thole, S["beta"],
                                        7.0, 16, 5)
    assert info0["converged"] == 1 and info0["iters"] == 0 and not np.any(np_(mu0))
    for K, p, beta in ((48, 5, S["beta"]), (16, 4, S["beta"]), (16, 5, 0.0)):
        with pytest.raises(tk.TkError):
            ctx.polarize_pcg_ewald(sysr, lst, w.mpole, w.polarity, w.thole, beta, 7.0, K, p)


def test_full_ewald_polarization_forces(ctx):
    # the composition of the oracle pin, on the device: real-space
    # polarization forces plus the difference of two PME force calls, at each
    # side's own converged full-Ewald dipoles
    w, sysr, lst, rp, cp = _ewald_case(ctx, "water216", 32, 5)
    beta, K, p = S["beta"], 32, 5
    mu, _ = ctx.polarize_pcg_ewald(sysr, lst, w.mpole, w.polarity, w.thole, beta, 7.0, K, p,
                                   tol_debye=1e-9)
    mo, _ = O.polarize_pcg_ewald(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole,
                                 beta, 7.0, K, p, tol_debye=1e-9)
    import torch
    mpg = torch.as_tensor(w.mpole, device=mu.device).clone()
    mpg[:, 1:4] += mu
    _, f, _ = ctx.epolar_real(sysr, lst, w.mpole, w.polarity, w.thole, mu, beta, 7.0)
    _, f1, _ = ctx.pme_mpole(sysr, mpg, beta, K, p, want_field=False)
    _, f0, _ = ctx.pme_mpole(sysr, w.mpole, beta, K, p, want_field=False)
    F = np_(f) + np_(f1) - np_(f0)
    _, fo, _ = O.epolar_real(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole, mo,
                             beta, 7.0)
    m2 = w.mpole.copy()
    m2[:, 1:4] += mo
    Fo = fo + O.pme_mpole(w.xyz, w.box, m2, beta, K, p)[1] - O.pme_mpole(w.xyz, w.box, w.mpole,
                                                                        beta, K, p)[1]
    assert fmax_rel(F, Fo) < 1e-8


def test_pme_point_charges_ewald_split(ctx):
    # the point-charge (CHARMM-style) path: PME of charges only, against the
    # oracle's PME, and the total Ewald energy (real space + PME + self term)
    # the same at two splitting parameters
    w = synth.charge_lj_water_box(4000, 49.4, 91)
    q = np.zeros((w.n, 10))
    q[:, 0] = w.charges
    sysr = ctx.system(w.xyz, w.box, w.molid)
    lst = ctx.nblist(sysr, 12.001, plan_slot=4)
    totals = []
    for beta in (0.34, 0.40):
        print(f"pme charges beta={beta}", flush=True)
        er, _, _ = ctx.echarge_real(sysr, lst, w.charges, beta, 12.0)
        ek, fk, _ = ctx.pme_mpole(sysr, q, beta, 64, 6, want_field=False)
        totals.append(float(np_(er)[0]) + float(np_(ek)[0]) + O.eself(q, beta))
        if beta == 0.34:
            eo, fo, _ = O.pme_mpole(w.xyz, w.box, q, beta, 64, 6)
            assert abs(np_(ek)[0] - eo) <= 1e-10 * abs(eo)
            assert fmax_rel(np_(fk), fo) < 1e-8
    assert abs(totals[0] - totals[1]) <= 1e-5 * abs(totals[0]), totals


def test_multipole_ewald_total_independent_of_split(ctx):
    # the AMOEBA multipoles of the water box: real space + PME + self energy
    # is the same at two splitting parameters.  Each piece is 1e4 to 1e5
    # times the total (the same-molecule terms cancel between the real-space
    # correction and the self energy), so the check needs a converged real
    # space (12 A) and PME error well below 1e-5 of the total (128^3, order
    # 8: at order 6 the totals of the oracle differ by 0.4 kcal/mol)
    w = _cache.setdefault("water7853", synth.make("water7853"))
    sysr = ctx.system(w.xyz, w.box, w.molid)
    lst = ctx.nblist(sysr, 12.001, plan_slot=4)
    totals, pieces = [], []
    for beta in (0.45, 0.50):
        print(f"multipole ewald split beta={beta}", flush=True)
        er, _, _ = ctx.empole_real(sysr, lst, w.mpole, beta, 12.0)
        ek, _, _ = ctx.pme_mpole(sysr, w.mpole, beta, 128, 8, want_field=False)
        pieces.append(float(np_(ek)[0]))
        totals.append(float(np_(er)[0]) + float(np_(ek)[0]) + O.eself(w.mpole, beta))
    assert abs(totals[0] - totals[1]) <= 1e-5 * abs(totals[0]), totals
    assert abs(pieces[0] - pieces[1]) > 1.0 * abs(totals[0])   # the pieces move by far more


@pytest.mark.parametrize("name,K", [("water216", 32), ("water7853", 64)])
def test_epolar_ewald_one_call(ctx, name, K):
    # tk_epolar_ewald against the oracle's composition: the real-space
    # polarization pair terms plus E_pme(M + mu) - E_pme(M) and its forces
    w, sysr, lst, rp, cp = _ewald_case(ctx, name, K, 5)
    print(f"epolar ewald {name} K={K}", flush=True)
    mu = np.random.default_rng(12).normal(0, 0.03, (w.n, 3))
    e, f = ctx.epolar_ewald(sysr, lst, w.mpole, w.polarity, w.thole, mu, S["beta"], 7.0, K, 5)
    er, fr, _ = O.epolar_real(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole, mu,
                              S["beta"], 7.0)
    m2 = w.mpole.copy()
    m2[:, 1:4] += mu
    ea, fa, _ = O.pme_mpole(w.xyz, w.box, m2, S["beta"], K, 5)
    eb, fb, _ = O.pme_mpole(w.xyz, w.box, w.mpole, S["beta"], K, 5)
    e = np_(e)
    assert abs(e[1] - er[0]) <= 1e-10 * abs(er[0])
    assert abs(e[2] - (ea - eb)) <= 1e-9 * abs(ea - eb)
    assert abs(e[0] - (er[0] + ea - eb)) <= 1e-9 * abs(er[0] + ea - eb)
    assert fmax_rel(np_(f), fr + fa - fb) < 1e-8
