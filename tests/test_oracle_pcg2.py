"""Pins of the oracle's two-right-hand-side solve: the field with a scaled
same-molecule part, the two dipole sets mu_d (field without same-molecule
pairs) and mu_p (field with them scaled by pscale) on one operator, and the
polarization forces with both sets."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1906_01211_amd import synth
from tests.test_oracle_polar import BETA, cself, near_cutoff
from tests.test_oracle_polar import small_water as water_skin

C, DEBYE = O.constants()


def small_water(n_w=27, box=9.4, seed=2, rc=4.6):
    wb = synth.amoeba_water_box(n_w, box, seed)
    rp, cp = O.nblist(wb.xyz, wb.box, rc)
    return wb, rp, cp, 0.5446, rc


def fields(wb, rp, cp, beta, rc, intra, molid=None):
    m = wb.molid if molid is None else molid
    return O.efield_intra(wb.xyz, wb.box, m, rp, cp, wb.mpole, wb.polarity, wb.thole, beta, rc,
                          intra)


def test_intra_field_endpoints_and_linearity():
    wb, rp, cp, beta, rc = small_water()
    e0 = fields(wb, rp, cp, beta, rc, 0.0)
    e1 = fields(wb, rp, cp, beta, rc, 1.0)
    # intra = 0 is the solver's field; intra = 1 treats every pair as intermolecular
    d = O.efield_direct(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole, beta, rc)
    assert np.array_equal(e0, d)
    distinct = np.arange(wb.n, dtype=np.int32)
    d1 = O.efield_direct(wb.xyz, wb.box, distinct, rp, cp, wb.mpole, wb.polarity, wb.thole, beta, rc)
    assert np.array_equal(e1, d1)
    scale = np.abs(e1).max()
    for s in (0.25, 0.5, 0.9):
        es = fields(wb, rp, cp, beta, rc, s)
        assert np.abs(es - ((1 - s) * e0 + s * e1)).max() <= 1e-13 * scale
    assert np.abs(e1 - e0).max() > 1e-2 * scale   # the same-molecule part is not small


def test_scaled_part_is_the_damped_bare_field_of_the_molecule():
    # E(1) - E(0) is the Thole-damped bare field of the same-molecule sites:
    # the same at any Ewald beta, and equal to the beta = 0 field with the
    # intermolecular pairs taken out.
    wb, rp, cp, beta, rc = small_water()
    diffs = [fields(wb, rp, cp, b, rc, 1.0) - fields(wb, rp, cp, b, rc, 0.0) for b in (0.3, beta)]
    scale = np.abs(diffs[1]).max()
    assert np.abs(diffs[0] - diffs[1]).max() <= 1e-12 * scale
    distinct = np.arange(wb.n, dtype=np.int32)
    all_pairs = O.efield_direct(wb.xyz, wb.box, distinct, rp, cp, wb.mpole, wb.polarity, wb.thole,
                                0.0, rc)
    inter = O.efield_direct(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                            0.0, rc)
    assert np.abs(diffs[1] - (all_pairs - inter)).max() <= 1e-12 * scale
    # inside one molecule, by hand: O at the origin of a lone molecule, its H's
    # dipole field with Thole damping only
    xyz = wb.xyz[:3].copy()
    rp1, cp1 = O.nblist(xyz, 60.0, 20.0)
    m = np.zeros((3, 10))
    m[1, 1:4] = [0.1, -0.05, 0.2]
    e = O.efield_intra(xyz, 60.0, np.zeros(3, np.int32), rp1, cp1, m, wb.polarity[:3],
                       wb.thole[:3], 0.0, 20.0, 1.0)
    r = xyz[0] - xyz[1]
    r = r - 60.0 * np.rint(r / 60.0)
    rn = np.linalg.norm(r)
    l3, l5, _ = O.thole(rn, wb.polarity[0], wb.polarity[1], wb.thole[0], wb.thole[1])
    mu = m[1, 1:4]
    want = l5 * 3 * r * (mu @ r) / rn ** 5 - l3 * mu / rn ** 3
    assert np.allclose(e[0], want, rtol=1e-13, atol=0)


def test_pcg2_matches_dense_solves():
    wb, rp, cp, beta, rc = small_water()
    A = O.dense_operator(wb.xyz, wb.box, rp, cp, wb.polarity, wb.thole, beta, rc)
    ed = fields(wb, rp, cp, beta, rc, 0.0).ravel()
    ep = fields(wb, rp, cp, beta, rc, 0.5).ravel()
    xd, xp = np.linalg.solve(A, ed), np.linalg.solve(A, ep)
    mu, info = O.polarize_pcg2(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                               beta, rc, 0.5, tol_debye=1e-12, maxiter=200)
    assert all(i["converged"] == 1 and i["status"] == 0 for i in info)
    assert np.allclose(mu[0].ravel(), xd, rtol=0, atol=1e-11 * np.abs(xd).max())
    assert np.allclose(mu[1].ravel(), xp, rtol=0, atol=1e-11 * np.abs(xp).max())
    assert np.abs(xd - xp).max() > 1e-3 * np.abs(xd).max()   # the two sets differ
    e_ref = -0.5 * C * ed @ xp                                 # = -C/2 E_d.A^-1 E_p
    assert info[0]["epol"] == pytest.approx(e_ref, rel=1e-11)
    assert info[1]["epol"] == pytest.approx(e_ref, rel=1e-11)
    assert ep @ xd == pytest.approx(ed @ xp, rel=1e-12)        # symmetry of A


def test_pcg2_reduces_to_the_one_rhs_solve():
    wb, rp, cp, beta, rc = small_water()
    kw = dict(tol_debye=1e-8, maxiter=100)
    mu1, info1 = O.polarize_pcg(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                                beta, rc, **kw)
    mu, info = O.polarize_pcg2(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                               beta, rc, 0.0, **kw)
    # pscale = 0: both fields are the solver's, both recurrences are its own
    assert np.array_equal(mu[0], mu1) and np.array_equal(mu[1], mu1)
    for i in info:
        assert i["iters"] == info1["iters"] and i["epol"] == info1["epol"]
    # pscale = 1: mu_p is the one-rhs solve with every pair intermolecular in
    # the field (the operator does not depend on molecules)
    distinct = np.arange(wb.n, dtype=np.int32)
    mu_all, info_all = O.polarize_pcg(wb.xyz, wb.box, distinct, rp, cp, wb.mpole, wb.polarity,
                                      wb.thole, beta, rc, **kw)
    mu, info = O.polarize_pcg2(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                               beta, rc, 1.0, **kw)
    assert np.array_equal(mu[1], mu_all) and info[1]["iters"] == info_all["iters"]
    assert np.array_equal(mu[0], mu1)


def test_pcg2_water216_energies_agree():
    wb = synth.make("water216")
    beta, rc = 0.5446, 7.0
    rp, cp = O.nblist(wb.xyz, wb.box, 7.001)
    mu, info = O.polarize_pcg2(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                               beta, rc, 0.5, tol_debye=1e-5, maxiter=100)
    for i in info:
        assert i["converged"] == 1 and 3 <= i["iters"] <= 12 and i["rms_true_debye"] < 2e-5
    # the two energy forms differ only by residual terms
    assert abs(info[0]["epol"] - info[1]["epol"]) <= 1e-5 * abs(info[0]["epol"])
    # guesses: the converged sets stop at once
    mu2, info2 = O.polarize_pcg2(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                                 beta, rc, 0.5, tol_debye=1e-5, maxiter=100, mu_guess=mu)
    assert [i["iters"] for i in info2] == [0, 0]


def test_pcg2_arguments_and_limits():
    wb, rp, cp, beta, rc = small_water(n_w=8, box=7.0, rc=3.4)
    for bad in (-0.1, 1.5, np.nan):
        with pytest.raises(O.OracleError):
            O.polarize_pcg2(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                            beta, rc, bad)
        with pytest.raises(O.OracleError):
            fields(wb, rp, cp, beta, rc, bad)
    mu, info = O.polarize_pcg2(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                               beta, rc, 0.5, tol_debye=1e-12, maxiter=1)
    assert all(i["status"] == O.E_NOCONV and i["iters"] == 1 for i in info)
    mu, info = O.polarize_pcg2(np.zeros((0, 3)), 20.0, np.zeros(0, np.int32),
                               np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros((0, 10)),
                               np.zeros(0), np.zeros(0), beta, rc, 0.5)
    assert mu.shape == (2, 0, 3) and all(i["converged"] == 1 for i in info)


# --- polarization forces with the two sets ---------------------------------


def lagrangian_pos(wb, rp, cp, rc, mu2, pscale, xyz):
    """Position-dependent part of 1/2 C [x.A y - x.E_p - y.E_d] at x = mu_d,
    y = mu_p, from the field routines."""
    c = cself(BETA)
    x, y = mu2
    ed = O.efield_intra(xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole, BETA, rc,
                        0.0)
    ep = O.efield_intra(xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole, BETA, rc,
                        pscale)
    ty = O.tmatvec(xyz, wb.box, rp, cp, wb.polarity, wb.thole, BETA, rc, y)
    p = wb.mpole[:, 1:4]
    return 0.5 * C * (-np.sum(x * (ty - c * y)) - np.sum(x * (ep - c * p)) -
                      np.sum(y * (ed - c * p)))


def test_two_set_forces_reduce_to_one_set():
    wb, rp, cp, rc = water_skin()
    mu = np.random.default_rng(3).normal(0, 0.02, (wb.n, 3))
    e1, f1, w1 = O.epolar_real(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                               mu, BETA, rc)
    e2, f2, w2 = O.epolar2_real(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                                np.stack([mu, mu]), BETA, rc, 0.0)
    assert np.allclose(e2, e1, rtol=1e-13, atol=0)
    assert np.abs(f2 - f1).max() <= 1e-13 * np.abs(f1).max()
    assert np.abs(w2 - w1).max() <= 1e-13 * np.abs(w1).max()


def test_two_set_forces_are_minus_gradient_at_fixed_sets():
    wb, rp, cp, rc = water_skin()
    rng = np.random.default_rng(8)
    mu2 = rng.normal(0, 0.02, (2, wb.n, 3))
    e, F, _ = O.epolar2_real(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                             mu2, BETA, rc, 0.6)
    # the pair energy is the Lagrangian's position-dependent part
    assert e[0] == pytest.approx(lagrangian_pos(wb, rp, cp, rc, mu2, 0.6, wb.xyz), rel=1e-12)
    atoms = [0, 1, 2, 31, 44]
    h = 1e-5
    assert not near_cutoff(wb, rc, atoms, 10 * h)
    for i in atoms:
        for a in range(3):
            xp, xm = wb.xyz.copy(), wb.xyz.copy()
            xp[i, a] += h
            xm[i, a] -= h
            g = (lagrangian_pos(wb, rp, cp, rc, mu2, 0.6, xp) -
                 lagrangian_pos(wb, rp, cp, rc, mu2, 0.6, xm)) / (2 * h)
            assert F[i, a] == pytest.approx(-g, rel=1e-6, abs=1e-8 * np.abs(F).max())
    assert np.allclose(F.sum(axis=0), 0.0, atol=1e-11 * np.abs(F).max())


def test_two_set_force_is_gradient_of_epol():
    # at the solved sets the fixed-set force is the gradient of
    # E_pol = -1/2 C E_d.A^-1 E_p with both sets re-solved at every geometry
    wb, rp, cp, rc = water_skin(n_w=20, box=8.6, seed=4, rc=3.6)

    def solve(xyz):
        mu2, info = O.polarize_pcg2(xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity,
                                    wb.thole, BETA, rc, 0.5, tol_debye=1e-12, maxiter=300)
        assert all(i["converged"] == 1 for i in info)
        return mu2, info[0]["epol"]
    mu2, _ = solve(wb.xyz)
    _, F, _ = O.epolar2_real(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                             mu2, BETA, rc, 0.5)
    _, F1, _ = O.epolar_real(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                             mu2[0], BETA, rc)
    assert np.abs(F - F1).max() > 1e-3 * np.abs(F).max()   # not the one-set force
    h = 1e-5
    atoms = [0, 5, 33]
    assert not near_cutoff(wb, rc, atoms, 10 * h)
    for i in atoms:
        for a in range(3):
            xp, xm = wb.xyz.copy(), wb.xyz.copy()
            xp[i, a] += h
            xm[i, a] -= h
            g = (solve(xp)[1] - solve(xm)[1]) / (2 * h)
            assert F[i, a] == pytest.approx(-g, rel=1e-6, abs=1e-8 * np.abs(F).max())


# --- both sets with the full Ewald operator ---------------------------------
def test_pcg2_ewald_reduces_to_the_one_set_ewald_solve():
    wb, rp, cp, beta, rc = small_water()
    kw = dict(tol_debye=1e-8, maxiter=100)
    mu1, info1 = O.polarize_pcg_ewald(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity,
                                      wb.thole, beta, rc, 16, order=5, **kw)
    mu, info = O.polarize_pcg2_ewald(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity,
                                     wb.thole, beta, rc, 16, 0.0, order=5, **kw)
    assert np.array_equal(mu[0], mu1) and np.array_equal(mu[1], mu1)
    assert all(i["iters"] == info1["iters"] and i["epol"] == info1["epol"] for i in info)
    distinct = np.arange(wb.n, dtype=np.int32)
    mu_all, info_all = O.polarize_pcg_ewald(wb.xyz, wb.box, distinct, rp, cp, wb.mpole,
                                            wb.polarity, wb.thole, beta, rc, 16, order=5, **kw)
    mu, info = O.polarize_pcg2_ewald(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity,
                                     wb.thole, beta, rc, 16, 1.0, order=5, **kw)
    assert np.array_equal(mu[1], mu_all) and info[1]["iters"] == info_all["iters"]
    assert np.array_equal(mu[0], mu1)


def test_pcg2_ewald_energy_forms_agree_and_differ_from_real_space():
    wb, rp, cp, beta, rc = small_water()
    mu, info = O.polarize_pcg2_ewald(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity,
                                     wb.thole, beta, rc, 16, 0.5, order=5, tol_debye=1e-10,
                                     maxiter=200)
    assert all(i["converged"] == 1 for i in info)
    # -C/2 mu_d.E_p = -C/2 mu_p.E_d for the symmetric full operator
    assert info[0]["epol"] == pytest.approx(info[1]["epol"], rel=1e-9)
    mr, ir = O.polarize_pcg2(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                             beta, rc, 0.5, tol_debye=1e-10, maxiter=200)
    assert abs(info[0]["epol"] - ir[0]["epol"]) > 1e-3 * abs(ir[0]["epol"])
    with pytest.raises(O.OracleError):
        O.polarize_pcg2_ewald(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                              beta, rc, 16, 1.5, order=5)


def test_two_set_full_ewald_forces_compose():
    # the reciprocal part of L = 1/2 C [x.A y - x.E_p - y.E_d] at fixed sets is
    # B(M, x) + B(M, y) + B(x, y) with Q(a) = B(a, a) the PME energy of the
    # multipoles a, i.e. 1/2 [Q(M + x + y) - Q(M) - Q(x) - Q(y)]; so the
    # two-set full-Ewald force is epolar2_real plus that combination of four
    # PME forces, and at the solved sets the gradient of E_pol re-solved
    w = synth.amoeba_water_box(20, 8.6, 4)
    rc, beta, K, p = 4.29, 0.9, 16, 5
    rp, cp = O.nblist(w.xyz, w.box, rc)

    def solve(xyz):
        mu2, info = O.polarize_pcg2_ewald(xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity,
                                          w.thole, beta, rc, K, 0.5, order=p, tol_debye=1e-12,
                                          maxiter=300)
        assert all(i["converged"] == 1 for i in info)
        return mu2, info[0]["epol"]

    def dip(v):
        m = np.zeros((w.n, 10))
        m[:, 1:4] = v
        return m
    mu2, _ = solve(w.xyz)
    _, F, _ = O.epolar2_real(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole, mu2,
                             beta, rc, 0.5)
    mxy = w.mpole.copy()
    mxy[:, 1:4] += mu2[0] + mu2[1]
    fq = lambda m: O.pme_mpole(w.xyz, w.box, m, beta, K, p)[1]
    F = F + 0.5 * (fq(mxy) - fq(w.mpole) - fq(dip(mu2[0])) - fq(dip(mu2[1])))
    h = 1e-5
    for i in (0, 5, 33):
        for a in range(3):
            xp, xm = w.xyz.copy(), w.xyz.copy()
            xp[i, a] += h
            xm[i, a] -= h
            g = (solve(xp)[1] - solve(xm)[1]) / (2 * h)
            assert abs(F[i, a] + g) <= 1e-8 * np.abs(F).max()
