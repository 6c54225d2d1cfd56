"""Pins of the oracle's reciprocal-space pieces: the exact Ewald k-sum's
forces and field, the cardinal B-splines and their moduli, and the smooth
PME (energy, forces, field) against the k-sum it approximates."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1906_01211_amd import synth

C, DEBYE = O.constants()


def small_box():
    return synth.amoeba_water_box(27, 9.4, 2)


def only(m, kind):
    m = m.copy()
    if kind == "q":
        m[:, 1:] = 0.0
    elif kind == "mu":
        m[:, 0] = 0.0
        m[:, 4:] = 0.0
    elif kind == "theta":
        m[:, :4] = 0.0
    return m


# ---------------------------------------------------------------- k-sum
def test_ksum_forces_are_minus_energy_gradient():
    w = small_box()
    beta, kmax = 0.5446, 9
    f, _ = O.erecip_grad(w.xyz, w.box, w.mpole, beta, kmax)
    h = 1e-5
    for i in (0, 4, 50):
        for a in range(3):
            xp, xm = w.xyz.copy(), w.xyz.copy()
            xp[i, a] += h
            xm[i, a] -= h
            g = (O.erecip(xp, w.box, w.mpole, beta, kmax) -
                 O.erecip(xm, w.box, w.mpole, beta, kmax)) / (2 * h)
            assert f[i, a] == pytest.approx(-g, rel=1e-6, abs=1e-8 * np.abs(f).max())


def test_ksum_field_is_minus_dipole_gradient():
    # dE/dmu_i = C grad phi(r_i) = -C field_i (E is quadratic in mu, so the
    # central difference is exact up to rounding at any step)
    w = small_box()
    beta, kmax = 0.5446, 9
    _, fld = O.erecip_grad(w.xyz, w.box, w.mpole, beta, kmax)
    h = 1e-3
    for i in (1, 33):
        for a in range(3):
            mp_, mm = w.mpole.copy(), w.mpole.copy()
            mp_[i, 1 + a] += h
            mm[i, 1 + a] -= h
            g = (O.erecip(w.xyz, w.box, mp_, beta, kmax) -
                 O.erecip(w.xyz, w.box, mm, beta, kmax)) / (2 * h)
            assert fld[i, a] == pytest.approx(-g / C, rel=1e-7, abs=1e-10)


# ---------------------------------------------------------------- B-splines
def test_bspline_values_and_identities():
    assert O.bspline(4, 1.0) == pytest.approx(1 / 6, rel=1e-15)
    assert O.bspline(4, 2.0) == pytest.approx(2 / 3, rel=1e-15)
    assert O.bspline(5, 1.0) == pytest.approx(1 / 24, rel=1e-15)
    assert O.bspline(5, 2.0) == pytest.approx(11 / 24, rel=1e-15)
    assert O.bspline(5, 2.5) == pytest.approx(115 / 192, rel=1e-15)
    assert O.bspline(5, 0.0) == 0.0 and O.bspline(5, 5.0) == 0.0
    rng = np.random.default_rng(0)
    for p in (5, 6, 8):
        for w in rng.uniform(0, 1, 5):
            # partition of unity; derivatives of a constant vanish
            assert sum(O.bspline(p, w + t) for t in range(p)) == pytest.approx(1.0, abs=1e-15)
            for d in (1, 2, 3):
                assert abs(sum(O.bspline(p, w + t, d) for t in range(p))) < 1e-13
            x = w + 1.7
            assert O.bspline(p, x) == pytest.approx(O.bspline(p, p - x), rel=1e-14)   # symmetric
            h = 1e-6
            for d in (0, 1, 2):
                fd = (O.bspline(p, x + h, d) - O.bspline(p, x - h, d)) / (2 * h)
                assert O.bspline(p, x, d + 1) == pytest.approx(fd, rel=1e-7, abs=1e-9)


def test_spline_moduli_interpolate_plane_waves():
    # exp(2 pi i m u/K) ~ b(m) sum_g M_p(u - g) exp(2 pi i m g/K), |b|^2 = 1/D(m);
    # the interpolant's modulus equals |b(m)|^-1 times the spline sum's modulus
    K, p = 32, 8
    for m in (1, 3, 7):
        D = O.spline_mod(p, K, m)
        for u in (3.3, 17.81):
            s = sum(O.bspline(p, u - g) * np.exp(2j * np.pi * m * g / K)
                    for g in range(int(np.floor(u)) - p, int(np.floor(u)) + 2))
            assert abs(s) ** 2 / D == pytest.approx(1.0, abs=1e-5 * m ** 2)
    # odd order: D(K/2) vanishes and is replaced by the mean of its neighbours
    D4 = [O.spline_mod(5, 16, m) for m in (7, 8, 9)]
    assert D4[1] == pytest.approx(0.5 * (D4[0] + D4[2]), rel=1e-14)
    assert all(O.spline_mod(6, 16, m) > 1e-3 for m in range(16))


# ---------------------------------------------------------------- PME
@pytest.mark.parametrize("kind", ["q", "mu", "theta", "all"])
def test_pme_converges_to_ksum(kind):
    # a smooth split (beta = 0.35) and order-8 splines: PME reproduces the
    # k-sum to its interpolation error
    w = small_box()
    m = only(w.mpole, kind)
    beta = 0.35
    ek = O.erecip(w.xyz, w.box, m, beta, 12)
    fk, Ek = O.erecip_grad(w.xyz, w.box, m, beta, 12)
    e, f, fld = O.pme_mpole(w.xyz, w.box, m, beta, 32, 8)
    assert e == pytest.approx(ek, rel=5e-8)
    assert np.abs(f - fk).max() <= 1e-5 * np.sqrt(np.mean(fk ** 2))
    assert np.abs(fld - Ek).max() <= 1e-6 * np.sqrt(np.mean(Ek ** 2))


def test_pme_order5_error_shrinks_with_grid():
    w = synth.make("water216")
    beta = 0.5446
    ek = O.erecip(w.xyz, w.box, w.mpole, beta, 20)
    errs = [abs(O.pme_mpole(w.xyz, w.box, w.mpole, beta, K, 5)[0] - ek) / abs(ek)
            for K in (16, 32, 48)]
    assert errs[0] > 10 * errs[1] > 10 * errs[2] and errs[2] < 1e-4


def test_pme_forces_and_field_are_its_own_gradients():
    # the PME energy is a smooth function of positions and dipoles; its
    # forces and field are exactly its gradients (not only the k-sum's)
    w = small_box()
    beta, K, p = 0.5446, 16, 5
    e0, f, fld = O.pme_mpole(w.xyz, w.box, w.mpole, beta, K, p)
    h = 1e-5
    for i in (0, 5, 40):
        for a in range(3):
            xp, xm = w.xyz.copy(), w.xyz.copy()
            xp[i, a] += h
            xm[i, a] -= h
            g = (O.pme_mpole(xp, w.box, w.mpole, beta, K, p)[0] -
                 O.pme_mpole(xm, w.box, w.mpole, beta, K, p)[0]) / (2 * h)
            assert abs(f[i, a] + g) <= 1e-8 * np.abs(f).max()
            mp_, mm = w.mpole.copy(), w.mpole.copy()
            mp_[i, 1 + a] += 1e-3
            mm[i, 1 + a] -= 1e-3
            gm = (O.pme_mpole(w.xyz, w.box, mp_, beta, K, p)[0] -
                  O.pme_mpole(w.xyz, w.box, mm, beta, K, p)[0]) / 2e-3
            assert fld[i, a] == pytest.approx(-gm / C, rel=1e-6, abs=1e-10)


def test_pme_grid_shift_invariance_and_arguments():
    w = small_box()
    beta, K, p = 0.5446, 16, 5
    e0, f0, _ = O.pme_mpole(w.xyz, w.box, w.mpole, beta, K, p)
    # a shift by whole grid spacings moves the spread pattern without change
    e1, f1, _ = O.pme_mpole(w.xyz + 3 * w.box / K, w.box, w.mpole, beta, K, p)
    assert e1 == pytest.approx(e0, rel=1e-12)
    assert np.allclose(f1, f0, rtol=0, atol=1e-10 * np.abs(f0).max())
    for K_, p_ in ((8, 5), (16, 4), (20, 9)):
        with pytest.raises(O.OracleError):
            O.pme_mpole(w.xyz, w.box, w.mpole, beta, K_, p_)


# ---------------------------------------------------------------- full-Ewald polarization
def _ewald_box():
    w = small_box()
    rc = 4.69
    rp, cp = O.nblist(w.xyz, w.box, rc)
    return w, rp, cp, rc


def _apply_full(w, rp, cp, rc, beta, K, p, v):
    """A v of the full operator from the separately pinned pieces."""
    Av = O.tmatvec(w.xyz, w.box, rp, cp, w.polarity, w.thole, beta, rc, v, include_diag=1)
    m = np.zeros((w.n, 10))
    m[:, 1:4] = v
    _, _, fld = O.pme_mpole(w.xyz, w.box, m, beta, K, p)
    return Av - np.where(w.polarity[:, None] > 0, fld, 0.0)


def test_ewald_pcg_solves_the_composed_system():
    # the converged dipoles satisfy A x = E_perm with A and E_perm composed of
    # the real-space mat-vec, the permanent field and the PME fields
    w, rp, cp, rc = _ewald_box()
    beta, K, p = 0.9, 16, 5
    mu, info = O.polarize_pcg_ewald(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole,
                                    beta, rc, K, p, tol_debye=1e-11, maxiter=200)
    assert info["converged"] == 1
    b = O.efield_direct(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole, beta, rc)
    b += O.pme_mpole(w.xyz, w.box, w.mpole, beta, K, p)[2]
    r = b - _apply_full(w, rp, cp, rc, beta, K, p, mu)
    assert DEBYE * np.sqrt(np.sum((w.polarity[:, None] * r) ** 2) / w.n) < 1e-10
    assert info["epol"] == pytest.approx(-0.5 * C * np.sum(mu * b), rel=1e-12)
    # the composed operator is symmetric (PME spreads and gathers with the same splines)
    rng = np.random.default_rng(5)
    u, v = rng.normal(size=(2, w.n, 3))
    Au = _apply_full(w, rp, cp, rc, beta, K, p, u)
    Av = _apply_full(w, rp, cp, rc, beta, K, p, v)
    assert np.sum(u * Av) == pytest.approx(np.sum(v * Au), rel=1e-12)


def test_ewald_polarization_energy_does_not_depend_on_the_split():
    # with the reciprocal part the polarization energy is the physical one:
    # changing beta moves work between real and reciprocal space only (here
    # limited by the PME error, ~1e-6); without it the energy moves by far more
    w, rp, cp, rc = _ewald_box()
    e = []
    for beta, K in ((0.9, 32), (1.0, 40)):
        _, info = O.polarize_pcg_ewald(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity,
                                       w.thole, beta, rc, K, 8, tol_debye=1e-10, maxiter=200)
        e.append(info["epol"])
    assert e[0] == pytest.approx(e[1], rel=2e-6)
    real = [O.polarize_pcg(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole, beta, rc,
                           tol_debye=1e-10, maxiter=200)[1]["epol"] for beta in (0.9, 1.0)]
    assert abs(real[0] - real[1]) > 1e3 * abs(e[0] - e[1])


def test_full_ewald_polarization_forces_compose():
    # at fixed mu the reciprocal part of the polarization energy is
    # E_pme(M + mu) - E_pme(M) (the cross term -C mu.E_perm_recip plus the
    # dipoles' own -1/2 C mu.R mu), so the full-Ewald polarization force is
    # the real-space one plus the difference of two PME forces; at converged
    # dipoles it is the gradient of E_pol with the dipoles re-solved
    w = synth.amoeba_water_box(20, 8.6, 4)
    rc, beta, K, p = 4.29, 0.9, 16, 5
    rp, cp = O.nblist(w.xyz, w.box, rc)

    def solve(xyz):
        mu, info = O.polarize_pcg_ewald(xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole,
                                        beta, rc, K, p, tol_debye=1e-12, maxiter=300)
        assert info["converged"] == 1
        return mu, info["epol"]
    mu, _ = solve(w.xyz)
    _, F, _ = O.epolar_real(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole, mu, beta,
                            rc)
    m2 = w.mpole.copy()
    m2[:, 1:4] += mu
    F += (O.pme_mpole(w.xyz, w.box, m2, beta, K, p)[1] -
          O.pme_mpole(w.xyz, w.box, w.mpole, beta, K, p)[1])
    h = 1e-5
    for i in (0, 5, 33):
        for a in range(3):
            xp, xm = w.xyz.copy(), w.xyz.copy()
            xp[i, a] += h
            xm[i, a] -= h
            g = (solve(xp)[1] - solve(xm)[1]) / (2 * h)
            assert abs(F[i, a] + g) <= 1e-8 * np.abs(F).max()
