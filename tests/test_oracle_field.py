"""Pins of the oracle's permanent field, Thole damping, mutual-field mat-vec and
induced-dipole PCG."""
import numpy as np
import pytest
from scipy import integrate

from oracle import oracle as O
from paper_1906_01211_amd import synth
from tests import _pointcharge as PC
from tests.test_oracle_multipole import rand_site

C, DEBYE = O.constants()


def test_thole_l3_is_enclosed_smeared_charge():
    # Thole's exponential model: unit charge smeared as rho(u) = (3a/4pi) exp(-a u^3),
    # u = r/(ai aj)^(1/6); the field factor l3 is the charge enclosed within r.
    ai, aj, a = 0.837, 0.496, 0.39
    A = (ai * aj) ** (1 / 6)
    for r in (0.5, 1.0, 2.0, 3.5):
        enc, _ = integrate.quad(lambda s: 4 * np.pi * s * s * 3 * a / (4 * np.pi) *
                                np.exp(-a * (s / A) ** 3) / A ** 3, 0, r, epsabs=1e-14,
                                epsrel=1e-13)
        l3, l5, l7 = O.thole(r, ai, aj, 0.39, 0.5)
        assert l3 == pytest.approx(enc, rel=1e-11)


def test_thole_family_obeys_radial_recursion():
    # l3 R1, l5 R2, l7 R3 obey f(n+1) = -(1/r) df(n)/dr like the bare family.
    ai, aj = 0.837, 0.496
    def fam(r):
        l3, l5, l7 = O.thole(r, ai, aj, 0.39, 0.39)
        return np.array([l3 / r ** 3, l5 * 3 / r ** 5, l7 * 15 / r ** 7])
    for r in (0.7, 1.3, 2.9):
        h = 1e-5
        d = (fam(r + h) - fam(r - h)) / (2 * h)
        f = fam(r)
        assert -d[0] / r == pytest.approx(f[1], rel=1e-8)
        assert -d[1] / r == pytest.approx(f[2], rel=1e-8)
    assert O.thole(1.0, 0.0, 0.5, 0.39, 0.39) == (1.0, 1.0, 1.0)
    assert O.thole(1.0, 0.5, 0.5, 0.39, 0.2)[0] == pytest.approx(1 - np.exp(-0.2 / 0.5), rel=1e-14)


@pytest.mark.parametrize("seed", range(4))
def test_bare_field_equals_point_charge_field(seed):
    # alpha = 0 gives l = 1; beta = 0 gives the bare multipole field of the other site.
    rng = np.random.default_rng(seed)
    mi, mj = rand_site(rng), rand_site(rng)
    r = rng.normal(size=3)
    r *= rng.uniform(1.5, 5) / np.linalg.norm(r)
    xyz = np.array([[50.0, 50, 50], 50 + r])
    rp, cp = O.nblist(xyz, 100.0, 49.0)
    fld = O.efield_direct(xyz, 100.0, np.array([0, 1], np.int32), rp, cp, np.stack([mi, mj]),
                          np.zeros(2), np.full(2, 0.39), 0.0, 49.0)
    ref_i = PC.field_at(xyz[0], PC.cluster(xyz[1], mj))
    ref_j = PC.field_at(xyz[1], PC.cluster(xyz[0], mi))
    assert np.allclose(fld[0], ref_i, rtol=1e-10, atol=1e-12)
    assert np.allclose(fld[1], ref_j, rtol=1e-10, atol=1e-12)


def test_field_is_minus_energy_gradient_in_dipoles():
    # With alpha = 0 (l = 1) efield uses the same kernels as the energy, so
    # E_i = -(1/C) d(E_real + E_self)/d mu_i, including the exclusion corrections.
    wb = synth.amoeba_water_box(27, 9.4, 13)
    beta, rc = 0.5446, 4.6
    rp, cp = O.nblist(wb.xyz, wb.box, rc)
    pol = np.zeros(wb.n)
    fld = O.efield_direct(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, pol, wb.thole, beta, rc)

    def Etot(m):
        e, _, _ = O.empole_real(wb.xyz, wb.box, wb.molid, rp, cp, m, beta, rc)
        return e[0] + O.eself(m, beta)
    h = 1e-6
    for i in (0, 1, 17, 50):
        for a in range(3):
            mp_, mm = wb.mpole.copy(), wb.mpole.copy()
            mp_[i, 1 + a] += h
            mm[i, 1 + a] -= h
            g = (Etot(mp_) - Etot(mm)) / (2 * h)
            assert -g / C == pytest.approx(fld[i, a], rel=1e-7, abs=1e-9)


def test_two_site_damped_closed_form():
    ai, aj, a = 0.837, 0.496, 0.39
    r = np.array([0.4, -1.1, 1.9])
    rr = np.linalg.norm(r)
    mu = np.array([0.2, 0.1, -0.3])
    xyz = np.array([[10.0, 10, 10], 10 + r])
    rp, cp = O.nblist(xyz, 40.0, 19.0)
    m = np.zeros((2, 10))
    m[1, 1:4] = mu
    fld = O.efield_direct(xyz, 40.0, np.array([0, 1], np.int32), rp, cp, m, np.array([ai, aj]),
                          np.full(2, a), 0.0, 19.0)
    l3, l5, _ = O.thole(rr, ai, aj, a, a)
    ref = 3 * l5 * r * (r @ mu) / rr ** 5 - l3 * mu / rr ** 3
    assert np.allclose(fld[0], ref, rtol=1e-13)
    out = O.tmatvec(xyz, 40.0, rp, cp, np.array([ai, aj]), np.full(2, a), 0.0, 19.0,
                    np.stack([np.zeros(3), mu]))
    assert np.allclose(out[0], ref, rtol=1e-13)


def small_water(n_w=27, box=9.4, seed=2, rc=4.6):
    wb = synth.amoeba_water_box(n_w, box, seed)
    rp, cp = O.nblist(wb.xyz, wb.box, rc)
    return wb, rp, cp, 0.5446, rc


def test_tmatvec_symmetric_and_matches_energy():
    wb, rp, cp, beta, rc = small_water()
    rng = np.random.default_rng(0)
    u, v = rng.normal(size=(2, wb.n, 3))
    Tu = O.tmatvec(wb.xyz, wb.box, rp, cp, wb.polarity, wb.thole, beta, rc, u)
    Tv = O.tmatvec(wb.xyz, wb.box, rp, cp, wb.polarity, wb.thole, beta, rc, v)
    assert np.sum(u * Tv) == pytest.approx(np.sum(v * Tu), rel=1e-13)
    # alpha = 0 (l = 1), distinct molecules: -(C/2) mu.(T + cI) mu = E_real + E_self (dipoles)
    m = np.zeros((wb.n, 10))
    m[:, 1:4] = u * 0.05
    pol0 = np.zeros(wb.n)
    T = O.tmatvec(wb.xyz, wb.box, rp, cp, pol0, wb.thole, beta, rc, m[:, 1:4])
    e, _, _ = O.empole_real(wb.xyz, wb.box, np.arange(wb.n, dtype=np.int32), rp, cp, m, beta, rc)
    assert -0.5 * C * np.sum(m[:, 1:4] * T) == pytest.approx(e[0] + O.eself(m, beta), rel=1e-12)
    # the mat-vec's dipole field equals efield's for intermolecular, damped pairs
    fld = O.efield_direct(wb.xyz, wb.box, np.arange(wb.n, dtype=np.int32), rp, cp, m, wb.polarity,
                          wb.thole, beta, rc)
    T2 = O.tmatvec(wb.xyz, wb.box, rp, cp, wb.polarity, wb.thole, beta, rc, m[:, 1:4])
    assert np.allclose(fld, T2, rtol=0, atol=1e-14 * np.abs(T2).max())


def test_operator_spd_and_pcg_matches_dense_solve():
    wb, rp, cp, beta, rc = small_water()
    A = O.dense_operator(wb.xyz, wb.box, rp, cp, wb.polarity, wb.thole, beta, rc)
    assert np.allclose(A, A.T, rtol=0, atol=1e-13)
    np.linalg.cholesky(A)                                   # SPD
    b = O.efield_direct(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole, beta,
                        rc).ravel()
    x = np.linalg.solve(A, b)
    mu, info = O.polarize_pcg(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                              beta, rc, tol_debye=1e-12, maxiter=200)
    assert info["converged"] == 1 and info["status"] == 0
    # stop rule: RMS of alpha*r <= 1e-12 D, so |x - A^-1 b| is of order cond(A) * 1e-12 / 4.8
    assert np.allclose(mu.ravel(), x, rtol=0, atol=1e-11 * np.abs(x).max())
    assert info["epol"] == pytest.approx(-0.5 * C * b @ x, rel=1e-11)
    # E_pol is variational: -1/2 b.A^-1 b is the minimum of 1/2 x.Ax - b.x (times C)
    y = x + 1e-3 * np.random.default_rng(1).normal(size=x.size)
    assert C * (0.5 * y @ A @ y - b @ y) > -0.5 * C * b @ x


def test_pcg_water216_iterations_and_true_error():
    wb = synth.make("water216")
    beta, rc = 0.5446, 7.0
    rp, cp = O.nblist(wb.xyz, wb.box, 7.001)
    mu, info = O.polarize_pcg(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                              beta, rc, tol_debye=1e-5, maxiter=100)
    assert info["converged"] == 1 and 3 <= info["iters"] <= 12
    assert info["rms_debye"] <= 1e-5 and info["rms_true_debye"] < 2e-5
    tight, _ = O.polarize_pcg(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                              beta, rc, tol_debye=1e-11, maxiter=100)
    err = DEBYE * np.sqrt(np.mean(np.sum((mu - tight) ** 2, axis=1)))
    assert err < 2e-5


def test_pcg_failure_modes():
    wb, rp, cp, beta, rc = small_water(n_w=8, box=7.0, rc=3.4)
    mu, info = O.polarize_pcg(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                              beta, 3.4, tol_debye=1e-12, maxiter=1)
    assert info["status"] == O.E_NOCONV and info["iters"] == 1 and info["converged"] == 0
    huge = np.full(wb.n, 50.0)   # 1/alpha - c < 0 on the diagonal: not positive definite
    mu, info = O.polarize_pcg(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, huge, np.full(wb.n, 1e-6),
                              2.0, 3.4, tol_debye=1e-12, maxiter=50)
    assert info["status"] in (O.E_BREAKDOWN, O.E_NOCONV)
    # zero iterations when the guess already satisfies the tolerance
    mu0, info0 = O.polarize_pcg(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                                beta, 3.4, tol_debye=1e-12, maxiter=100)
    mu1, info1 = O.polarize_pcg(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                                beta, 3.4, tol_debye=1e-6, maxiter=100, mu_guess=mu0)
    assert info1["iters"] == 0 and info1["converged"] == 1


@pytest.mark.parametrize("part", ["dipole", "quadrupole"])
def test_damped_field_is_gradient_of_damped_potential(part):
    # Thole-damped potential of a site at s = y - r_j (traceless Theta):
    #   dipole: (mu.s) l3 R1,   quadrupole: (s.Theta.s) l5 R2;
    # the field at i is minus its gradient.  Checks how efield uses l3, l5, l7.
    ai, aj, a = 0.837, 0.496, 0.39
    rng = np.random.default_rng(5)
    m = rand_site(rng, q=False, mu=(part == "dipole"), th=(part == "quadrupole"))
    rj = np.array([20.0, 20.0, 20.0])
    ri = rj + np.array([0.9, -1.3, 1.6])
    Th = np.array([[m[4], m[5], m[6]], [m[5], m[7], m[8]], [m[6], m[8], m[9]]])

    def phi(y):
        s = y - rj
        r = np.linalg.norm(s)
        l3, l5, _ = O.thole(r, ai, aj, a, a)
        if part == "dipole":
            return (m[1:4] @ s) * l3 / r ** 3
        return (s @ Th @ s) * l5 * 3 / r ** 5
    h = 1e-5
    grad = np.array([(phi(ri + h * e) - phi(ri - h * e)) / (2 * h) for e in np.eye(3)])
    grad2 = np.array([(phi(ri + 2 * h * e) - phi(ri - 2 * h * e)) / (4 * h) for e in np.eye(3)])
    grad = (4 * grad - grad2) / 3
    xyz = np.stack([ri, rj])
    rp, cp = O.nblist(xyz, 60.0, 29.0)
    mp = np.stack([np.zeros(10), m])
    fld = O.efield_direct(xyz, 60.0, np.array([0, 1], np.int32), rp, cp, mp, np.array([ai, aj]),
                          np.full(2, a), 0.0, 29.0)
    assert np.allclose(fld[0], -grad, rtol=1e-8, atol=1e-10)


def test_converged_dipoles_satisfy_self_consistency():
    # induced dipoles: mu_i = alpha_i (E_perm_i + [(T + cI) mu]_i)
    wb, rp, cp, beta, rc = small_water()
    mu, info = O.polarize_pcg(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                              beta, rc, tol_debye=1e-12, maxiter=200)
    E = O.efield_direct(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole, beta, rc)
    F = O.tmatvec(wb.xyz, wb.box, rp, cp, wb.polarity, wb.thole, beta, rc, mu, include_diag=0)
    assert np.allclose(mu, wb.polarity[:, None] * (E + F), rtol=0, atol=1e-11)


@pytest.mark.parametrize("k", [1, 2, 4])
def test_pcg_iterate_is_krylov_optimal(k):
    # In exact arithmetic the k-th PCG iterate minimises the A-norm error over
    # x0 + span{z0, (M A) z0, ..., (M A)^(k-1) z0}, M = diag(alpha).
    wb, rp, cp, beta, rc = small_water(n_w=8, box=7.0, seed=4, rc=3.4)
    A = O.dense_operator(wb.xyz, wb.box, rp, cp, wb.polarity, wb.thole, beta, rc)
    b = O.efield_direct(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole, beta,
                        rc).ravel()
    Mdiag = np.repeat(wb.polarity, 3)
    x0 = Mdiag * b
    r0 = b - A @ x0
    V = [Mdiag * r0]
    for _ in range(k - 1):
        V.append(Mdiag * (A @ V[-1]))
    V = np.linalg.qr(np.array(V).T)[0]
    y = np.linalg.solve(V.T @ A @ V, V.T @ r0)
    xk = x0 + V @ y
    mu, info = O.polarize_pcg(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                              beta, rc, tol_debye=0.0, maxiter=k)
    assert info["iters"] == k
    assert np.allclose(mu.ravel(), xk, rtol=0, atol=1e-12 * np.abs(xk).max())
