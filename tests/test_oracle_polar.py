"""Pins of the oracle's polarization forces (or_epolar_real): the pair
energies against the field routines, forces against finite differences of
the field routines' energy at fixed dipoles and of the solver's E_pol with
re-solved dipoles, textbook two-site closed forms, and the virial."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1906_01211_amd import synth

C, DEBYE = O.constants()
BETA = 0.5446


def cself(beta):
    return 4.0 * beta ** 3 / (3.0 * np.sqrt(np.pi))


def small_water(n_w=27, box=9.4, seed=2, rc=4.0, skin=0.6):
    # list built with a skin so that small displacements keep the same pairs
    wb = synth.amoeba_water_box(n_w, box, seed)
    rp, cp = O.nblist(wb.xyz, wb.box, rc + skin)
    return wb, rp, cp, rc


def rand_mu(n, seed, scale=0.02):
    return np.random.default_rng(seed).normal(0.0, scale, size=(n, 3))


def field_energy(wb, rp, cp, rc, mu, xyz=None, box=None):
    """E(r, mu) minus its position-independent parts, from the field routines:
    -C mu.(E_p - c p) - 1/2 C mu.((T + cI) mu - c mu)."""
    xyz = wb.xyz if xyz is None else xyz
    box = wb.box if box is None else box
    c = cself(BETA)
    ep = O.efield_direct(xyz, box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole, BETA, rc)
    tm = O.tmatvec(xyz, box, rp, cp, wb.polarity, wb.thole, BETA, rc, mu)
    e_ip = -C * np.sum(mu * (ep - c * wb.mpole[:, 1:4]))
    e_ii = -0.5 * C * np.sum(mu * (tm - c * mu))
    return e_ip, e_ii


def near_cutoff(wb, rc, atoms, margin):
    """True if an atom of `atoms` has a partner within `margin` of the cutoff."""
    for i in atoms:
        d = wb.xyz - wb.xyz[i]
        d -= wb.box * np.rint(d / wb.box)
        r = np.linalg.norm(d, axis=1)
        if np.any(np.abs(r - rc) < margin):
            return True
    return False


def test_thole_l9_obeys_radial_recursion():
    # (l7 R3)' = -r l9 R4 with R3 = 15/r^7, R4 = 105/r^9: the factor that the
    # gradient of the damped quadrupole field needs.
    ai, aj = 0.837, 0.496
    for r in (0.6, 1.1, 1.9, 3.3):
        h = 1e-5
        f = lambda s: O.thole(s, ai, aj, 0.39, 0.5)[2] * 15 / s ** 7
        d = (f(r + h) - f(r - h)) / (2 * h)
        assert -d / r == pytest.approx(O.thole_l9(r, ai, aj, 0.39, 0.5) * 105 / r ** 9, rel=1e-8)
    assert O.thole_l9(1.0, 0.0, 0.5, 0.39, 0.39) == 1.0
    # large x: every factor tends to 1; small x: the series of
    # 1 - (1 + x + 18/35 x^2 + 9/35 x^3) e^-x starts -x^2/70 - 8 x^3/105
    assert O.thole_l9(8.0, 0.8, 0.5, 0.39, 0.39) == pytest.approx(1.0, abs=1e-12)
    x = 1e-2
    l9 = O.thole_l9(x ** (1 / 3), 1.0, 1.0, 1.0, 1.0)
    assert l9 == pytest.approx(-x * x / 70 - 8 * x ** 3 / 105, rel=1e-3)


@pytest.mark.parametrize("seed", [0, 1])
def test_pair_energies_match_field_routines(seed):
    wb, rp, cp, rc = small_water(seed=seed + 2)
    mu = rand_mu(wb.n, seed)
    e, _, _ = O.epolar_real(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole, mu,
                            BETA, rc)
    e_ip, e_ii = field_energy(wb, rp, cp, rc, mu)
    assert e[1] == pytest.approx(e_ip, rel=1e-12)
    assert e[2] == pytest.approx(e_ii, rel=1e-12)
    assert e[0] == e[1] + e[2]


def test_forces_are_minus_gradient_at_fixed_mu():
    # any mu: F = -dE(r, mu)/dx, E from the field routines (both damped
    # families, same-molecule pairs, quadrupole field gradient through l9)
    wb, rp, cp, rc = small_water()
    mu = rand_mu(wb.n, 7)
    _, F, _ = O.epolar_real(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole, mu,
                            BETA, rc)
    atoms = [0, 1, 2, 31, 44, 80]
    h = 1e-5
    assert not near_cutoff(wb, rc, atoms, 10 * h)
    for i in atoms:
        for a in range(3):
            xp, xm = wb.xyz.copy(), wb.xyz.copy()
            xp[i, a] += h
            xm[i, a] -= h
            g = (sum(field_energy(wb, rp, cp, rc, mu, xyz=xp)) -
                 sum(field_energy(wb, rp, cp, rc, mu, xyz=xm))) / (2 * h)
            assert F[i, a] == pytest.approx(-g, rel=1e-6, abs=1e-8 * np.abs(F).max())
    # Newton's third law: the pair forces sum to zero
    assert np.allclose(F.sum(axis=0), 0.0, atol=1e-11 * np.abs(F).max())


def test_variational_force_is_gradient_of_epol():
    # at converged dipoles the fixed-mu force is the gradient of the solver's
    # E_pol = -1/2 C mu.E_p with the dipoles re-solved at every geometry
    wb, rp, cp, rc = small_water(n_w=20, box=8.6, seed=4, rc=3.6)

    def solve(xyz):
        mu, info = O.polarize_pcg(xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                                  BETA, rc, tol_debye=1e-12, maxiter=300)
        assert info["converged"] == 1
        return mu, info["epol"]
    mu, _ = solve(wb.xyz)
    _, F, _ = O.epolar_real(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole, mu,
                            BETA, rc)
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


def test_point_charge_and_induced_dipole_closed_form():
    # beta = 0, alpha_i alpha_j = 0 (no damping), different molecules: the
    # textbook energy of a dipole p in the field of a charge q at r = x_j - x_i,
    # U = C q p.r / r^3, and the force on the charge -grad_j U.
    q, p = 0.73, np.array([0.21, -0.4, 0.15])
    r = np.array([1.3, 0.6, -2.2])
    xyz = np.array([[20.0, 20, 20], 20 + r])
    rp, cp = O.nblist(xyz, 60.0, 29.0)
    m = np.zeros((2, 10))
    m[1, 0] = q
    mu = np.stack([p, np.zeros(3)])
    e, F, W = O.epolar_real(xyz, 60.0, np.array([0, 1], np.int32), rp, cp, m, np.zeros(2),
                            np.full(2, 0.39), mu, 0.0, 29.0)
    rr = np.linalg.norm(r)
    assert e[1] == pytest.approx(C * q * (p @ r) / rr ** 3, rel=1e-13)
    assert e[2] == 0.0
    Fj = -C * q * (p / rr ** 3 - 3 * (p @ r) * r / rr ** 5)
    assert np.allclose(F[1], Fj, rtol=1e-12, atol=0)
    assert np.allclose(F[0], -Fj, rtol=1e-12, atol=0)
    # W = sum over pairs r (x) de/dr = r (x) (-F_j)
    assert np.allclose(W, np.outer(r, -Fj), rtol=1e-12, atol=1e-15)


def test_two_damped_induced_dipoles_closed_form():
    # beta = 0: e_ii = C [pi.pj l3/r^3 - 3 l5 (pi.r)(pj.r)/r^5] (the Thole-damped
    # dipole-dipole energy); forces by differencing that formula.
    ai, aj, a = 0.837, 0.496, 0.39
    pi, pj = np.array([0.12, -0.3, 0.25]), np.array([-0.2, 0.05, 0.31])

    def u(r):
        rr = np.linalg.norm(r)
        l3, l5, _ = O.thole(rr, ai, aj, a, a)
        return C * ((pi @ pj) * l3 / rr ** 3 - 3 * l5 * (pi @ r) * (pj @ r) / rr ** 5)
    r = np.array([0.9, -1.2, 1.4])
    xyz = np.array([[20.0, 20, 20], 20 + r])
    rp, cp = O.nblist(xyz, 60.0, 29.0)
    e, F, _ = O.epolar_real(xyz, 60.0, np.array([0, 0], np.int32), rp, cp, np.zeros((2, 10)),
                            np.array([ai, aj]), np.full(2, a), np.stack([pi, pj]), 0.0, 29.0)
    assert e[1] == 0.0
    assert e[2] == pytest.approx(u(r), rel=1e-13)
    h = 1e-6
    g = np.array([(u(r + h * v) - u(r - h * v)) / (2 * h) for v in np.eye(3)])
    assert np.allclose(F[1], -g, rtol=1e-7, atol=0)


def test_virial_is_minus_sum_of_x_outer_f_without_images():
    # no periodic images in play (all pairs well inside half the box): the
    # pair virial sum_pairs r (x) de/dr equals -sum_i x_i (x) F_i
    wb = synth.amoeba_water_box(12, 8.0, 9)
    box = 40.0
    xyz = wb.xyz + 16.0
    rp, cp = O.nblist(xyz, box, 19.0)
    mu = rand_mu(wb.n, 3)
    _, F, W = O.epolar_real(xyz, box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole, mu,
                            BETA, 19.0)
    ref = -np.einsum("ia,ib->ab", xyz, F)
    assert np.allclose(W, ref, rtol=0, atol=1e-10 * np.abs(ref).max())


def test_virial_trace_is_isotropic_strain_derivative():
    # x -> (1 + e) x and L -> (1 + e) L scale every pair vector: dE/de = tr W
    wb, rp, cp, rc = small_water(seed=6)
    mu = rand_mu(wb.n, 11)
    _, _, W = O.epolar_real(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                            mu, BETA, rc)
    eps = 1e-6

    def E(s):
        return O.epolar_real(wb.xyz * s, wb.box * s, wb.molid, rp, cp, wb.mpole, wb.polarity,
                             wb.thole, mu, BETA, rc)[0][0]
    d = (E(1 + eps) - E(1 - eps)) / (2 * eps)
    assert np.trace(W) == pytest.approx(d, rel=1e-6)


def test_zero_dipoles_and_bad_arguments():
    wb, rp, cp, rc = small_water(n_w=8, box=7.0, rc=2.8)
    e, F, W = O.epolar_real(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                            np.zeros((wb.n, 3)), BETA, rc)
    assert np.all(e == 0.0) and np.all(F == 0.0) and np.all(W == 0.0)
    with pytest.raises(O.OracleError):
        O.epolar_real(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, wb.polarity, wb.thole,
                      np.zeros((wb.n, 3)), BETA, 0.6 * wb.box)
