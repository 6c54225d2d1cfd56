"""Pins of the oracle's permanent-multipole energy, forces and virial against
Coulomb's law, closed forms, finite differences, symmetry and Ewald identities."""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from paper_1906_01211_amd import synth
from tests import _pointcharge as PC

C, DEBYE = O.constants()


def rand_site(rng, q=True, mu=True, th=True):
    m = np.zeros(10)
    if q:
        m[0] = rng.normal(0, 0.5)
    if mu:
        m[1:4] = rng.normal(0, 0.3, 3)
    if th:
        T = rng.normal(0, 0.3, (3, 3))
        T = 0.5 * (T + T.T)
        T -= np.trace(T) / 3 * np.eye(3)
        m[4:] = [T[0, 0], T[0, 1], T[0, 2], T[1, 1], T[1, 2], T[2, 2]]
    return m


def two_site(r_vec, mi, mj, beta=0.0, same_mol=False, box=100.0):
    xyz = np.array([[50.0, 50.0, 50.0], 50.0 + np.asarray(r_vec)])
    molid = np.array([0, 0 if same_mol else 1], dtype=np.int32)
    rp, cp = O.nblist(xyz, box, 49.0)
    return O.empole_real(xyz, box, molid, rp, cp, np.stack([mi, mj]), beta, 49.0)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("kind", ["qq", "q-mu", "mu-mu", "q-th", "full"])
def test_pair_energy_equals_point_charge_coulomb(seed, kind):
    rng = np.random.default_rng(100 + seed)
    flags = {"qq": (1, 0, 0, 1, 0, 0), "q-mu": (1, 0, 0, 0, 1, 0), "mu-mu": (0, 1, 0, 0, 1, 0),
             "q-th": (1, 0, 0, 0, 0, 1), "full": (1, 1, 1, 1, 1, 1)}[kind]
    mi = rand_site(rng, *flags[:3])
    mj = rand_site(rng, *flags[3:])
    r = rng.normal(size=3)
    r *= rng.uniform(1.5, 6.0) / np.linalg.norm(r)
    e, f, w = two_site(r, mi, mj)
    ref = PC.coulomb_energy(PC.cluster(np.zeros(3), mi), PC.cluster(r, mj), C)
    assert e[0] == pytest.approx(ref, rel=1e-11, abs=1e-13)


def test_closed_forms():
    r = 3.1
    q, th = 0.7, 0.4
    Th = np.array([-0.5 * th, 0, 0, -0.5 * th, 0, th])  # theta diag(-1/2,-1/2,1) along z
    mq = np.r_[q, 0, 0, 0, 0, 0, 0, 0, 0, 0]
    mth = np.r_[0, 0, 0, 0, Th]
    e, _, _ = two_site([0, 0, r], mq, mth)
    assert e[0] == pytest.approx(3 * C * q * th / r ** 3, rel=1e-13)
    mth2 = np.r_[0, 0, 0, 0, 0.3 * Th / th]
    e, _, _ = two_site([0, 0, r], mth, mth2)
    assert e[0] == pytest.approx(54 * C * th * 0.3 / r ** 5, rel=1e-13)
    mu_i, mu_j = np.array([0.1, -0.2, 0.3]), np.array([-0.3, 0.1, 0.25])
    rv = np.array([1.0, 2.0, -2.0])
    rr = np.linalg.norm(rv)
    e, _, _ = two_site(rv, np.r_[0, mu_i, np.zeros(6)], np.r_[0, mu_j, np.zeros(6)])
    ref = C * (mu_i @ mu_j / rr ** 3 - 3 * (mu_i @ rv) * (mu_j @ rv) / rr ** 5)
    assert e[0] == pytest.approx(ref, rel=1e-13)
    e, _, _ = two_site(rv, np.r_[0.6, np.zeros(9)], np.r_[0, mu_j, np.zeros(6)])
    assert e[0] == pytest.approx(-C * 0.6 * (mu_j @ rv) / rr ** 3, rel=1e-13)
    # screened charge pair: C q q erfc(beta r)/r
    from math import erfc
    e, _, _ = two_site([0, 0, r], mq, np.r_[-0.4, np.zeros(9)], beta=0.5446)
    assert e[0] == pytest.approx(C * q * -0.4 * erfc(0.5446 * r) / r, rel=1e-14)
    # excluded pair: the correction is -C q q erf(beta r)/r
    e, _, _ = two_site([0, 0, 0.9572], mq, np.r_[-0.4, np.zeros(9)], beta=0.5446, same_mol=True)
    from math import erf
    assert e[1] == 0.0
    assert e[2] == pytest.approx(-C * q * -0.4 * erf(0.5446 * 0.9572) / 0.9572, rel=1e-13)


def test_radial_recursion_fd_and_bare_limit():
    beta = 0.5446
    for r in (0.9, 2.5, 6.3):
        h = 1e-5
        Bp, _ = O.radial(r + h, beta)
        Bm, _ = O.radial(r - h, beta)
        B, R = O.radial(r, beta)
        for n in range(5):
            d = (Bp[n] - Bm[n]) / (2 * h)
            assert -d / r == pytest.approx(B[n + 1], rel=1e-8)
        B0, R0 = O.radial(r, 0.0)
        assert np.allclose(B0, R0, rtol=0, atol=0)
        assert np.allclose(R, [1 / r, 1 / r ** 3, 3 / r ** 5, 15 / r ** 7, 105 / r ** 9,
                               945 / r ** 11], rtol=1e-15)
        Bs, _ = O.radial(r, 1e-7)          # B_n -> R_n as beta -> 0 (B0 - R0 = O(beta))
        assert np.allclose(Bs, R, rtol=1e-6)
        assert np.allclose(Bs[1:], R[1:], rtol=1e-12)


def small_system(seed=3, n_w=6, box=40.0, spread=7.0):
    rng = np.random.default_rng(seed)
    wb = synth.amoeba_water_box(n_w, spread, seed)
    xyz = wb.xyz + (box - spread) / 2
    mpole = wb.mpole.copy()
    mpole[:, 1:4] *= 4
    mpole[:, 4:] *= 3
    return xyz, box, wb.molid, mpole, wb


def test_fd_forces_net_force_virial_isolated_cluster():
    xyz, box, molid, mpole, _ = small_system()
    beta, rc = 0.5446, 19.0
    rp, cp = O.nblist(xyz, box, rc)
    e, f, w = O.empole_real(xyz, box, molid, rp, cp, mpole, beta, rc)
    assert abs(e[1]) > 1e-3 and abs(e[2]) > 1.0

    def E(x):
        return O.empole_real(x, box, molid, rp, cp, mpole, beta, rc)[0][0]

    h = 1e-4
    for i in range(0, xyz.shape[0], 2):
        for a in range(3):
            def d(hh):
                xp, xm = xyz.copy(), xyz.copy()
                xp[i, a] += hh
                xm[i, a] -= hh
                return (E(xp) - E(xm)) / (2 * hh)
            fd = (4 * d(h / 2) - d(h)) / 3
            assert -fd == pytest.approx(f[i, a], rel=1e-7, abs=1e-7)
    assert np.abs(f.sum(axis=0)).max() < 1e-12 * np.abs(f).sum()
    # tr W = dE/dlambda under r -> lambda r with multipoles fixed
    c = xyz.mean(axis=0)

    def Es(lam):
        return O.empole_real(c + lam * (xyz - c), box, molid, rp, cp, mpole, beta, rc)[0][0]
    h = 1e-5
    dEdl = (8 * (Es(1 + h) - Es(1 - h)) - (Es(1 + 2 * h) - Es(1 - 2 * h))) / (12 * h)
    assert np.trace(w) == pytest.approx(dEdl, rel=1e-8)


def test_fd_forces_periodic_box():
    wb = synth.amoeba_water_box(27, 9.4, 11)
    beta, rc = 0.5446, 4.6
    rp, cp = O.nblist(wb.xyz, wb.box, rc)
    e, f, w = O.empole_real(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, beta, rc)
    # no pair within 1e-3 A of the cutoff, so small displacements keep the pair set
    i = np.repeat(np.arange(wb.n), np.diff(rp))
    d = wb.xyz[cp] - wb.xyz[i]
    d -= wb.box * np.rint(d / wb.box)
    r = np.linalg.norm(d, axis=1)
    assert np.min(np.abs(r - rc)) > 1e-3
    h = 1e-5
    for atom in (0, 5, 40):
        for a in range(3):
            xp, xm = wb.xyz.copy(), wb.xyz.copy()
            xp[atom, a] += h
            xm[atom, a] -= h
            ep = O.empole_real(xp, wb.box, wb.molid, rp, cp, wb.mpole, beta, rc)[0][0]
            em = O.empole_real(xm, wb.box, wb.molid, rp, cp, wb.mpole, beta, rc)[0][0]
            assert -(ep - em) / (2 * h) == pytest.approx(f[atom, a], rel=1e-6, abs=1e-6)
    assert np.abs(f.sum(axis=0)).max() < 1e-11 * np.abs(f).sum()


def _rot_mpole(m, R):
    out = m.copy()
    out[:, 1:4] = m[:, 1:4] @ R.T
    T = np.zeros((m.shape[0], 3, 3))
    T[:, 0, 0], T[:, 0, 1], T[:, 0, 2] = m[:, 4], m[:, 5], m[:, 6]
    T[:, 1, 1], T[:, 1, 2], T[:, 2, 2] = m[:, 7], m[:, 8], m[:, 9]
    T[:, 1, 0], T[:, 2, 0], T[:, 2, 1] = m[:, 5], m[:, 6], m[:, 8]
    T = R[None] @ T @ R.T[None]
    out[:, 4:] = np.stack([T[:, 0, 0], T[:, 0, 1], T[:, 0, 2], T[:, 1, 1], T[:, 1, 2],
                           T[:, 2, 2]], axis=1)
    return out


def cube_rotations():
    mats = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product([1, -1], repeat=3):
            R = np.zeros((3, 3))
            for a in range(3):
                R[a, perm[a]] = signs[a]
            if np.linalg.det(R) > 0:
                mats.append(R)
    return mats


def test_translation_and_cubic_rotation_invariance():
    wb = synth.amoeba_water_box(27, 9.4, 5)
    beta, rc = 0.5446, 4.6
    rp, cp = O.nblist(wb.xyz, wb.box, rc)
    e0, f0, _ = O.empole_real(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, beta, rc)
    x1 = (wb.xyz + np.array([1.3, -2.2, 0.7])) % wb.box
    rp1, cp1 = O.nblist(x1, wb.box, rc)
    e1, f1, _ = O.empole_real(x1, wb.box, wb.molid, rp1, cp1, wb.mpole, beta, rc)
    assert e1[0] == pytest.approx(e0[0], rel=1e-12)
    assert np.allclose(f1, f0, rtol=0, atol=1e-10 * np.abs(f0).max())
    rots = cube_rotations()
    assert len(rots) == 24
    for R in rots:
        xr = ((wb.xyz - wb.box / 2) @ R.T + wb.box / 2) % wb.box
        mr = _rot_mpole(wb.mpole, R)
        rpr, cpr = O.nblist(xr, wb.box, rc)
        er, fr, _ = O.empole_real(xr, wb.box, wb.molid, rpr, cpr, mr, beta, rc)
        assert er[0] == pytest.approx(e0[0], rel=1e-12)
        assert np.allclose(fr, f0 @ R.T, atol=1e-10 * np.abs(f0).max())


def test_arbitrary_rotation_isolated_cluster():
    xyz, box, molid, mpole, _ = small_system(seed=9)
    rp, cp = O.nblist(xyz, box, 19.0)
    e0, f0, _ = O.empole_real(xyz, box, molid, rp, cp, mpole, 0.3, 19.0)
    rng = np.random.default_rng(0)
    for _ in range(3):
        q = rng.normal(size=4)
        R = synth._rotations(q[None])[0]
        c = np.full(3, box / 2)
        xr = (xyz - c) @ R.T + c
        mr = _rot_mpole(mpole, R)
        rpr, cpr = O.nblist(xr, box, 19.0)
        er, fr, _ = O.empole_real(xr, box, molid, rpr, cpr, mr, 0.3, 19.0)
        assert er[0] == pytest.approx(e0[0], rel=1e-12)
        assert np.allclose(fr, f0 @ R.T, atol=1e-10 * np.abs(f0).max())


def ewald_total(xyz, box, molid, mpole, beta, kmax=40):
    rc = box / 2
    rp, cp = O.nblist(xyz, box, rc)
    e, _, _ = O.empole_real(xyz, box, molid, rp, cp, mpole, beta, rc)
    return e[0] + O.erecip(xyz, box, mpole, beta, kmax) + O.eself(mpole, beta)


def test_ewald_beta_independence_with_quadrupoles_and_exclusions():
    wb = synth.amoeba_water_box(4, 10.0, 21)
    mpole = wb.mpole.copy()
    mpole[:, 1:4] *= 4
    mpole[:, 4:] *= 2
    tots = [ewald_total(wb.xyz, wb.box, wb.molid, mpole, b) for b in (1.45, 1.6, 1.8)]
    scale = abs(O.eself(mpole, 1.45))
    assert max(tots) - min(tots) < 1e-12 * scale


def test_nacl_madelung():
    a = 2.8
    pts, q = [], []
    for ix, iy, iz in itertools.product(range(4), repeat=3):
        pts.append([ix * a, iy * a, iz * a])
        q.append(1.0 if (ix + iy + iz) % 2 == 0 else -1.0)
    xyz = np.array(pts) + 0.1
    mpole = np.zeros((64, 10))
    mpole[:, 0] = q
    molid = np.arange(64, dtype=np.int32)
    E = ewald_total(xyz, 4 * a, molid, mpole, 1.5)
    madelung = float(open(__file__.replace("test_oracle_multipole.py",
                                           "golden/nacl_madelung.txt")).read().split()[0])
    assert E / 32 == pytest.approx(-madelung * C / a, rel=1e-10)


def test_simple_cubic_dipole_lattice():
    a, mu = 3.0, 0.3
    pts = [[ix * a, iy * a, iz * a] for ix, iy, iz in itertools.product(range(3), repeat=3)]
    xyz = np.array(pts) + 0.2
    mpole = np.zeros((27, 10))
    mpole[:, 3] = mu
    E = ewald_total(xyz, 3 * a, np.arange(27, dtype=np.int32), mpole, 1.6)
    assert E / 27 == pytest.approx(-2 * np.pi / 3 * C * mu ** 2 / a ** 3, rel=1e-10)


def test_charge_path_equals_multipole_path():
    wb = synth.charge_lj_water_box(64, 12.5, 3)
    rp, cp = O.nblist(wb.xyz, wb.box, 6.001)
    e1, f1, w1 = O.echarge_real(wb.xyz, wb.box, wb.molid, rp, cp, wb.charges, 0.34, 6.0)
    e2, f2, w2 = O.empole_real(wb.xyz, wb.box, wb.molid, rp, cp, wb.mpole, 0.34, 6.0)
    assert np.allclose(e1, e2, rtol=1e-14)
    assert np.allclose(f1, f2, rtol=0, atol=1e-13 * np.abs(f1).max())
    assert np.allclose(w1, w2, rtol=0, atol=1e-13 * np.abs(w1).max())


def test_full_virial_tensor_is_strain_derivative():
    # Under r -> (I + e) r (multipoles fixed), dE/de_ab = sum r_b de/dr_a = W_ba.
    xyz, box, molid, mpole, _ = small_system(seed=12)
    beta, rc = 0.5446, 19.0
    rp, cp = O.nblist(xyz, box, rc)
    _, _, W = O.empole_real(xyz, box, molid, rp, cp, mpole, beta, rc)
    c = xyz.mean(axis=0)
    h = 1e-6
    for a in range(3):
        for b in range(3):
            def E(s):
                eps = np.zeros((3, 3))
                eps[a, b] = s
                return O.empole_real(c + (xyz - c) @ (np.eye(3) + eps).T, box, molid, rp, cp,
                                     mpole, beta, rc)[0][0]
            d = (E(h) - E(-h)) / (2 * h)
            assert W[b, a] == pytest.approx(d, rel=1e-6, abs=1e-6)
    assert np.abs(W - W.T).max() > 1e-3       # not symmetric without torques
