"""Pins of the oracle's Halgren 14-7 and LJ 12-6 terms and the taper."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1906_01211_amd import synth


def pair_energy(r, form, Ri, Rj, ei, ej, rc=20.0, dhal=0.07, ghal=0.12, molid=(0, 1)):
    box = max(50.0, 2 * rc + 10.0)
    xyz = np.array([[20.0, 20, 20], [20.0 + r, 20, 20]])
    rp, cp = O.nblist(xyz, box, rc + 0.001)
    e, f, w = O.evdw(xyz, box, np.array(molid, np.int32), rp, cp, form, np.array([Ri, Rj]),
                     np.array([ei, ej]), rc, 0.9, dhal, ghal)
    return e, f


def test_hal_special_values():
    R, eps = 3.405, 0.11
    e, f = pair_energy(R, O.VDW_HAL, R, R, eps, eps)
    assert e == pytest.approx(-eps, rel=1e-14)                 # e(R_ij) = -eps_ij
    # slope at R_ij in closed form: 7 eps/R [1/(1+d) - 1/(1+g)]
    slope = 7 * eps / R * (1 / 1.07 - 1 / 1.12)
    assert f[1, 0] == pytest.approx(-slope, rel=1e-12)
    # long range: e ~ -2 eps (1+d)^7 (R/r)^7
    r = 100 * R
    e, _ = pair_energy(r, O.VDW_HAL, R, R, eps, eps, rc=r + 10.0)
    assert e == pytest.approx(-2 * eps * 1.07 ** 7 * (R / r) ** 7, rel=2e-3)
    # combining rules: cubic mean radius, HHG epsilon, at unequal parameters
    Ri, Rj, ei, ej = 3.405, 2.655, 0.11, 0.0135
    Rij = (Ri ** 3 + Rj ** 3) / (Ri ** 2 + Rj ** 2)
    eij = 4 * ei * ej / (np.sqrt(ei) + np.sqrt(ej)) ** 2
    e, _ = pair_energy(Rij, O.VDW_HAL, Ri, Rj, ei, ej)
    assert e == pytest.approx(-eij, rel=1e-13)


def test_lj_special_values():
    s, eps = 3.15, 0.152
    e, _ = pair_energy(s, O.VDW_LJ, s, s, eps, eps)
    assert abs(e) < 1e-14
    rmin = 2 ** (1 / 6) * s
    e, f = pair_energy(rmin, O.VDW_LJ, s, s, eps, eps)
    assert e == pytest.approx(-eps, rel=1e-14)
    assert abs(f[0, 0]) < 1e-14
    e, _ = pair_energy(rmin, O.VDW_LJ, s, 2.0, eps, 0.0)      # eps_ij = sqrt(ei ej) = 0
    assert e == 0.0


@pytest.mark.parametrize("si,sj,ei,ej", [(3.15, 1.2, 0.152, 0.046), (2.0, 4.5, 0.3, 0.01),
                                         (3.4, 3.0, 0.1, 0.2)])
def test_lj_unequal_sigma(si, sj, ei, ej):
    # Lorentz-Berthelot at unequal sigma and nonzero eps on both sites: the
    # arithmetic-mean sigma puts the zero at (si+sj)/2 and the minimum -sqrt(ei ej)
    # at 2^(1/6) (si+sj)/2 with zero slope.  A geometric-mean sigma (or an
    # arithmetic-mean eps) fails each of these by far more than the tolerance.
    s = 0.5 * (si + sj)
    eij = np.sqrt(ei * ej)
    e0, _ = pair_energy(s, O.VDW_LJ, si, sj, ei, ej)
    assert abs(e0) < 1e-14
    rmin = 2 ** (1 / 6) * s
    e, f = pair_energy(rmin, O.VDW_LJ, si, sj, ei, ej)
    assert e == pytest.approx(-eij, rel=1e-13)
    assert abs(f[0, 0]) < 1e-13
    # away from the special points: the closed form 4 eps_ij [(s/r)^12 - (s/r)^6]
    r = 1.37 * s
    e, f = pair_energy(r, O.VDW_LJ, si, sj, ei, ej)
    sr6 = (s / r) ** 6
    assert e == pytest.approx(4 * eij * (sr6 * sr6 - sr6), rel=1e-13)
    # force on the second site along +x: -de/dr
    assert f[1, 0] == pytest.approx(24 * eij * (2 * sr6 * sr6 - sr6) / r, rel=1e-12)
    assert abs(s - np.sqrt(si * sj)) > 1e-3   # the cases do separate the two means


@pytest.mark.parametrize("form", [O.VDW_HAL, O.VDW_LJ])
def test_taper(form):
    rc = 9.0
    ron = 0.9 * rc
    e_on, _ = pair_energy(ron - 1e-9, form, 3.4, 3.4, 0.1, 0.1, rc=rc)
    e_on2, _ = pair_energy(ron + 1e-9, form, 3.4, 3.4, 0.1, 0.1, rc=rc)
    assert e_on2 == pytest.approx(e_on, rel=1e-7)
    e_end, f_end = pair_energy(rc - 1e-6, form, 3.4, 3.4, 0.1, 0.1, rc=rc)
    assert abs(e_end) < 1e-12 and abs(f_end[0, 0]) < 1e-8
    # taper at the midpoint is S(1/2) = 1/2 of the bare energy
    mid = ron + 0.05 * rc
    e_mid, _ = pair_energy(mid, form, 3.4, 3.4, 0.1, 0.1, rc=rc)
    e_bare, _ = pair_energy(mid, form, 3.4, 3.4, 0.1, 0.1, rc=50.0 / 2 - 0.01)
    assert e_mid == pytest.approx(0.5 * e_bare, rel=1e-12)
    # same-molecule pairs are skipped
    e, f = pair_energy(3.0, form, 3.4, 3.4, 0.1, 0.1, molid=(4, 4))
    assert e == 0.0 and np.all(f == 0)


@pytest.mark.parametrize("form", [O.VDW_HAL, O.VDW_LJ])
def test_fd_forces_net_force_virial(form):
    wb = synth.amoeba_water_box(27, 9.6, 17)
    rc = 4.7
    rp, cp = O.nblist(wb.xyz, wb.box, rc + 0.001)
    rad = wb.vdw_rad if form == O.VDW_HAL else np.where(np.arange(wb.n) % 3 == 0, 3.15, 1.0)
    eps = wb.vdw_eps
    e, f, w = O.evdw(wb.xyz, wb.box, wb.molid, rp, cp, form, rad, eps, rc)
    h = 1e-5
    for atom in (0, 4, 30):
        for a in range(3):
            xp, xm = wb.xyz.copy(), wb.xyz.copy()
            xp[atom, a] += h
            xm[atom, a] -= h
            ep = O.evdw(xp, wb.box, wb.molid, rp, cp, form, rad, eps, rc)[0]
            em = O.evdw(xm, wb.box, wb.molid, rp, cp, form, rad, eps, rc)[0]
            assert -(ep - em) / (2 * h) == pytest.approx(f[atom, a], rel=1e-6, abs=1e-8)
    assert np.abs(f.sum(axis=0)).max() < 1e-12 * np.abs(f).sum()
    c = wb.box / 2

    def Es(lam):
        x = c + lam * (wb.xyz - c)
        return O.evdw(x, wb.box * lam, wb.molid, rp, cp, form, rad, eps, rc)[0]
    hh = 1e-6
    assert np.trace(w) == pytest.approx((Es(1 + hh) - Es(1 - hh)) / (2 * hh), rel=1e-6)
