"""Pins of the oracle's one-step truncated conjugate gradient (TCG1): its
dipoles are the first preconditioned-CG iterate from the direct guess, one
step is exact when the preconditioned operator is a multiple of the
identity, and its forces are the total derivative of its (non-variational)
energy."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1906_01211_amd import synth

C, DEBYE = O.constants()
BETA = 0.5446


def box27():
    w = synth.amoeba_water_box(27, 9.4, 2)
    rc = 4.0
    rp, cp = O.nblist(w.xyz, w.box, rc + 0.6)
    return w, rp, cp, rc


def test_tcg1_dipoles_are_the_first_cg_iterate():
    w, rp, cp, rc = box27()
    mu, U, _ = O.polarize_tcg1(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole, BETA,
                               rc, forces=False)
    m1, info = O.polarize_pcg(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole, BETA,
                              rc, tol_debye=0.0, maxiter=1)
    assert info["iters"] == 1
    assert np.allclose(mu, m1, rtol=0, atol=1e-14 * np.abs(m1).max())
    E = O.efield_direct(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole, BETA, rc)
    assert U == pytest.approx(-0.5 * C * np.sum(mu * E), rel=1e-14)


def test_tcg1_exact_for_a_scaled_identity():
    # no pairs within the cutoff and one polarizability: alpha A = (1 - c alpha) I,
    # so one step reaches A mu = E exactly
    rng = np.random.default_rng(3)
    n = 6
    xyz = np.array([[2.0 + 9.0 * k, 3.0, 4.0] for k in range(n)]) + rng.normal(0, 0.1, (n, 3))
    box = 60.0
    m = np.zeros((n, 10))
    m[:, 0] = rng.normal(0, 0.5, n)
    m[:, 1:4] = rng.normal(0, 0.1, (n, 3))
    pol = np.full(n, 0.8)
    rp, cp = O.nblist(xyz, box, 3.0)
    molid = np.arange(n, dtype=np.int32)
    mu, U, F = O.polarize_tcg1(xyz, box, molid, rp, cp, m, pol, np.full(n, 0.39), BETA, 3.0)
    c = 4 * BETA ** 3 / (3 * np.sqrt(np.pi))
    E = O.efield_direct(xyz, box, molid, rp, cp, m, pol, np.full(n, 0.39), BETA, 3.0)
    assert np.allclose(mu, E / (1 / 0.8 - c), rtol=1e-13)
    assert np.all(F == 0.0)


def test_tcg1_forces_are_minus_energy_gradient():
    w, rp, cp, rc = box27()
    _, _, F = O.polarize_tcg1(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole, BETA,
                              rc)

    def U(xyz):
        return O.polarize_tcg1(xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole, BETA, rc,
                               forces=False)[1]
    h = 1e-5
    for i in (0, 1, 2, 31, 50):
        for a in range(3):
            xp, xm = w.xyz.copy(), w.xyz.copy()
            xp[i, a] += h
            xm[i, a] -= h
            g = (U(xp) - U(xm)) / (2 * h)
            assert F[i, a] == pytest.approx(-g, rel=1e-6, abs=1e-8 * np.abs(F).max())
    assert np.allclose(F.sum(axis=0), 0.0, atol=1e-11 * np.abs(F).max())
    # not the variational force: the fixed-mu polarization force differs
    mu, _, _ = O.polarize_tcg1(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole, BETA,
                               rc, forces=False)
    _, Fv, _ = O.epolar_real(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole, mu,
                             BETA, rc)
    assert np.abs(Fv - F).max() > 1e-3 * np.abs(F).max()


def test_tcg1_no_polarizability():
    w, rp, cp, rc = box27()
    mu, U, F = O.polarize_tcg1(w.xyz, w.box, w.molid, rp, cp, w.mpole, np.zeros(w.n), w.thole,
                               BETA, rc)
    assert np.all(mu == 0.0) and U == 0.0 and np.all(F == 0.0)
