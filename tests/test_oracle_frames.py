"""Pins of the oracle's local-frame multipoles: the frame axes, the rotation
to the lab frame, rigid-rotation invariance of the energy, and the forces
(torques included) against finite differences of the energy."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1906_01211_amd import synth

BETA = 0.5446


def waters(n_w=27, box=9.4, seed=2, frames="water"):
    w = synth.amoeba_water_box(n_w, box, seed)
    ft, fa = (synth.water_frames if frames == "water" else synth.mixed_frames)(n_w)
    loc = synth.water_local_multipoles(n_w, seed)
    return w, ft, fa, loc


FRAME_SETS = ["water", "mixed"]


def unit_dipoles_rotated(w, ft, fa, axis):
    loc = np.zeros((w.n, 10))
    loc[:, 1 + axis] = 1.0
    return O.rotate_mpole(w.xyz, w.box, ft, fa, loc)[:, 1:4]


def test_frame_axes_orthonormal_and_defined_as_stated():
    w, ft, fa, _ = waters()
    X, Y, Z = (unit_dipoles_rotated(w, ft, fa, a) for a in range(3))
    for A in (X, Y, Z):
        assert np.allclose(np.sum(A * A, axis=1), 1.0, atol=1e-14)
    assert np.allclose(np.sum(X * Y, axis=1), 0.0, atol=1e-14)
    assert np.allclose(np.sum(X * Z, axis=1), 0.0, atol=1e-14)
    assert np.allclose(np.cross(Z, X), Y, atol=1e-14)   # right-handed
    d = lambda i, j: (w.xyz[j] - w.xyz[i]) - w.box * np.rint((w.xyz[j] - w.xyz[i]) / w.box)
    for m in (0, 7, 20):
        o, h1, h2 = 3 * m, 3 * m + 1, 3 * m + 2
        u1, u2 = d(o, h1), d(o, h2)
        u1, u2 = u1 / np.linalg.norm(u1), u2 / np.linalg.norm(u2)
        bis = (u1 + u2) / np.linalg.norm(u1 + u2)
        assert np.allclose(Z[o], bis, atol=1e-14)               # bisector
        assert abs(X[o] @ np.cross(u1, u2)) < 1e-14             # x in the HOH plane
        assert X[o] @ u2 > 0
        zh = d(h1, o) / np.linalg.norm(d(h1, o))
        assert np.allclose(Z[h1], zh, atol=1e-14)               # Z-then-X
        assert abs(X[h1] @ zh) < 1e-14 and X[h1] @ d(h1, h2) > 0


def test_mixed_frame_axes_defined_as_stated():
    w, ft, fa, _ = waters(frames="mixed")
    assert set(ft.tolist()) == {1, 2, 3, 4, 5}
    X, Y, Z = (unit_dipoles_rotated(w, ft, fa, a) for a in range(3))
    for A in (X, Y, Z):
        assert np.allclose(np.sum(A * A, axis=1), 1.0, atol=1e-14)
    assert np.allclose(np.cross(Z, X), Y, atol=1e-14)
    d = lambda i, j: (w.xyz[j] - w.xyz[i]) - w.box * np.rint((w.xyz[j] - w.xyz[i]) / w.box)
    u = lambda i, j: d(i, j) / np.linalg.norm(d(i, j))
    seen = set()
    for i in range(w.n):
        t, (iz, ix, iy) = int(ft[i]), fa[i]
        if t == synth.FRAME_Z_ONLY:          # z to the z atom; x from a global axis
            assert np.allclose(Z[i], u(i, iz), atol=1e-14)
            ref = np.eye(3)[1] if abs(Z[i][0]) > 0.866 else np.eye(3)[0]
            assert abs(X[i] @ np.cross(Z[i], ref)) < 1e-14 and X[i] @ ref > 0
        elif t == synth.FRAME_Z_BISECTOR:    # x in the plane of z and u_x + u_y
            b = u(i, ix) + u(i, iy)
            assert np.allclose(Z[i], u(i, iz), atol=1e-14)
            assert abs(X[i] @ np.cross(Z[i], b)) < 1e-13 and X[i] @ b > 0
        elif t == synth.FRAME_3FOLD:         # z along u_z + u_x + u_y, x towards u_x
            s3 = u(i, iz) + u(i, ix) + u(i, iy)
            assert np.allclose(Z[i], s3 / np.linalg.norm(s3), atol=1e-14)
            assert abs(X[i] @ np.cross(Z[i], u(i, ix))) < 1e-13 and X[i] @ u(i, ix) > 0
        seen.add(t)
    assert {3, 4, 5} <= seen


@pytest.mark.parametrize("frames", FRAME_SETS)
def test_rotation_keeps_invariants_and_none_is_identity(frames):
    w, ft, fa, loc = waters(frames=frames)
    g = O.rotate_mpole(w.xyz, w.box, ft, fa, loc)
    assert np.array_equal(g[:, 0], loc[:, 0])
    assert np.allclose(np.linalg.norm(g[:, 1:4], axis=1), np.linalg.norm(loc[:, 1:4], axis=1),
                       rtol=1e-14)
    def full(m):
        T = np.zeros((len(m), 3, 3))
        T[:, 0, 0], T[:, 0, 1], T[:, 0, 2] = m[:, 4], m[:, 5], m[:, 6]
        T[:, 1, 1], T[:, 1, 2], T[:, 2, 2] = m[:, 7], m[:, 8], m[:, 9]
        return T + np.transpose(T, (0, 2, 1)) - T * np.eye(3)
    Tl, Tg = full(loc), full(g)
    assert np.allclose(np.trace(Tg, axis1=1, axis2=2), 0.0, atol=1e-14)
    assert np.allclose(np.einsum("nab,nab->n", Tg, Tg), np.einsum("nab,nab->n", Tl, Tl),
                       rtol=1e-13)
    none = O.rotate_mpole(w.xyz, w.box, np.zeros(w.n, np.int32), fa, loc)
    assert np.array_equal(none, loc)


@pytest.mark.parametrize("frames", FRAME_SETS)
def test_energy_invariant_under_rigid_rotation_with_frames(frames):
    # isolated cluster in a large box: rotating every position rigidly leaves
    # the local-frame energy unchanged; lab-frame multipoles would not follow
    # (Z-only sites excepted: their x comes from a global axis)
    w, ft, fa, loc = waters(n_w=8, box=7.0, seed=3, frames=frames)
    ft = np.where(ft == synth.FRAME_Z_ONLY, synth.FRAME_Z_THEN_X, ft).astype(np.int32)
    fa = fa.copy()
    for i in np.nonzero((ft == synth.FRAME_Z_THEN_X) & (fa[:, 1] < 0))[0]:
        fa[i, 1] = 3 * (i // 3) + (2 if i % 3 == 1 else 1)
    box = 60.0
    xyz = w.xyz + 26.0
    rp, cp = O.nblist(xyz, box, 29.0)
    th = 0.7
    Rz = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1.0]])
    Rx = np.array([[1.0, 0, 0], [0, np.cos(1.1), -np.sin(1.1)], [0, np.sin(1.1), np.cos(1.1)]])
    c = xyz.mean(axis=0)
    xyz2 = (xyz - c) @ (Rx @ Rz).T + c
    e1, _, _ = O.empole_frames(xyz, box, w.molid, rp, cp, ft, fa, loc, 0.0, 29.0)
    e2, _, _ = O.empole_frames(xyz2, box, w.molid, rp, cp, ft, fa, loc, 0.0, 29.0)
    assert e2[0] == pytest.approx(e1[0], rel=1e-12)
    lab = O.rotate_mpole(xyz, box, ft, fa, loc)
    e3, _, _ = O.empole_real(xyz2, box, w.molid, rp, cp, lab, 0.0, 29.0)
    assert abs(e3[0] - e1[0]) > 1e-3 * abs(e1[0])


@pytest.mark.parametrize("frames", FRAME_SETS)
def test_forces_with_torques_are_minus_energy_gradient(frames):
    # E(x) = real-space multipole energy at the multipoles rotated from the
    # current positions, from the separately pinned rotation and energy
    w, ft, fa, loc = waters(frames=frames)
    rc = 4.0
    rp, cp = O.nblist(w.xyz, w.box, rc + 0.5)
    e, F, _ = O.empole_frames(w.xyz, w.box, w.molid, rp, cp, ft, fa, loc, BETA, rc)

    def E(xyz):
        g = O.rotate_mpole(xyz, w.box, ft, fa, loc)
        return O.empole_real(xyz, w.box, w.molid, rp, cp, g, BETA, rc)[0][0]
    assert e[0] == pytest.approx(E(w.xyz), rel=1e-14)
    h = 1e-5
    for i in (0, 1, 2, 31, 45):
        for a in range(3):
            xp, xm = w.xyz.copy(), w.xyz.copy()
            xp[i, a] += h
            xm[i, a] -= h
            g = (E(xp) - E(xm)) / (2 * h)
            assert F[i, a] == pytest.approx(-g, rel=1e-6, abs=1e-7 * np.abs(F).max())
    assert np.allclose(F.sum(axis=0), 0.0, atol=1e-10 * np.abs(F).max())


def test_no_frames_is_plain_multipoles_and_bad_frames():
    w, ft, fa, loc = waters(n_w=8, box=7.0)
    rp, cp = O.nblist(w.xyz, w.box, 3.4)
    zero = np.zeros(w.n, np.int32)
    e, F, _ = O.empole_frames(w.xyz, w.box, w.molid, rp, cp, zero, fa, loc, BETA, 3.4)
    e0, F0, _ = O.empole_real(w.xyz, w.box, w.molid, rp, cp, loc, BETA, 3.4)
    assert np.array_equal(e, e0) and np.array_equal(F, F0)
    bad = fa.copy()
    bad[0, 0] = 0   # the site itself
    with pytest.raises(O.OracleError):
        O.rotate_mpole(w.xyz, w.box, ft, bad, loc)
    badt = ft.copy()
    badt[3] = 7
    with pytest.raises(O.OracleError):
        O.empole_frames(w.xyz, w.box, w.molid, rp, cp, badt, fa, loc, BETA, 3.4)
    # types that take a y atom refuse a missing or repeated one
    mt, ma = synth.mixed_frames(8)
    k = int(np.nonzero(mt == synth.FRAME_Z_BISECTOR)[0][0])
    for y in (-1, ma[k, 0], k):
        bad = ma.copy()
        bad[k, 2] = y
        with pytest.raises(O.OracleError):
            O.rotate_mpole(w.xyz, w.box, mt, bad, loc)
    O.rotate_mpole(w.xyz, w.box, mt, ma, loc)   # the clean topology is accepted


# ---------------------------------------------------------------- vdW hydrogen reduction
def test_vdw_reduction_sites_and_forces():
    w = synth.amoeba_water_box(27, 9.4, 2)
    parent, red = synth.water_vdw_reduction(27)
    sites = O.vdw_sites(w.xyz, w.box, parent, red)
    # O at its atom; each H site on its O-H bond at 0.91 of the bond length
    assert np.array_equal(sites[0::3], w.xyz[0::3])
    for h in (1, 2):
        d = w.xyz[h::3] - w.xyz[0::3]
        d -= w.box * np.rint(d / w.box)
        s = sites[h::3] - w.xyz[0::3]
        assert np.allclose(np.linalg.norm(s, axis=1), 0.91 * np.linalg.norm(d, axis=1), rtol=1e-14)
        assert np.allclose(np.cross(s, d), 0.0, atol=1e-14)
    # forces on atoms are minus the gradient of E(sites(x))
    rc = 4.0
    rp, cp = O.nblist(sites, w.box, rc + 0.5)

    def E(xyz):
        return O.evdw(O.vdw_sites(xyz, w.box, parent, red), w.box, w.molid, rp, cp, 0, w.vdw_rad,
                      w.vdw_eps, rc)[0]
    _, fs, _ = O.evdw(sites, w.box, w.molid, rp, cp, 0, w.vdw_rad, w.vdw_eps, rc)
    F = O.vdw_forces_to_atoms(parent, red, fs)
    assert np.allclose(F.sum(axis=0), fs.sum(axis=0), atol=1e-12 * np.abs(fs).max())
    h = 1e-5
    for i in (0, 1, 2, 40):
        for a in range(3):
            xp, xm = w.xyz.copy(), w.xyz.copy()
            xp[i, a] += h
            xm[i, a] -= h
            g = (E(xp) - E(xm)) / (2 * h)
            assert F[i, a] == pytest.approx(-g, rel=1e-6, abs=1e-8 * np.abs(F).max())
    # red = 1 everywhere: sites are the atoms, forces unchanged
    ones = np.ones(w.n)
    assert np.array_equal(O.vdw_sites(w.xyz, w.box, parent, ones), w.xyz)
    assert np.array_equal(O.vdw_forces_to_atoms(parent, ones, fs), fs)
    bad = parent.copy()
    bad[4] = 4
    with pytest.raises(O.OracleError):
        O.vdw_sites(w.xyz, w.box, bad, red)


@pytest.mark.parametrize("frames", FRAME_SETS)
def test_polarization_forces_with_frames_are_minus_gradient(frames):
    # at fixed induced dipoles, the polarization pair energy depends on the
    # frame atoms through the rotated permanent multipoles as well
    w, ft, fa, loc = waters(frames=frames)
    rc = 4.0
    rp, cp = O.nblist(w.xyz, w.box, rc + 0.5)
    mu = np.random.default_rng(4).normal(0, 0.03, (w.n, 3))
    e, F, _ = O.epolar_frames(w.xyz, w.box, w.molid, rp, cp, ft, fa, loc, w.polarity, w.thole, mu,
                           BETA, rc)

    def E(xyz):
        g = O.rotate_mpole(xyz, w.box, ft, fa, loc)
        return O.epolar_real(xyz, w.box, w.molid, rp, cp, g, w.polarity, w.thole, mu, BETA, rc)[0][0]
    assert e[0] == pytest.approx(E(w.xyz), rel=1e-14)
    h = 1e-5
    for i in (0, 1, 2, 31):
        for a in range(3):
            xp, xm = w.xyz.copy(), w.xyz.copy()
            xp[i, a] += h
            xm[i, a] -= h
            g = (E(xp) - E(xm)) / (2 * h)
            assert F[i, a] == pytest.approx(-g, rel=1e-6, abs=1e-8 * np.abs(F).max())
    # the frame part is not negligible
    g = O.rotate_mpole(w.xyz, w.box, ft, fa, loc)
    _, F0, _ = O.epolar_real(w.xyz, w.box, w.molid, rp, cp, g, w.polarity, w.thole, mu, BETA, rc)
    assert np.abs(F0 - F).max() > 1e-3 * np.abs(F).max()


@pytest.mark.parametrize("frames", FRAME_SETS)
@pytest.mark.parametrize("term", ["empole", "epolar"])
def test_frame_virial_is_minus_sum_of_x_outer_f(frames, term):
    # an isolated cluster in a large box: the energy is a function of relative
    # vectors only (pair vectors and frame vectors), so W = -sum_i x_i (x) F_i
    # holds for the full tensor, frame part included
    w, ft, fa, loc = waters(n_w=8, box=7.0, seed=3, frames=frames)
    box = 60.0
    xyz = w.xyz + 26.0
    rp, cp = O.nblist(xyz, box, 29.0)
    if term == "empole":
        e, F, W = O.empole_frames(xyz, box, w.molid, rp, cp, ft, fa, loc, BETA, 29.0)
        _, F0, W0 = O.empole_real(xyz, box, w.molid, rp, cp,
                                  O.rotate_mpole(xyz, box, ft, fa, loc), BETA, 29.0)
    else:
        mu = np.random.default_rng(5).normal(0, 0.03, (w.n, 3))
        e, F, W = O.epolar_frames(xyz, box, w.molid, rp, cp, ft, fa, loc, w.polarity, w.thole,
                                  mu, BETA, 29.0)
        _, F0, W0 = O.epolar_real(xyz, box, w.molid, rp, cp,
                                  O.rotate_mpole(xyz, box, ft, fa, loc), w.polarity, w.thole, mu,
                                  BETA, 29.0)
    ref = -np.einsum("ia,ib->ab", xyz, F)
    assert np.abs(W - ref).max() <= 1e-10 * np.abs(ref).max()
    assert np.abs(W - W0).max() > 1e-4 * np.abs(W).max()   # the frame part is not small
    # no frames: the plain pair virial
    zero = np.zeros(w.n, np.int32)
    if term == "empole":
        _, _, Wn = O.empole_frames(xyz, box, w.molid, rp, cp, zero, fa, loc, BETA, 29.0)
        _, _, Wr = O.empole_real(xyz, box, w.molid, rp, cp, loc, BETA, 29.0)
        assert np.array_equal(Wn, Wr)
