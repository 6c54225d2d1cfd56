"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the package smoke check and the CPU leg of the benchmark
may import this module.  It loads ``liboracle.so`` (built from
``tk_oracle.c`` by ``oracle/build.py``) and exposes numpy-level functions
with the call shapes of the GPU library's C-ABI, on host arrays.

The functions here add no arithmetic of their own beyond argument marshalling,
except ``dense_operator`` (assembles the polarization operator column by column
from the oracle's mat-vec, for direct-solve pins).
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

OK, E_ARG, E_CUTOFF, E_CAPACITY, E_NOCONV, E_BREAKDOWN = 0, -1, -2, -3, -4, -5
VDW_HAL, VDW_LJ = 0, 1

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_up = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_i64p = C.POINTER(C.c_int64)


class PcgInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("refinements", C.c_int32),
                ("converged", C.c_int32), ("rms_debye", C.c_double),
                ("rms_true_debye", C.c_double), ("epol", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from oracle import build as _b  # noqa: WPS433
            _b.build()
        _lib = configure(C.CDLL(LIB_PATH))
    return _lib


def configure(L):
    """Declare the argument and result types of the oracle's C functions on a
    loaded library (the plain build, or its op-counting build)."""
    if True:   # one block of declarations
        L.or_coulomb_constant.restype = C.c_double
        L.or_debye_factor.restype = C.c_double
        L.or_quantize.argtypes = [C.c_int, _dp, C.c_double, _up]
        L.or_cutoff_quantum.argtypes = [C.c_double, C.c_double]
        L.or_cutoff_quantum.restype = C.c_uint32
        for f in (L.or_nblist_brute, L.or_nblist_cell):
            f.argtypes = [C.c_int, _dp, C.c_double, C.c_double, _ip, _ip, C.c_int64, _i64p]
        L.or_radial.argtypes = [C.c_double, C.c_double, C.c_int, _dp, _dp]
        L.or_thole.argtypes = [C.c_double] * 5 + [C.POINTER(C.c_double)] * 3
        L.or_mpole_pair.argtypes = [_dp, _dp, _dp, _dp, C.POINTER(C.c_double), _dp]
        L.or_empole_real.argtypes = [C.c_int, _dp, C.c_double, _ip, _ip, _ip, _dp, C.c_double,
                                     C.c_double, _dp, _dp, _dp]
        L.or_echarge_real.argtypes = [C.c_int, _dp, C.c_double, _ip, _ip, _ip, _dp, C.c_double,
                                      C.c_double, _dp, _dp, _dp]
        L.or_efield_direct.argtypes = [C.c_int, _dp, C.c_double, _ip, _ip, _ip, _dp, _dp, _dp,
                                       C.c_double, C.c_double, _dp]
        L.or_efield_intra.argtypes = [C.c_int, _dp, C.c_double, _ip, _ip, _ip, _dp, _dp, _dp,
                                      C.c_double, C.c_double, C.c_double, _dp]
        L.or_polarize_pcg2.argtypes = [C.c_int, _dp, C.c_double, _ip, _ip, _ip, _dp, _dp, _dp,
                                       C.c_double, C.c_double, C.c_double, C.c_double, C.c_int,
                                       C.c_void_p, _dp, C.POINTER(PcgInfo * 2)]
        L.or_polarize_pcg2_ewald.argtypes = [C.c_int, _dp, C.c_double, _ip, _ip, _ip, _dp, _dp,
                                             _dp, C.c_double, C.c_double, C.c_int, C.c_int,
                                             C.c_double, C.c_double, C.c_int, C.c_void_p, _dp,
                                             C.POINTER(PcgInfo * 2)]
        L.or_tmatvec.argtypes = [C.c_int, _dp, C.c_double, _ip, _ip, _dp, _dp, C.c_double,
                                 C.c_double, C.c_int, _dp, _dp]
        L.or_polarize_pcg.argtypes = [C.c_int, _dp, C.c_double, _ip, _ip, _ip, _dp, _dp, _dp,
                                      C.c_double, C.c_double, C.c_double, C.c_int, C.c_void_p,
                                      _dp, C.POINTER(PcgInfo)]
        L.or_thole_l9.argtypes = [C.c_double] * 5
        L.or_thole_l9.restype = C.c_double
        L.or_epolar_real.argtypes = [C.c_int, _dp, C.c_double, _ip, _ip, _ip, _dp, _dp, _dp, _dp,
                                     C.c_double, C.c_double, _dp, _dp, _dp]
        L.or_epolar2_real.argtypes = [C.c_int, _dp, C.c_double, _ip, _ip, _ip, _dp, _dp, _dp,
                                      _dp, C.c_double, C.c_double, C.c_double, _dp, _dp, _dp]
        L.or_evdw.argtypes = [C.c_int, _dp, C.c_double, _ip, _ip, _ip, C.c_int, _dp, _dp,
                              C.c_double, C.c_double, C.c_double, C.c_double, _dp, _dp, _dp]
        L.or_eself.argtypes = [C.c_int, _dp, C.c_double]
        L.or_eself.restype = C.c_double
        L.or_erecip.argtypes = [C.c_int, _dp, C.c_double, _dp, C.c_double, C.c_int]
        L.or_erecip.restype = C.c_double
        L.or_erecip_grad.argtypes = [C.c_int, _dp, C.c_double, _dp, C.c_double, C.c_int, _dp, _dp]
        L.or_bspline.argtypes = [C.c_int, C.c_double, C.c_int]
        L.or_bspline.restype = C.c_double
        L.or_spline_mod.argtypes = [C.c_int, C.c_int, C.c_int]
        L.or_spline_mod.restype = C.c_double
        L.or_pme_mpole.argtypes = [C.c_int, _dp, C.c_double, _dp, C.c_double, C.c_int, C.c_int,
                                   C.POINTER(C.c_double), _dp, C.c_void_p]
        L.or_polarize_pcg_ewald.argtypes = [C.c_int, _dp, C.c_double, _ip, _ip, _ip, _dp, _dp,
                                            _dp, C.c_double, C.c_double, C.c_int, C.c_int,
                                            C.c_double, C.c_int, C.c_void_p, _dp,
                                            C.POINTER(PcgInfo)]
        L.or_rotate_mpole.argtypes = [C.c_int, _dp, C.c_double, _ip, _ip, _dp, _dp]
        L.or_empole_frames.argtypes = [C.c_int, _dp, C.c_double, _ip, _ip, _ip, _ip, _ip, _dp,
                                       C.c_double, C.c_double, _dp, _dp, _dp]
        L.or_vdw_sites.argtypes = [C.c_int, _dp, C.c_double, _ip, _dp, _dp]
        L.or_vdw_forces_to_atoms.argtypes = [C.c_int, _ip, _dp, _dp, _dp]
        L.or_polarize_tcg1.argtypes = [C.c_int, _dp, C.c_double, _ip, _ip, _ip, _dp, _dp, _dp,
                                       C.c_double, C.c_double, _dp, C.POINTER(C.c_double),
                                       C.c_void_p]
        L.or_epolar_frames.argtypes = [C.c_int, _dp, C.c_double, _ip, _ip, _ip, _ip, _ip, _dp,
                                       _dp, _dp, _dp, C.c_double, C.c_double, _dp, _dp, _dp]
    return L


def _d(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a if shape is None else a.reshape(shape)


def _i(a):
    return np.ascontiguousarray(a, dtype=np.int32)


COULOMB = None
DEBYE = None


def constants():
    return lib().or_coulomb_constant(), lib().or_debye_factor()


class OracleError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"oracle status {status} {msg}")
        self.status = status


def quantize(xyz, box):
    xyz = _d(xyz)
    n = xyz.shape[0]
    u = np.zeros((n, 3), dtype=np.uint32)
    st = lib().or_quantize(n, xyz, box, u)
    if st:
        raise OracleError(st)
    return u


def cutoff_quantum(rc, box):
    return int(lib().or_cutoff_quantum(rc, box))


def nblist(xyz, box, cutoff, method="cell", cap=None):
    """Canonical half list: (row_ptr[n+1], col[npairs]) with j > i ascending."""
    xyz = _d(xyz)
    n = xyz.shape[0]
    if cap is None:
        cap = max(16, n * (n - 1) // 2) if n < 4000 else int(
            n * (2.0 * np.pi / 3.0) * cutoff ** 3 * (n / box ** 3) * 1.5 + 4096)
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    col = np.zeros(max(cap, 1), dtype=np.int32)
    npairs = C.c_int64(0)
    f = lib().or_nblist_cell if method == "cell" else lib().or_nblist_brute
    st = f(n, xyz, box, cutoff, row_ptr, col, cap, C.byref(npairs))
    if st == E_CAPACITY:
        return nblist(xyz, box, cutoff, method, cap=int(npairs.value))
    if st:
        raise OracleError(st)
    return row_ptr, col[: npairs.value].copy()


def radial(r, beta, nmax=5):
    B = np.zeros(nmax + 1)
    R = np.zeros(nmax + 1)
    lib().or_radial(r, beta, nmax, B, R)
    return B, R


def thole(r, ai, aj, ti, tj):
    l3, l5, l7 = C.c_double(), C.c_double(), C.c_double()
    lib().or_thole(r, ai, aj, ti, tj, C.byref(l3), C.byref(l5), C.byref(l7))
    return l3.value, l5.value, l7.value


def mpole_pair(r, mi, mj, g):
    e = C.c_double()
    de = np.zeros(3)
    lib().or_mpole_pair(_d(r), _d(mi), _d(mj), _d(g), C.byref(e), de)
    return e.value, de


def empole_real(xyz, box, molid, row_ptr, col, mpole, beta, cutoff):
    xyz = _d(xyz)
    n = xyz.shape[0]
    energy = np.zeros(3)
    force = np.zeros((n, 3))
    virial = np.zeros((3, 3))
    st = lib().or_empole_real(n, xyz, box, _i(molid), _i(row_ptr), _i(col), _d(mpole), beta,
                              cutoff, energy, force, virial)
    if st:
        raise OracleError(st)
    return energy, force, virial


def echarge_real(xyz, box, molid, row_ptr, col, q, beta, cutoff):
    xyz = _d(xyz)
    n = xyz.shape[0]
    energy = np.zeros(3)
    force = np.zeros((n, 3))
    virial = np.zeros((3, 3))
    st = lib().or_echarge_real(n, xyz, box, _i(molid), _i(row_ptr), _i(col), _d(q), beta, cutoff,
                               energy, force, virial)
    if st:
        raise OracleError(st)
    return energy, force, virial


def efield_direct(xyz, box, molid, row_ptr, col, mpole, polarity, thole_a, beta, cutoff):
    xyz = _d(xyz)
    n = xyz.shape[0]
    field = np.zeros((n, 3))
    st = lib().or_efield_direct(n, xyz, box, _i(molid), _i(row_ptr), _i(col), _d(mpole),
                                _d(polarity), _d(thole_a), beta, cutoff, field)
    if st:
        raise OracleError(st)
    return field


def efield_intra(xyz, box, molid, row_ptr, col, mpole, polarity, thole_a, beta, cutoff, intra):
    """The permanent field with same-molecule pairs scaled by intra (0: the
    field of efield_direct)."""
    xyz = _d(xyz)
    n = xyz.shape[0]
    field = np.zeros((n, 3))
    st = lib().or_efield_intra(n, xyz, box, _i(molid), _i(row_ptr), _i(col), _d(mpole),
                               _d(polarity), _d(thole_a), beta, cutoff, float(intra), field)
    if st:
        raise OracleError(st)
    return field


def tmatvec(xyz, box, row_ptr, col, polarity, thole_a, beta, cutoff, mu, include_diag=0):
    xyz = _d(xyz)
    n = xyz.shape[0]
    out = np.zeros((n, 3))
    st = lib().or_tmatvec(n, xyz, box, _i(row_ptr), _i(col), _d(polarity), _d(thole_a), beta,
                          cutoff, int(include_diag), _d(mu), out)
    if st:
        raise OracleError(st)
    return out


def thole_l9(r, ai, aj, ti, tj):
    return lib().or_thole_l9(r, ai, aj, ti, tj)


def epolar_real(xyz, box, molid, row_ptr, col, mpole, polarity, thole_a, mu, beta, cutoff):
    """Polarization pair energies {total, induced-permanent, induced-induced},
    forces and virial at fixed induced dipoles mu (or_epolar_real)."""
    xyz = _d(xyz)
    n = xyz.shape[0]
    energy = np.zeros(3)
    force = np.zeros((n, 3))
    virial = np.zeros((3, 3))
    st = lib().or_epolar_real(n, xyz, box, _i(molid), _i(row_ptr), _i(col), _d(mpole),
                              _d(polarity), _d(thole_a), _d(mu), beta, cutoff, energy, force,
                              virial)
    if st:
        raise OracleError(st)
    return energy, force, virial


def polarize_pcg(xyz, box, molid, row_ptr, col, mpole, polarity, thole_a, beta, cutoff,
                 tol_debye=1e-5, maxiter=100, mu_guess=None):
    """Returns (mu[n,3], info dict).  Non-convergence is reported in info, not raised."""
    xyz = _d(xyz)
    n = xyz.shape[0]
    mu = np.zeros((n, 3))
    info = PcgInfo()
    guess = None
    if mu_guess is not None:
        guess_arr = _d(mu_guess)
        guess = guess_arr.ctypes.data_as(C.c_void_p)
    st = lib().or_polarize_pcg(n, xyz, box, _i(molid), _i(row_ptr), _i(col), _d(mpole),
                               _d(polarity), _d(thole_a), beta, cutoff, tol_debye, int(maxiter),
                               guess, mu, C.byref(info))
    if st not in (OK, E_NOCONV, E_BREAKDOWN):
        raise OracleError(st)
    return mu, {k: getattr(info, k) for k, _ in PcgInfo._fields_}


def polarize_pcg_ewald(xyz, box, molid, row_ptr, col, mpole, polarity, thole_a, beta, cutoff,
                       grid, order=5, tol_debye=1e-5, maxiter=100, mu_guess=None):
    """The solve with the full Ewald operator (PME reciprocal part on a grid^3
    mesh); returns (mu[n,3], info dict) as polarize_pcg."""
    xyz = _d(xyz)
    n = xyz.shape[0]
    mu = np.zeros((n, 3))
    info = PcgInfo()
    guess = None
    if mu_guess is not None:
        guess_arr = _d(mu_guess)
        guess = guess_arr.ctypes.data_as(C.c_void_p)
    st = lib().or_polarize_pcg_ewald(n, xyz, box, _i(molid), _i(row_ptr), _i(col), _d(mpole),
                                     _d(polarity), _d(thole_a), beta, cutoff, int(grid),
                                     int(order), tol_debye, int(maxiter), guess, mu,
                                     C.byref(info))
    if st not in (OK, E_NOCONV, E_BREAKDOWN):
        raise OracleError(st)
    return mu, {k: getattr(info, k) for k, _ in PcgInfo._fields_}


def epolar2_real(xyz, box, molid, row_ptr, col, mpole, polarity, thole_a, mu2, beta, cutoff,
                 pscale):
    """Polarization forces at fixed dipole sets mu2[2,n,3] (mu_d, mu_p):
    (energy[3], force[n,3], virial[3,3]) as epolar_real."""
    xyz = _d(xyz)
    n = xyz.shape[0]
    energy = np.zeros(3)
    force = np.zeros((n, 3))
    virial = np.zeros((3, 3))
    st = lib().or_epolar2_real(n, xyz, box, _i(molid), _i(row_ptr), _i(col), _d(mpole),
                               _d(polarity), _d(thole_a), _d(np.asarray(mu2).reshape(2, n, 3)),
                               beta, cutoff, float(pscale), energy, force, virial)
    if st:
        raise OracleError(st)
    return energy, force, virial


def polarize_pcg2(xyz, box, molid, row_ptr, col, mpole, polarity, thole_a, beta, cutoff, pscale,
                  tol_debye=1e-5, maxiter=100, mu_guess=None):
    """Both dipole sets: mu_d from the field without same-molecule pairs,
    mu_p from the field with them scaled by pscale.  Returns (mu[2,n,3],
    [info_d, info_p]); info_d's epol is -C/2 mu_d.E_p, info_p's -C/2 mu_p.E_d."""
    xyz = _d(xyz)
    n = xyz.shape[0]
    mu = np.zeros((2, n, 3))
    info = (PcgInfo * 2)()
    guess = None
    if mu_guess is not None:
        guess_arr = _d(np.asarray(mu_guess).reshape(2, n, 3))
        guess = guess_arr.ctypes.data_as(C.c_void_p)
    st = lib().or_polarize_pcg2(n, xyz, box, _i(molid), _i(row_ptr), _i(col), _d(mpole),
                                _d(polarity), _d(thole_a), beta, cutoff, float(pscale), tol_debye,
                                int(maxiter), guess, mu, C.byref(info))
    if st not in (OK, E_NOCONV, E_BREAKDOWN):
        raise OracleError(st)
    return mu, [{k: getattr(info[v], k) for k, _ in PcgInfo._fields_} for v in range(2)]


def polarize_pcg2_ewald(xyz, box, molid, row_ptr, col, mpole, polarity, thole_a, beta, cutoff,
                        grid, pscale, order=5, tol_debye=1e-5, maxiter=100, mu_guess=None):
    """Both dipole sets with the full Ewald operator; returns as polarize_pcg2."""
    xyz = _d(xyz)
    n = xyz.shape[0]
    mu = np.zeros((2, n, 3))
    info = (PcgInfo * 2)()
    guess = None
    if mu_guess is not None:
        guess_arr = _d(np.asarray(mu_guess).reshape(2, n, 3))
        guess = guess_arr.ctypes.data_as(C.c_void_p)
    st = lib().or_polarize_pcg2_ewald(n, xyz, box, _i(molid), _i(row_ptr), _i(col), _d(mpole),
                                      _d(polarity), _d(thole_a), beta, cutoff, int(grid),
                                      int(order), float(pscale), tol_debye, int(maxiter), guess,
                                      mu, C.byref(info))
    if st not in (OK, E_NOCONV, E_BREAKDOWN):
        raise OracleError(st)
    return mu, [{k: getattr(info[v], k) for k, _ in PcgInfo._fields_} for v in range(2)]


def evdw(xyz, box, molid, row_ptr, col, form, rad, eps, cutoff, taper_frac=0.9, dhal=0.07,
         ghal=0.12):
    xyz = _d(xyz)
    n = xyz.shape[0]
    energy = np.zeros(1)
    force = np.zeros((n, 3))
    virial = np.zeros((3, 3))
    st = lib().or_evdw(n, xyz, box, _i(molid), _i(row_ptr), _i(col), int(form), _d(rad), _d(eps),
                       cutoff, taper_frac, dhal, ghal, energy, force, virial)
    if st:
        raise OracleError(st)
    return energy[0], force, virial


def eself(mpole, beta):
    mpole = _d(mpole)
    return lib().or_eself(mpole.shape[0], mpole, beta)


def erecip(xyz, box, mpole, beta, kmax):
    xyz = _d(xyz)
    return lib().or_erecip(xyz.shape[0], xyz, box, _d(mpole), beta, int(kmax))


def dense_operator(xyz, box, row_ptr, col, polarity, thole_a, beta, cutoff):
    """The 3n x 3n polarization operator A, one column per unit vector."""
    n = np.asarray(xyz).shape[0]
    A = np.zeros((3 * n, 3 * n))
    e = np.zeros(3 * n)
    for k in range(3 * n):
        e[:] = 0.0
        e[k] = 1.0
        A[:, k] = tmatvec(xyz, box, row_ptr, col, polarity, thole_a, beta, cutoff,
                          e.reshape(n, 3), include_diag=1).ravel()
    return A


def erecip_grad(xyz, box, mpole, beta, kmax):
    """Reciprocal-space forces and field by the plain k-sum (or_erecip_grad)."""
    xyz = _d(xyz)
    n = xyz.shape[0]
    force = np.zeros((n, 3))
    field = np.zeros((n, 3))
    st = lib().or_erecip_grad(n, xyz, box, _d(mpole), beta, kmax, force, field)
    if st:
        raise OracleError(st)
    return force, field


def bspline(p, x, deriv=0):
    return lib().or_bspline(p, x, deriv)


def spline_mod(p, K, m):
    return lib().or_spline_mod(p, K, m)


def pme_mpole(xyz, box, mpole, beta, K, order=5):
    """Smooth-PME reciprocal energy, forces and field (or_pme_mpole)."""
    xyz = _d(xyz)
    n = xyz.shape[0]
    e = C.c_double()
    force = np.zeros((n, 3))
    field = np.zeros((n, 3))
    st = lib().or_pme_mpole(n, xyz, box, _d(mpole), beta, K, order, C.byref(e), force,
                            field.ctypes.data_as(C.c_void_p))
    if st:
        raise OracleError(st)
    return e.value, force, field


FRAME_NONE, FRAME_Z_THEN_X, FRAME_BISECTOR = 0, 1, 2
FRAME_Z_ONLY, FRAME_Z_BISECTOR, FRAME_3FOLD = 3, 4, 5


def rotate_mpole(xyz, box, ftype, fatoms, local):
    """Lab-frame multipoles from local-frame ones (or_rotate_mpole)."""
    xyz = _d(xyz)
    n = xyz.shape[0]
    out = np.zeros((n, 10))
    st = lib().or_rotate_mpole(n, xyz, box, _i(ftype), _i(fatoms), _d(local), out)
    if st:
        raise OracleError(st)
    return out


def empole_frames(xyz, box, molid, row_ptr, col, ftype, fatoms, local, beta, cutoff):
    """Energies, forces (torques included) and virial (frame part included)
    with local-frame multipoles."""
    xyz = _d(xyz)
    n = xyz.shape[0]
    energy = np.zeros(3)
    force = np.zeros((n, 3))
    virial = np.zeros((3, 3))
    st = lib().or_empole_frames(n, xyz, box, _i(molid), _i(row_ptr), _i(col), _i(ftype),
                                _i(fatoms), _d(local), beta, cutoff, energy, force, virial)
    if st:
        raise OracleError(st)
    return energy, force, virial


def vdw_sites(xyz, box, parent, red):
    """vdW site positions with hydrogen reduction (or_vdw_sites)."""
    xyz = _d(xyz)
    n = xyz.shape[0]
    out = np.zeros((n, 3))
    st = lib().or_vdw_sites(n, xyz, box, _i(parent), _d(red), out)
    if st:
        raise OracleError(st)
    return out


def vdw_forces_to_atoms(parent, red, fsite):
    fsite = _d(fsite)
    n = fsite.shape[0]
    out = np.zeros((n, 3))
    st = lib().or_vdw_forces_to_atoms(n, _i(parent), _d(red), fsite, out)
    if st:
        raise OracleError(st)
    return out


def polarize_tcg1(xyz, box, molid, row_ptr, col, mpole, polarity, thole_a, beta, cutoff,
                  forces=True):
    """One-step truncated CG (or_polarize_tcg1): (mu1[n,3], U, force[n,3] or None)."""
    xyz = _d(xyz)
    n = xyz.shape[0]
    mu = np.zeros((n, 3))
    e = C.c_double()
    f = np.zeros((n, 3)) if forces else None
    st = lib().or_polarize_tcg1(n, xyz, box, _i(molid), _i(row_ptr), _i(col), _d(mpole),
                                _d(polarity), _d(thole_a), beta, cutoff, mu, C.byref(e),
                                None if f is None else f.ctypes.data_as(C.c_void_p))
    if st:
        raise OracleError(st)
    return mu, e.value, f


def epolar_frames(xyz, box, molid, row_ptr, col, ftype, fatoms, local, polarity, thole_a, mu, beta,
                  cutoff):
    """Polarization pair energies, forces and virial at fixed mu with
    local-frame multipoles."""
    xyz = _d(xyz)
    n = xyz.shape[0]
    energy = np.zeros(3)
    force = np.zeros((n, 3))
    virial = np.zeros((3, 3))
    st = lib().or_epolar_frames(n, xyz, box, _i(molid), _i(row_ptr), _i(col), _i(ftype),
                                _i(fatoms), _d(local), _d(polarity), _d(thole_a), _d(mu), beta,
                                cutoff, energy, force, virial)
    if st:
        raise OracleError(st)
    return energy, force, virial
