"""Thin ctypes binding of libtk.so (declared in include/tk.h).

Argument marshalling only: torch CUDA tensors provide device memory and the
stream; every step of the computation runs in the library's HIP kernels.
There is no CPU fallback: ``load()`` raises if the library or a GPU is
missing.
"""
import ctypes as C
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtk.so")

OK, E_ARG, E_CUTOFF, E_CAPACITY, E_NOCONV, E_BREAKDOWN, E_NOMEM, E_HIP, E_BUSY, E_PLAN = (
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9)
FP64, MIXED = 0, 1
VDW_HAL, VDW_LJ = 0, 1
MAX_PLANS = 8


class System(C.Structure):
    _fields_ = [("n", C.c_int32), ("xyz", C.c_void_p), ("box", C.c_double), ("molid", C.c_void_p)]


class NbList(C.Structure):
    _fields_ = [("row_ptr", C.c_void_p), ("col", C.c_void_p), ("npairs", C.c_int64),
                ("cutoff", C.c_double), ("plan", C.c_int32)]


class PcgInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("refinements", C.c_int32),
                ("converged", C.c_int32), ("rms_debye", C.c_double),
                ("rms_true_debye", C.c_double), ("epol", C.c_double)]


class TkError(RuntimeError):
    def __init__(self, status, where=""):
        msg = load().tk_strerror(status).decode() if _lib is not None else str(status)
        super().__init__(f"{where}: {msg} ({status})")
        self.status = status


_lib = None
_vp, _i32, _i64, _d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
_SIGS = {
    "tk_create": [C.c_int, C.POINTER(C.c_void_p)],
    "tk_destroy": [_vp],
    "tk_strerror": [_i32],
    "tk_nblist_build": [_vp, _vp, C.POINTER(System), _d, _i32, _vp, _vp, _i64, C.POINTER(_i64)],
    "tk_empole_real": [_vp, _vp, C.POINTER(System), C.POINTER(NbList), _vp, _d, _d, C.c_int, _vp,
                       _vp, _vp],
    "tk_echarge_real": [_vp, _vp, C.POINTER(System), C.POINTER(NbList), _vp, _d, _d, C.c_int, _vp,
                        _vp, _vp],
    "tk_efield_direct": [_vp, _vp, C.POINTER(System), C.POINTER(NbList), _vp, _vp, _vp, _d, _d,
                         C.c_int, _vp],
    "tk_tmatvec": [_vp, _vp, C.POINTER(System), C.POINTER(NbList), _vp, _vp, _d, _d, C.c_int,
                   C.c_int, _vp, _vp],
    "tk_polarize_pcg": [_vp, _vp, C.POINTER(System), C.POINTER(NbList), _vp, _vp, _vp, _d, _d, _d,
                        _i32, C.c_int, _vp, _vp, C.POINTER(PcgInfo)],
    "tk_evdw": [_vp, _vp, C.POINTER(System), C.POINTER(NbList), C.c_int, _vp, _vp, _d, _d, _d, _d,
                C.c_int, _vp, _vp, _vp],
    "tk_profile_enable": [_vp, C.c_int, C.c_char_p],
    "tk_profile_read": [_vp, _i32, C.c_char_p, _i32, C.POINTER(_i64), C.POINTER(_d)],
    "tk_profile_reset": [_vp],
}


def exported_symbols():
    return list(_SIGS)


def load(path: str = LIB_PATH):
    """Load libtk.so (no compute).  Raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"libtk.so not built ({path}); run __graft_entry__.build()")
        L = C.CDLL(path)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int32 if name not in ("tk_destroy", "tk_strerror") else None
        L.tk_strerror.restype = C.c_char_p
        _lib = L
    return _lib


def _check(st, where):
    if st != OK:
        raise TkError(st, where)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev(t, dtype, device):
    t = torch.as_tensor(t)
    return t.to(device=device, dtype=dtype).contiguous()


def _stream(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Context:
    """A libtk context on one GPU (owns scratch memory and list plans)."""

    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("libtk needs a ROCm GPU; none is visible")
        self.device = torch.device("cuda", device)
        self._h = C.c_void_p()
        torch.cuda.set_device(self.device)
        _check(load().tk_create(device, C.byref(self._h)), "tk_create")

    def close(self):
        if self._h:
            load().tk_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- kernel timing -----------------------------------------------------------
    def profile(self, on=True, only=None):
        """Time kernel launches with HIP events on their stream (optionally one kernel)."""
        if on:
            _check(load().tk_profile_reset(self._h), "tk_profile_reset")
        _check(load().tk_profile_enable(self._h, int(on), None if only is None else only.encode()),
               "tk_profile_enable")

    def profile_read(self):
        out = {}
        buf = C.create_string_buffer(128)
        n, ms = C.c_int64(0), C.c_double(0.0)
        k = 0
        while load().tk_profile_read(self._h, k, buf, 128, C.byref(n), C.byref(ms)) == OK:
            out[buf.value.decode()] = {"launches": int(n.value), "ms": float(ms.value)}
            k += 1
        return out

    # -- systems and lists ---------------------------------------------------
    def system(self, xyz, box, molid):
        """Device copies of coordinates and molecule ids; returns a SystemRef."""
        x = _dev(xyz, torch.float64, self.device)
        m = _dev(molid, torch.int32, self.device)
        return SystemRef(x, float(box), m)

    def nblist(self, sysref, cutoff, plan_slot=0, cap=None, want_csr=True):
        n = sysref.n
        if cap is None:
            rho = n / sysref.box ** 3
            cap = int(n * (2.0 * 3.141592653589793 / 3.0) * cutoff ** 3 * rho * 1.3 + 4096)
        row_ptr = torch.zeros(n + 1, dtype=torch.int32, device=self.device) if want_csr else None
        col = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device) if want_csr else None
        npairs = C.c_int64(0)
        st = load().tk_nblist_build(self._h, _stream(self.device), C.byref(sysref.c), cutoff,
                                    plan_slot, _ptr(row_ptr), _ptr(col), cap if want_csr else 0,
                                    C.byref(npairs))
        if st == E_CAPACITY and want_csr and npairs.value > cap:
            return self.nblist(sysref, cutoff, plan_slot, cap=int(npairs.value), want_csr=True)
        _check(st, "tk_nblist_build")
        return ListRef(row_ptr, None if col is None else col[: npairs.value], int(npairs.value),
                       float(cutoff), int(plan_slot))

    # -- pair terms ------------------------------------------------------------
    def empole_real(self, sysref, lst, mpole, beta, cutoff, prec=FP64):
        mp = _dev(mpole, torch.float64, self.device)
        e = torch.zeros(3, dtype=torch.float64, device=self.device)
        f = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        w = torch.zeros((3, 3), dtype=torch.float64, device=self.device)
        _check(load().tk_empole_real(self._h, _stream(self.device), C.byref(sysref.c),
                                     C.byref(lst.c), _ptr(mp), beta, cutoff, prec, _ptr(e), _ptr(f),
                                     _ptr(w)), "tk_empole_real")
        return e, f, w

    def echarge_real(self, sysref, lst, q, beta, cutoff, prec=FP64):
        qq = _dev(q, torch.float64, self.device)
        e = torch.zeros(3, dtype=torch.float64, device=self.device)
        f = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        w = torch.zeros((3, 3), dtype=torch.float64, device=self.device)
        _check(load().tk_echarge_real(self._h, _stream(self.device), C.byref(sysref.c),
                                      C.byref(lst.c), _ptr(qq), beta, cutoff, prec, _ptr(e),
                                      _ptr(f), _ptr(w)), "tk_echarge_real")
        return e, f, w

    def efield_direct(self, sysref, lst, mpole, polarity, thole, beta, cutoff, prec=FP64):
        mp = _dev(mpole, torch.float64, self.device)
        pol = _dev(polarity, torch.float64, self.device)
        th = _dev(thole, torch.float64, self.device)
        out = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        _check(load().tk_efield_direct(self._h, _stream(self.device), C.byref(sysref.c),
                                       C.byref(lst.c), _ptr(mp), _ptr(pol), _ptr(th), beta, cutoff,
                                       prec, _ptr(out)), "tk_efield_direct")
        return out

    def tmatvec(self, sysref, lst, polarity, thole, beta, cutoff, mu, include_diag=0, prec=FP64):
        pol = _dev(polarity, torch.float64, self.device)
        th = _dev(thole, torch.float64, self.device)
        m = _dev(mu, torch.float64, self.device)
        out = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        _check(load().tk_tmatvec(self._h, _stream(self.device), C.byref(sysref.c), C.byref(lst.c),
                                 _ptr(pol), _ptr(th), beta, cutoff, int(include_diag), prec,
                                 _ptr(m), _ptr(out)), "tk_tmatvec")
        return out

    def polarize_pcg(self, sysref, lst, mpole, polarity, thole, beta, cutoff, tol_debye=1e-5,
                     maxiter=100, prec=FP64, mu_guess=None):
        mp = _dev(mpole, torch.float64, self.device)
        pol = _dev(polarity, torch.float64, self.device)
        th = _dev(thole, torch.float64, self.device)
        g = None if mu_guess is None else _dev(mu_guess, torch.float64, self.device)
        out = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        info = PcgInfo()
        st = load().tk_polarize_pcg(self._h, _stream(self.device), C.byref(sysref.c),
                                    C.byref(lst.c), _ptr(mp), _ptr(pol), _ptr(th), beta, cutoff,
                                    tol_debye, int(maxiter), prec, _ptr(g), _ptr(out),
                                    C.byref(info))
        if st not in (OK, E_NOCONV, E_BREAKDOWN):
            _check(st, "tk_polarize_pcg")
        return out, {k: getattr(info, k) for k, _ in PcgInfo._fields_}

    def evdw(self, sysref, lst, form, rad, eps, cutoff, taper_frac=0.9, dhal=0.07, ghal=0.12,
             prec=FP64):
        r = _dev(rad, torch.float64, self.device)
        ep = _dev(eps, torch.float64, self.device)
        e = torch.zeros(1, dtype=torch.float64, device=self.device)
        f = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        w = torch.zeros((3, 3), dtype=torch.float64, device=self.device)
        _check(load().tk_evdw(self._h, _stream(self.device), C.byref(sysref.c), C.byref(lst.c),
                              int(form), _ptr(r), _ptr(ep), cutoff, taper_frac, dhal, ghal, prec,
                              _ptr(e), _ptr(f), _ptr(w)), "tk_evdw")
        return e[0], f, w


@dataclass
class SystemRef:
    xyz: torch.Tensor
    box: float
    molid: torch.Tensor

    def __post_init__(self):
        self.c = System(self.xyz.shape[0], self.xyz.data_ptr(), self.box, self.molid.data_ptr())

    @property
    def n(self):
        return int(self.xyz.shape[0])


@dataclass
class ListRef:
    row_ptr: torch.Tensor
    col: torch.Tensor
    npairs: int
    cutoff: float
    plan: int

    def __post_init__(self):
        self.c = NbList(None if self.row_ptr is None else self.row_ptr.data_ptr(),
                        None if self.col is None else self.col.data_ptr(), self.npairs,
                        self.cutoff, self.plan)
