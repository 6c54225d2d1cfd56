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
E_TOOBIG = -10
FP64, MIXED = 0, 1
VDW_HAL, VDW_LJ = 0, 1
MAX_PLANS = 8


class System(C.Structure):
    _fields_ = [("n", C.c_int32), ("xyz", C.c_void_p), ("box", C.c_double), ("molid", C.c_void_p)]


class NbList(C.Structure):
    _fields_ = [("row_ptr", C.c_void_p), ("col", C.c_void_p), ("npairs", C.c_int64),
                ("cutoff", C.c_double), ("plan", C.c_int32)]


class NbBounds(C.Structure):
    _fields_ = [("max_occ", C.c_int32), ("max_row", C.c_int32), ("max_nbhd", C.c_int32),
                ("reserved", C.c_int32), ("windows", C.c_int64), ("npairs", C.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_ if k != "reserved"}


class PcgInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("refinements", C.c_int32),
                ("converged", C.c_int32), ("rms_debye", C.c_double),
                ("rms_true_debye", C.c_double), ("epol", C.c_double)]


class StepParams(C.Structure):
    _fields_ = [("rc_ewald", C.c_double), ("rc_vdw", C.c_double), ("skin", C.c_double),
                ("ewald_beta", C.c_double), ("tol_debye", C.c_double),
                ("taper_on_frac", C.c_double), ("hal_delta", C.c_double),
                ("hal_gamma", C.c_double), ("maxiter", C.c_int32), ("prec", C.c_int32)]


class Batch(C.Structure):
    _fields_ = [("nsys", C.c_int32), ("atom_off", C.c_void_p), ("box", C.c_void_p),
                ("xyz", C.c_void_p), ("molid", C.c_void_p)]


class StepResult(C.Structure):
    _fields_ = [("e_mpole", C.c_double * 3), ("w_mpole", C.c_double * 9), ("e_vdw", C.c_double),
                ("w_vdw", C.c_double * 9), ("rc_vdw", C.c_double), ("pcg", PcgInfo)]

    def as_dict(self):
        return {"e_mpole": list(self.e_mpole), "w_mpole": list(self.w_mpole),
                "e_vdw": self.e_vdw, "w_vdw": list(self.w_vdw), "rc_vdw": self.rc_vdw,
                "pcg": {k: getattr(self.pcg, k) for k, _ in PcgInfo._fields_}}


class Request(C.Structure):
    _fields_ = [("n", C.c_int32), ("box", C.c_double), ("xyz", C.c_void_p), ("molid", C.c_void_p),
                ("mpole", C.c_void_p), ("polarity", C.c_void_p), ("thole", C.c_void_p),
                ("vdw_rad", C.c_void_p), ("vdw_eps", C.c_void_p), ("session", C.c_uint64)]


class Timing(C.Structure):
    _fields_ = [("t_submit", C.c_int64), ("t_start", C.c_int64), ("t_done", C.c_int64),
                ("batch_size", C.c_int32), ("batch_index", C.c_int32), ("lane", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("lanes", C.c_int32), ("batches", C.c_int32), ("budget", C.c_size_t),
                ("peak_device_bytes", C.c_size_t), ("device_bytes", C.c_size_t),
                ("bytes_per_atom", C.c_double)]


def step_params(s, prec=FP64):
    """StepParams from a settings dict (synth.AMOEBA_SETTINGS keys)."""
    return StepParams(s["rc_ewald"], s["rc_vdw"], s["skin"], s["beta"], s["tol_debye"],
                      s["taper_frac"], s["dhal"], s["ghal"], int(s["maxiter"]), int(prec))


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
    "tk_nblist_build_multi": [_vp, _i32, _vp, C.POINTER(System), _vp, _vp, _vp, _vp, _vp,
                              C.POINTER(_i64)],
    "tk_nblist_bounds_get": [_vp, _i32, _d, C.POINTER(NbBounds)],
    "tk_nblist_build_async": [_vp, _vp, C.POINTER(System), _d, _i32, C.POINTER(NbBounds), _vp,
                              _vp, _i64, _vp, _vp, _vp],
    "tk_empole_real": [_vp, _vp, C.POINTER(System), C.POINTER(NbList), _vp, _d, _d, C.c_int, _vp,
                       _vp, _vp],
    "tk_echarge_real": [_vp, _vp, C.POINTER(System), C.POINTER(NbList), _vp, _d, _d, C.c_int, _vp,
                        _vp, _vp],
    "tk_efield_direct": [_vp, _vp, C.POINTER(System), C.POINTER(NbList), _vp, _vp, _vp, _d, _d,
                         C.c_int, _vp],
    "tk_tmatvec": [_vp, _vp, C.POINTER(System), C.POINTER(NbList), _vp, _vp, _d, _d, C.c_int,
                   C.c_int, _vp, _vp],
    "tk_tmatvec_noalloc": [_vp, _vp, C.POINTER(System), C.POINTER(NbList), _vp, _vp, _d, _d,
                           C.c_int, C.c_int, _vp, _vp],
    "tk_tmatvec_noalloc_max_atoms": [],
    "tk_polarize_pcg": [_vp, _vp, C.POINTER(System), C.POINTER(NbList), _vp, _vp, _vp, _d, _d, _d,
                        _i32, C.c_int, _vp, _vp, C.POINTER(PcgInfo)],
    "tk_polarize_pcg_queued": [_vp, _vp, C.POINTER(System), C.POINTER(NbList), _vp, _vp, _vp,
                               _d, _d, _d, _i32, C.c_int, _vp, _vp, _vp],
    "tk_empole_polarize_queued": [_vp, _vp, C.POINTER(System), C.POINTER(NbList), _vp, _vp,
                                  _vp, _d, _d, _d, _i32, C.c_int, _vp, _vp, _vp, _vp, _vp, _vp],
    "tk_epolar_real": [_vp, _vp, C.POINTER(System), C.POINTER(NbList), _vp, _vp, _vp, _vp, _d,
                       _d, C.c_int, _vp, _vp, _vp],
    "tk_pme_mpole": [_vp, _vp, C.POINTER(System), _vp, _d, _i32, _i32, _vp, _vp, _vp],
    "tk_empole_polarize": [_vp, _vp, C.POINTER(System), C.POINTER(NbList), _vp, _vp, _vp, _d,
                           _d, _d, _i32, C.c_int, _vp, _vp, C.POINTER(PcgInfo), _vp, _vp, _vp],
    "tk_polarize_pcg_ewald": [_vp, _vp, C.POINTER(System), C.POINTER(NbList), _vp, _vp, _vp, _d,
                              _d, _i32, _i32, _d, _i32, _vp, _vp, C.POINTER(PcgInfo)],
    "tk_polarize_pcg2": [_vp, _vp, C.POINTER(System), C.POINTER(NbList), _vp, _vp, _vp, _d, _d,
                         _d, _d, _i32, _vp, _vp, C.POINTER(PcgInfo * 2)],
    "tk_polarize_pcg2_ewald": [_vp, _vp, C.POINTER(System), C.POINTER(NbList), _vp, _vp, _vp,
                               _d, _d, _i32, _i32, _d, _d, _i32, _vp, _vp,
                               C.POINTER(PcgInfo * 2)],
    "tk_epolar_ewald": [_vp, _vp, C.POINTER(System), C.POINTER(NbList), _vp, _vp, _vp, _vp, _d,
                        _d, _i32, _i32, _vp, _vp],
    "tk_epolar2_real": [_vp, _vp, C.POINTER(System), C.POINTER(NbList), _vp, _vp, _vp, _vp, _d,
                        _d, _d, _vp, _vp, _vp],
    "tk_rotate_mpole": [_vp, _vp, C.POINTER(System), _vp, _vp, _vp, _vp],
    "tk_empole_frames": [_vp, _vp, C.POINTER(System), C.POINTER(NbList), _vp, _vp, _vp, _d, _d,
                         _vp, _vp, _vp, _vp],
    "tk_vdw_sites": [_vp, _vp, C.POINTER(System), _vp, _vp, _vp],
    "tk_vdw_site_forces": [_vp, _vp, _i32, _vp, _vp, _vp, _vp],
    "tk_polarize_tcg1": [_vp, _vp, C.POINTER(System), C.POINTER(NbList), _vp, _vp, _vp, _d, _d,
                         _vp, _vp, _vp],
    "tk_epolar_frames": [_vp, _vp, C.POINTER(System), C.POINTER(NbList), _vp, _vp, _vp, _vp, _vp,
                         _vp, _d, _d, _vp, _vp, _vp],
    "tk_evdw": [_vp, _vp, C.POINTER(System), C.POINTER(NbList), C.c_int, _vp, _vp, _d, _d, _d, _d,
                C.c_int, _vp, _vp, _vp],
    "tk_batch_step": [_vp, _vp, C.POINTER(Batch), C.POINTER(StepParams), _vp, _vp, _vp, _vp, _vp,
                      _vp, _vp, _vp, _vp, _vp, _vp],
    "tk_server_create": [C.c_int, C.POINTER(StepParams), C.c_size_t, _i32, C.POINTER(_vp)],
    "tk_server_create_lanes": [C.c_int, C.POINTER(StepParams), C.c_size_t, _i32, _i32,
                               C.POINTER(_vp)],
    "tk_server_footprint": [_i32],
    "tk_server_submit": [_vp, C.POINTER(Request), C.POINTER(C.c_uint64)],
    "tk_server_poll": [_vp, C.c_uint64, C.POINTER(StepResult), C.POINTER(Timing), _vp, _vp, _vp],
    "tk_server_release": [_vp, C.c_uint64],
    "tk_server_stats": [_vp, C.POINTER(ServerStats)],
    "tk_server_destroy": [_vp],
    "tk_set_arena_budget": [_vp, C.c_size_t],
    "tk_arena_bytes": [_vp],
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
            f.restype = C.c_int32 if name not in ("tk_destroy", "tk_strerror",
                                                  "tk_server_destroy") else None
        L.tk_strerror.restype = C.c_char_p
        L.tk_server_footprint.restype = C.c_size_t
        L.tk_arena_bytes.restype = C.c_size_t
        _lib = L
    return _lib


def _check(st, where):
    if st != OK:
        raise TkError(st, where)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev(t, dtype, device, shape=None, what="array"):
    """A contiguous device tensor of `dtype`; with `shape`, refused (ValueError)
    unless it has exactly that shape: the kernels index every array by the
    system's atom count, so a shorter one would be read out of bounds."""
    t = torch.as_tensor(t)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} must have shape {tuple(shape)}; got {tuple(t.shape)}")
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

    # -- device-memory budget ------------------------------------------------------
    def set_arena_budget(self, nbytes):
        """Bound the device bytes this context may hold (0: no bound)."""
        _check(load().tk_set_arena_budget(self._h, int(nbytes)), "tk_set_arena_budget")

    def arena_bytes(self):
        return int(load().tk_arena_bytes(self._h))

    # -- kernel timing -----------------------------------------------------------
    def profile(self, on=True, only=None, reset=True):
        """Time kernel launches with HIP events on their stream (optionally one
        kernel).  Switching on clears the counters (which waits for the timed
        work) unless reset is False."""
        if on and reset:
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
        if x.dim() != 2 or x.shape[1] != 3:
            raise ValueError(f"xyz must have shape (n, 3); got {tuple(x.shape)}")
        m = _dev(molid, torch.int32, self.device, (x.shape[0],), "molid")
        return SystemRef(x, float(box), m)

    def nblist(self, sysref, cutoff, plan_slot=0, cap=None, want_csr=True):
        n = sysref.n
        if cap is None:
            rho = n / sysref.box ** 3
            cap = int(n * (2.0 * 3.141592653589793 / 3.0) * cutoff ** 3 * rho * 1.3 + 4096)
        row_ptr = torch.empty(n + 1, dtype=torch.int32, device=self.device) if want_csr else None
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

    def nblists(self, sysref, cutoffs, plan_slots, streams=None, want_csr=True):
        """Several lists of the same atoms with one host synchronisation
        (tk_nblist_build_multi).  streams: one torch stream per list (None: the
        current stream for all); list k's outputs are ready in streams[k]'s
        order."""
        n, k = sysref.n, len(cutoffs)
        cur = torch.cuda.current_stream(self.device)
        strs = list(streams) if streams is not None else [cur] * k
        rho = n / sysref.box ** 3
        caps = [int(n * (2.0 * 3.141592653589793 / 3.0) * c ** 3 * rho * 1.3 + 4096)
                for c in cutoffs]
        while True:
            rps = [torch.empty(n + 1, dtype=torch.int32, device=self.device) if want_csr else None
                   for _ in range(k)]
            cols = [torch.empty(max(c, 1), dtype=torch.int32, device=self.device) if want_csr
                    else None for c in caps]
            for t, st in zip(rps + cols, strs + strs):
                if t is not None and st != cur:
                    t.record_stream(st)   # written (and maybe read) on another stream
            npairs = (C.c_int64 * k)()
            arr_st = (C.c_void_p * k)(*[st.cuda_stream for st in strs])
            arr_cut = (C.c_double * k)(*[float(c) for c in cutoffs])
            arr_slot = (C.c_int32 * k)(*[int(x) for x in plan_slots])
            arr_rp = (C.c_void_p * k)(*[None if t is None else t.data_ptr() for t in rps])
            arr_col = (C.c_void_p * k)(*[None if t is None else t.data_ptr() for t in cols])
            arr_cap = (C.c_int64 * k)(*[c if want_csr else 0 for c in caps])
            st = load().tk_nblist_build_multi(self._h, k, arr_st, C.byref(sysref.c), arr_cut,
                                              arr_slot, arr_rp, arr_col, arr_cap, npairs)
            if st == E_CAPACITY and want_csr and any(npairs[i] > caps[i] for i in range(k)):
                caps = [max(caps[i], int(npairs[i])) for i in range(k)]
                continue
            _check(st, "tk_nblist_build_multi")
            return [ListRef(rps[i], None if cols[i] is None else cols[i][: npairs[i]],
                            int(npairs[i]), float(cutoffs[i]), int(plan_slots[i]))
                    for i in range(k)]

    def nblist_bounds(self, plan_slot, headroom=0.1):
        """Bounds for stream-ordered builds of a slot, from its last synchronous build."""
        b = NbBounds()
        _check(load().tk_nblist_bounds_get(self._h, int(plan_slot), float(headroom), C.byref(b)),
               "tk_nblist_bounds_get")
        return b

    def nblist_async(self, sysref, cutoff, plan_slot, bounds, cap=None, want_csr=True,
                     stream=None, report=True):
        """The list queued on `stream` (default: the current one) with no host
        synchronisation (tk_nblist_build_async); its pair count and status
        stay on the device (AsyncListRef)."""
        n = sysref.n
        if cap is None:
            cap = int(bounds.npairs)
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        with torch.cuda.stream(st):
            row_ptr = torch.empty(n + 1, dtype=torch.int32, device=self.device) if want_csr else None
            col = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device) if want_csr else None
            npd = torch.empty(1, dtype=torch.int64, device=self.device)
            std = torch.empty(1, dtype=torch.int32, device=self.device)
            rep = torch.empty(4, dtype=torch.int64, device=self.device) if report else None
        _check(load().tk_nblist_build_async(self._h, st.cuda_stream, C.byref(sysref.c), cutoff,
                                            int(plan_slot), C.byref(bounds), _ptr(row_ptr),
                                            _ptr(col), int(cap), _ptr(npd), _ptr(std), _ptr(rep)),
               "tk_nblist_build_async")
        return AsyncListRef(row_ptr, col, -1, float(cutoff), int(plan_slot), npd, std, rep)

    # -- pair terms ------------------------------------------------------------
    def empole_real(self, sysref, lst, mpole, beta, cutoff, prec=FP64):
        mp = _dev(mpole, torch.float64, self.device, (sysref.n, 10), "mpole")
        e = torch.empty(3, dtype=torch.float64, device=self.device)
        f = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        w = torch.empty((3, 3), dtype=torch.float64, device=self.device)
        _check(load().tk_empole_real(self._h, _stream(self.device), C.byref(sysref.c),
                                     C.byref(lst.c), _ptr(mp), beta, cutoff, prec, _ptr(e), _ptr(f),
                                     _ptr(w)), "tk_empole_real")
        return e, f, w

    def echarge_real(self, sysref, lst, q, beta, cutoff, prec=FP64):
        qq = _dev(q, torch.float64, self.device, (sysref.n,), "q")
        e = torch.empty(3, dtype=torch.float64, device=self.device)
        f = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        w = torch.empty((3, 3), dtype=torch.float64, device=self.device)
        _check(load().tk_echarge_real(self._h, _stream(self.device), C.byref(sysref.c),
                                      C.byref(lst.c), _ptr(qq), beta, cutoff, prec, _ptr(e),
                                      _ptr(f), _ptr(w)), "tk_echarge_real")
        return e, f, w

    def efield_direct(self, sysref, lst, mpole, polarity, thole, beta, cutoff, prec=FP64):
        mp = _dev(mpole, torch.float64, self.device, (sysref.n, 10), "mpole")
        pol = _dev(polarity, torch.float64, self.device, (sysref.n,), "polarity")
        th = _dev(thole, torch.float64, self.device, (sysref.n,), "thole")
        out = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        _check(load().tk_efield_direct(self._h, _stream(self.device), C.byref(sysref.c),
                                       C.byref(lst.c), _ptr(mp), _ptr(pol), _ptr(th), beta, cutoff,
                                       prec, _ptr(out)), "tk_efield_direct")
        return out

    def tmatvec(self, sysref, lst, polarity, thole, beta, cutoff, mu, include_diag=0, prec=FP64):
        pol = _dev(polarity, torch.float64, self.device, (sysref.n,), "polarity")
        th = _dev(thole, torch.float64, self.device, (sysref.n,), "thole")
        m = _dev(mu, torch.float64, self.device, (sysref.n, 3), "mu")
        out = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        _check(load().tk_tmatvec(self._h, _stream(self.device), C.byref(sysref.c), C.byref(lst.c),
                                 _ptr(pol), _ptr(th), beta, cutoff, int(include_diag), prec,
                                 _ptr(m), _ptr(out)), "tk_tmatvec")
        return out

    def tmatvec_noalloc(self, sysref, lst, polarity, thole, beta, cutoff, mu, out,
                        include_diag=0, prec=FP64):
        """tk_tmatvec_noalloc into the caller's `out` (device [n][3] float64);
        returns the status (no allocation on the library side)."""
        return load().tk_tmatvec_noalloc(self._h, _stream(self.device), C.byref(sysref.c),
                                         C.byref(lst.c), _ptr(polarity), _ptr(thole), beta,
                                         cutoff, int(include_diag), prec, _ptr(mu), _ptr(out))

    def polarize_pcg(self, sysref, lst, mpole, polarity, thole, beta, cutoff, tol_debye=1e-5,
                     maxiter=100, prec=FP64, mu_guess=None):
        mp = _dev(mpole, torch.float64, self.device, (sysref.n, 10), "mpole")
        pol = _dev(polarity, torch.float64, self.device, (sysref.n,), "polarity")
        th = _dev(thole, torch.float64, self.device, (sysref.n,), "thole")
        g = None if mu_guess is None else _dev(mu_guess, torch.float64, self.device,
                                               (sysref.n, 3), "mu_guess")
        out = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        info = PcgInfo()
        st = load().tk_polarize_pcg(self._h, _stream(self.device), C.byref(sysref.c),
                                    C.byref(lst.c), _ptr(mp), _ptr(pol), _ptr(th), beta, cutoff,
                                    tol_debye, int(maxiter), prec, _ptr(g), _ptr(out),
                                    C.byref(info))
        if st not in (OK, E_NOCONV, E_BREAKDOWN):
            _check(st, "tk_polarize_pcg")
        return out, {k: getattr(info, k) for k, _ in PcgInfo._fields_}

    def polarize_pcg_queued(self, sysref, lst, mpole, polarity, thole, beta, cutoff, iterations,
                            tol_debye=1e-5, prec=FP64, mu_guess=None, info_dev=None):
        """tk_polarize_pcg_queued: (mu, info_dev), both written in stream order
        on the current stream; info_dev is a device uint8 tensor holding one
        tk_pcg_info (read it with pcg_info)."""
        mp = _dev(mpole, torch.float64, self.device, (sysref.n, 10), "mpole")
        pol = _dev(polarity, torch.float64, self.device, (sysref.n,), "polarity")
        th = _dev(thole, torch.float64, self.device, (sysref.n,), "thole")
        g = None if mu_guess is None else _dev(mu_guess, torch.float64, self.device,
                                               (sysref.n, 3), "mu_guess")
        out = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        info_dev = self._info_dev(info_dev)
        st = load().tk_polarize_pcg_queued(self._h, _stream(self.device), C.byref(sysref.c),
                                           C.byref(lst.c), _ptr(mp), _ptr(pol), _ptr(th), beta,
                                           cutoff, tol_debye, int(iterations), prec, _ptr(g),
                                           _ptr(out), _ptr(info_dev))
        _check(st, "tk_polarize_pcg_queued")
        return out, info_dev

    def empole_polarize_queued(self, sysref, lst, mpole, polarity, thole, beta, cutoff,
                               iterations, tol_debye=1e-5, prec=FP64, mu_guess=None,
                               info_dev=None):
        """tk_empole_polarize_queued: (energy[3], force, virial), (mu, info_dev), all
        written in stream order on the current stream."""
        mp = _dev(mpole, torch.float64, self.device, (sysref.n, 10), "mpole")
        pol = _dev(polarity, torch.float64, self.device, (sysref.n,), "polarity")
        th = _dev(thole, torch.float64, self.device, (sysref.n,), "thole")
        g = None if mu_guess is None else _dev(mu_guess, torch.float64, self.device,
                                               (sysref.n, 3), "mu_guess")
        out = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        e = torch.empty(3, dtype=torch.float64, device=self.device)
        f = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        v = torch.empty(9, dtype=torch.float64, device=self.device)
        info_dev = self._info_dev(info_dev)
        st = load().tk_empole_polarize_queued(self._h, _stream(self.device), C.byref(sysref.c),
                                              C.byref(lst.c), _ptr(mp), _ptr(pol), _ptr(th),
                                              beta, cutoff, tol_debye, int(iterations), prec,
                                              _ptr(g), _ptr(out), _ptr(info_dev), _ptr(e),
                                              _ptr(f), _ptr(v))
        _check(st, "tk_empole_polarize_queued")
        return (e, f, v), (out, info_dev)

    def _info_dev(self, info_dev):
        if info_dev is None:
            return torch.empty(C.sizeof(PcgInfo), dtype=torch.uint8, device=self.device)
        if (info_dev.device != self.device or info_dev.dtype != torch.uint8
                or info_dev.numel() < C.sizeof(PcgInfo) or not info_dev.is_contiguous()):
            raise ValueError("info_dev: contiguous device uint8 tensor of sizeof(tk_pcg_info)")
        return info_dev

    @staticmethod
    def pcg_info(info_dev):
        """Decode a device tk_pcg_info (synchronises with its writer)."""
        raw = bytes(info_dev[:C.sizeof(PcgInfo)].cpu().numpy().tobytes())
        info = PcgInfo.from_buffer_copy(raw)
        return {k: getattr(info, k) for k, _ in PcgInfo._fields_}

    def empole_polarize(self, sysref, lst, mpole, polarity, thole, beta, cutoff, tol_debye=1e-5,
                        maxiter=100, prec=FP64, mu_guess=None):
        """tk_empole_polarize: (energy[3], force, virial), (mu, info)."""
        mp = _dev(mpole, torch.float64, self.device, (sysref.n, 10), "mpole")
        pol = _dev(polarity, torch.float64, self.device, (sysref.n,), "polarity")
        th = _dev(thole, torch.float64, self.device, (sysref.n,), "thole")
        g = None if mu_guess is None else _dev(mu_guess, torch.float64, self.device,
                                               (sysref.n, 3), "mu_guess")
        out = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        e = torch.empty(3, dtype=torch.float64, device=self.device)
        f = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        v = torch.empty(9, dtype=torch.float64, device=self.device)
        info = PcgInfo()
        st = load().tk_empole_polarize(self._h, _stream(self.device), C.byref(sysref.c),
                                       C.byref(lst.c), _ptr(mp), _ptr(pol), _ptr(th), beta, cutoff,
                                       tol_debye, int(maxiter), prec, _ptr(g), _ptr(out),
                                       C.byref(info), _ptr(e), _ptr(f), _ptr(v))
        if st not in (OK, E_NOCONV, E_BREAKDOWN):
            _check(st, "tk_empole_polarize")
        return (e, f, v), (out, {k: getattr(info, k) for k, _ in PcgInfo._fields_})

    def polarize_pcg_ewald(self, sysref, lst, mpole, polarity, thole, beta, cutoff, grid,
                           order=5, tol_debye=1e-5, maxiter=100, mu_guess=None):
        mp = _dev(mpole, torch.float64, self.device, (sysref.n, 10), "mpole")
        pol = _dev(polarity, torch.float64, self.device, (sysref.n,), "polarity")
        th = _dev(thole, torch.float64, self.device, (sysref.n,), "thole")
        g = None if mu_guess is None else _dev(mu_guess, torch.float64, self.device,
                                               (sysref.n, 3), "mu_guess")
        out = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        info = PcgInfo()
        st = load().tk_polarize_pcg_ewald(self._h, _stream(self.device), C.byref(sysref.c),
                                          C.byref(lst.c), _ptr(mp), _ptr(pol), _ptr(th), beta,
                                          cutoff, int(grid), int(order), tol_debye, int(maxiter),
                                          _ptr(g), _ptr(out), C.byref(info))
        if st not in (OK, E_NOCONV, E_BREAKDOWN):
            _check(st, "tk_polarize_pcg_ewald")
        return out, {k: getattr(info, k) for k, _ in PcgInfo._fields_}

    def polarize_pcg2(self, sysref, lst, mpole, polarity, thole, beta, cutoff, pscale,
                      tol_debye=1e-5, maxiter=100, mu_guess=None):
        """Both dipole sets: returns (mu[2,n,3] with mu_d first, [info_d, info_p])."""
        mp = _dev(mpole, torch.float64, self.device, (sysref.n, 10), "mpole")
        pol = _dev(polarity, torch.float64, self.device, (sysref.n,), "polarity")
        th = _dev(thole, torch.float64, self.device, (sysref.n,), "thole")
        g = None if mu_guess is None else _dev(mu_guess, torch.float64, self.device,
                                               (2, sysref.n, 3), "mu_guess")
        out = torch.empty((2, sysref.n, 3), dtype=torch.float64, device=self.device)
        info = (PcgInfo * 2)()
        st = load().tk_polarize_pcg2(self._h, _stream(self.device), C.byref(sysref.c),
                                     C.byref(lst.c), _ptr(mp), _ptr(pol), _ptr(th), beta, cutoff,
                                     float(pscale), tol_debye, int(maxiter), _ptr(g), _ptr(out),
                                     C.byref(info))
        if st not in (OK, E_NOCONV, E_BREAKDOWN):
            _check(st, "tk_polarize_pcg2")
        return out, [{k: getattr(info[v], k) for k, _ in PcgInfo._fields_} for v in range(2)]

    def epolar_real(self, sysref, lst, mpole, polarity, thole, mu, beta, cutoff, prec=FP64):
        mp = _dev(mpole, torch.float64, self.device, (sysref.n, 10), "mpole")
        pol = _dev(polarity, torch.float64, self.device, (sysref.n,), "polarity")
        th = _dev(thole, torch.float64, self.device, (sysref.n,), "thole")
        m = _dev(mu, torch.float64, self.device, (sysref.n, 3), "mu")
        e = torch.empty(3, dtype=torch.float64, device=self.device)
        f = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        w = torch.empty((3, 3), dtype=torch.float64, device=self.device)
        _check(load().tk_epolar_real(self._h, _stream(self.device), C.byref(sysref.c),
                                     C.byref(lst.c), _ptr(mp), _ptr(pol), _ptr(th), _ptr(m), beta,
                                     cutoff, prec, _ptr(e), _ptr(f), _ptr(w)), "tk_epolar_real")
        return e, f, w

    def polarize_pcg2_ewald(self, sysref, lst, mpole, polarity, thole, beta, cutoff, grid,
                            pscale, order=5, tol_debye=1e-5, maxiter=100, mu_guess=None):
        """Both dipole sets with the full Ewald operator; returns as polarize_pcg2."""
        mp = _dev(mpole, torch.float64, self.device, (sysref.n, 10), "mpole")
        pol = _dev(polarity, torch.float64, self.device, (sysref.n,), "polarity")
        th = _dev(thole, torch.float64, self.device, (sysref.n,), "thole")
        g = None if mu_guess is None else _dev(mu_guess, torch.float64, self.device,
                                               (2, sysref.n, 3), "mu_guess")
        out = torch.empty((2, sysref.n, 3), dtype=torch.float64, device=self.device)
        info = (PcgInfo * 2)()
        st = load().tk_polarize_pcg2_ewald(self._h, _stream(self.device), C.byref(sysref.c),
                                           C.byref(lst.c), _ptr(mp), _ptr(pol), _ptr(th), beta,
                                           cutoff, int(grid), int(order), float(pscale),
                                           tol_debye, int(maxiter), _ptr(g), _ptr(out),
                                           C.byref(info))
        if st not in (OK, E_NOCONV, E_BREAKDOWN):
            _check(st, "tk_polarize_pcg2_ewald")
        return out, [{k: getattr(info[v], k) for k, _ in PcgInfo._fields_} for v in range(2)]

    def epolar_ewald(self, sysref, lst, mpole, polarity, thole, mu, beta, cutoff, grid, order=5):
        """Polarization energies [total, real space, reciprocal] and forces at
        fixed dipoles with the full Ewald operator."""
        mp = _dev(mpole, torch.float64, self.device, (sysref.n, 10), "mpole")
        pol = _dev(polarity, torch.float64, self.device, (sysref.n,), "polarity")
        th = _dev(thole, torch.float64, self.device, (sysref.n,), "thole")
        m = _dev(mu, torch.float64, self.device, (sysref.n, 3), "mu")
        e = torch.empty(3, dtype=torch.float64, device=self.device)
        f = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        _check(load().tk_epolar_ewald(self._h, _stream(self.device), C.byref(sysref.c),
                                      C.byref(lst.c), _ptr(mp), _ptr(pol), _ptr(th), _ptr(m), beta,
                                      cutoff, int(grid), int(order), _ptr(e), _ptr(f)),
               "tk_epolar_ewald")
        return e, f

    def epolar2_real(self, sysref, lst, mpole, polarity, thole, mu2, beta, cutoff, pscale):
        """Polarization forces with both dipole sets mu2[2,n,3] (mu_d first)."""
        mp = _dev(mpole, torch.float64, self.device, (sysref.n, 10), "mpole")
        pol = _dev(polarity, torch.float64, self.device, (sysref.n,), "polarity")
        th = _dev(thole, torch.float64, self.device, (sysref.n,), "thole")
        m = _dev(mu2, torch.float64, self.device, (2, sysref.n, 3), "mu2")
        e = torch.empty(3, dtype=torch.float64, device=self.device)
        f = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        w = torch.empty((3, 3), dtype=torch.float64, device=self.device)
        _check(load().tk_epolar2_real(self._h, _stream(self.device), C.byref(sysref.c),
                                      C.byref(lst.c), _ptr(mp), _ptr(pol), _ptr(th), _ptr(m), beta,
                                      cutoff, float(pscale), _ptr(e), _ptr(f), _ptr(w)),
               "tk_epolar2_real")
        return e, f, w

    def pme_mpole(self, sysref, mpole, beta, grid, order=5, want_field=True):
        mp = _dev(mpole, torch.float64, self.device, (sysref.n, 10), "mpole")
        e = torch.empty(1, dtype=torch.float64, device=self.device)
        f = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        fld = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device) if want_field \
            else None
        _check(load().tk_pme_mpole(self._h, _stream(self.device), C.byref(sysref.c), _ptr(mp), beta,
                                   int(grid), int(order), _ptr(e), _ptr(f),
                                   None if fld is None else _ptr(fld)), "tk_pme_mpole")
        return e, f, fld

    def _frames(self, sysref, frame_type, frame_atoms):
        """Device frame types [n] and frame atoms [n, 3]; the kernels read three
        atoms per site, so other shapes are refused here."""
        ft = _dev(frame_type, torch.int32, self.device)
        fa = _dev(frame_atoms, torch.int32, self.device)
        if tuple(ft.shape) != (sysref.n,) or tuple(fa.shape) != (sysref.n, 3):
            raise ValueError(f"frame_type must be [{sysref.n}] and frame_atoms [{sysref.n}, 3]; "
                             f"got {tuple(ft.shape)} and {tuple(fa.shape)}")
        return ft, fa

    def rotate_mpole(self, sysref, frame_type, frame_atoms, mpole_local):
        ft, fa = self._frames(sysref, frame_type, frame_atoms)
        ml = _dev(mpole_local, torch.float64, self.device, (sysref.n, 10), "mpole_local")
        out = torch.empty((sysref.n, 10), dtype=torch.float64, device=self.device)
        _check(load().tk_rotate_mpole(self._h, _stream(self.device), C.byref(sysref.c), _ptr(ft),
                                      _ptr(fa), _ptr(ml), _ptr(out)), "tk_rotate_mpole")
        return out

    def empole_frames(self, sysref, lst, frame_type, frame_atoms, mpole_local, beta, cutoff):
        ft, fa = self._frames(sysref, frame_type, frame_atoms)
        ml = _dev(mpole_local, torch.float64, self.device, (sysref.n, 10), "mpole_local")
        e = torch.empty(3, dtype=torch.float64, device=self.device)
        f = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        w = torch.empty((3, 3), dtype=torch.float64, device=self.device)
        mg = torch.empty((sysref.n, 10), dtype=torch.float64, device=self.device)
        _check(load().tk_empole_frames(self._h, _stream(self.device), C.byref(sysref.c),
                                       C.byref(lst.c), _ptr(ft), _ptr(fa), _ptr(ml), beta, cutoff,
                                       _ptr(e), _ptr(f), _ptr(w), _ptr(mg)), "tk_empole_frames")
        return e, f, mg, w

    def vdw_sites(self, sysref, parent, red):
        par = _dev(parent, torch.int32, self.device, (sysref.n,), "parent")
        rd = _dev(red, torch.float64, self.device, (sysref.n,), "red")
        out = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        _check(load().tk_vdw_sites(self._h, _stream(self.device), C.byref(sysref.c), _ptr(par),
                                   _ptr(rd), _ptr(out)), "tk_vdw_sites")
        return out

    def vdw_site_forces(self, parent, red, site_force):
        fs = _dev(site_force, torch.float64, self.device)
        n = fs.shape[0]
        if fs.dim() != 2 or fs.shape[1] != 3:
            raise ValueError(f"site_force must have shape (n, 3); got {tuple(fs.shape)}")
        par = _dev(parent, torch.int32, self.device, (n,), "parent")
        rd = _dev(red, torch.float64, self.device, (n,), "red")
        out = torch.empty_like(fs)
        _check(load().tk_vdw_site_forces(self._h, _stream(self.device), int(fs.shape[0]), _ptr(par),
                                         _ptr(rd), _ptr(fs), _ptr(out)), "tk_vdw_site_forces")
        return out

    def polarize_tcg1(self, sysref, lst, mpole, polarity, thole, beta, cutoff, forces=True):
        mp = _dev(mpole, torch.float64, self.device, (sysref.n, 10), "mpole")
        pol = _dev(polarity, torch.float64, self.device, (sysref.n,), "polarity")
        th = _dev(thole, torch.float64, self.device, (sysref.n,), "thole")
        mu = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        e = torch.empty(1, dtype=torch.float64, device=self.device)
        f = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device) if forces else None
        _check(load().tk_polarize_tcg1(self._h, _stream(self.device), C.byref(sysref.c),
                                       C.byref(lst.c), _ptr(mp), _ptr(pol), _ptr(th), beta, cutoff,
                                       _ptr(mu), _ptr(e), _ptr(f)), "tk_polarize_tcg1")
        return mu, e, f

    def epolar_frames(self, sysref, lst, frame_type, frame_atoms, mpole_local, polarity, thole, mu,
                      beta, cutoff):
        ft, fa = self._frames(sysref, frame_type, frame_atoms)
        ml = _dev(mpole_local, torch.float64, self.device, (sysref.n, 10), "mpole_local")
        pol = _dev(polarity, torch.float64, self.device, (sysref.n,), "polarity")
        th = _dev(thole, torch.float64, self.device, (sysref.n,), "thole")
        m = _dev(mu, torch.float64, self.device, (sysref.n, 3), "mu")
        e = torch.empty(3, dtype=torch.float64, device=self.device)
        f = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        w = torch.empty((3, 3), dtype=torch.float64, device=self.device)
        _check(load().tk_epolar_frames(self._h, _stream(self.device), C.byref(sysref.c),
                                       C.byref(lst.c), _ptr(ft), _ptr(fa), _ptr(ml), _ptr(pol),
                                       _ptr(th), _ptr(m), beta, cutoff, _ptr(e), _ptr(f), _ptr(w)),
               "tk_epolar_frames")
        return e, f, w

    def evdw(self, sysref, lst, form, rad, eps, cutoff, taper_frac=0.9, dhal=0.07, ghal=0.12,
             prec=FP64):
        r = _dev(rad, torch.float64, self.device, (sysref.n,), "rad")
        ep = _dev(eps, torch.float64, self.device, (sysref.n,), "eps")
        e = torch.empty(1, dtype=torch.float64, device=self.device)
        f = torch.empty((sysref.n, 3), dtype=torch.float64, device=self.device)
        w = torch.empty((3, 3), dtype=torch.float64, device=self.device)
        _check(load().tk_evdw(self._h, _stream(self.device), C.byref(sysref.c), C.byref(lst.c),
                              int(form), _ptr(r), _ptr(ep), cutoff, taper_frac, dhal, ghal, prec,
                              _ptr(e), _ptr(f), _ptr(w)), "tk_evdw")
        return e[0], f, w


    # -- batches of systems ----------------------------------------------------
    def batch_step(self, systems, params, mu_guess=None, use_guess=None):
        """One step (lists, multipoles, dipoles, HAL) for a list of systems in
        one batch.  systems: objects with xyz, box, molid, mpole, polarity,
        thole, vdw_rad, vdw_eps (host arrays).  Returns (results, forces_mpole,
        mu, forces_vdw) with per-system dicts and per-system [n][3] tensors."""
        import numpy as np
        off = np.zeros(len(systems) + 1, dtype=np.int32)
        off[1:] = np.cumsum([len(w.xyz) for w in systems])
        box = np.array([w.box for w in systems], dtype=np.float64)
        cat = lambda f, dt: _dev(np.concatenate([np.asarray(getattr(w, f)) for w in systems]),
                                 dt, self.device)
        xyz, molid = cat("xyz", torch.float64), cat("molid", torch.int32)
        mp, pol, th = cat("mpole", torch.float64), cat("polarity", torch.float64), cat(
            "thole", torch.float64)
        rad, eps = cat("vdw_rad", torch.float64), cat("vdw_eps", torch.float64)
        n = int(off[-1])
        g = None if mu_guess is None else _dev(mu_guess, torch.float64, self.device)
        ug = None if use_guess is None else np.ascontiguousarray(use_guess, dtype=np.int32)
        fm = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        mu = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        fv = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        res = (StepResult * len(systems))()
        b = Batch(len(systems), off.ctypes.data, box.ctypes.data, xyz.data_ptr(), molid.data_ptr())
        _check(load().tk_batch_step(self._h, _stream(self.device), C.byref(b), C.byref(params),
                                    _ptr(mp), _ptr(pol), _ptr(th), _ptr(rad), _ptr(eps), _ptr(g),
                                    None if ug is None else C.c_void_p(ug.ctypes.data), _ptr(fm),
                                    _ptr(mu), _ptr(fv), res), "tk_batch_step")
        split = lambda t: [t[off[k]:off[k + 1]] for k in range(len(systems))]
        return [r.as_dict() for r in res], split(fm), split(mu), split(fv)


class Server:
    """Continuous-batching server (three lanes unless `lanes` says fewer: a
    thread, context and stream each)."""

    def __init__(self, params, hbm_budget, max_batch=256, device=0, lanes=3):
        if not torch.cuda.is_available():
            raise RuntimeError("libtk needs a ROCm GPU; none is visible")
        self._h = C.c_void_p()
        self._keep = {}
        _check(load().tk_server_create_lanes(device, C.byref(params), int(hbm_budget),
                                             int(max_batch), int(lanes), C.byref(self._h)),
               "tk_server_create_lanes")

    @staticmethod
    def footprint(n):
        return int(load().tk_server_footprint(int(n)))

    def submit(self, w, session=0):
        """Queue one system (host arrays); returns the request id."""
        import numpy as np
        arr = [np.ascontiguousarray(w.xyz, dtype=np.float64),
               np.ascontiguousarray(w.molid, dtype=np.int32),
               np.ascontiguousarray(w.mpole, dtype=np.float64),
               np.ascontiguousarray(w.polarity, dtype=np.float64),
               np.ascontiguousarray(w.thole, dtype=np.float64),
               np.ascontiguousarray(w.vdw_rad, dtype=np.float64),
               np.ascontiguousarray(w.vdw_eps, dtype=np.float64)]
        q = Request(len(arr[0]), float(w.box), *[a.ctypes.data for a in arr], int(session))
        rid = C.c_uint64(0)
        _check(load().tk_server_submit(self._h, C.byref(q), C.byref(rid)), "tk_server_submit")
        self._keep[rid.value] = len(arr[0])
        return rid.value

    def poll(self, rid, arrays=True):
        """None while running; else (result dict, timing dict, f_mpole, mu, f_vdw)."""
        import numpy as np
        n = self._keep[rid]
        res, tim = StepResult(), Timing()
        outs = [np.empty((n, 3)) for _ in range(3)] if arrays else [None] * 3
        st = load().tk_server_poll(self._h, rid, C.byref(res), C.byref(tim),
                                   *[None if a is None else C.c_void_p(a.ctypes.data) for a in outs])
        if st == E_BUSY:
            return None
        _check(st, "tk_server_poll")
        t = {k: getattr(tim, k) for k, _ in Timing._fields_}
        return (res.as_dict(), t, *outs)

    def release(self, rid):
        _check(load().tk_server_release(self._h, rid), "tk_server_release")
        self._keep.pop(rid, None)

    def stats(self):
        st = ServerStats()
        _check(load().tk_server_stats(self._h, C.byref(st)), "tk_server_stats")
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def close(self):
        if self._h:
            load().tk_server_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


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


@dataclass
class AsyncListRef(ListRef):
    """A list from tk_nblist_build_async: npairs is -1 on the host; the count,
    the status and the measured sizes are device tensors (reading them
    synchronises)."""
    npairs_dev: torch.Tensor = None
    status_dev: torch.Tensor = None
    report_dev: torch.Tensor = None

    def status(self):
        return int(self.status_dev.item())

    def count(self):
        return int(self.npairs_dev.item())

    def report(self):
        r = self.report_dev.cpu()
        i32 = r[:2].view(torch.int32)
        return {"max_occ": int(i32[0]), "max_row": int(i32[1]), "max_nbhd": int(i32[2]),
                "windows": int(r[2]), "npairs": int(r[3])}

    def resolved(self):
        """The same list with its pair count read back (col cut to it)."""
        m = self.count()
        return ListRef(self.row_ptr, None if self.col is None else self.col[:m], m, self.cutoff,
                       self.plan)
