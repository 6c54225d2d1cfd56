"""Floating-point work per pair of each real-space routine, counted by the
oracle's op-counting build (oracle/opcount.cpp).  TEST INFRASTRUCTURE ONLY.

The counting build is the oracle's own source with a counting scalar in place
of double, so the counts are those of the plain definitions the oracle
evaluates (section "Hotspots" names the routines: the polarization mat-vec,
the permanent-field right-hand side, the multipole energy, the 14-7 and 12-6
van der Waals energies and the point-charge energy, plus the polarization
forces).  Counts per pair come from two-atom systems in different molecules:

  per evaluated pair = ops(pair inside the cutoff) - ops(pair listed, beyond it)
  per listed pair    = ops(pair listed, beyond it) - ops(no pair listed)

(3.1 A inside; 7.5 A beyond the 7 A cutoff, 9.5 A beyond the 9 A one.)

``flops`` adds +, -, *, / (one each) and fma (two); the library calls (sqrt,
exp, erfc, pow) are listed apart.  ``python -m oracle.opcount --write``
writes tests/golden/pair_opcounts.json (read by the benchmark for its
algorithmic flop rates and pinned by the tests).
"""
import contextlib
import ctypes as C
import json
import os
import subprocess
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "opcount.cpp")
LIB = os.path.join(HERE, "liboracle_ops.so")
GOLDEN = os.path.join(ROOT, "tests", "golden", "pair_opcounts.json")
KINDS = ("add", "mul", "div", "fma", "sqrt", "exp", "erfc", "trig", "pow", "other")

_L = None


def build(verbose=False):
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-w", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def counting_lib():
    global _L
    if _L is None:
        from oracle import oracle as O
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
                os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "tk_oracle.c"))):
            build()
        L = O.configure(C.CDLL(LIB))
        L.or_ops_read.argtypes = [C.POINTER(C.c_longlong)]
        L.or_ops_reset.argtypes = []
        _L = L
    return _L


@contextlib.contextmanager
def counting():
    """Within the block the oracle's Python functions run on the counting build."""
    from oracle import oracle as O
    saved = O._lib
    O._lib = counting_lib()
    try:
        yield O
    finally:
        O._lib = saved


def ops():
    buf = (C.c_longlong * len(KINDS))()
    counting_lib().or_ops_read(buf)
    return dict(zip(KINDS, (int(v) for v in buf)))


def reset():
    counting_lib().or_ops_reset()


def flops(c):
    return c["add"] + c["mul"] + c["div"] + 2 * c["fma"]


def _diff(a, b):
    return {k: a[k] - b[k] for k in KINDS}


BETA, RC = 0.5446, 7.0
POL = np.array([0.837, 0.496])
THOLE = np.array([0.39, 0.39])
MOLID = np.array([0, 1], dtype=np.int32)
BOX = 30.0


def _xyz(r):
    u = np.array([0.48, -0.36, 0.8])
    u /= np.linalg.norm(u)
    return np.array([[1.0, 2.0, 3.0], [1.0, 2.0, 3.0]]) + np.outer([0.0, r], u)


def _pair_list(listed):
    return (np.array([0, 1, 1], dtype=np.int32), np.array([1], dtype=np.int32)) if listed else \
        (np.array([0, 0, 0], dtype=np.int32), np.zeros(0, dtype=np.int32))


def _counts(call, r_out=7.5):
    """ops of call(xyz, row_ptr, col) at r = 3.1 (in), r = r_out (listed, beyond the
    cutoff) and with no pair listed."""
    res = []
    for r, listed in ((3.1, True), (r_out, True), (r_out, False)):
        rp, cp = _pair_list(listed)
        reset()
        call(_xyz(r), rp, cp)
        res.append(ops())
    ev, lst = _diff(res[0], res[1]), _diff(res[1], res[2])
    return {"evaluated_pair": ev, "listed_pair": lst,
            "flops_per_evaluated_pair": flops(ev), "flops_per_listed_pair": flops(lst)}


def pair_counts():
    rng = np.random.default_rng(5)
    mpole = rng.normal(0.0, 0.1, (2, 10))
    mpole[:, 9] = -(mpole[:, 4] + mpole[:, 7])   # traceless quadrupoles
    mu = rng.normal(0.0, 0.05, (2, 3))
    q = np.array([-0.834, 0.417])
    rad = np.array([3.405, 2.655])
    eps = np.array([0.11, 0.0135])
    out = {}
    with counting() as O:
        out["tmatvec"] = _counts(lambda x, rp, cp: O.tmatvec(x, BOX, rp, cp, POL, THOLE, BETA, RC,
                                                             mu, 0))
        out["efield_direct"] = _counts(lambda x, rp, cp: O.efield_direct(
            x, BOX, MOLID, rp, cp, mpole, POL, THOLE, BETA, RC))
        out["empole_real"] = _counts(lambda x, rp, cp: O.empole_real(x, BOX, MOLID, rp, cp, mpole,
                                                                     BETA, RC))
        out["epolar_real"] = _counts(lambda x, rp, cp: O.epolar_real(
            x, BOX, MOLID, rp, cp, mpole, POL, THOLE, mu, BETA, RC))
        out["evdw_hal"] = _counts(lambda x, rp, cp: O.evdw(x, BOX, MOLID, rp, cp, O.VDW_HAL, rad,
                                                           eps, 9.0), r_out=9.5)
        out["evdw_lj"] = _counts(lambda x, rp, cp: O.evdw(x, BOX, MOLID, rp, cp, O.VDW_LJ,
                                                          np.array([3.15, 3.15]), eps, 9.0),
                                  r_out=9.5)
        out["echarge_real"] = _counts(lambda x, rp, cp: O.echarge_real(x, BOX, MOLID, rp, cp, q,
                                                                       0.34, RC))
    return out


def main():
    res = pair_counts()
    for k, v in res.items():
        e = v["evaluated_pair"]
        print(f"{k:14s} flops/evaluated pair {v['flops_per_evaluated_pair']:4d} "
              f"(+ sqrt {e['sqrt']}, exp {e['exp']}, erfc {e['erfc']}, pow {e['pow']}); "
              f"per listed pair {v['flops_per_listed_pair']}")
    if "--write" in sys.argv:
        doc = {"about": "floating-point operations per pair of each real-space routine, counted "
                        "by the oracle's op-counting build (oracle/opcount.py): + - * / one "
                        "each, fma two; library calls apart",
               "counts": res}
        with open(GOLDEN, "w") as f:
            json.dump(doc, f, indent=1, sort_keys=True)
            f.write("\n")
        print("wrote", GOLDEN)


if __name__ == "__main__":
    main()
