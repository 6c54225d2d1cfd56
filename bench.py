"""Benchmark: one step = one pass of the real-space AMOEBA hot path on one GPU.

Step (23,559-atom water box, FP64 unless --prec mixed):
  neighbour list at 7 A (CSR + cell-pair plan), neighbour list at 9 A,
  permanent-multipole energy/forces/virial and the permanent field (7 A, one
  fused pass), induced dipoles by PCG to 1e-5 D RMS (mat-vecs + FP64 true
  residual), Halgren 14-7 energy/forces/virial (9 A).
value = real-space pair interactions per second over the whole step (each
listed pair with r <= rc counted once per routine that evaluates it: the
multipole energy and the permanent field once each, the mat-vec once per
call, HAL once).  Inputs are resident in HBM before the timed region.

The step is stream-ordered: the lists come from the stream-ordered build
(bounds from a synchronous build of the same box plus 10 %), the solve runs
the iteration count that the synchronous solve took (a caller carries it from
step to step) and stops on convergence, and nothing inside a step waits for
the host.  After the timed loop every step's list status and solve outcome
are read back: a failed list or an unconverged solve fails the run.

Prints ONE JSON line.  Extra keys: polarization solves/s, the mixed-precision
step, the point-charge + LJ path (96,000 atoms, 12 A), the roofline of the
dominant kernel (HIP events inside the library, on the launch stream) and the
CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1906_01211_amd import synth  # noqa: E402

# Compulsory HBM bytes of one solver mat-vec launch (iteration k): per listed
# pair its 4-byte pair code and its two cached radial factors (8 bytes each in
# FP64, 4 in the mixed form); per atom the coordinates (24), z (24), the
# previous direction (24) and alpha (8) read, p (24) and q (24) written.
MV_BYTES_PER_PAIR = {"fp64": 4 + 16, "mixed": 4 + 8}
MV_BYTES_PER_ATOM = 24 + 24 + 24 + 8 + 24 + 24
# Floating-point operations per listed pair of the same launch (both atoms'
# fields: pair vector 9, two dot products 10, two field updates 12, scale 2).
MV_FLOPS_PER_PAIR = 33
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
# Unpacked FP32 vector issue (the form this library is built for) runs at the
# FP64 vector rate: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz.
PEAK_FP32_UNPACKED_TFLOPS = 78.6
# Floating-point operations per pair of each routine, counted by the oracle's
# op-counting build (+ - * / one each, fma two; sqrt, exp, erfc and pow
# apart): per evaluated pair (r <= rc) and per listed pair (image, distance).
OPCOUNTS = os.path.join(ROOT, "tests", "golden", "pair_opcounts.json")


def algorithmic_flops(routines, evaluated, listed):
    """Algorithmic FLOPs of one pass over a list: the listed routines' counts
    per evaluated pair times the evaluated pairs, plus theirs per listed
    pair times the listed pairs."""
    with open(OPCOUNTS) as f:
        c = json.load(f)["counts"]
    return sum(c[r]["flops_per_evaluated_pair"] * evaluated + c[r]["flops_per_listed_pair"] * listed
               for r in routines)


def valu_entry(prof, name, routines, evaluated, listed, peak, per_launch=1):
    """Algorithmic FLOP rate of one VALU-bound pair kernel from its HIP-event
    time (per_launch: passes over the list per launch)."""
    if name not in prof or prof[name]["launches"] == 0:
        return None
    us = prof[name]["ms"] / prof[name]["launches"] * 1e3
    fl = algorithmic_flops(routines, evaluated, listed) * per_launch
    return {"routines": list(routines), "avg_launch_us": round(us, 2),
            "algorithmic_gflop_per_launch": round(fl / 1e9, 4),
            "tflops": round(fl / (us * 1e-6) / 1e12, 3), "peak_tflops": peak,
            "frac": round(fl / (us * 1e-6) / 1e12 / peak, 4)}
PEAK_HBM_GBS = 8000.0


def committed_traffic(prec):
    """HBM bytes per launch of the FP64 solver mat-vec from the committed
    counter summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when
    the kernel source has changed since the counters were taken."""
    import hashlib
    if prec != "fp64":
        return None
    path = os.path.join(ROOT, "profiles", "pcg_mv_water7853_fp64_traffic.txt")
    src = os.path.join(ROOT, "paper_1906_01211_amd", "csrc", "pcg.hip")
    try:
        kv = dict(line.split(": ", 1) for line in open(path).read().splitlines()
                  if line.startswith(("kernel_source_sha256", "fetch_bytes", "write_bytes")))
        if kv["kernel_source_sha256"].strip() != hashlib.sha256(open(src, "rb").read()).hexdigest():
            return None
        return int(kv["fetch_bytes_per_launch"]) + int(kv["write_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def count_pairs(xyz, box, row_ptr, col, rc, molid=None, skip_same=False):
    n = len(row_ptr) - 1
    i = np.repeat(np.arange(n), np.diff(row_ptr))
    d = xyz[col] - xyz[i]
    d -= box * np.rint(d / box)
    ok = np.einsum("ij,ij->i", d, d) <= rc * rc
    if skip_same:
        ok &= molid[i] != molid[col]
    return int(ok.sum())


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--prec", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--serial-step", action="store_true",
                    help="run HAL after the solve on one stream (each kernel alone; for "
                         "kernel traces)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=512)
    ap.add_argument("--no-solve-rates", action="store_true",
                    help="skip the solve-alone rates (kept out of the profiled step traces)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run device-to-device copies of this many MiB (a kernel of known "
                         "traffic for scaling HBM counters)")
    return ap.parse_args()


class AmoebaStep:
    def __init__(self, ctx, tk, w, prec):
        import torch
        self.ctx, self.tk, self.w, self.prec = ctx, tk, w, prec
        s = synth.AMOEBA_SETTINGS
        self.s = s
        dev = ctx.device
        self.sys = ctx.system(w.xyz, w.box, w.molid)
        self.mpole = torch.as_tensor(w.mpole, device=dev)
        self.pol = torch.as_tensor(w.polarity, device=dev)
        self.thole = torch.as_tensor(w.thole, device=dev)
        self.rad = torch.as_tensor(w.vdw_rad, device=dev)
        self.eps = torch.as_tensor(w.vdw_eps, device=dev)
        self.side = torch.cuda.Stream(device=dev)   # default priority
        self.info = None
        self.out = None   # the last step's outputs (device tensors), for the accuracy check

    def __call__(self):
        import torch
        c, s, p = self.ctx, self.s, self.prec
        main = torch.cuda.current_stream(c.device)
        # the two lists are built concurrently (the 9 A one on a second stream),
        # with one host synchronisation; the second stream first waits for the
        # previous step's use of its plan slot.  (Running the multipole and
        # HAL kernels concurrently as well was measured slower: each fills
        # the GPU on its own.)
        self.side.wait_stream(main)
        l7, l9 = c.nblists(self.sys, [s["rc_ewald"] + s["skin"], s["rc_vdw"] + s["skin"]],
                           [0, 1], streams=[main, self.side])
        main.wait_stream(self.side)   # the 9 A list is complete before the solver starts
        # multipole energy/forces/virial and the induced dipoles: one call, the
        # multipole terms and the permanent field from one pass over the list
        em, (mu, self.info) = c.empole_polarize(self.sys, l7, self.mpole, self.pol, self.thole,
                                                s["beta"], s["rc_ewald"],
                                                tol_debye=s["tol_debye"], maxiter=s["maxiter"],
                                                prec=p)
        ev = c.evdw(self.sys, l9, self.tk.VDW_HAL, self.rad, self.eps, s["rc_vdw"],
                    s["taper_frac"], s["dhal"], s["ghal"], prec=p)
        self.out = (em, mu, ev)
        return l7, l9

    def pair_counts(self):
        l7, l9 = self()
        self.l7_pairs = l7.npairs
        self.l9_pairs = l9.npairs
        w, s = self.w, self.s
        n7 = count_pairs(w.xyz, w.box, l7.row_ptr.cpu().numpy(), l7.col.cpu().numpy(),
                         s["rc_ewald"])
        n9 = count_pairs(w.xyz, w.box, l9.row_ptr.cpu().numpy(), l9.col.cpu().numpy(), s["rc_vdw"],
                         w.molid, skip_same=True)
        return n7, n9


class QueuedAmoebaStep(AmoebaStep):
    """The same step with no host synchronisation inside it: both lists from
    the stream-ordered build (bounds: the synchronous build's sizes plus 10 %),
    the multipole terms and dipoles from the queued fused call with the
    synchronous solve's iteration count (the count a caller carries from one
    step to the next) on the first stream, HAL on the second.  Every list
    status and solve outcome stays on the device; `check` reads them after
    the timed loop."""

    def __init__(self, ctx, tk, w, prec, iters, serial=False):
        super().__init__(ctx, tk, w, prec)
        self.serial = serial   # HAL after the solve on the first stream (each kernel alone)
        s = self.s
        ctx.nblists(self.sys, [s["rc_ewald"] + s["skin"], s["rc_vdw"] + s["skin"]], [6, 7])
        self.b7, self.b9 = ctx.nblist_bounds(6, 0.1), ctx.nblist_bounds(7, 0.1)
        self.iters = int(iters)
        self.flags = []   # per step: both list statuses and the solve outcome (device)

    def __call__(self):
        import torch
        c, s, p = self.ctx, self.s, self.prec
        main = torch.cuda.current_stream(c.device)
        self.side.wait_stream(main)
        l7 = c.nblist_async(self.sys, s["rc_ewald"] + s["skin"], 6, self.b7, stream=main,
                            report=False)
        l9 = c.nblist_async(self.sys, s["rc_vdw"] + s["skin"], 7, self.b9, stream=self.side,
                            report=False)
        # HAL on the second stream behind its list, beside the solve: the
        # solve's launches are latency-bound and leave room on the GPU
        # (0.601 against 0.660 ms with HAL after the solve on one stream)
        hal = lambda: c.evdw(self.sys, l9, self.tk.VDW_HAL, self.rad, self.eps, s["rc_vdw"],
                             s["taper_frac"], s["dhal"], s["ghal"], prec=p)
        if not self.serial:
            with torch.cuda.stream(self.side):
                ev = hal()
        else:
            main.wait_stream(self.side)
        em, (mu, info_dev) = c.empole_polarize_queued(self.sys, l7, self.mpole, self.pol,
                                                      self.thole, s["beta"], s["rc_ewald"],
                                                      self.iters, tol_debye=s["tol_debye"],
                                                      prec=p)
        if self.serial:
            ev = hal()
        main.wait_stream(self.side)
        self.flags.append((l7.status_dev, l9.status_dev, info_dev))   # read after the loop
        self.out = (em, mu, ev)
        return l7, l9

    def check(self):
        """Every step since the last check: lists built, solve converged."""
        last = None
        for s7, s9, info_dev in self.flags:
            last = self.ctx.pcg_info(info_dev)
            assert int(s7.item()) == 0 and int(s9.item()) == 0, "a queued step's list failed"
            assert last["converged"] == 1, "a queued step's solve did not converge"
        self.flags = []
        if last is not None:
            self.info = last
        return last


class EveryKth:
    """Runs `step`, timing the dominant kernel's launches with HIP events in
    every k-th call only: an event-timed dispatch costs the GPU about 5 us, so
    timing all eight mat-vecs of every step would add about 40 us to it."""

    def __init__(self, ctx, step, dom, k):
        self.ctx, self.step, self.dom, self.k = ctx, step, dom, k
        self.calls = 0
        self.sampled = 0

    def __call__(self):
        on = self.calls % self.k == 0
        if on:
            self.ctx.profile(True, only=self.dom, reset=False)
            self.sampled += 1
        r = self.step()
        if on:
            self.ctx.profile(False)
        self.calls += 1
        return r


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# Row-block workers of the all-core leg (forked before the GPU is touched; each
# runs the unchanged oracle on its block of CSR rows).
_blk = {}


def _block_rows(row_ptr, parts):
    """Row boundaries splitting the listed pairs into `parts` nearly equal blocks."""
    n = len(row_ptr) - 1
    tgt = np.linspace(0, row_ptr[-1], parts + 1)
    b = np.searchsorted(row_ptr, tgt, side="left")
    b[0], b[-1] = 0, n
    return np.maximum.accumulate(b)


def _sub_csr(row_ptr, col, r0, r1):
    base = row_ptr[r0]
    rp = np.clip(row_ptr, row_ptr[r0], row_ptr[r1]) - base
    return rp.astype(np.int32), np.ascontiguousarray(col[row_ptr[r0]:row_ptr[r1]])


def _blk_work(k):
    """One worker's share of the step's pair kernels: rows of block k of the
    7 A list (multipoles, permanent field, `mv` mat-vecs) and of the 9 A list
    (HAL).  Returns its multipole energy (the blocks' sum is the full one)."""
    from oracle import oracle as O
    d = _blk
    w, s = d["w"], synth.AMOEBA_SETTINGS
    rp, cp = d["b7"][k]
    rp9, cp9 = d["b9"][k]
    e, _, _ = O.empole_real(w.xyz, w.box, w.molid, rp, cp, w.mpole, s["beta"], s["rc_ewald"])
    O.efield_direct(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole, s["beta"],
                    s["rc_ewald"])
    v = d["mu"]
    for _ in range(d["mv"]):
        O.tmatvec(w.xyz, w.box, rp, cp, w.polarity, w.thole, s["beta"], s["rc_ewald"], v, 1)
    O.evdw(w.xyz, w.box, w.molid, rp9, cp9, 0, w.vdw_rad, w.vdw_eps, s["rc_vdw"])
    return float(e[0])


def cpu_baseline(w):
    """The CPU oracle on the benchmark's step, serial (one full step: lists,
    multipoles, PCG solve, HAL) and on all the host's cores (the same step's
    pair kernels split by CSR row blocks over one process per core, the unchanged
    oracle in each; the lists and the PCG vector algebra, a few percent of the
    serial time, are left out there).  Runs before the GPU is touched (the
    workers are forked).  Returns the record, the reference outputs and the
    pair counts at 7 A (r <= 7) and 9 A (r <= 9, other molecules)."""
    import multiprocessing as mp
    from oracle import oracle as O
    s = synth.AMOEBA_SETTINGS
    # whole steps, repeated until at least 10 s have been timed (at most 8)
    reps, dt = 0, 0.0
    while reps == 0 or (dt < 10.0 and reps < 8):
        t0 = time.perf_counter()
        rp7, cp7 = O.nblist(w.xyz, w.box, s["rc_ewald"] + s["skin"])
        rp9, cp9 = O.nblist(w.xyz, w.box, s["rc_vdw"] + s["skin"])
        em = O.empole_real(w.xyz, w.box, w.molid, rp7, cp7, w.mpole, s["beta"], s["rc_ewald"])
        mu, info = O.polarize_pcg(w.xyz, w.box, w.molid, rp7, cp7, w.mpole, w.polarity,
                                  w.thole, s["beta"], s["rc_ewald"], tol_debye=s["tol_debye"])
        ev = O.evdw(w.xyz, w.box, w.molid, rp9, cp9, 0, w.vdw_rad, w.vdw_eps, s["rc_vdw"])
        dt += time.perf_counter() - t0
        reps += 1
    n7 = count_pairs(w.xyz, w.box, rp7, cp7, s["rc_ewald"])
    n9 = count_pairs(w.xyz, w.box, rp9, cp9, s["rc_vdw"], w.molid, skip_same=True)
    mv = info["iters"] + 2
    pairs = n7 * (2 + mv) + n9
    base = {"value": pairs * reps / dt, "unit": "pair-interactions/s", "cores": 1,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{reps} full FP64 steps of the 23,559-atom water box (serial C oracle, "
                      f"{dt:.2f} s in all, {info['iters']} PCG iterations each)", "seconds": dt}
    # all cores: the machine's CPU share (at most 16 workers per GPU)
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    P = max(1, min(16, avail))
    b7, b9 = _block_rows(rp7, P), _block_rows(rp9, P)
    _blk.update(w=w, mu=mu, mv=mv,
                b7=[_sub_csr(rp7, cp7, b7[k], b7[k + 1]) for k in range(P)],
                b9=[_sub_csr(rp9, cp9, b9[k], b9[k + 1]) for k in range(P)])
    with mp.get_context("fork").Pool(P) as pool:
        pool.map(_blk_work, range(P))          # warm-up: workers load the oracle
        reps_all, dt_all = 0, 0.0              # repeated until at least 2 s (at most 16)
        while reps_all == 0 or (dt_all < 2.0 and reps_all < 16):
            t1 = time.perf_counter()
            parts = pool.map(_blk_work, range(P))
            dt_all += time.perf_counter() - t1
            reps_all += 1
    e_sum = float(np.sum(parts))
    base["all_cores"] = {
        "value": pairs * reps_all / dt_all, "unit": "pair-interactions/s", "cores": P,
        "host_cpus_visible": avail, "seconds": dt_all,
        "sample": f"the step's pair kernels (multipoles, permanent field, {mv} mat-vecs, HAL) "
                  f"split by CSR row blocks over {P} processes, {reps_all} times",
        "check_multipole_energy_rel": abs(e_sum - em[0][0]) / abs(em[0][0])}
    _blk.clear()
    # not timed: dipoles converged far below the tolerance, the reference that
    # the mixed form's dipole error is stated against
    tight, _ = O.polarize_pcg(w.xyz, w.box, w.molid, rp7, cp7, w.mpole, w.polarity, w.thole,
                              s["beta"], s["rc_ewald"], tol_debye=1e-10, maxiter=200)
    return base, (em, (mu, info), ev, tight), (n7, n9)


def copy_rate(ctx, mib=1024):
    """Achievable HBM rate: a device-to-device copy of `mib` MiB (bytes read +
    written per second, GB/s), best of 5."""
    import torch
    src = torch.ones(mib << 17, dtype=torch.float64, device=ctx.device)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = 0.0
    for _ in range(5):
        t0 = time.perf_counter()
        dst.copy_(src)
        torch.cuda.synchronize()
        best = max(best, 2 * src.numel() * 8 / (time.perf_counter() - t0) / 1e9)
    del src, dst
    return round(best, 1)


def accuracy(step, ref):
    """A timed step's outputs against the oracle's step on the same inputs:
    relative energy errors, force errors (max over RMS, and the RMS over atoms
    of |dF| in kcal/mol/A), dipoles against the oracle's step and against
    dipoles converged to 1e-10 D (max and RMS, Debye)."""
    (e_g, f_g, _), mu_g, (ev_g, fv_g, _) = step.out
    (e_o, f_o, _), (mu_o, info_o), (ev_o, fv_o, _), tight = ref
    debye = 4.80320

    def frel(g, o):
        return float(np.abs(g.cpu().numpy() - o).max() / np.sqrt(np.mean(o ** 2)))

    def rms(g, o):
        return float(np.sqrt(np.mean(np.sum((np.asarray(g) - o) ** 2, axis=1))))
    e = e_g.cpu().numpy()
    mu = mu_g.cpu().numpy()
    return {"empole_energy_rel": float(abs(e[0] - e_o[0]) / abs(e_o[0])),
            "empole_energy_parts_rel": [float(abs(e[k] - e_o[k]) / abs(e_o[0])) for k in (1, 2)],
            "empole_force_max_over_rms": frel(f_g, f_o),
            "empole_force_rms_err": rms(f_g.cpu().numpy(), f_o),
            "dipole_max_debye": float(debye * np.abs(mu - mu_o).max()),
            "dipole_rms_debye": debye * rms(mu, mu_o),
            "dipole_rms_debye_vs_converged": debye * rms(mu, tight),
            "dipole_rms_true_residual_debye": step.info["rms_true_debye"],
            "epol_rel": float(abs(step.info["epol"] - info_o["epol"]) / abs(info_o["epol"])),
            "pcg_iters_gpu_oracle": [step.info["iters"], info_o["iters"]],
            "pcg_refinements": step.info["refinements"],
            "hal_energy_rel": float(abs(float(ev_g.cpu()) - ev_o) / abs(ev_o)),
            "hal_force_max_over_rms": frel(fv_g, fv_o),
            "hal_force_rms_err": rms(fv_g.cpu().numpy(), fv_o)}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported "
              f"(the path runs on one GPU; its value is one GPU's throughput)",
              file=sys.stderr)
        sys.exit(2)
    w = synth.make("water7853")
    cpu = None
    if not a.no_cpu_baseline:   # before the GPU is touched: its workers are forked
        cpu = cpu_baseline(w)
    import torch
    from paper_1906_01211_amd import tk
    tk.load()
    ctx = tk.Context(0)
    if a.calibrate_copy > 0:
        src = torch.ones(a.calibrate_copy << 17, dtype=torch.float64, device=ctx.device)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    prec = tk.FP64 if a.prec == "fp64" else tk.MIXED
    # the synchronous step once: exact pair counts from its host-sized lists,
    # and the iteration count its solve takes (the count a stream-ordered
    # step carries from the previous step)
    ref_step = AmoebaStep(ctx, tk, w, prec)
    n7, n9 = ref_step.pair_counts()
    step = QueuedAmoebaStep(ctx, tk, w, prec, ref_step.info["iters"], serial=a.serial_step)
    step.l7_pairs, step.l9_pairs = ref_step.l7_pairs, ref_step.l9_pairs

    # timed region: the dominant kernel (the solver's per-cell mat-vec) is
    # timed by HIP events that the library records on its launch stream
    dom = "pcg_mv_fp64" if prec == tk.FP64 else "pcg_mv_fp32"
    ctx.profile(True, only=dom)   # clears the counters
    ctx.profile(False)
    sampler = EveryKth(ctx, step, dom, 10)
    ms = timed(sampler, a.steps, a.warmup) * 1e3
    dprof = ctx.profile_read()
    step.check()   # every timed step: both lists built, the solve converged
    # full kernel breakdown from a separate pass (not used for `value`), with
    # HAL after the solve on one stream, so that each kernel runs alone
    lone = QueuedAmoebaStep(ctx, tk, w, prec, ref_step.info["iters"], serial=True)
    ctx.profile(True)
    timed(lone, max(2, a.steps // 4), 0)
    prof = ctx.profile_read()
    ctx.profile(False)
    lone.check()
    # per-step wall times of a further pass (a synchronisation after each step)
    per = []
    for _ in range(max(20, a.steps)):
        t0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        per.append((time.perf_counter() - t0) * 1e3)
    q10, q50, q90 = np.percentile(per, [10, 50, 90])
    iters = step.check()["iters"]
    # the polarization solve alone (right-hand side, PCG to tolerance, FP64
    # true residual) on the step's 7 A list, FP64 and mixed
    sv = None if a.no_solve_rates else {}
    if not a.no_solve_rates:
        l7 = ctx.nblist(step.sys,
                        synth.AMOEBA_SETTINGS["rc_ewald"] + synth.AMOEBA_SETTINGS["skin"],
                        plan_slot=5)
    for name, pr in (() if a.no_solve_rates else (("fp64", tk.FP64), ("mixed", tk.MIXED))):
        s_ = synth.AMOEBA_SETTINGS
        solve_ms = timed(lambda: ctx.polarize_pcg(step.sys, l7, step.mpole, step.pol, step.thole,
                                                  s_["beta"], s_["rc_ewald"],
                                                  tol_debye=s_["tol_debye"],
                                                  maxiter=s_["maxiter"], prec=pr),
                         max(10, a.steps), 2) * 1e3
        sv[name] = round(1e3 / solve_ms, 1)
    mv_calls = iters + 2          # initial residual + iterations + final FP64 residual
    pairs = n7 * (1 + 1 + mv_calls) + n9   # empole + efield + mat-vecs + HAL
    value = pairs / (ms * 1e-3)

    roof = None
    if dom in dprof and dprof[dom]["launches"] > 0:
        launches = dprof[dom]["launches"]
        avg_ms = dprof[dom]["ms"] / launches
        # launches per solve: iterations 0..iters-1 each do one mat-vec (the
        # queued solve takes the last stopping test inside its FP64 residual
        # launch; the mixed form keeps a launch for it, timed but not counted
        # as work).  Timed solves: every tenth.
        solves = sampler.sampled
        working = iters * solves
        nl7 = int(step.l7_pairs)
        bpl = MV_BYTES_PER_PAIR[a.prec] * nl7 + MV_BYTES_PER_ATOM * w.n
        ach = bpl * working / (dprof[dom]["ms"] * 1e-3) / 1e9
        fl = MV_FLOPS_PER_PAIR * n7 * working / (dprof[dom]["ms"] * 1e-3) / 1e12
        peak_fl = PEAK_FP64_TFLOPS if prec == tk.FP64 else PEAK_FP32_TFLOPS
        roof = {"bound": "hbm", "kernel": "k_pcg_mv (solver mat-vec, iteration form)",
                "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": committed_traffic(a.prec),
                "bytes_per_launch": bpl, "launches": launches, "working_launches": working,
                "timed_steps": f"{solves} of {a.steps + a.warmup} (every tenth)",
                "avg_launch_us": round(avg_ms * 1e3, 3),
                "alu_tflops": round(fl, 3), "alu_frac": round(fl / peak_fl, 4),
                # what the counters say binds it (HBM is not saturated)
                "limiter": "LDS issue and latency: about a quarter VALU busy, a quarter of "
                           "LDS cycles bank-conflicted, a fifth of wave time waiting on LDS "
                           "(profiles/valu_counters_water7853.txt)"}
    out = {
        "metric": "real-space pair-interactions/s + polarization solves/s (mixed vs FP64); p99 lat",
        "value": value, "unit": "pair-interactions/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if prec == tk.FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "water box, 7,853 waters (23,559 atoms), 62.23 A, AMOEBA-style "
                               "multipoles + Thole polarization + HAL, rc 7/9 A",
                   "atoms": w.n, "pairs_7A": n7, "pairs_9A_hal": n9,
                   "pcg_iters": iters, "prec": a.prec,
                   "step": "stream-ordered: no host synchronisation inside a step; HAL "
                           + ("after the solve on one stream" if a.serial_step
                              else "on a second stream beside the solve")},
        "solves_per_s": 1e3 / ms,   # one solve per step
        "polarization_solves_per_s": sv,   # the solve alone
        "step_ms_p10_p50_p90": [round(q10, 4), round(q50, 4), round(q90, 4)],
        "kernel_ms_per_step": {k: round(v["ms"] / max(2, a.steps // 4), 5) for k, v in prof.items()},
        "roofline": roof,
    }
    # the VALU-bound pair kernels of the step: algorithmic FLOP rate (oracle
    # op counts x exact pair counts / HIP-event time) against the vector peak
    tag = "fp64" if prec == tk.FP64 else "fp32"
    pk = PEAK_FP64_TFLOPS if prec == tk.FP64 else PEAK_FP32_UNPACKED_TFLOPS
    out["valu_kernels"] = {
        "units_mpole_field_" + tag: valu_entry(prof, "units_mpole_field_" + tag,
                                               ("empole_real", "efield_direct"), n7,
                                               step.l7_pairs, pk),
        "units_vdw_" + tag: valu_entry(prof, "units_vdw_" + tag, ("evdw_hal",), n9,
                                       step.l9_pairs, pk),
        "units_tmat_fp64": valu_entry(prof, "units_tmat_fp64", ("tmatvec",), n7, step.l7_pairs,
                                      PEAK_FP64_TFLOPS),
    }
    other_step = None
    if not a.no_extras:
        out["extras"], other_step = extras(ctx, tk, w, a, prec, n7, iters)
    if not a.no_serving:
        out["serving"] = serving(tk, a.serving_requests)
    if roof is not None:
        roof["achievable_copy_gbs"] = copy_rate(ctx)
        roof["frac_of_achievable"] = round(roof["achieved"] / roof["achievable_copy_gbs"], 4)
    if cpu is not None:
        out["cpu_baseline"], ref, (n7o, n9o) = cpu
        assert (n7o, n9o) == (n7, n9), "GPU and oracle lists count different pairs"
        # the last timed-pass step's outputs, and those of the other precision's step
        acc = {a.prec: accuracy(step, ref)}
        if other_step is not None:
            acc["mixed" if a.prec == "fp64" else "fp64"] = accuracy(other_step, ref)
        out["accuracy_vs_oracle"] = acc
    ctx.close()
    print(json.dumps(out))


def extras(ctx, tk, w, a, prec, n7, iters):
    """Mixed-vs-FP64 step, the charge + LJ path, the polarization forces, the
    reciprocal-space PME, the local frames and the truncated CG (not part of
    `value`)."""
    import torch
    res = {}
    other = tk.MIXED if prec == tk.FP64 else tk.FP64
    ref_o = AmoebaStep(ctx, tk, w, other)
    ref_o()
    if ref_o.info["refinements"] == 0:   # the queued solve has no FP64 refinement
        st = QueuedAmoebaStep(ctx, tk, w, other, ref_o.info["iters"])
        res["other_step_form"] = "stream-ordered"
    else:
        st = ref_o
        res["other_step_form"] = "synchronous (its solve needed FP64 refinement)"
    ms = timed(st, max(3, a.steps // 2), 2) * 1e3
    if st is not ref_o:
        st.check()
    res["amoeba_step_ms_" + ("mixed" if other == tk.MIXED else "fp64")] = ms
    res["pcg_iters_other"] = st.info["iters"]
    # the synchronous step (lists sized through the host, the solve's
    # outcome read on the host) against the stream-ordered one, interleaved
    qs = QueuedAmoebaStep(ctx, tk, w, prec, iters)
    sync_step = AmoebaStep(ctx, tk, w, prec)
    qms, sms = [], []
    for _ in range(3):
        qms.append(timed(qs, max(10, a.steps), 2) * 1e3)
        qs.check()
        sms.append(timed(sync_step, max(10, a.steps), 2) * 1e3)
    res["sync_step"] = {"ms_runs": [round(x, 4) for x in sms],
                        "stream_ordered_ms_runs": [round(x, 4) for x in qms]}
    wc = synth.make("water32000_charge_lj")
    s = synth.CHARGE_SETTINGS
    sysr = ctx.system(wc.xyz, wc.box, wc.molid)
    q = torch.as_tensor(wc.charges, device=ctx.device)
    rad = torch.as_tensor(wc.vdw_rad, device=ctx.device)
    eps = torch.as_tensor(wc.vdw_eps, device=ctx.device)
    for name, pr in (("fp64", tk.FP64), ("mixed", tk.MIXED)):
        def cstep():
            l12 = ctx.nblist(sysr, s["rc_ewald"] + s["skin"], plan_slot=2)
            ctx.echarge_real(sysr, l12, q, s["beta"], s["rc_ewald"], prec=pr)
            ctx.evdw(sysr, l12, tk.VDW_LJ, rad, eps, s["rc_vdw"], s["taper_frac"], prec=pr)
            return l12
        l12 = cstep()
        ms = timed(cstep, 3, 1) * 1e3
        res[f"charge_lj_step_ms_{name}"] = ms
        res["charge_lj_pairs_12A"] = int(l12.npairs)
        res[f"charge_lj_pairs_per_s_{name}"] = 2 * l12.npairs / (ms * 1e-3)
    res["epolar"] = epolar_leg(ctx, tk, w, n7)
    res["pme"] = pme_leg(ctx, tk, w)
    res["frames"] = frames_leg(ctx, tk, w)
    res["tcg1"] = tcg_leg(ctx, tk, w)
    return res, st


def tcg_leg(ctx, tk, w):
    """One-step truncated CG on the water box: dipoles and energy, and with
    its forces (the total derivative), beside the converged PCG solve."""
    import torch
    s = synth.AMOEBA_SETTINGS
    dev = ctx.device
    sysw = ctx.system(w.xyz, w.box, w.molid)
    l7 = ctx.nblist(sysw, s["rc_ewald"] + s["skin"], plan_slot=3)
    mp = torch.as_tensor(w.mpole, device=dev)
    pol = torch.as_tensor(w.polarity, device=dev)
    th = torch.as_tensor(w.thole, device=dev)
    out = {}
    out["solve_ms"] = round(timed(lambda: ctx.polarize_tcg1(sysw, l7, mp, pol, th, s["beta"],
                                                            s["rc_ewald"], forces=False),
                                  20, 3) * 1e3, 4)
    out["solve_forces_ms"] = round(timed(lambda: ctx.polarize_tcg1(sysw, l7, mp, pol, th, s["beta"],
                                                                   s["rc_ewald"]), 20, 3) * 1e3, 4)
    out["pcg_ms"] = round(timed(lambda: ctx.polarize_pcg(sysw, l7, mp, pol, th, s["beta"],
                                                         s["rc_ewald"], tol_debye=s["tol_debye"],
                                                         maxiter=s["maxiter"]), 20, 3) * 1e3, 4)
    _, e, _ = ctx.polarize_tcg1(sysw, l7, mp, pol, th, s["beta"], s["rc_ewald"], forces=False)
    _, info = ctx.polarize_pcg(sysw, l7, mp, pol, th, s["beta"], s["rc_ewald"],
                               tol_debye=s["tol_debye"], maxiter=s["maxiter"])
    out["epol_tcg1"] = float(e.cpu()[0])
    out["epol_pcg"] = info["epol"]
    # both dipole sets in one solve (same-molecule factor 0.5 in the second
    # field), beside the one-set solve; per-launch times of the two mat-vecs
    def two():
        return ctx.polarize_pcg2(sysw, l7, mp, pol, th, s["beta"], s["rc_ewald"], 0.5,
                                 tol_debye=s["tol_debye"], maxiter=s["maxiter"])
    def one():
        return ctx.polarize_pcg(sysw, l7, mp, pol, th, s["beta"], s["rc_ewald"],
                                tol_debye=s["tol_debye"], maxiter=s["maxiter"])
    out["pcg2_ms"] = round(timed(two, 20, 3) * 1e3, 4)
    mu2, i2 = two()
    out["epolar2_ms"] = round(timed(lambda: ctx.epolar2_real(sysw, l7, mp, pol, th, mu2, s["beta"],
                                                             s["rc_ewald"], 0.5), 20, 3) * 1e3, 4)
    out["pcg2_iters"] = [i2[0]["iters"], i2[1]["iters"]]
    out["epol_pcg2"] = [i2[0]["epol"], i2[1]["epol"]]
    ctx.profile(True)
    for _ in range(5):
        two()
        one()
    prof = ctx.profile_read()
    ctx.profile(False)
    for k in ("pcg_mv_fp64", "pcg2_mv_fp64"):
        if k in prof:
            out[k + "_us"] = round(prof[k]["ms"] / prof[k]["launches"] * 1e3, 2)
    return out


def frames_leg(ctx, tk, w):
    """Local-frame multipoles on the water box: rotation, and the multipole
    energy and forces with the frame part, beside the lab-frame call."""
    import torch
    s = synth.AMOEBA_SETTINGS
    n_w = w.n // 3
    ft, fa = synth.water_frames(n_w)
    dev = ctx.device
    ft = torch.as_tensor(ft, device=dev)
    fa = torch.as_tensor(fa, device=dev)
    loc = torch.as_tensor(synth.water_local_multipoles(n_w, 7), device=dev)
    sysw = ctx.system(w.xyz, w.box, w.molid)
    l7 = ctx.nblist(sysw, s["rc_ewald"] + s["skin"], plan_slot=3)
    mg = ctx.rotate_mpole(sysw, ft, fa, loc)
    out = {"rotate_ms": round(timed(lambda: ctx.rotate_mpole(sysw, ft, fa, loc), 20, 3) * 1e3, 4)}
    out["empole_frames_ms"] = round(timed(lambda: ctx.empole_frames(sysw, l7, ft, fa, loc, s["beta"],
                                                                    s["rc_ewald"]), 20, 3) * 1e3, 4)
    out["empole_lab_ms"] = round(timed(lambda: ctx.empole_real(sysw, l7, mg, s["beta"],
                                                               s["rc_ewald"]), 20, 3) * 1e3, 4)
    # polarization forces at fixed dipoles, with the frame part
    mu = torch.as_tensor(np.random.default_rng(9).normal(0, 0.03, (w.n, 3)), device=dev)
    pol = torch.as_tensor(w.polarity, device=dev)
    th = torch.as_tensor(w.thole, device=dev)
    out["epolar_frames_ms"] = round(timed(lambda: ctx.epolar_frames(sysw, l7, ft, fa, loc, pol, th,
                                                                    mu, s["beta"], s["rc_ewald"]),
                                          20, 3) * 1e3, 4)
    return out


def pme_leg(ctx, tk, w, grid=64, order=5):
    """Reciprocal-space multipoles by smooth PME on the water box (64^3 mesh,
    order-5 splines): whole call and its three stages (spread, the five FFT
    passes with the convolution, gather + energy); and the induced-dipole
    solve with the full Ewald operator beside the real-space one."""
    import torch
    s = synth.AMOEBA_SETTINGS
    sysw = ctx.system(w.xyz, w.box, w.molid)
    mp = torch.as_tensor(w.mpole, device=ctx.device)

    def call():
        ctx.pme_mpole(sysw, mp, s["beta"], grid, order)
    ms = timed(call, 20, 3) * 1e3
    ctx.profile(True)
    timed(call, 20, 0)
    prof = ctx.profile_read()
    ctx.profile(False)
    out = {"grid": grid, "order": order, "atoms": w.n, "call_ms": round(ms, 4)}
    for k in ("pme_spread", "pme_fft", "pme_gather"):
        if k in prof:
            out[k + "_us"] = round(prof[k]["ms"] / prof[k]["launches"] * 1e3, 2)
    # the five FFT passes each read and write the complex mesh (the first reads
    # the 8-byte fixed-point mesh, the last writes the 8-byte real potential)
    kk = grid ** 3
    fft_bytes = kk * (8 + 16) + 3 * kk * 32 + kk * (16 + 8)
    if "pme_fft_us" in out:
        out["fft_bytes"] = fft_bytes
        out["fft_hbm_frac"] = round(fft_bytes / (out["pme_fft_us"] * 1e-6) / 1e9 / PEAK_HBM_GBS, 4)
    # induced dipoles with the full Ewald operator beside the real-space solve
    # (same list, tolerance and guess; the right-hand sides included)
    l7 = ctx.nblist(sysw, s["rc_ewald"] + s["skin"], plan_slot=3)
    pol = torch.as_tensor(w.polarity, device=ctx.device)
    th = torch.as_tensor(w.thole, device=ctx.device)
    info = {}

    def ewald():
        _, info["ewald"] = ctx.polarize_pcg_ewald(sysw, l7, mp, pol, th, s["beta"], s["rc_ewald"],
                                                  grid, order, tol_debye=s["tol_debye"],
                                                  maxiter=s["maxiter"])

    def real():
        _, info["real"] = ctx.polarize_pcg(sysw, l7, mp, pol, th, s["beta"], s["rc_ewald"],
                                           tol_debye=s["tol_debye"], maxiter=s["maxiter"])
    out["pcg_ewald_ms"] = round(timed(ewald, 10, 2) * 1e3, 4)
    out["pcg_ewald_iters"] = info["ewald"]["iters"]
    out["pcg_real_ms"] = round(timed(real, 10, 2) * 1e3, 4)
    out["pcg_real_iters"] = info["real"]["iters"]

    def ewald2():   # both dipole sets (same-molecule factor 0.5 in the second field)
        _, info["ewald2"] = ctx.polarize_pcg2_ewald(sysw, l7, mp, pol, th, s["beta"],
                                                    s["rc_ewald"], grid, 0.5, order=order,
                                                    tol_debye=s["tol_debye"], maxiter=s["maxiter"])
    out["pcg2_ewald_ms"] = round(timed(ewald2, 10, 2) * 1e3, 4)
    out["pcg2_ewald_iters"] = [i["iters"] for i in info["ewald2"]]
    # polarization forces with the full Ewald operator: one call (both PME
    # evaluations in one packed mesh pass) beside the three-call composition
    mu = torch.as_tensor(np.random.default_rng(12).normal(0, 0.03, (w.n, 3)), device=ctx.device)
    mpm = mp.clone()
    mpm[:, 1:4] += mu
    out["epolar_ewald_ms"] = round(timed(lambda: ctx.epolar_ewald(sysw, l7, mp, pol, th, mu,
                                                                  s["beta"], s["rc_ewald"], grid,
                                                                  order), 20, 3) * 1e3, 4)

    def composed():
        ctx.epolar_real(sysw, l7, mp, pol, th, mu, s["beta"], s["rc_ewald"])
        ctx.pme_mpole(sysw, mpm, s["beta"], grid, order, want_field=False)
        ctx.pme_mpole(sysw, mp, s["beta"], grid, order, want_field=False)
    out["epolar_ewald_composed_ms"] = round(timed(composed, 20, 3) * 1e3, 4)
    return out


def epolar_leg(ctx, tk, w, n7):
    """Polarization forces at the converged dipoles of the water box: one call
    (gather, pair kernel, reduction) and its pair kernel alone, FP64 and mixed."""
    import torch
    s = synth.AMOEBA_SETTINGS
    dev = ctx.device
    sysw = ctx.system(w.xyz, w.box, w.molid)
    l7 = ctx.nblist(sysw, s["rc_ewald"] + s["skin"], plan_slot=3)
    mp = torch.as_tensor(w.mpole, device=dev)
    pol = torch.as_tensor(w.polarity, device=dev)
    th = torch.as_tensor(w.thole, device=dev)
    out = {"pairs": n7}
    for name, pr, tag in (("fp64", tk.FP64, "fp64"), ("mixed", tk.MIXED, "fp32")):
        mu, _ = ctx.polarize_pcg(sysw, l7, mp, pol, th, s["beta"], s["rc_ewald"],
                                 tol_debye=s["tol_debye"], maxiter=s["maxiter"], prec=pr)

        def call():
            ctx.epolar_real(sysw, l7, mp, pol, th, mu, s["beta"], s["rc_ewald"], prec=pr)
        kname = "units_epolar_" + tag
        ctx.profile(True, only=kname)
        ms = timed(call, 20, 3) * 1e3
        kp = ctx.profile_read()
        ctx.profile(False)
        kus = kp[kname]["ms"] / kp[kname]["launches"] * 1e3
        out[f"call_ms_{name}"] = round(ms, 4)
        out[f"kernel_us_{name}"] = round(kus, 2)
        out[f"pairs_per_s_{name}"] = n7 / (kus * 1e-6)
        fl = algorithmic_flops(("epolar_real",), n7, l7.npairs)
        out[f"algorithmic_tflops_{name}"] = round(fl / (kus * 1e-6) / 1e12, 3)
        out[f"algorithmic_frac_{name}"] = round(fl / (kus * 1e-6) / 1e12 / PEAK_FP64_TFLOPS, 4)
    return out


_serving_systems = {}


def serving_systems(count):
    """The request stream's systems (log-uniform 300-30,000 atoms, water density)."""
    if count not in _serving_systems:
        reqs = synth.serving_requests(count)
        _serving_systems[count] = [synth.amoeba_water_box(r["n_w"], r["box"], r["seed"])
                                   for r in reqs]
    return _serving_systems[count]


def run_stream(srv, systems, arrivals=None):
    """Submit every system (all at once, or at the given offsets in seconds)
    and wait for all; returns latencies (ms), wall time (s) and batch count."""
    import threading
    ids = [None] * len(systems)
    err = []

    def feed():
        t0 = time.perf_counter()
        try:
            for k, w in enumerate(systems):
                if arrivals is not None:
                    dt = arrivals[k] - (time.perf_counter() - t0)
                    if dt > 0:
                        time.sleep(dt)
                ids[k] = srv.submit(w)
        except Exception as e:   # re-raised below, after the submitted requests are drained
            err.append(e)

    th = threading.Thread(target=feed)
    th.start()
    th.join()
    if err:
        for rid in ids:
            if rid is not None:
                while srv.poll(rid, arrays=False) is None:
                    time.sleep(2e-4)
        raise err[0]
    lat, first, last, batches = [], None, None, {}
    for rid in ids:
        while True:
            out = srv.poll(rid, arrays=False)
            if out is not None:
                break
            time.sleep(2e-4)
        t = out[1]
        lat.append((t["t_done"] - t["t_submit"]) * 1e-6)
        first = t["t_submit"] if first is None else min(first, t["t_submit"])
        last = t["t_done"] if last is None else max(last, t["t_done"])
        batches[t["batch_index"]] = (t["t_done"] - t["t_start"]) * 1e-9
        srv.release(rid)
    return np.array(lat), (last - first) * 1e-9, len(batches), sum(batches.values())


def serving(tk, count):
    """Serving form on the request stream: capacity (all requests queued at
    once) and p50/p99 latency under Poisson arrivals at 0.5, 0.8, 1.0 and 1.2
    times that capacity, for FP64 and mixed; a 1 GiB device budget; and the
    baseline of one request at a time (FP64) under the same arrivals."""
    systems = serving_systems(count)
    atoms = sum(w.n for w in systems)
    loads = (0.5, 0.8, 1.0, 1.2)
    out = {"requests": count, "atoms": atoms,
           "sizes": "log-uniform 300-30,000 atoms, water-box density, seeds 20000+k; Poisson "
                    "arrivals seed 1004"}

    def arrivals(rate):
        return [r["arrival"] for r in synth.serving_requests(count, rate=rate)]

    def one(prec, budget, max_batch, fracs, base=None, lanes=3):
        """fracs: offered loads as fractions of `base` req/s (default: this
        configuration's own capacity)."""
        srv = tk.Server(tk.step_params(synth.AMOEBA_SETTINGS, prec), budget, max_batch,
                        lanes=lanes)
        try:
            for _ in range(2):                          # warm-up: grows the device arena
                run_stream(srv, systems)
            lat, wall, nb, busy = run_stream(srv, systems)   # capacity: all queued at once
            res = {"capacity_req_s": count / wall, "atoms_per_s": atoms / wall, "batches": nb,
                   "busy_atoms_per_s": atoms / busy,
                   "closed_p50_ms": float(np.percentile(lat, 50)),
                   "closed_p99_ms": float(np.percentile(lat, 99))}
            ref = res["capacity_req_s"] if base is None else base
            for f in fracs:
                rate = f * ref
                lat, wall, nb, busy = run_stream(srv, systems, arrivals(rate))
                res[f"load_{f}"] = {"rate_req_s": rate, "p50_ms": float(np.percentile(lat, 50)),
                                    "p99_ms": float(np.percentile(lat, 99)),
                                    "throughput_req_s": count / wall, "batches": nb}
            st = srv.stats()
            res["server"] = {"lanes": st["lanes"], "batches_run": st["batches"],
                             "peak_device_MiB": round(st["peak_device_bytes"] / 2 ** 20, 1),
                             "budget_MiB": round(st["budget"] / 2 ** 20, 1),
                             "measured_bytes_per_atom": round(st["bytes_per_atom"], 1)}
            return res
        finally:
            srv.close()

    # "unconstrained": a 16 GiB device budget and at most 64 requests per
    # batch (a bound on the batch's scratch, so the warm-up passes grow the
    # arena to its final size before the timed passes)
    big, mb = 16 << 30, 64
    out["batch_limit"] = {"budget_GiB": 16, "max_requests": mb}

    def guarded(key, *args, **kw):
        try:
            out[key] = one(*args, **kw)
        except Exception as e:   # a failed configuration is reported, not fatal to the line
            out[key] = {"error": f"{type(e).__name__}: {e}"}

    guarded("fp64", tk.FP64, big, mb, loads)
    guarded("mixed", tk.MIXED, big, mb, loads)
    cap = out["fp64"].get("capacity_req_s")
    if cap:   # loads below are fractions of the unconstrained FP64 capacity
        # a tight budget: room for the largest request (30,000 atoms, about
        # 18 KB per atom measured) and little more
        guarded("fp64_budget_1GiB", tk.FP64, 1 << 30, mb, (0.5, 0.8), base=cap)
        # the baseline: one lane, one request per batch (one request at a time)
        guarded("fp64_one_at_a_time", tk.FP64, big, 1, (0.5, 1.0), base=cap, lanes=1)
    return out


if __name__ == "__main__":
    main()
