"""Mixed precision (FP32 pair arithmetic, FP64 accumulation and FP64 residual
refinement) against the FP64 CPU oracle, at the stated error budget:
energy relative error <= 1e-6, force RMS error <= 1e-4 kcal/mol/A, induced
dipoles within 1e-5 D RMS of a tightly converged FP64 solve."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1906_01211_amd import synth

pytestmark = pytest.mark.gpu

C, DEBYE = O.constants()
S = synth.AMOEBA_SETTINGS
_cache = {}


@pytest.fixture(scope="module")
def tk():
    import torch
    from paper_1906_01211_amd import tk as _tk
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _tk.load()
    return _tk


@pytest.fixture(scope="module")
def ctx(tk):
    c = tk.Context(0)
    yield c
    c.close()


def setup(ctx, name, rc_list, slot):
    w = _cache.setdefault(name, synth.make(name))
    sysr = ctx.system(w.xyz, w.box, w.molid)
    lst = ctx.nblist(sysr, rc_list, plan_slot=slot)
    key = (name, rc_list)
    if key not in _cache:
        _cache[key] = O.nblist(w.xyz, w.box, rc_list)
    rp, cp = _cache[key]
    return w, sysr, lst, rp, cp


def rms_err(a, b):
    return float(np.sqrt(np.mean(np.sum((np.asarray(a) - np.asarray(b)) ** 2, axis=1))))


@pytest.mark.parametrize("name", ["water216", "water7853"])
def test_empole_mixed(ctx, tk, name):
    w, sysr, lst, rp, cp = setup(ctx, name, 7.001, 2)
    e, f, vir = ctx.empole_real(sysr, lst, w.mpole, S["beta"], 7.0, prec=tk.MIXED)
    eo, fo, vo = O.empole_real(w.xyz, w.box, w.molid, rp, cp, w.mpole, S["beta"], 7.0)
    e = e.cpu().numpy()
    # the returned energy (total) within 1e-6; the split into intermolecular sum
    # and intramolecular corrections within 1e-6 of that energy
    assert abs(e[0] - eo[0]) <= 1e-6 * abs(eo[0]), (e[0], eo[0])
    for k in (1, 2):
        assert abs(e[k] - eo[k]) <= 1e-6 * abs(eo[0]), (k, e[k], eo[k])
    assert rms_err(f.cpu().numpy(), fo) <= 1e-4


def field_budget(polarity):
    # A field error dE moves a dipole by alpha dE.  The dipole budget is 1e-5 D
    # RMS; the field and the mat-vec must stay ten times inside it:
    # RMS|dE| * max(alpha) * 4.80320 D/(e A) <= 1e-6 D.
    return 1e-6 / (DEBYE * float(np.max(polarity)))


@pytest.mark.parametrize("name", ["water216", "water7853"])
def test_efield_mixed(ctx, tk, name):
    # the mixed permanent field (the solver's right-hand side) element by element
    w, sysr, lst, rp, cp = setup(ctx, name, 7.001, 2)
    fld = ctx.efield_direct(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0,
                            prec=tk.MIXED).cpu().numpy()
    fo = O.efield_direct(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole,
                         S["beta"], 7.0)
    assert rms_err(fld, fo) <= field_budget(w.polarity), rms_err(fld, fo)
    # and no single atom far outside it (FP32 rounding is spread, not concentrated)
    assert np.abs(fld - fo).max() <= 20 * field_budget(w.polarity)
    # it is the FP32 form: close to, but not bitwise, the FP64 one
    f64 = ctx.efield_direct(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0).cpu().numpy()
    assert not np.array_equal(fld, f64)


@pytest.mark.parametrize("name", ["water216", "water7853"])
@pytest.mark.parametrize("diag", [0, 1])
def test_tmatvec_mixed(ctx, tk, name, diag):
    w, sysr, lst, rp, cp = setup(ctx, name, 7.001, 2)
    mu = np.random.default_rng(11).normal(0, 0.05, size=(w.n, 3))
    out = ctx.tmatvec(sysr, lst, w.polarity, w.thole, S["beta"], 7.0, mu, include_diag=diag,
                      prec=tk.MIXED).cpu().numpy()
    oo = O.tmatvec(w.xyz, w.box, rp, cp, w.polarity, w.thole, S["beta"], 7.0, mu, diag)
    assert rms_err(out, oo) <= field_budget(w.polarity), rms_err(out, oo)
    assert np.abs(out - oo).max() <= 20 * field_budget(w.polarity)
    o64 = ctx.tmatvec(sysr, lst, w.polarity, w.thole, S["beta"], 7.0, mu,
                      include_diag=diag).cpu().numpy()
    assert not np.array_equal(out, o64)


@pytest.mark.parametrize("name", ["water216", "water7853"])
def test_pcg_mixed_dipoles(ctx, tk, name):
    w, sysr, lst, rp, cp = setup(ctx, name, 7.001, 2)
    mu, info = ctx.polarize_pcg(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0,
                                tol_debye=S["tol_debye"], prec=tk.MIXED)
    tight, io = O.polarize_pcg(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole,
                               S["beta"], 7.0, tol_debye=1e-10, maxiter=200)
    assert io["converged"] == 1
    assert info["converged"] == 1 and info["rms_true_debye"] <= S["tol_debye"]
    err_d = DEBYE * rms_err(mu.cpu().numpy(), tight)
    assert err_d <= 1e-5, err_d
    # E_pol = -1/2 C mu.E_perm is first order in the solver's truncation, so
    # its precision error is compared at a tolerance where truncation is small
    mu2, info2 = ctx.polarize_pcg(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0,
                                  tol_debye=1e-8, prec=tk.MIXED)
    assert abs(info2["epol"] - io["epol"]) <= 1e-6 * abs(io["epol"])


def test_pcg_mixed_refinement_triggers(ctx, tk):
    # a tolerance below what FP32 pair arithmetic resolves (the FP32 operator
    # differs from the FP64 one by ~1e-8 D in the residual) forces FP64 refinement
    w, sysr, lst, rp, cp = setup(ctx, "water216", 7.001, 2)
    mu, info = ctx.polarize_pcg(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0,
                                tol_debye=1e-10, maxiter=100, prec=tk.MIXED)
    assert info["refinements"] >= 1
    tight, _ = O.polarize_pcg(w.xyz, w.box, w.molid, rp, cp, w.mpole, w.polarity, w.thole,
                              S["beta"], 7.0, tol_debye=1e-11, maxiter=300)
    assert DEBYE * rms_err(mu.cpu().numpy(), tight) <= 1e-6


@pytest.mark.parametrize("form", [0, 1])
def test_evdw_mixed(ctx, tk, form):
    w, sysr, lst, rp, cp = setup(ctx, "water7853", 9.001, 3)
    rad = w.vdw_rad if form == 0 else np.where(np.arange(w.n) % 3 == 0, 3.15, 1.2)
    e, f, _ = ctx.evdw(sysr, lst, form, rad, w.vdw_eps, 9.0, prec=tk.MIXED)
    eo, fo, _ = O.evdw(w.xyz, w.box, w.molid, rp, cp, form, rad, w.vdw_eps, 9.0)
    assert abs(float(e) - eo) <= 1e-6 * abs(eo)
    assert rms_err(f.cpu().numpy(), fo) <= 1e-4


def test_charge_lj_mixed(ctx, tk):
    w = synth.charge_lj_water_box(4000, 49.4, 91)
    sysr = ctx.system(w.xyz, w.box, w.molid)
    lst = ctx.nblist(sysr, 12.001, plan_slot=4)
    rp, cp = O.nblist(w.xyz, w.box, 12.001)
    e, f, _ = ctx.echarge_real(sysr, lst, w.charges, 0.34, 12.0, prec=tk.MIXED)
    eo, fo, _ = O.echarge_real(w.xyz, w.box, w.molid, rp, cp, w.charges, 0.34, 12.0)
    e = e.cpu().numpy()
    for k in range(3):
        assert abs(e[k] - eo[k]) <= 1e-6 * abs(eo[k])
    assert rms_err(f.cpu().numpy(), fo) <= 1e-4
    e2, f2, _ = ctx.evdw(sysr, lst, 1, w.vdw_rad, w.vdw_eps, 12.0, prec=tk.MIXED)
    eo2, fo2, _ = O.evdw(w.xyz, w.box, w.molid, rp, cp, 1, w.vdw_rad, w.vdw_eps, 12.0)
    assert abs(float(e2) - eo2) <= 1e-6 * abs(eo2)
    assert rms_err(f2.cpu().numpy(), fo2) <= 1e-4


def test_pcg_mixed_reports_failed_check(ctx, tk):
    # one iteration per solve cannot reach 1e-5 D even with three refinement
    # rounds (the FP64 solve needs 7): the outcome must say so, from the FP64
    # residual, not from the FP32 recurrence
    w, sysr, lst, rp, cp = setup(ctx, "water216", 7.001, 2)
    mu, info = ctx.polarize_pcg(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0,
                                tol_debye=S["tol_debye"], maxiter=1, prec=tk.MIXED)
    assert info["refinements"] == 3
    assert info["rms_true_debye"] > S["tol_debye"]
    assert info["converged"] == 0 and info["status"] == tk.E_NOCONV
    # the same call with room to converge reports success from the same check
    mu, info = ctx.polarize_pcg(sysr, lst, w.mpole, w.polarity, w.thole, S["beta"], 7.0,
                                tol_debye=S["tol_debye"], maxiter=100, prec=tk.MIXED)
    assert info["converged"] == 1 and info["status"] == tk.OK
    assert info["rms_true_debye"] <= S["tol_debye"]
