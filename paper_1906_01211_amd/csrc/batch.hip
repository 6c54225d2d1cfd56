// One AMOEBA real-space step for a batch of independent systems: both
// neighbour lists, Halgren 14-7, and the permanent multipoles with the
// induced dipoles (one pass over the 7 A list gives the multipole terms and
// the solver's right-hand side), each as a single set of launches over all
// systems.
#include <cmath>
#include <cstring>
#include <vector>

#include "terms.hpp"

using namespace tk;

namespace {

tk_status check_params(const tk_step_params* p) {
  if (!p) return TK_E_ARG;
  const double v[] = {p->rc_ewald, p->rc_vdw, p->skin, p->ewald_beta, p->tol_debye,
                      p->taper_on_frac, p->hal_delta, p->hal_gamma};
  for (double x : v)
    if (!std::isfinite(x)) return TK_E_ARG;
  if (!(p->rc_ewald > 0.0) || !(p->rc_vdw > 0.0) || p->skin < 0.0 || p->ewald_beta < 0.0 ||
      p->tol_debye < 0.0 || p->taper_on_frac < 0.0 || p->taper_on_frac > 1.0 || p->maxiter < 0)
    return TK_E_ARG;
  if (p->prec != TK_FP64 && p->prec != TK_MIXED) return TK_E_ARG;
  return TK_OK;
}

// rc0: the first system's vdW cutoff (the functor's own geometry, used as
// is when the plan holds one system); sys_cut: every system's, per unit.
template <class R>
tk_status run_vdw(tk_ctx* ctx, hipStream_t st, const Plan& P, const tk_batch* b,
                  const double* rad, const double* eps, const tk_step_params* p, double rc0,
                  const double* sys_cut, double* force, double* energy, double* virial) {
  VdwPh<R> ph;
  const tk_system s1{P.n, b->xyz, b->box[0], b->molid};
  ph.set(&s1, TK_VDW_HAL, rad, eps, rc0, p->taper_on_frac, p->hal_delta, p->hal_gamma);
  ph.sys_cut = sys_cut;
  return run_term(ctx, st, P, ph, EpiForce{force}, energy, virial);
}

}  // namespace

extern "C" tk_status tk_batch_step(tk_ctx* ctx, void* stream, const tk_batch* b,
                                   const tk_step_params* p, const double* mpole,
                                   const double* polarity, const double* thole,
                                   const double* vdw_rad, const double* vdw_eps,
                                   const double* mu_guess, const int32_t* use_guess,
                                   double* force_mpole, double* mu, double* force_vdw,
                                   tk_step_result* res) {
  if (!ctx || !b || !res) return TK_E_ARG;
  tk_status s = check_params(p);
  if (s) return s;
  const int nsys = b->nsys;
  if (nsys < 1 || !b->atom_off || !b->box || b->atom_off[0] != 0) return TK_E_ARG;
  for (int k = 0; k < nsys; ++k)
    if (b->atom_off[k + 1] < b->atom_off[k] || !(b->box[k] > 0.0) || !std::isfinite(b->box[k]))
      return TK_E_ARG;
  const int n = b->atom_off[nsys];
  if (n > 0 && (!b->xyz || !b->molid || !mpole || !polarity || !thole || !vdw_rad || !vdw_eps ||
                !force_mpole || !mu || !force_vdw))
    return TK_E_ARG;
  // per-system cutoffs: Ewald fixed, vdW clamped to the box
  std::vector<double> c7(nsys), c9(nsys), r9(nsys);
  for (int k = 0; k < nsys; ++k) {
    c7[k] = p->rc_ewald + p->skin;
    if (c7[k] > 0.5 * b->box[k]) return TK_E_CUTOFF;
    r9[k] = std::fmin(p->rc_vdw, 0.5 * b->box[k] - p->skin);
    if (!(r9[k] > 0.0)) return TK_E_CUTOFF;
    c9[k] = r9[k] + p->skin;
  }
  hipStream_t st = (hipStream_t)stream;
  int64_t npairs[2] = {0, 0};
  const PlanSpec specs[2] = {{nsys, b->atom_off, b->box, c7.data()},
                             {nsys, b->atom_off, b->box, c9.data()}};
  const int slots[2] = {kBatchPlan7, kBatchPlan9};
  if ((s = build_plans(ctx, st, 2, slots, n, b->xyz, specs, npairs))) return s;
  const Plan& P7 = ctx->plans[kBatchPlan7];
  const Plan& P9 = ctx->plans[kBatchPlan9];
  // device outputs of the per-system scalars: e3 | w3 | e1 | w1, then vdW cutoffs
  const size_t nout = (size_t)nsys * (3 + 9 + 1 + 9);
  void *outd, *cutd, *gon = nullptr;
  if (mu_guess && use_guess) {
    if ((s = scratch(ctx, "batch_guess_on", sizeof(int32_t) * nsys, &gon))) return s;
    TK_HIP(hipMemcpyAsync(gon, use_guess, sizeof(int32_t) * nsys, hipMemcpyHostToDevice, st));
  }
  if ((s = scratch(ctx, "batch_out", sizeof(double) * nout, &outd)) ||
      (s = scratch(ctx, "batch_cut", sizeof(double) * nsys, &cutd)))
    return s;
  double* e3 = (double*)outd;
  double* w3 = e3 + 3 * nsys;
  double* e1 = w3 + 9 * nsys;
  double* w1 = e1 + nsys;
  TK_HIP(hipMemcpyAsync(cutd, r9.data(), sizeof(double) * nsys, hipMemcpyHostToDevice, st));
  if (n > 0) {
    if (unit_lds_bytes<EmpolePh<double>>(P7, 1) > kMaxLds ||
        unit_lds_bytes<VdwPh<double>>(P9, 1) > kMaxLds)
      return TK_E_CAPACITY;
    s = p->prec == TK_FP64 ? run_vdw<double>(ctx, st, P9, b, vdw_rad, vdw_eps, p, r9[0],
                                             (const double*)cutd, force_vdw, e1, w1)
                           : run_vdw<float>(ctx, st, P9, b, vdw_rad, vdw_eps, p, r9[0],
                                            (const double*)cutd, force_vdw, e1, w1);
    if (s) return s;
  } else {
    TK_HIP(hipMemsetAsync(outd, 0, sizeof(double) * nout, st));
  }
  std::vector<tk_pcg_info> info(nsys);
  if (n > 0) {
    // the multipole energies, forces and virial come out of the solver's
    // right-hand-side pass (one pass over the 7 A list for both)
    if ((s = solve_dipoles(ctx, st, &P7, b->xyz, b->molid, mpole, polarity, thole, p->ewald_beta,
                           p->rc_ewald, p->tol_debye, p->maxiter, p->prec, mu_guess,
                           (const int32_t*)gon, mu, info.data(), 0, 0, 1, 0.0, e3, force_mpole,
                           w3)))
      return s;
  } else {
    for (auto& i : info) i.converged = 1;
  }
  std::vector<double> out(nout);
  TK_HIP(hipMemcpyAsync(out.data(), outd, sizeof(double) * nout, hipMemcpyDeviceToHost, st));
  TK_HIP(hipStreamSynchronize(st));
  for (int k = 0; k < nsys; ++k) {
    tk_step_result& r = res[k];
    std::memcpy(r.e_mpole, out.data() + 3 * k, sizeof(r.e_mpole));
    std::memcpy(r.w_mpole, out.data() + 3 * nsys + 9 * k, sizeof(r.w_mpole));
    r.e_vdw = out[12 * nsys + k];
    std::memcpy(r.w_vdw, out.data() + 13 * nsys + 9 * k, sizeof(r.w_vdw));
    r.rc_vdw = r9[k];
    r.pcg = info[k];
  }
  return TK_OK;
}
