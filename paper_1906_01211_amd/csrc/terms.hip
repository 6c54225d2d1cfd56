// Pair terms on the cell-pair tile skeleton: permanent multipoles (energy,
// forces, virial), point charges, permanent field, induced-dipole field
// mat-vec, Halgren 14-7 / LJ 12-6 van der Waals; their C-ABI entry points.
#include <cmath>

#include "pairs.hpp"
#include "terms.hpp"

namespace tk {

namespace {

}  // namespace

namespace {

tk_status common_args(tk_ctx* ctx, const tk_system* sys, const tk_nblist* list, double cutoff,
                      int prec, const Plan** plan) {
  if (!ctx) return TK_E_ARG;
  tk_status s = check_system(sys);
  if (s) return s;
  if (prec != TK_FP64 && prec != TK_MIXED) return TK_E_ARG;
  if (!std::isfinite(cutoff)) return TK_E_ARG;
  return get_plan(ctx, sys, list, cutoff, plan);
}

}  // namespace

template <class R>
tk_status launch_tmat(tk_ctx* ctx, hipStream_t st, const Plan& P, const tk_system* sys,
                      const double* polarity, const double* thole, double beta, double cutoff,
                      int include_diag, const double* mu, double* out, const TermWs* ws) {
  TmatPh<R> ph;
  ph.xyz = sys->xyz;
  ph.mu = mu;
  ph.mu_sorted = 0;
  ph.polarity = polarity;
  ph.thole = thole;
  ph.g.set(sys->box, cutoff, beta);
  ph.molid = sys->molid;
  ph.perm_ = (const int32_t*)P.perm.p;
  EpiMutual epi{out, mu, polarity, ph.g.cself, include_diag};
  return run_term(ctx, st, P, ph, epi, nullptr, nullptr, ws);
}

size_t tmatvec_ws_doubles(const Plan& P) { return term_ws_doubles<TmatPh<double>>(P); }
size_t tmatvec_ws_doubles_n(long n) {
  return (size_t)pad64(n) * (kMaxSlots * TmatPh<double>::NA + TmatPh<double>::NG);
}
static_assert(TmatPh<double>::NA == TmatPh<float>::NA && TmatPh<double>::NG == TmatPh<float>::NG,
              "both precisions take the same buffers");

tk_status tmatvec_checked(tk_ctx* ctx, hipStream_t st, const tk_system* sys,
                          const tk_nblist* list, const double* polarity, const double* thole,
                          double ewald_beta, double cutoff, int include_diag, int prec,
                          const double* mu, double* out, const TermWs* ws,
                          size_t ws_limit_doubles) {
  const Plan* P;
  tk_status s = common_args(ctx, sys, list, cutoff, prec, &P);
  if (s) return s;
  if (!(ewald_beta >= 0.0) || !std::isfinite(ewald_beta)) return TK_E_ARG;
  if (include_diag != 0 && include_diag != 1) return TK_E_ARG;
  if (sys->n == 0) return TK_OK;
  if (!polarity || !thole || !mu || !out) return TK_E_ARG;
  if (ws && tmatvec_ws_doubles(*P) > ws_limit_doubles) return TK_E_TOOBIG;
  return prec == TK_FP64 ? launch_tmat<double>(ctx, st, *P, sys, polarity, thole, ewald_beta,
                                               cutoff, include_diag, mu, out, ws)
                         : launch_tmat<float>(ctx, st, *P, sys, polarity, thole, ewald_beta,
                                              cutoff, include_diag, mu, out, ws);
}


}  // namespace tk

using namespace tk;

namespace tk {
namespace {
// M + (0, mu, 0): the permanent multipoles with the induced dipoles added
__global__ void k_mpole_plus_dipoles(int n, const double* __restrict__ mpole,
                                     const double* __restrict__ mu, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int c = 0; c < 10; ++c) out[10 * i + c] = mpole[10 * i + c];
#pragma unroll
  for (int c = 0; c < 3; ++c) out[10 * i + 1 + c] += mu[3 * i + c];
}

// force += F_pme(M + mu) - F_pme(M); energy = {real + recip, real, recip}
__global__ void k_epolar_ewald_sum(int n, const double* __restrict__ fa,
                                   const double* __restrict__ fb, const double* __restrict__ er,
                                   const double* __restrict__ ek, double* __restrict__ force,
                                   double* __restrict__ energy) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    const double rec = ek[0] - ek[1];
    energy[0] = er[0] + rec;
    energy[1] = er[0];
    energy[2] = rec;
  }
  if (i >= n) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) force[3 * i + c] += fa[3 * i + c] - fb[3 * i + c];
}
}  // namespace
}  // namespace tk

extern "C" {

tk_status tk_empole_real(tk_ctx* ctx, void* stream, const tk_system* sys, const tk_nblist* list,
                         const double* mpole, double ewald_beta, double cutoff, int prec,
                         double* energy, double* force, double* virial) {
  const Plan* P;
  tk_status s = common_args(ctx, sys, list, cutoff, prec, &P);
  if (s) return s;
  if (!(ewald_beta >= 0.0) || !std::isfinite(ewald_beta) || !energy || !virial) return TK_E_ARG;
  if (sys->n > 0 && (!mpole || !force)) return TK_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  if (sys->n == 0) {
    TK_HIP(hipMemsetAsync(energy, 0, 3 * sizeof(double), st));
    TK_HIP(hipMemsetAsync(virial, 0, 9 * sizeof(double), st));
    return TK_OK;
  }
  if (prec == TK_FP64) {
    EmpolePh<double> ph;
    ph.xyz = sys->xyz; ph.mpole = mpole; ph.molid = sys->molid;
    ph.g.set(sys->box, cutoff, ewald_beta);
    s = run_term(ctx, st, *P, ph, EpiForce{force}, energy, virial);
  } else {
    EmpolePh<float> ph;
    ph.xyz = sys->xyz; ph.mpole = mpole; ph.molid = sys->molid;
    ph.g.set(sys->box, cutoff, ewald_beta);
    s = run_term(ctx, st, *P, ph, EpiForce{force}, energy, virial);
  }
  return s;
}

tk_status tk_echarge_real(tk_ctx* ctx, void* stream, const tk_system* sys, const tk_nblist* list,
                          const double* q, double ewald_beta, double cutoff, int prec,
                          double* energy, double* force, double* virial) {
  const Plan* P;
  tk_status s = common_args(ctx, sys, list, cutoff, prec, &P);
  if (s) return s;
  if (!(ewald_beta >= 0.0) || !std::isfinite(ewald_beta) || !energy || !virial) return TK_E_ARG;
  if (sys->n > 0 && (!q || !force)) return TK_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  if (sys->n == 0) {
    TK_HIP(hipMemsetAsync(energy, 0, 3 * sizeof(double), st));
    TK_HIP(hipMemsetAsync(virial, 0, 9 * sizeof(double), st));
    return TK_OK;
  }
  if (prec == TK_FP64) {
    ChargePh<double> ph;
    ph.xyz = sys->xyz; ph.q = q; ph.molid = sys->molid;
    ph.g.set(sys->box, cutoff, ewald_beta);
    s = run_term(ctx, st, *P, ph, EpiForce{force}, energy, virial);
  } else {
    ChargePh<float> ph;
    ph.xyz = sys->xyz; ph.q = q; ph.molid = sys->molid;
    ph.g.set(sys->box, cutoff, ewald_beta);
    s = run_term(ctx, st, *P, ph, EpiForce{force}, energy, virial);
  }
  return s;
}

tk_status tk_efield_direct(tk_ctx* ctx, void* stream, const tk_system* sys, const tk_nblist* list,
                           const double* mpole, const double* polarity, const double* thole,
                           double ewald_beta, double cutoff, int prec, double* field) {
  const Plan* P;
  tk_status s = common_args(ctx, sys, list, cutoff, prec, &P);
  if (s) return s;
  if (!(ewald_beta >= 0.0) || !std::isfinite(ewald_beta)) return TK_E_ARG;
  if (sys->n == 0) return TK_OK;
  if (!mpole || !polarity || !thole || !field) return TK_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  return prec == TK_FP64
             ? launch_efield<double>(ctx, st, *P, sys, mpole, polarity, thole, ewald_beta, cutoff,
                                     field, 0)
             : launch_efield<float>(ctx, st, *P, sys, mpole, polarity, thole, ewald_beta, cutoff,
                                    field, 0);
}

tk_status tk_tmatvec(tk_ctx* ctx, void* stream, const tk_system* sys, const tk_nblist* list,
                     const double* polarity, const double* thole, double ewald_beta,
                     double cutoff, int include_diag, int prec, const double* mu, double* out) {
  return tmatvec_checked(ctx, (hipStream_t)stream, sys, list, polarity, thole, ewald_beta, cutoff,
                         include_diag, prec, mu, out, nullptr, 0);
}

tk_status tk_epolar_real(tk_ctx* ctx, void* stream, const tk_system* sys, const tk_nblist* list,
                         const double* mpole, const double* polarity, const double* thole,
                         const double* mu, double ewald_beta, double cutoff, int prec,
                         double* energy, double* force, double* virial) {
  const Plan* P;
  tk_status s = common_args(ctx, sys, list, cutoff, prec, &P);
  if (s) return s;
  if (!(ewald_beta >= 0.0) || !std::isfinite(ewald_beta) || !energy || !virial) return TK_E_ARG;
  if (sys->n > 0 && (!mpole || !polarity || !thole || !mu || !force)) return TK_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  if (sys->n == 0) {
    TK_HIP(hipMemsetAsync(energy, 0, 3 * sizeof(double), st));
    TK_HIP(hipMemsetAsync(virial, 0, 9 * sizeof(double), st));
    return TK_OK;
  }
  auto run = [&](auto ph) {
    ph.xyz = sys->xyz;
    ph.mpole = mpole;
    ph.molid = sys->molid;
    ph.polarity = polarity;
    ph.thole = thole;
    ph.mu = mu;
    ph.g.set(sys->box, cutoff, ewald_beta);
    return run_term(ctx, st, *P, ph, EpiForce{force}, energy, virial);
  };
  return prec == TK_FP64 ? run(EpolarPh<double>{}) : run(EpolarPh<float>{});
}

tk_status tk_epolar2_real(tk_ctx* ctx, void* stream, const tk_system* sys, const tk_nblist* list,
                          const double* mpole, const double* polarity, const double* thole,
                          const double* mu2, double ewald_beta, double cutoff, double pscale,
                          double* energy, double* force, double* virial) {
  const Plan* P;
  tk_status s = common_args(ctx, sys, list, cutoff, TK_FP64, &P);
  if (s) return s;
  if (!(ewald_beta >= 0.0) || !std::isfinite(ewald_beta) || !(pscale >= 0.0 && pscale <= 1.0) ||
      !energy || !virial)
    return TK_E_ARG;
  if (sys->n > 0 && (!mpole || !polarity || !thole || !mu2 || !force)) return TK_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  if (sys->n == 0) {
    TK_HIP(hipMemsetAsync(energy, 0, 3 * sizeof(double), st));
    TK_HIP(hipMemsetAsync(virial, 0, 9 * sizeof(double), st));
    return TK_OK;
  }
  Epolar2Ph ph;
  ph.xyz = sys->xyz;
  ph.mpole = mpole;
  ph.molid = sys->molid;
  ph.polarity = polarity;
  ph.thole = thole;
  ph.mu2 = mu2;
  ph.n2 = 3L * sys->n;
  ph.pscale = pscale;
  ph.g.set(sys->box, cutoff, ewald_beta);
  return run_term(ctx, st, *P, ph, EpiForce{force}, energy, virial);
}

tk_status tk_epolar_ewald(tk_ctx* ctx, void* stream, const tk_system* sys,
                          const tk_nblist* list, const double* mpole, const double* polarity,
                          const double* thole, const double* mu, double ewald_beta, double cutoff,
                          int32_t grid, int32_t order, double* energy, double* force) {
  const Plan* P;
  tk_status s = common_args(ctx, sys, list, cutoff, TK_FP64, &P);
  if (s) return s;
  if (!(ewald_beta > 0.0) || !std::isfinite(ewald_beta) || !pme_args_ok(grid, order) || !energy)
    return TK_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int n = sys->n;
  if (n == 0) {
    TK_HIP(hipMemsetAsync(energy, 0, 3 * sizeof(double), st));
    return TK_OK;
  }
  if (!mpole || !polarity || !thole || !mu || !force) return TK_E_ARG;
  void* buf;   // real-space energies [3] and virial [9], PME energies [2], M + mu, PME forces [2]
  const size_t nn = (size_t)n;
  if ((s = scratch(ctx, per_stream("epolar_ewald", st).c_str(),
                   sizeof(double) * (16 + 10 * nn + 6 * nn), &buf)))
    return s;
  double* er = (double*)buf;
  double* vir = er + 3;
  double* ek = vir + 9;        // [2]: E_pme(M + mu), E_pme(M)
  double* msum = ek + 4;       // padded to 16 doubles
  double* fk = msum + 10 * nn; // [2][n][3]
  EpolarPh<double> ph;
  ph.xyz = sys->xyz;
  ph.mpole = mpole;
  ph.molid = sys->molid;
  ph.polarity = polarity;
  ph.thole = thole;
  ph.mu = mu;
  ph.g.set(sys->box, cutoff, ewald_beta);
  if ((s = run_term(ctx, st, *P, ph, EpiForce{force}, er, vir))) return s;
  k_mpole_plus_dipoles<<<ceil_div(n, 256), 256, 0, st>>>(n, mpole, mu, msum);
  if ((s = pme_mpole_pair(ctx, st, sys, msum, mpole, ewald_beta, grid, order, ek, fk, ek + 1,
                          fk + 3 * nn)))
    return s;
  k_epolar_ewald_sum<<<ceil_div(n, 256), 256, 0, st>>>(n, fk, fk + 3 * nn, er, ek, force, energy);
  TK_HIP(hipGetLastError());
  return TK_OK;
}

tk_status tk_evdw(tk_ctx* ctx, void* stream, const tk_system* sys, const tk_nblist* list,
                  int form, const double* radius_or_sigma, const double* eps, double cutoff,
                  double taper_on_frac, double hal_delta, double hal_gamma, int prec,
                  double* energy, double* force, double* virial) {
  const Plan* P;
  tk_status s = common_args(ctx, sys, list, cutoff, prec, &P);
  if (s) return s;
  if (form != TK_VDW_HAL && form != TK_VDW_LJ) return TK_E_ARG;
  if (!(taper_on_frac >= 0.0 && taper_on_frac <= 1.0) || !std::isfinite(hal_delta) ||
      !std::isfinite(hal_gamma) || !energy || !virial)
    return TK_E_ARG;
  if (sys->n > 0 && (!radius_or_sigma || !eps || !force)) return TK_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  if (sys->n == 0) {
    TK_HIP(hipMemsetAsync(energy, 0, sizeof(double), st));
    TK_HIP(hipMemsetAsync(virial, 0, 9 * sizeof(double), st));
    return TK_OK;
  }
  auto run = [&](auto ph) {
    ph.set(sys, form, radius_or_sigma, eps, cutoff, taper_on_frac, hal_delta, hal_gamma);
    return run_term(ctx, st, *P, ph, EpiForce{force}, energy, virial);
  };
  if (form == TK_VDW_HAL)
    return prec == TK_FP64 ? run(VdwPh<double>{}) : run(VdwPh<float>{});
  return prec == TK_FP64 ? run(VdwLjPh<double>{}) : run(VdwLjPh<float>{});
}

}  // extern "C"
