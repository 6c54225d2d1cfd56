// Induced dipoles by preconditioned conjugate gradient, resident on the device
// (the polarization solver of section "Hotspots": its mat-vec is the paper's
// largest hotspot and is called up to 12 times per step).
//
// All solver vectors live in the plan's sorted atom order.  One iteration is
// four kernels:
//   mat-vec tiles on p = z + beta p (formed while staging),
//   per-atom apply: p stored, q = A p, block partials of p.q,
//   update: gamma = p.q (every block sums the partials in the same order),
//           alpha = rho/gamma, x += alpha p, r -= alpha q, z = alpha_i r,
//           block partials of r.z and |z|^2,
//   finish (one block): beta, rho, RMS, convergence flag, iteration count,
//           mirrored into pinned host memory.
// No grid-wide fences (a device-scope fence writes back the L2 of every XCD);
// kernel boundaries order the reductions.  Every sum runs in a fixed order, so
// iterates are bitwise reproducible.  The host queues iterations in chunks and
// reads the mirrored state once per chunk; kernels queued after convergence
// return at once.
#include <cmath>

#include "terms.hpp"

namespace tk {
namespace {

constexpr int kBlk = 256;
constexpr int kChunk = 6;

struct PcgState {
  double rho, gamma, alpha, beta, zz, rms, rms_true, epol, tol;
  int32_t iters, done, npol, maxiter;
};
// done: 0 running, 1 converged, 2 iteration limit, 3 breakdown

__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = kBlk / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double fixed_sum(const double* part, int nblk, double* sh) {
  double v = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kBlk) v += part[b];
  return block_sum(v, sh);
}

// Solver state initialisation (one thread): keeps npol, resets the rest.
__global__ void k_pcg_init(PcgState* st, double tol, int maxiter) {
  const int npol = st->npol;
  PcgState s0 = {};
  s0.npol = npol;
  s0.tol = tol;
  s0.maxiter = maxiter;
  *st = s0;
}

// gather sorted-order per-atom data: alpha, x0 (guess or alpha * b); block
// counts of polarizable atoms into part (summed by k_pcg_count).
__global__ __launch_bounds__(kBlk) void k_pcg_setup(int n, const int32_t* __restrict__ perm,
                                                    const double* __restrict__ pol,
                                                    const double* __restrict__ guess,
                                                    const double* __restrict__ b,
                                                    double* __restrict__ alpha_s,
                                                    double* __restrict__ x, double* __restrict__ part) {
  __shared__ double sh[kBlk];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  double c = 0.0;
  if (s < n) {
    const int i = perm[s];
    const double a = pol[i];
    alpha_s[s] = a;
    c = a > 0.0 ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
      x[3 * s + k] = guess ? (a > 0.0 ? guess[3 * i + k] : 0.0) : a * b[3 * s + k];
  }
  const double tot = block_sum(c, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlk) void k_pcg_count(const double* __restrict__ part, int nblk,
                                                    PcgState* st) {
  __shared__ double sh[kBlk];
  const double t = fixed_sum(part, nblk, sh);
  if (threadIdx.x == 0) st->npol = (int)t;
}

// Per atom: (A v)_s = v_s/alpha_s - (field_s + c v_s) from the partial slots.
// mode 0: initial residual r = b - A x, z = alpha r, p = z; partials r.z, |z|^2.
// mode 1: v = previous direction; p = z + beta v is formed exactly as the
//         mat-vec staged it and stored; q = A p; partial p.q.
// mode 2: true residual of x: partials |alpha (b - A x)|^2 and x.b.
template <int kMode>
__global__ __launch_bounds__(kBlk) void k_pcg_apply(PlanView pv, const double* __restrict__ partial,
                                                    long pstride, double cself,
                                                    const double* __restrict__ alpha_s,
                                                    const double* v, const double* __restrict__ b,
                                                    double* __restrict__ q, double* __restrict__ r,
                                                    double* __restrict__ z, double* p,
                                                    double* __restrict__ part,
                                                    const PcgState* __restrict__ st) {
  __shared__ double sh[kBlk];
  if (kMode == 1 && st->done) return;
  const int s = blockIdx.x * kBlk + threadIdx.x;
  const int nblk = gridDim.x;
  double s0 = 0.0, s1 = 0.0;
  if (s < pv.n) {
    const int ns = pv.cell_nslot[pv.scell[s]];
    double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < kMaxSlots; ++k)   // unrolled: all slot loads in flight at once
      if (k < ns)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] += partial[((long)k * 3 + c) * pstride + s];
    const double a = alpha_s[s];
    const double bd = kMode == 1 ? st->beta : 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double vv = kMode == 1 ? fma(bd, v[3 * s + c], z[3 * s + c]) : v[3 * s + c];
      const double av = a > 0.0 ? vv / a - (acc[c] + cself * vv) : 0.0;   // (A v)_s
      if (kMode == 1) {
        p[3 * s + c] = vv;
        q[3 * s + c] = av;
        s0 += vv * av;
      } else {
        const double rr = a > 0.0 ? b[3 * s + c] - av : 0.0;
        const double zz = a * rr;
        if (kMode == 0) {
          r[3 * s + c] = rr;
          z[3 * s + c] = zz;
          p[3 * s + c] = zz;
          s0 += rr * zz;
          s1 += zz * zz;
        } else {
          s0 += zz * zz;
          s1 += vv * b[3 * s + c];
        }
      }
    }
  }
  const double t0 = block_sum(s0, sh), t1 = block_sum(s1, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = t0;
    part[nblk + blockIdx.x] = t1;
  }
}

// gamma from the apply partials (same order in every block), then the
// x, r, z update and partials of r.z and |z|^2.
__global__ __launch_bounds__(kBlk) void k_pcg_update(int n, const double* __restrict__ alpha_s,
                                                     const double* __restrict__ p,
                                                     const double* __restrict__ q,
                                                     double* __restrict__ x, double* __restrict__ r,
                                                     double* __restrict__ z,
                                                     const double* __restrict__ part_g,
                                                     double* __restrict__ part, PcgState* st) {
  __shared__ double sh[kBlk];
  if (st->done) return;
  const int nblk = gridDim.x;
  const double gam = fixed_sum(part_g, nblk, sh);
  if (!(gam > 0.0)) {   // p.Ap <= 0: not positive definite
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->gamma = gam;
      st->done = 3;
    }
    return;
  }
  const double al = st->rho / gam;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->gamma = gam;
    st->alpha = al;
  }
  const int s = blockIdx.x * kBlk + threadIdx.x;
  double s0 = 0.0, s1 = 0.0;
  if (s < n) {
    const double a = alpha_s[s];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int k = 3 * s + c;
      x[k] += al * p[k];
      const double rr = r[k] - al * q[k];
      r[k] = rr;
      const double zz = a * rr;
      z[k] = zz;
      s0 += rr * zz;
      s1 += zz * zz;
    }
  }
  const double t0 = block_sum(s0, sh), t1 = block_sum(s1, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = t0;
    part[nblk + blockIdx.x] = t1;
  }
}

// One block: finish a reduction and update the state; mirror it to the host.
// mode 0: after the initial residual; mode 1: after an update (beta, rho, RMS,
// iteration count, convergence); mode 2: after the true residual.
template <int kMode>
__global__ __launch_bounds__(kBlk) void k_pcg_finish(const double* __restrict__ part, int nblk,
                                                     PcgState* st, PcgState* host) {
  __shared__ double sh[kBlk];
  if (kMode == 1 && st->done) {
    if (threadIdx.x == 0) *host = *st;
    return;
  }
  const double S0 = fixed_sum(part, nblk, sh), S1 = fixed_sum(part + nblk, nblk, sh);
  if (threadIdx.x != 0) return;
  const double npol = st->npol > 0 ? (double)st->npol : 1.0;
  if (kMode == 0) {
    st->rho = S0;
    st->zz = S1;
    st->rms = kDebye * sqrt(S1 / npol);
    st->iters = 0;
    if (st->rms <= st->tol) st->done = 1;
    else if (st->maxiter == 0) st->done = 2;
  } else if (kMode == 1) {
    st->beta = S0 / st->rho;
    st->rho = S0;
    st->zz = S1;
    st->rms = kDebye * sqrt(S1 / npol);
    st->iters += 1;
    if (st->rms <= st->tol) st->done = 1;
    else if (st->iters >= st->maxiter) st->done = 2;
  } else {
    st->rms_true = kDebye * sqrt(S0 / npol);
    st->epol = -0.5 * kCoulomb * S1;
  }
  *host = *st;
}

__global__ void k_add_into(int n3, double* __restrict__ x, const double* __restrict__ d) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n3) x[k] += d[k];
}

__global__ void k_scatter_out(int n, const int32_t* __restrict__ perm, const double* __restrict__ x,
                              double* __restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int i = perm[s];
#pragma unroll
  for (int c = 0; c < 3; ++c) out[3 * i + c] = x[3 * s + c];
}

struct Solver {
  tk_ctx* ctx;
  hipStream_t st;
  const Plan* P;
  const tk_system* sys;
  const double* polarity;
  const double* thole;
  double beta, cutoff, cself;
  double *alpha_s, *b, *x, *r, *z, *p, *q, *part, *partg, *partial, *gathered;
  PcgState* state;
  PcgState* host;       // pinned host mirror
  PcgState* host_dev;   // its device address
  long pstride;
  int nblk;

  template <class R>
  TmatPh<R> tmat(const double* v, const int* done, bool dir) const {
    TmatPh<R> ph;
    ph.xyz = sys->xyz;
    ph.mu = v;
    ph.mu_sorted = 1;
    ph.polarity = polarity;
    ph.thole = thole;
    ph.molid = sys->molid;
    ph.g.set(sys->box, cutoff, beta);
    ph.done = done;
    ph.sorted = gathered;
    ph.gstride = pstride;
    ph.perm_ = (const int32_t*)P->perm.p;
    if (dir) {
      ph.zdir = z;
      ph.beta_dir = &state->beta;
    }
    return ph;
  }

  // static per-atom fields of the mat-vec, gathered once per solve
  void gather_geometry() {
    TmatPh<double> ph = tmat<double>(nullptr, nullptr, false);
    k_gather<TmatPh<double>><<<ceil_div(P->n, 256), 256, 0, st>>>(P->view(), ph, gathered, pstride);
  }

  template <class R>
  void matvec_units(const double* v, const int* done, bool dir = false) {
    TmatPh<R> ph = tmat<R>(v, done, dir);
    ProfScope ps(ctx, st, std::string("units_tmat") + TmatPh<R>::kTag);
    k_units<TmatPh<R>><<<P->nunits, 64, unit_lds_bytes<TmatPh<R>>(*P), st>>>(P->view(), ph, partial,
                                                                            pstride, nullptr);
  }

  tk_status sync_state() {
    TK_HIP(hipGetLastError());
    TK_HIP(hipStreamSynchronize(st));
    return TK_OK;
  }

  // PCG on A x = rhs, x holding the initial guess; leaves the result in x.
  template <class R>
  tk_status run(const double* rhs, double tol, int maxiter) {
    const int n = P->n;
    k_pcg_init<<<1, 1, 0, st>>>(state, tol, maxiter);
    matvec_units<R>(x, nullptr);
    k_pcg_apply<0><<<nblk, kBlk, 0, st>>>(P->view(), partial, pstride, cself, alpha_s, x, rhs, q, r,
                                          z, p, part, state);
    k_pcg_finish<0><<<1, kBlk, 0, st>>>(part, nblk, state, host_dev);
    int queued = 0;
    for (;;) {
      const int chunk = maxiter - queued < kChunk ? maxiter - queued : kChunk;
      for (int c = 0; c < chunk; ++c) {
        matvec_units<R>(p, &state->done, true);
        {
          ProfScope ps(ctx, st, "pcg_apply");
          k_pcg_apply<1><<<nblk, kBlk, 0, st>>>(P->view(), partial, pstride, cself, alpha_s, p,
                                                nullptr, q, nullptr, z, p, partg, state);
        }
        {
          ProfScope ps(ctx, st, "pcg_update");
          k_pcg_update<<<nblk, kBlk, 0, st>>>(n, alpha_s, p, q, x, r, z, partg, part, state);
        }
        k_pcg_finish<1><<<1, kBlk, 0, st>>>(part, nblk, state, host_dev);
      }
      queued += chunk;
      tk_status s = sync_state();
      if (s) return s;
      if (host->done || queued >= maxiter) break;
    }
    return TK_OK;
  }

  // FP64 residual of x against rhs: rms_true and epol (x.rhs) into the state.
  tk_status true_residual(const double* rhs) {
    matvec_units<double>(x, nullptr);
    k_pcg_apply<2><<<nblk, kBlk, 0, st>>>(P->view(), partial, pstride, cself, alpha_s, x, rhs,
                                          nullptr, nullptr, nullptr, nullptr, part, state);
    k_pcg_finish<2><<<1, kBlk, 0, st>>>(part, nblk, state, host_dev);
    return sync_state();
  }
};

}  // namespace
}  // namespace tk

using namespace tk;

extern "C" tk_status tk_polarize_pcg(tk_ctx* ctx, void* stream, const tk_system* sys,
                                     const tk_nblist* list, const double* mpole,
                                     const double* polarity, const double* thole,
                                     double ewald_beta, double cutoff, double tol_debye,
                                     int32_t maxiter, int prec, const double* mu_guess,
                                     double* mu_out, tk_pcg_info* info) {
  if (!ctx || !info) return TK_E_ARG;
  tk_status s = check_system(sys);
  if (s) return s;
  if (prec != TK_FP64 && prec != TK_MIXED) return TK_E_ARG;
  if (!(ewald_beta >= 0.0) || !std::isfinite(ewald_beta) || !(tol_debye >= 0.0) || maxiter < 0)
    return TK_E_ARG;
  const Plan* P;
  if ((s = get_plan(ctx, sys, list, cutoff, &P))) return s;
  *info = tk_pcg_info{};
  const int n = sys->n;
  if (n == 0) {
    info->converged = 1;
    return TK_OK;
  }
  if (!mpole || !polarity || !thole || !mu_out) return TK_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  Solver S;
  S.ctx = ctx;
  S.st = st;
  S.P = P;
  S.sys = sys;
  S.polarity = polarity;
  S.thole = thole;
  S.beta = ewald_beta;
  S.cutoff = cutoff;
  S.cself = 4.0 * ewald_beta * ewald_beta * ewald_beta / (3.0 * kSqrtPi);
  S.pstride = pad64(n);
  S.nblk = ceil_div(n, kBlk);
  const size_t v3 = sizeof(double) * 3 * (size_t)n;
  void *alpha_s, *b, *x, *r, *z, *p, *q, *part, *partg, *partial, *state, *dx, *rt, *gath;
  if ((s = scratch(ctx, "pcg_alpha", sizeof(double) * n, &alpha_s)) ||
      (s = scratch(ctx, "pcg_b", v3, &b)) || (s = scratch(ctx, "pcg_x", v3, &x)) ||
      (s = scratch(ctx, "pcg_r", v3, &r)) || (s = scratch(ctx, "pcg_z", v3, &z)) ||
      (s = scratch(ctx, "pcg_p", v3, &p)) || (s = scratch(ctx, "pcg_q", v3, &q)) ||
      (s = scratch(ctx, "pcg_dx", v3, &dx)) || (s = scratch(ctx, "pcg_rt", v3, &rt)) ||
      (s = scratch(ctx, "pcg_part", sizeof(double) * 2 * S.nblk, &part)) ||
      (s = scratch(ctx, "pcg_partg", sizeof(double) * 2 * S.nblk, &partg)) ||
      (s = scratch(ctx, "partial", sizeof(double) * kMaxSlots * 3 * S.pstride, &partial)) ||
      (s = scratch(ctx, "pcg_gathered", sizeof(double) * TmatPh<double>::NG * S.pstride, &gath)) ||
      (s = scratch(ctx, "pcg_state", sizeof(PcgState), &state)))
    return s;
  S.alpha_s = (double*)alpha_s; S.b = (double*)b; S.x = (double*)x; S.r = (double*)r;
  S.z = (double*)z; S.p = (double*)p; S.q = (double*)q; S.part = (double*)part;
  S.partg = (double*)partg; S.partial = (double*)partial; S.state = (PcgState*)state;
  S.gathered = (double*)gath;
  if (unit_lds_bytes<EfieldPh<double>>(*P) > kMaxLds) return TK_E_CAPACITY;
  void *hbase, *hdev;
  if ((s = pinned(ctx, 4096, &hbase, &hdev))) return s;
  S.host = (PcgState*)((char*)hbase + 1024);
  S.host_dev = (PcgState*)((char*)hdev + 1024);

  // right-hand side: permanent field (sorted order)
  s = prec == TK_FP64 ? launch_efield<double>(ctx, st, *P, sys, mpole, polarity, thole, ewald_beta,
                                              cutoff, S.b, 1)
                      : launch_efield<float>(ctx, st, *P, sys, mpole, polarity, thole, ewald_beta,
                                             cutoff, S.b, 1);
  if (s) return s;
  S.gather_geometry();
  k_pcg_setup<<<S.nblk, kBlk, 0, st>>>(n, (const int32_t*)P->perm.p, polarity, mu_guess, S.b,
                                        S.alpha_s, S.x, S.part);
  k_pcg_count<<<1, kBlk, 0, st>>>(S.part, S.nblk, S.state);
  s = prec == TK_FP64 ? S.run<double>(S.b, tol_debye, maxiter)
                      : S.run<float>(S.b, tol_debye, maxiter);
  if (s) return s;
  const int done = S.host->done;
  info->iters = S.host->iters;
  info->rms_debye = S.host->rms;
  info->converged = done == 1;
  info->status = done == 1 ? TK_OK : done == 3 ? TK_E_BREAKDOWN : TK_E_NOCONV;
  if ((s = S.true_residual(S.b))) return s;
  info->rms_true_debye = S.host->rms_true;
  info->epol = S.host->epol;
  if (prec == TK_MIXED && done != 3) {
    // FP64-residual refinement: solve A d = b - A x with the mixed solver, x += d.
    for (int ref = 0; ref < 3 && S.host->rms_true > tol_debye; ++ref) {
      // r_t = b - A x in FP64 (sorted); d0 = alpha r_t is left in z
      S.matvec_units<double>(S.x, nullptr);
      k_pcg_apply<0><<<S.nblk, kBlk, 0, st>>>(P->view(), S.partial, S.pstride, S.cself, S.alpha_s,
                                              S.x, S.b, S.q, (double*)rt, S.z, S.p, S.part, S.state);
      TK_HIP(hipMemcpyAsync(dx, x, v3, hipMemcpyDeviceToDevice, st));   // keep x
      TK_HIP(hipMemcpyAsync(x, S.z, v3, hipMemcpyDeviceToDevice, st));
      if ((s = S.run<float>((double*)rt, tol_debye, maxiter))) return s;
      info->iters += S.host->iters;
      info->refinements = ref + 1;
      k_add_into<<<ceil_div(3L * n, kBlk), kBlk, 0, st>>>(3 * n, (double*)dx, S.x);
      TK_HIP(hipMemcpyAsync(x, dx, v3, hipMemcpyDeviceToDevice, st));
      if ((s = S.true_residual(S.b))) return s;
      info->rms_true_debye = S.host->rms_true;
      info->epol = S.host->epol;
      if (S.host->rms_true <= tol_debye) {
        info->converged = 1;
        info->status = TK_OK;
      }
    }
  }
  k_scatter_out<<<ceil_div(n, kBlk), kBlk, 0, st>>>(n, (const int32_t*)P->perm.p, S.x, mu_out);
  TK_HIP(hipGetLastError());
  TK_HIP(hipStreamSynchronize(st));
  return info->status;
}
