// Induced dipoles by preconditioned conjugate gradient, resident on the device
// (the polarization solver of section "Hotspots": its mat-vec is the paper's
// largest hotspot and is called up to 12 times per step).
//
// All solver vectors live in the plan's sorted atom order.  One iteration is
// four kernels: the mutual-field mat-vec on the tile skeleton, a per-atom
// reduce that forms q = A p and p.q, the x/r/z update with r.z and |z|^2, and
// p = z + beta p.  Scalars (rho, gamma, alpha, beta, the convergence flag) stay
// on the device; each reduction is finished by the last block to arrive, in a
// fixed order, so the iterates are bitwise reproducible.  The host queues
// iterations in chunks and reads the flag once per chunk; kernels queued after
// convergence return at once.
#include <cmath>

#include "terms.hpp"

namespace tk {
namespace {

constexpr int kBlk = 256;
constexpr int kChunk = 6;

struct PcgState {
  double rho, gamma, alpha, beta, zz, rms, rms_true, epol, tol;
  int32_t iters, done, npol, maxiter, ticket, status, pad0, pad1;
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

// Returns true in the one thread of the last block to finish; the block
// partial `v` (per block) has been stored to part[k * nblk + blockIdx.x].
__device__ __forceinline__ bool last_block(PcgState* st) {
  __shared__ int is_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) is_last = atomicAdd(&st->ticket, 1) == (int)gridDim.x - 1;
  __syncthreads();
  return is_last;
}

__device__ __forceinline__ double fixed_sum(double* part, int nblk, double* sh) {
  double v = 0.0;   // other blocks' partials: device-scope loads, not the local cache
  for (int b = threadIdx.x; b < nblk; b += kBlk)
    v += __hip_atomic_load(&part[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return block_sum(v, sh);
}

// gather sorted-order per-atom data: alpha, and x0 (guess or alpha * b)
__global__ void k_pcg_setup(int n, const int32_t* __restrict__ perm, const double* __restrict__ pol,
                            const double* __restrict__ guess, const double* __restrict__ b,
                            double* __restrict__ alpha_s, double* __restrict__ x) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  int i = perm[s];
  double a = pol[i];
  alpha_s[s] = a;
#pragma unroll
  for (int c = 0; c < 3; ++c)
    x[3 * s + c] = guess ? (a > 0.0 ? guess[3 * i + c] : 0.0) : a * b[3 * s + c];
}

// mode 0: initial residual r = b - A x, z = alpha r, p = z; sums rho = r.z, zz.
// mode 1: q = A p and gamma = p.q; last block forms alpha or flags breakdown.
// mode 2: true residual from A x: zz of alpha (b - A x) and epol sum x.b.
template <int kMode>
__global__ __launch_bounds__(kBlk) void k_pcg_apply(PlanView pv, const double* __restrict__ partial,
                                                    long pstride, double cself,
                                                    const double* __restrict__ alpha_s,
                                                    const double* __restrict__ v,   // x or p
                                                    const double* __restrict__ b,
                                                    double* __restrict__ q, double* __restrict__ r,
                                                    double* __restrict__ z, double* __restrict__ p,
                                                    double* __restrict__ part, PcgState* st) {
  __shared__ double sh[kBlk];
  if (kMode == 1 && st->done) return;
  const int s = blockIdx.x * kBlk + threadIdx.x;
  const int nblk = gridDim.x;
  double s0 = 0.0, s1 = 0.0;
  if (s < pv.n) {
    const int ns = pv.cell_nslot[pv.scell[s]];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < ns; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c] += partial[((long)k * 3 + c) * pstride + s];
    const double a = alpha_s[s];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double vv = v[3 * s + c];
      const double av = a > 0.0 ? vv / a - (acc[c] + cself * vv) : 0.0;   // (A v)_s
      if (kMode == 1) {
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
  double t0 = block_sum(s0, sh), t1 = block_sum(s1, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = t0;
    part[nblk + blockIdx.x] = t1;
  }
  if (!last_block(st)) return;
  const double S0 = fixed_sum(part, nblk, sh), S1 = fixed_sum(part + nblk, nblk, sh);
  if (threadIdx.x != 0) return;
  st->ticket = 0;
  const double npol = st->npol > 0 ? (double)st->npol : 1.0;
  if (kMode == 0) {
    st->rho = S0;
    st->zz = S1;
    st->rms = kDebye * sqrt(S1 / npol);
    st->iters = 0;
    if (st->rms <= st->tol) st->done = 1;
    else if (st->maxiter == 0) st->done = 2;
  } else if (kMode == 1) {
    st->gamma = S0;
    if (!(S0 > 0.0)) {
      st->done = 3;
    } else {
      st->alpha = st->rho / S0;
    }
  } else {
    st->rms_true = kDebye * sqrt(S0 / npol);
    st->epol = -0.5 * kCoulomb * S1;
  }
}

__global__ __launch_bounds__(kBlk) void k_pcg_update(int n, const double* __restrict__ alpha_s,
                                                     const double* __restrict__ p,
                                                     const double* __restrict__ q,
                                                     double* __restrict__ x, double* __restrict__ r,
                                                     double* __restrict__ z,
                                                     double* __restrict__ part, PcgState* st) {
  __shared__ double sh[kBlk];
  if (st->done) return;
  const double al = st->alpha;
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
  const int nblk = gridDim.x;
  double t0 = block_sum(s0, sh), t1 = block_sum(s1, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = t0;
    part[nblk + blockIdx.x] = t1;
  }
  if (!last_block(st)) return;
  const double S0 = fixed_sum(part, nblk, sh), S1 = fixed_sum(part + nblk, nblk, sh);
  if (threadIdx.x != 0) return;
  st->ticket = 0;
  st->beta = S0 / st->rho;
  st->rho = S0;
  st->zz = S1;
  const double npol = st->npol > 0 ? (double)st->npol : 1.0;
  st->rms = kDebye * sqrt(S1 / npol);
  st->iters += 1;
  if (st->rms <= st->tol) st->done = 1;
  else if (st->iters >= st->maxiter) st->done = 2;
}

// p = z + beta p; it runs for the iteration that just updated (done may have
// just been set, which is harmless: p is not used after the loop).
__global__ void k_pcg_p(int n3, const double* __restrict__ z, double* __restrict__ p,
                        const PcgState* st) {
  if (st->done) return;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n3) return;
  p[k] = z[k] + st->beta * p[k];
}

__global__ void k_count_pol(int n, const double* __restrict__ pol, PcgState* st, double tol,
                            int maxiter) {
  __shared__ int cnt[kBlk];
  int c = 0;
  for (int i = threadIdx.x; i < n; i += kBlk) c += pol[i] > 0.0;
  cnt[threadIdx.x] = c;
  __syncthreads();
  for (int o = kBlk / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) cnt[threadIdx.x] += cnt[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    PcgState s0 = {};
    s0.npol = cnt[0];
    s0.tol = tol;
    s0.maxiter = maxiter;
    *st = s0;
  }
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
  double beta, cutoff;
  double *alpha_s, *b, *x, *r, *z, *p, *q, *part, *partial;
  PcgState* state;
  long pstride;
  int nblk;

  template <class R>
  TmatPh<R> tmat(const double* v, const int* done) const {
    TmatPh<R> ph;
    ph.xyz = sys->xyz;
    ph.mu = v;
    ph.mu_sorted = 1;
    ph.polarity = polarity;
    ph.thole = thole;
    ph.molid = sys->molid;
    ph.g.set(sys->box, cutoff, beta);
    ph.done = done;
    return ph;
  }

  template <class R>
  void matvec_units(const double* v, const int* done) {
    TmatPh<R> ph = tmat<R>(v, done);
    k_units<TmatPh<R>><<<P->nunits, 64, unit_lds_bytes<TmatPh<R>>(*P), st>>>(P->view(), ph, partial,
                                                                            pstride, nullptr);
  }

  // PCG on A x = rhs, x holding the initial guess; leaves the result in x.
  template <class R>
  tk_status run(const double* rhs, double tol, int maxiter, PcgState* host) {
    const int n = P->n;
    const double cself = 4.0 * beta * beta * beta / (3.0 * kSqrtPi);
    k_count_pol<<<1, kBlk, 0, st>>>(n, polarity, state, tol, maxiter);
    matvec_units<R>(x, nullptr);
    k_pcg_apply<0><<<nblk, kBlk, 0, st>>>(P->view(), partial, pstride, cself, alpha_s, x, rhs, q, r,
                                          z, p, part, state);
    int queued = 0;
    for (;;) {
      int chunk = maxiter - queued < kChunk ? maxiter - queued : kChunk;
      for (int c = 0; c < chunk; ++c) {
        matvec_units<R>(p, &state->done);
        k_pcg_apply<1><<<nblk, kBlk, 0, st>>>(P->view(), partial, pstride, cself, alpha_s, p,
                                              nullptr, q, nullptr, nullptr, nullptr, part, state);
        k_pcg_update<<<nblk, kBlk, 0, st>>>(n, alpha_s, p, q, x, r, z, part, state);
        k_pcg_p<<<ceil_div(3L * n, kBlk), kBlk, 0, st>>>(3 * n, z, p, state);
      }
      queued += chunk;
      TK_HIP(hipGetLastError());
      TK_HIP(hipMemcpyAsync(host, state, sizeof(PcgState), hipMemcpyDeviceToHost, st));
      TK_HIP(hipStreamSynchronize(st));
      if (host->done || queued >= maxiter) break;
    }
    return TK_OK;
  }

  // FP64 residual of x against rhs: rms_true and epol (x.rhs) into the state.
  tk_status true_residual(const double* rhs, PcgState* host) {
    const double cself = 4.0 * beta * beta * beta / (3.0 * kSqrtPi);
    matvec_units<double>(x, nullptr);
    k_pcg_apply<2><<<nblk, kBlk, 0, st>>>(P->view(), partial, pstride, cself, alpha_s, x, rhs,
                                          nullptr, nullptr, nullptr, nullptr, part, state);
    TK_HIP(hipGetLastError());
    TK_HIP(hipMemcpyAsync(host, state, sizeof(PcgState), hipMemcpyDeviceToHost, st));
    TK_HIP(hipStreamSynchronize(st));
    return TK_OK;
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
  S.pstride = pad64(n);
  S.nblk = ceil_div(n, kBlk);
  const size_t v3 = sizeof(double) * 3 * (size_t)n;
  void *alpha_s, *b, *x, *r, *z, *p, *q, *part, *partial, *state, *dx, *rt;
  if ((s = scratch(ctx, "pcg_alpha", sizeof(double) * n, &alpha_s)) ||
      (s = scratch(ctx, "pcg_b", v3, &b)) || (s = scratch(ctx, "pcg_x", v3, &x)) ||
      (s = scratch(ctx, "pcg_r", v3, &r)) || (s = scratch(ctx, "pcg_z", v3, &z)) ||
      (s = scratch(ctx, "pcg_p", v3, &p)) || (s = scratch(ctx, "pcg_q", v3, &q)) ||
      (s = scratch(ctx, "pcg_dx", v3, &dx)) || (s = scratch(ctx, "pcg_rt", v3, &rt)) ||
      (s = scratch(ctx, "pcg_part", sizeof(double) * 2 * S.nblk, &part)) ||
      (s = scratch(ctx, "partial", sizeof(double) * kMaxSlots * 3 * S.pstride, &partial)) ||
      (s = scratch(ctx, "pcg_state", sizeof(PcgState), &state)))
    return s;
  S.alpha_s = (double*)alpha_s; S.b = (double*)b; S.x = (double*)x; S.r = (double*)r;
  S.z = (double*)z; S.p = (double*)p; S.q = (double*)q; S.part = (double*)part;
  S.partial = (double*)partial; S.state = (PcgState*)state;
  if (unit_lds_bytes<EfieldPh<double>>(*P) > kMaxLds) return TK_E_CAPACITY;
  PcgState* host;
  if ((s = pinned(ctx, sizeof(PcgState), (void**)&host))) return s;
  TK_HIP(hipMemsetAsync(state, 0, sizeof(PcgState), st));

  // right-hand side: permanent field (sorted order)
  s = prec == TK_FP64 ? launch_efield<double>(ctx, st, *P, sys, mpole, polarity, thole, ewald_beta,
                                              cutoff, S.b, 1)
                      : launch_efield<float>(ctx, st, *P, sys, mpole, polarity, thole, ewald_beta,
                                             cutoff, S.b, 1);
  if (s) return s;
  k_pcg_setup<<<ceil_div(n, kBlk), kBlk, 0, st>>>(n, P->perm.p ? (const int32_t*)P->perm.p : nullptr,
                                                   polarity, mu_guess, S.b, S.alpha_s, S.x);
  s = prec == TK_FP64 ? S.run<double>(S.b, tol_debye, maxiter, host)
                      : S.run<float>(S.b, tol_debye, maxiter, host);
  if (s) return s;
  const int done = host->done;
  info->iters = host->iters;
  info->rms_debye = host->rms;
  info->converged = done == 1;
  info->status = done == 1 ? TK_OK : done == 3 ? TK_E_BREAKDOWN : TK_E_NOCONV;
  if ((s = S.true_residual(S.b, host))) return s;
  info->rms_true_debye = host->rms_true;
  info->epol = host->epol;
  if (prec == TK_MIXED && done != 3) {
    // FP64-residual refinement: solve A d = b - A x with the mixed solver, x += d.
    const double cself = 4.0 * ewald_beta * ewald_beta * ewald_beta / (3.0 * kSqrtPi);
    for (int ref = 0; ref < 3 && host->rms_true > tol_debye; ++ref) {
      // r_t = b - A x in FP64 (sorted), written to rt via mode 0 on a scratch copy
      double* xs = S.x;
      S.matvec_units<double>(xs, nullptr);
      k_pcg_apply<0><<<S.nblk, kBlk, 0, st>>>(P->view(), S.partial, S.pstride, cself, S.alpha_s,
                                              xs, S.b, S.q, (double*)rt, S.z, S.p, S.part, S.state);
      TK_HIP(hipMemcpyAsync(dx, x, v3, hipMemcpyDeviceToDevice, st));   // keep x
      // correction solve from d0 = alpha * r_t (= z of the mode-0 pass)
      TK_HIP(hipMemcpyAsync(x, S.z, v3, hipMemcpyDeviceToDevice, st));
      s = S.run<float>((double*)rt, tol_debye, maxiter, host);
      if (s) return s;
      info->iters += host->iters;
      info->refinements = ref + 1;
      k_add_into<<<ceil_div(3L * n, kBlk), kBlk, 0, st>>>(3 * n, (double*)dx, S.x);
      TK_HIP(hipMemcpyAsync(x, dx, v3, hipMemcpyDeviceToDevice, st));
      if ((s = S.true_residual(S.b, host))) return s;
      info->rms_true_debye = host->rms_true;
      info->epol = host->epol;
      if (host->rms_true <= tol_debye) {
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
