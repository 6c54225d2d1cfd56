// One-step truncated conjugate gradient (TCG1): a fixed-cost polarization
// solve (two mat-vecs) with the exact derivative of its energy (the
// fixed-cost solvers of the paper's later versions).  Diagonal
// preconditioner alpha, direct guess, no "peek" step:
//   mu0 = alpha E,  r0 = E - A mu0,  p0 = alpha r0,
//   gamma = r0.p0,  delta = p0.A p0,  a = gamma/delta,  mu1 = mu0 + a p0,
//   U = -1/2 C mu1.E.
// U is not variational in mu; its total derivative, with s = p0.E,
//   w = 2 p0/delta - 2 gamma alpha A p0/delta^2,  v = s w + a mu0,
//   u = mu0 + mu1 + v - alpha A v,
// is dU = -1/2 C [u.dE + v.dT mu0 + s gamma/delta^2 p0.dT p0], which one
// pass of the PolGradPh pair term evaluates (a = u/2, (b1, c1) = (v/2, mu0),
// (b2, c2) = (s gamma/(2 delta^2) p0, p0)).
//
// All vectors in the caller's order; the scalars stay on the device (fixed-
// order block sums, then one block), so the call queues its work without a
// host synchronisation.
#include <cmath>

#include "pairs.hpp"
#include "terms.hpp"

namespace tk {

namespace {

constexpr int kDotBlocks = 256;

// Epilogue of the field pass: E (permanent field + Ewald self field, as
// tk_efield_direct) and the direct guess mu0 = alpha E, caller order.
struct EpiFieldGuess {
  double* E;
  double* mu0;
  const double* mpole;
  const double* alpha;
  double cself;
  __device__ void operator()(int, int i, const double* a) const {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double e = a[c] + cself * mpole[10 * i + 1 + c];
      E[3 * i + c] = e;
      mu0[3 * i + c] = alpha[i] * e;
    }
  }
};

// Epilogue of the first mat-vec: q = A mu0 (as tk_tmatvec with the
// diagonal), r0 = E - q (zero rows for alpha = 0), p0 = alpha r0.
struct EpiResidual {
  const double* mu;
  const double* alpha;
  const double* E;
  double cself;
  double* r0;
  double* p0;
  __device__ void operator()(int, int i, const double* a) const {
    const double al = alpha[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double m = mu[3 * i + c];
      const double f = a[c] + cself * m;
      const double q = al > 0.0 ? m / al - f : 0.0;
      const double r = al > 0.0 ? E[3 * i + c] - q : 0.0;
      r0[3 * i + c] = r;
      p0[3 * i + c] = al * r;
    }
  }
};

// Up to four dot products of [3n] vectors: block partials (threads in
// order, waves in order), then one block sums the partials in order.
struct Dots {
  const double* a[4];
  const double* b[4];
};

__global__ __launch_bounds__(256) void k_dots(long m, int nd, Dots D, double* __restrict__ part) {
  __shared__ double sh[4][4];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int d = 0; d < 4; ++d)
      if (d < nd) v[d] += D.a[d][k] * D.b[d][k];
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    for (int o = 32; o > 0; o >>= 1) v[d] += __shfl_xor(v[d], o);
    if (lane == 0) sh[d][w] = v[d];
  }
  __syncthreads();
  if ((int)threadIdx.x < nd)
    part[threadIdx.x * kDotBlocks + blockIdx.x] =
        ((sh[threadIdx.x][0] + sh[threadIdx.x][1]) + sh[threadIdx.x][2]) + sh[threadIdx.x][3];
}

__global__ __launch_bounds__(256) void k_dots_finish(int nd, const double* __restrict__ part,
                                                     double* __restrict__ out) {
  __shared__ double sh[4];
  for (int d = 0; d < nd; ++d) {
    double v = part[d * kDotBlocks + threadIdx.x];   // kDotBlocks == blockDim.x
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) out[d] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    __syncthreads();
  }
}

// S = {gamma, delta, s, mu0.E}: mu1 = mu0 + a p0; block 0 writes
// U = -1/2 C mu1.E = -1/2 C (mu0.E + a s).
__global__ __launch_bounds__(256) void k_tcg_mu1(int n, const double* __restrict__ S,
                                                 const double* __restrict__ mu0,
                                                 const double* __restrict__ p0,
                                                 double* __restrict__ mu1,
                                                 double* __restrict__ epol) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const double a = S[1] != 0.0 ? S[0] / S[1] : 0.0;
  if (i == 0) epol[0] = -0.5 * kCoulomb * (S[3] + a * S[2]);
  if (i >= n) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) mu1[3 * i + c] = mu0[3 * i + c] + a * p0[3 * i + c];
}

// v = s w + a mu0, w = 2 p0/delta - 2 gamma alpha P/delta^2
__global__ __launch_bounds__(256) void k_tcg_v(int n, const double* __restrict__ S,
                                               const double* __restrict__ alpha,
                                               const double* __restrict__ mu0,
                                               const double* __restrict__ p0,
                                               const double* __restrict__ P,
                                               double* __restrict__ v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double g = S[0], dl = S[1], s = S[2];
  const double a = dl != 0.0 ? g / dl : 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int k = 3 * i + c;
    const double w = dl != 0.0 ? 2.0 * p0[k] / dl - 2.0 * g * alpha[i] * P[k] / (dl * dl) : 0.0;
    v[k] = s * w + a * mu0[k];
  }
}

// The gradient pass's inputs: a = u/2 with u = mu0 + mu1 + v - alpha A v,
// b1 = v/2, b2 = s gamma/(2 delta^2) p0 (c1 = mu0, c2 = p0 as they are).
__global__ __launch_bounds__(256) void k_tcg_grad_in(int n, const double* __restrict__ S,
                                                     const double* __restrict__ alpha,
                                                     const double* __restrict__ mu0,
                                                     const double* __restrict__ mu1,
                                                     const double* __restrict__ v,
                                                     const double* __restrict__ Av,
                                                     const double* __restrict__ p0,
                                                     double* __restrict__ ga,
                                                     double* __restrict__ gb1,
                                                     double* __restrict__ gb2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double dl = S[1];
  const double cb = dl != 0.0 ? S[2] * S[0] / (dl * dl) : 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int k = 3 * i + c;
    ga[k] = 0.5 * (mu0[k] + mu1[k] + v[k] - alpha[i] * Av[k]);
    gb1[k] = 0.5 * v[k];
    gb2[k] = 0.5 * cb * p0[k];
  }
}

// TmatPh for A v in the caller's order
TmatPh<double> tmat_of(const tk_system* sys, const Plan& P, const double* polarity,
                       const double* thole, double beta, double cutoff, const double* v) {
  TmatPh<double> ph;
  ph.xyz = sys->xyz;
  ph.mu = v;
  ph.mu_sorted = 0;
  ph.polarity = polarity;
  ph.thole = thole;
  ph.g.set(sys->box, cutoff, beta);
  ph.molid = sys->molid;
  ph.perm_ = (const int32_t*)P.perm.p;
  return ph;
}

}  // namespace

}  // namespace tk

using namespace tk;

extern "C" tk_status tk_polarize_tcg1(tk_ctx* ctx, void* stream, const tk_system* sys,
                                      const tk_nblist* list, const double* mpole,
                                      const double* polarity, const double* thole,
                                      double ewald_beta, double cutoff, double* mu_out,
                                      double* epol, double* force) {
  if (!ctx) return TK_E_ARG;
  tk_status s = check_system(sys);
  if (s) return s;
  const Plan* P;
  if ((s = get_plan(ctx, sys, list, cutoff, &P))) return s;
  if (!(ewald_beta >= 0.0) || !std::isfinite(ewald_beta) || !epol) return TK_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int n = sys->n;
  if (n == 0) {
    TK_HIP(hipMemsetAsync(epol, 0, sizeof(double), st));
    return TK_OK;
  }
  if (!mpole || !polarity || !thole || !mu_out) return TK_E_ARG;
  const size_t v3 = sizeof(double) * 3 * (size_t)n;
  void *buf, *part, *S;
  if ((s = scratch(ctx, per_stream("tcg_vec", st).c_str(), 10 * v3, &buf)) ||
      (s = scratch(ctx, per_stream("tcg_part", st).c_str(), sizeof(double) * 4 * kDotBlocks, &part)) ||
      (s = scratch(ctx, per_stream("tcg_S", st).c_str(), sizeof(double) * 8, &S)))
    return s;
  double* V = (double*)buf;
  const size_t m3 = 3 * (size_t)n;
  double *E = V, *mu0 = V + m3, *r0 = V + 2 * m3, *p0 = V + 3 * m3, *Pv = V + 4 * m3,
         *v = V + 5 * m3, *Av = V + 6 * m3, *ga = V + 7 * m3, *gb1 = V + 8 * m3,
         *gb2 = V + 9 * m3;
  double* Sd = (double*)S;   // gamma, delta, s, mu0.E
  const int nb = ceil_div(n, 256);
  // E and mu0 (field pass), r0 and p0 (first mat-vec), P = A p0
  EfieldPh<double> ef;
  ef.xyz = sys->xyz;
  ef.mpole = mpole;
  ef.molid = sys->molid;
  ef.polarity = polarity;
  ef.thole = thole;
  ef.g.set(sys->box, cutoff, ewald_beta);
  const double cself = ef.g.cself;
  if ((s = run_term(ctx, st, *P, ef, EpiFieldGuess{E, mu0, mpole, polarity, cself}, nullptr,
                    nullptr)))
    return s;
  if ((s = run_term(ctx, st, *P, tmat_of(sys, *P, polarity, thole, ewald_beta, cutoff, mu0),
                    EpiResidual{mu0, polarity, E, cself, r0, p0}, nullptr, nullptr)))
    return s;
  if ((s = run_term(ctx, st, *P, tmat_of(sys, *P, polarity, thole, ewald_beta, cutoff, p0),
                    EpiMutual{Pv, p0, polarity, cself, 1}, nullptr, nullptr)))
    return s;
  // gamma, delta, s, mu0.E in one pass; mu1 and U
  k_dots<<<kDotBlocks, 256, 0, st>>>((long)m3, 4, Dots{{r0, p0, p0, mu0}, {p0, Pv, E, E}},
                                     (double*)part);
  k_dots_finish<<<1, kDotBlocks, 0, st>>>(4, (const double*)part, Sd);
  k_tcg_mu1<<<nb, 256, 0, st>>>(n, Sd, mu0, p0, mu_out, epol);
  if (force) {
    k_tcg_v<<<nb, 256, 0, st>>>(n, Sd, polarity, mu0, p0, Pv, v);
    if ((s = run_term(ctx, st, *P, tmat_of(sys, *P, polarity, thole, ewald_beta, cutoff, v),
                      EpiMutual{Av, v, polarity, cself, 1}, nullptr, nullptr)))
      return s;
    k_tcg_grad_in<<<nb, 256, 0, st>>>(n, Sd, polarity, mu0, mu_out, v, Av, p0, ga, gb1, gb2);
    PolGradPh<double> ph;
    ph.xyz = sys->xyz;
    ph.mpole = mpole;
    ph.molid = sys->molid;
    ph.polarity = polarity;
    ph.thole = thole;
    ph.vec[0] = ga;
    ph.vec[1] = gb1;
    ph.vec[2] = mu0;
    ph.vec[3] = gb2;
    ph.vec[4] = p0;
    ph.g.set(sys->box, cutoff, ewald_beta);
    if ((s = run_term(ctx, st, *P, ph, EpiForce{force}, nullptr, nullptr))) return s;
  }
  TK_HIP(hipGetLastError());
  return TK_OK;
}
