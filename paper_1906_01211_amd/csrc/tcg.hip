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

template <class R>
tk_status launch_tmat(tk_ctx* ctx, hipStream_t st, const Plan& P, const tk_system* sys,
                      const double* polarity, const double* thole, double beta, double cutoff,
                      int include_diag, const double* mu, double* out);

namespace {

constexpr int kDotBlocks = 256;

// Up to three dot products of [3n] vectors: block partials (threads in
// order, waves in order), then one block sums the partials in order.
__global__ __launch_bounds__(256) void k_dots(long m, int nd, const double* __restrict__ a0,
                                              const double* __restrict__ b0,
                                              const double* __restrict__ a1,
                                              const double* __restrict__ b1,
                                              const double* __restrict__ a2,
                                              const double* __restrict__ b2,
                                              double* __restrict__ part) {
  __shared__ double sh[3][4];
  double v[3] = {0.0, 0.0, 0.0};
  for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (long)gridDim.x * blockDim.x) {
    v[0] += a0[k] * b0[k];
    if (nd > 1) v[1] += a1[k] * b1[k];
    if (nd > 2) v[2] += a2[k] * b2[k];
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    for (int o = 32; o > 0; o >>= 1) v[d] += __shfl_xor(v[d], o);
    if (lane == 0) sh[d][w] = v[d];
  }
  __syncthreads();
  if (threadIdx.x < 3)
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

// mu0 = alpha E
__global__ __launch_bounds__(256) void k_tcg_mu0(int n, const double* __restrict__ alpha,
                                                 const double* __restrict__ E,
                                                 double* __restrict__ mu0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) mu0[3 * i + c] = alpha[i] * E[3 * i + c];
}

// r0 = E - A mu0 (zero rows for alpha = 0), p0 = alpha r0
__global__ __launch_bounds__(256) void k_tcg_r0(int n, const double* __restrict__ alpha,
                                                const double* __restrict__ E,
                                                const double* __restrict__ q,
                                                double* __restrict__ r0, double* __restrict__ p0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double al = alpha[i];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double r = al > 0.0 ? E[3 * i + c] - q[3 * i + c] : 0.0;
    r0[3 * i + c] = r;
    p0[3 * i + c] = al * r;
  }
}

// S = {gamma, delta, s}: mu1 = mu0 + a p0
__global__ __launch_bounds__(256) void k_tcg_mu1(int n, const double* __restrict__ S,
                                                 const double* __restrict__ mu0,
                                                 const double* __restrict__ p0,
                                                 double* __restrict__ mu1) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = S[1] != 0.0 ? S[0] / S[1] : 0.0;
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

__global__ void k_tcg_energy(const double* __restrict__ d, double* __restrict__ epol) {
  if (threadIdx.x == 0) epol[0] = -0.5 * kCoulomb * d[0];
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
  if ((s = scratch(ctx, per_stream("tcg_vec", st).c_str(), 12 * v3, &buf)) ||
      (s = scratch(ctx, per_stream("tcg_part", st).c_str(), sizeof(double) * 3 * kDotBlocks, &part)) ||
      (s = scratch(ctx, per_stream("tcg_S", st).c_str(), sizeof(double) * 8, &S)))
    return s;
  double* V = (double*)buf;
  const size_t m3 = 3 * (size_t)n;
  double *E = V, *mu0 = V + m3, *q = V + 2 * m3, *r0 = V + 3 * m3, *p0 = V + 4 * m3,
         *Pv = V + 5 * m3, *v = V + 6 * m3, *Av = V + 7 * m3, *ga = V + 8 * m3,
         *gb1 = V + 9 * m3, *gb2 = V + 10 * m3;
  double* Sd = (double*)S;   // gamma, delta, s, mu1.E
  const int nb = ceil_div(n, 256);
  const tk_system s1{n, sys->xyz, sys->box, sys->molid};
  if ((s = launch_efield<double>(ctx, st, *P, &s1, mpole, polarity, thole, ewald_beta, cutoff, E,
                                 0)))
    return s;
  k_tcg_mu0<<<nb, 256, 0, st>>>(n, polarity, E, mu0);
  if ((s = launch_tmat<double>(ctx, st, *P, &s1, polarity, thole, ewald_beta, cutoff, 1, mu0, q)))
    return s;
  k_tcg_r0<<<nb, 256, 0, st>>>(n, polarity, E, q, r0, p0);
  if ((s = launch_tmat<double>(ctx, st, *P, &s1, polarity, thole, ewald_beta, cutoff, 1, p0, Pv)))
    return s;
  k_dots<<<kDotBlocks, 256, 0, st>>>((long)m3, 3, r0, p0, p0, Pv, p0, E, (double*)part);
  k_dots_finish<<<1, kDotBlocks, 0, st>>>(3, (const double*)part, Sd);
  k_tcg_mu1<<<nb, 256, 0, st>>>(n, Sd, mu0, p0, mu_out);
  k_dots<<<kDotBlocks, 256, 0, st>>>((long)m3, 1, mu_out, E, nullptr, nullptr, nullptr, nullptr,
                                     (double*)part);
  k_dots_finish<<<1, kDotBlocks, 0, st>>>(1, (const double*)part, Sd + 3);
  k_tcg_energy<<<1, 64, 0, st>>>(Sd + 3, epol);
  if (force) {
    k_tcg_v<<<nb, 256, 0, st>>>(n, Sd, polarity, mu0, p0, Pv, v);
    if ((s = launch_tmat<double>(ctx, st, *P, &s1, polarity, thole, ewald_beta, cutoff, 1, v, Av)))
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
