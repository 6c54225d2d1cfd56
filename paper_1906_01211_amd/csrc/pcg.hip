// Induced dipoles by preconditioned conjugate gradient, resident on the device
// (the polarization solver of section "Hotspots": its mat-vec is the paper's
// largest hotspot and is called up to 12 times per step).
//
// All solver vectors live in the plan's sorted atom order.  The right-hand
// side pass (permanent field) also stores each listed pair's two mutual-field
// radial factors, so the mat-vec tiles only recompute the pair vector and
// contract it with the dipoles.  One iteration is four kernels:
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
#include <algorithm>
#include <cmath>

#include "terms.hpp"

namespace tk {
namespace {

constexpr int kBlk = 256;
constexpr int kChunk = 6;

struct PcgState {
  double rho, gamma, alpha, beta, zz, rms, rms0, rms_true, epol, tol;
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
  if (kMode == 2 && !st->done) return;   // residual queued ahead of convergence
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
  __shared__ int s_done;
  if (threadIdx.x == 0) s_done = st->done;   // one read per block: all its waves agree
  __syncthreads();
  if (s_done) return;
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
// iteration count, convergence); mode 2: after the true residual (only once
// the solver has stopped: the host queues it behind each chunk).
template <int kMode>
__global__ __launch_bounds__(kBlk) void k_pcg_finish(const double* __restrict__ part, int nblk,
                                                     PcgState* st, PcgState* host) {
  __shared__ double sh[kBlk];
  if (kMode == 1 && st->done) {
    if (threadIdx.x == 0) *host = *st;
    return;
  }
  if (kMode == 2 && !st->done) return;   // residual queued ahead of convergence
  const double S0 = fixed_sum(part, nblk, sh), S1 = fixed_sum(part + nblk, nblk, sh);
  if (threadIdx.x != 0) return;
  const double npol = st->npol > 0 ? (double)st->npol : 1.0;
  if (kMode == 0) {
    st->rho = S0;
    st->zz = S1;
    st->rms = kDebye * sqrt(S1 / npol);
    st->rms0 = st->rms;
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

// ---------------------------------------------------------------------------
// Per-cell mat-vec with the iteration's bookkeeping folded in.
//
// One workgroup per cell C owns C's atoms.  It stages the coordinates and the
// operand of every neighbour cell of C into LDS, then walks the pair codes of
// all units C takes part in (each unordered pair is therefore visited from
// both of its cells) and accumulates only C's side; each wave keeps its own
// accumulator copy, summed in wave order, so sums are reproducible.  The
// epilogue applies A to C's atoms directly: no partial slots, no separate
// per-atom pass.  Radial factors come from the right-hand-side pass cache.
//
// kMode 0: v = x:  r = b - A x, z = alpha r; partials r.z, z.z.
// kMode 1: iteration k.  Every workgroup first sums the partials of r.z and
//          z.z (and of the previous r.z) in a fixed order, so all of them
//          take the same decisions: stop (converged or k = maxiter), else
//          beta = rho_k / rho_{k-1} and p_k = z_k + beta p_{k-1}, staged as
//          the operand; outputs p_k, q = A p_k and partials of p.q.
//          Workgroup 0 records the state and mirrors it to the host.
// kMode 2: v = x (only once the solver has stopped): partials of
//          |alpha (b - A x)|^2 and x.b.
constexpr int kMvThreads = 256;
constexpr int kMvWaves = kMvThreads / 64;

template <class R>
struct MvArgs {
  PlanView pv;
  const R* gc;
  long gcs;
  double box, inv_box, cself;
  const double* pos;   // sorted SoA coordinates, stride pstride
  long pstride;
  const double* alpha_s;
  const double* rhs;    // modes 0, 2
  const double* v;      // modes 0, 2: x; mode 1: z
  const double* pold;   // mode 1, k >= 1
  double* pnew;         // mode 1
  double* q;            // mode 1
  double* r;            // mode 0
  double* z;            // mode 0
  double* part;         // [2][ncells] workgroup partials
  const double* pz_cur;
  int npz_cur;
  const double* pz_prev;
  int npz_prev;
  int k;
  int stage_cap, own_cap;
  PcgState* st;
  PcgState* host;
};

// Three fixed-order sums in one pass: a[0..na), b[0..na), c[0..nc).
__device__ __forceinline__ void mv_fixed_sum3(const double* a, const double* b, int na,
                                              const double* c, int nc, double* sh, double& sa,
                                              double& sb, double& sc) {
  double va = 0.0, vb = 0.0, vc = 0.0;
  for (int i = threadIdx.x; i < na; i += kMvThreads) {
    va += a[i];
    vb += b[i];
  }
  for (int i = threadIdx.x; i < nc; i += kMvThreads) vc += c[i];
  sh[threadIdx.x] = va;
  sh[kMvThreads + threadIdx.x] = vb;
  sh[2 * kMvThreads + threadIdx.x] = vc;
  __syncthreads();
  for (int o = kMvThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sh[threadIdx.x] += sh[threadIdx.x + o];
      sh[kMvThreads + threadIdx.x] += sh[kMvThreads + threadIdx.x + o];
      sh[2 * kMvThreads + threadIdx.x] += sh[2 * kMvThreads + threadIdx.x + o];
    }
    __syncthreads();
  }
  sa = sh[0];
  sb = sh[kMvThreads];
  sc = sh[2 * kMvThreads];
  __syncthreads();
}

// Pairs per thread whose loads are issued together (latency hiding).
constexpr int kMvBatch = 4;
// Staged atoms per thread whose loads are issued together.
constexpr int kMvStageBatch = 4;

template <class R, int kMode>
__global__ __launch_bounds__(kMvThreads) void k_pcg_mv(MvArgs<R> A) {
  extern __shared__ double lds[];
  __shared__ double red[3 * kMvThreads];
  __shared__ int e_unit[kCellUnitStride], e_role[kCellUnitStride], e_cs[kCellUnitStride];
  __shared__ int e_off[kCellUnitStride + 1], e_pre[kCellUnitStride + 1];
  __shared__ long e_uoff[kCellUnitStride];
  __shared__ int self_j;
  const int c = blockIdx.x, tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  PcgState* st = A.st;
  __shared__ int s_done;
  if (tid == 0) s_done = st->done;   // one read per workgroup: all its waves agree
  __syncthreads();
  if (kMode == 1 && s_done) return;
  if (kMode == 2 && !s_done) return;
  double beta = 0.0;
  if (kMode == 1) {
    double rz, zz, rzp;
    mv_fixed_sum3(A.pz_cur, A.pz_cur + A.npz_cur, A.npz_cur, A.pz_prev,
                  A.k >= 1 ? A.npz_prev : 0, red, rz, zz, rzp);
    const double npol = st->npol > 0 ? (double)st->npol : 1.0;
    const double rms = kDebye * sqrt(zz / npol);
    const int stop = rms <= st->tol ? 1 : A.k >= st->maxiter ? 2 : 0;
    if (A.k >= 1) beta = rz / rzp;
    if (c == 0 && tid == 0) {
      st->rho = rz;
      st->zz = zz;
      st->rms = rms;
      if (A.k == 0) st->rms0 = rms;
      st->beta = beta;
      st->iters = A.k;
      if (stop) st->done = stop;
      *A.host = *st;
    }
    if (stop) return;
  }
  // the cell's units: other cell start, staging offset, pair-code prefix
  const PlanView& pv = A.pv;
  const int32_t* cu = pv.cell_units + (long)c * kCellUnitStride;
  const int ne = cu[0];
  if (w == 0) {
    int no = 0, cnt = 0, u = 0, role = 0, cs = 0;
    if (lane < ne) {
      const int e = cu[1 + lane];
      u = e >> 2;
      role = e & 3;
      const Unit un = pv.units[u];
      const int oc = role == 1 ? un.h : un.k;
      cs = pv.cell_start[oc];
      no = pv.cell_start[oc + 1] - cs;
      cnt = pv.unit_cnt[u];
      e_uoff[lane] = pv.unit_off[u];
    }
    int io = no, ic = cnt;
    for (int o = 1; o < 64; o <<= 1) {
      const int t1 = __shfl_up(io, o), t2 = __shfl_up(ic, o);
      if (lane >= o) {
        io += t1;
        ic += t2;
      }
    }
    if (lane < ne) {
      e_unit[lane] = u;
      e_role[lane] = role;
      e_cs[lane] = cs;
      e_off[lane] = io - no;
      e_pre[lane] = ic - cnt;
      if (role == 2) self_j = lane;
    }
    if (lane == ne - 1) {
      e_off[ne] = io;
      e_pre[ne] = ic;
    }
  }
  __syncthreads();
  const int SC = A.stage_cap, OC = A.own_cap;
  double* L = lds;                 // x y z v0 v1 v2, stride SC
  double* ACC = L + 6 * SC;        // [wave][3][OC]
  const int total = e_off[ne];
  const long ps = A.pstride;
  // operand v + beta * pold: for k = 0 (and modes 0, 2) beta = 0 and pold = v
  const double* pold = (kMode == 1 && A.k >= 1) ? A.pold : A.v;
  for (int i0 = tid; i0 < total; i0 += kMvThreads * kMvStageBatch) {
    int src[kMvStageBatch];
#pragma unroll
    for (int m = 0; m < kMvStageBatch; ++m) {
      const int i = i0 + m * kMvThreads;
      int lo = 0, hi = ne - 1;   // last entry starting at or before i
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (e_off[mid] <= i) lo = mid;
        else hi = mid - 1;
      }
      src[m] = i < total ? e_cs[lo] + (i - e_off[lo]) : -1;
    }
    double f[kMvStageBatch][6];
#pragma unroll
    for (int m = 0; m < kMvStageBatch; ++m) {
      const int s = src[m];
      if (s < 0) continue;
      f[m][0] = A.pos[s];
      f[m][1] = A.pos[ps + s];
      f[m][2] = A.pos[2 * ps + s];
#pragma unroll
      for (int d = 0; d < 3; ++d)
        f[m][3 + d] = fma(beta, pold[3 * s + d], A.v[3 * s + d]);
    }
#pragma unroll
    for (int m = 0; m < kMvStageBatch; ++m) {
      const int i = i0 + m * kMvThreads;
      if (src[m] < 0) continue;
#pragma unroll
      for (int d = 0; d < 6; ++d) L[d * SC + i] = f[m][d];
    }
  }
  const int js = self_j;
  const int own0 = e_off[js], nown = e_off[js + 1] - own0;
  for (int i = tid; i < kMvWaves * 3 * nown; i += kMvThreads) {
    const int ww = i / (3 * nown), rem = i - ww * 3 * nown;
    ACC[ww * 3 * OC + rem] = 0.0;   // [ww][d][t] with rem = d * nown + t
  }
  __syncthreads();
  // accumulator of wave w, component d, own atom t: ACC[(w * 3 + d) * nown + t]
  double* MY = ACC + w * 3 * OC;
  const int T = e_pre[ne];
  int j = 0;
  for (int v0 = tid; v0 < T; v0 += kMvThreads * kMvBatch) {
    // issue the batch's code and factor loads together
    uint32_t codes[kMvBatch];
    R g1s[kMvBatch], g2s[kMvBatch];
    int roles[kMvBatch], offs[kMvBatch];   // kept in registers: no LDS reads after the atomics
#pragma unroll
    for (int m = 0; m < kMvBatch; ++m) {
      const int vix = v0 + m * kMvThreads;
      roles[m] = -1;
      if (vix < T) {
        while (vix >= e_pre[j + 1]) ++j;
        roles[m] = e_role[j];
        offs[m] = e_off[j];
        const long p = e_uoff[j] + (vix - e_pre[j]);
        codes[m] = pv.codes[p];
        g1s[m] = A.gc[p];
        g2s[m] = A.gc[A.gcs + p];
      }
    }
#pragma unroll
    for (int m = 0; m < kMvBatch; ++m) {
    if (roles[m] < 0) continue;
    const int role = roles[m];
    const uint32_t code = codes[m];
    const int a = (int)(code & 0xffffu), b = (int)(code >> 16);
    const int own = role == 1 ? b : a;
    const int oth = offs[m] + (role == 1 ? a : b);
    const int ownL = own0 + own;
    const R g1 = g1s[m], g2 = g2s[m];
    R dv[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double t = L[d * SC + oth] - L[d * SC + ownL];
      dv[d] = R(fma(-A.box, rint(t * A.inv_box), t));
    }
    const R vo[3] = {R(L[3 * SC + oth]), R(L[4 * SC + oth]), R(L[5 * SC + oth])};
    const R so = (vo[0] * dv[0] + vo[1] * dv[1] + vo[2] * dv[2]) * g2;
#pragma unroll
    for (int d = 0; d < 3; ++d) lds_add(&MY[d * nown + own], (double)(dv[d] * so - vo[d] * g1));
    if (role == 2) {
      const R va[3] = {R(L[3 * SC + ownL]), R(L[4 * SC + ownL]), R(L[5 * SC + ownL])};
      const R sa = (va[0] * dv[0] + va[1] * dv[1] + va[2] * dv[2]) * g2;
#pragma unroll
      for (int d = 0; d < 3; ++d) lds_add(&MY[d * nown + b], (double)(dv[d] * sa - va[d] * g1));
    }
    }
  }
  __syncthreads();
  const int hs = pv.cell_start[c];
  double s0 = 0.0, s1 = 0.0;
  for (int t = tid; t < nown; t += kMvThreads) {
    const int s = hs + t;
    const double al = A.alpha_s[s];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double f = 0.0;
#pragma unroll
      for (int ww = 0; ww < kMvWaves; ++ww) f += ACC[ww * 3 * OC + d * nown + t];
      const double vv = L[(3 + d) * SC + own0 + t];
      const double av = al > 0.0 ? vv / al - (f + A.cself * vv) : 0.0;   // (A v)_s
      if (kMode == 1) {
        A.pnew[3 * s + d] = vv;
        A.q[3 * s + d] = av;
        s0 += vv * av;
      } else {
        const double rr = al > 0.0 ? A.rhs[3 * s + d] - av : 0.0;
        const double zz = al * rr;
        if (kMode == 0) {
          A.r[3 * s + d] = rr;
          A.z[3 * s + d] = zz;
          s0 += rr * zz;
          s1 += zz * zz;
        } else {
          s0 += zz * zz;
          s1 += vv * A.rhs[3 * s + d];
        }
      }
    }
  }
  const int ncells = gridDim.x;
  red[tid] = s0;
  __syncthreads();
  for (int o = kMvThreads / 2; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  if (tid == 0) A.part[c] = red[0];
  __syncthreads();
  if (kMode != 1) {
    red[tid] = s1;
    __syncthreads();
    for (int o = kMvThreads / 2; o > 0; o >>= 1) {
      if (tid < o) red[tid] += red[tid + o];
      __syncthreads();
    }
    if (tid == 0) A.part[ncells + c] = red[0];
  }
}

// Iteration k, second half: gamma = p.q and rho_k from their partials (fixed
// order, in every block), alpha = rho/gamma, x += alpha p, r -= alpha q,
// z = alpha_i r; partials of r.z and z.z for iteration k + 1.
__global__ __launch_bounds__(kBlk) void k_pcg_update_fused(
    int n, const double* __restrict__ alpha_s, const double* __restrict__ p,
    const double* __restrict__ q, double* __restrict__ x, double* __restrict__ r,
    double* __restrict__ z, const double* __restrict__ pg, int npg,
    const double* __restrict__ pz_cur, int npz_cur, double* __restrict__ pz_next, int k,
    PcgState* st, PcgState* host) {
  __shared__ double sh[kBlk];
  __shared__ int s_done;
  if (threadIdx.x == 0) s_done = st->done;   // one read per block: all its waves agree
  __syncthreads();
  if (s_done) return;
  const double gam = fixed_sum(pg, npg, sh);
  const double rho = fixed_sum(pz_cur, npz_cur, sh);
  if (!(gam > 0.0)) {   // p.Ap <= 0: not positive definite
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->gamma = gam;
      st->iters = k;
      st->done = 3;
      *host = *st;
    }
    return;
  }
  const double al = rho / gam;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->gamma = gam;
    st->alpha = al;
  }
  const int nblk = gridDim.x;
  const int s = blockIdx.x * kBlk + threadIdx.x;
  double s0 = 0.0, s1 = 0.0;
  if (s < n) {
    const double a = alpha_s[s];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int e = 3 * s + c;
      x[e] += al * p[e];
      const double rr = r[e] - al * q[e];
      r[e] = rr;
      const double zz = a * rr;
      z[e] = zz;
      s0 += rr * zz;
      s1 += zz * zz;
    }
  }
  const double t0 = block_sum(s0, sh), t1 = block_sum(s1, sh);
  if (threadIdx.x == 0) {
    pz_next[blockIdx.x] = t0;
    pz_next[nblk + blockIdx.x] = t1;
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
  double beta, cutoff, cself;
  double *alpha_s, *b, *x, *r, *z, *p, *q, *part, *partg, *partial, *gathered;
  PcgState* state;
  PcgState* host;       // pinned host mirror
  PcgState* host_dev;   // its device address
  long pstride;
  int nblk;
  int prec;
  void* gc = nullptr;   // cached radial factors g1 | g2 per pair code (solver precision)
  long gcs = 0;
  // per-cell fused path
  bool fused = false;
  int ncells = 0;
  size_t mv_lds = 0;
  double* pbuf[2] = {nullptr, nullptr};   // search directions p_k (k even, odd)
  double* pz[2] = {nullptr, nullptr};     // partials of r.z | z.z (k even, odd)
  double* pg = nullptr;                   // partials of p.q (per cell)

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

  template <class R>
  TmatCachedPh<R> tmat_cached(const double* v, const int* done, bool dir) const {
    TmatCachedPh<R> ph;
    ph.gc = (const R*)gc;
    ph.gcs = gcs;
    ph.box = sys->box;
    ph.inv_box = 1.0 / sys->box;
    ph.xyz = sys->xyz;
    ph.mu = v;
    ph.done = done;
    ph.sorted = gathered;
    ph.gstride = pstride;
    if (dir) {
      ph.zdir = z;
      ph.beta_dir = &state->beta;
    }
    return ph;
  }

  // Static per-atom fields of the mat-vec, gathered once per solve: the
  // coordinates for the cached mat-vec; for the mixed form also the damping
  // fields of the on-the-fly FP64 mat-vec (the first three fields coincide).
  void gather_geometry() {
    if (prec == TK_MIXED) {
      TmatPh<double> ph = tmat<double>(nullptr, nullptr, false);
      k_gather<TmatPh<double>><<<ceil_div(P->n, 256), 256, 0, st>>>(P->view(), ph, gathered,
                                                                    pstride);
    } else {
      TmatCachedPh<double> ph = tmat_cached<double>(nullptr, nullptr, false);
      k_gather<TmatCachedPh<double>><<<ceil_div(P->n, 256), 256, 0, st>>>(P->view(), ph, gathered,
                                                                          pstride);
    }
  }

  // Mat-vec tiles into the partial slots.  The solver's own precision uses
  // the radial factors cached by the right-hand-side pass; the FP64 residual
  // of the mixed form is evaluated on the fly in FP64.
  template <class R>
  void matvec_units(const double* v, const int* done, bool dir = false) {
    if (std::is_same<R, double>::value && prec == TK_MIXED) {
      TmatPh<double> ph = tmat<double>(v, done, dir);
      ProfScope ps(ctx, st, "units_tmat_fp64");
      k_units<TmatPh<double>><<<P->nunits, 64, unit_lds_bytes<TmatPh<double>>(*P), st>>>(
          P->view(), ph, partial, pstride, nullptr);
      return;
    }
    TmatCachedPh<R> ph = tmat_cached<R>(v, done, dir);
    ProfScope ps(ctx, st, std::string("units_tmatc") + TmatCachedPh<R>::kTag);
    k_units<TmatCachedPh<R>><<<P->nunits, 64, unit_lds_bytes<TmatCachedPh<R>>(*P), st>>>(
        P->view(), ph, partial, pstride, nullptr);
  }

  tk_status sync_state() {
    TK_HIP(hipGetLastError());
    TK_HIP(hipStreamSynchronize(st));
    return TK_OK;
  }

  // One PCG iteration: mat-vec on p = z + beta p, apply, update, finish.
  template <class R>
  void iteration() {
    matvec_units<R>(p, &state->done, true);
    {
      ProfScope ps(ctx, st, "pcg_apply");
      k_pcg_apply<1><<<nblk, kBlk, 0, st>>>(P->view(), partial, pstride, cself, alpha_s, p, nullptr,
                                            q, nullptr, z, p, partg, state);
    }
    {
      ProfScope ps(ctx, st, "pcg_update");
      k_pcg_update<<<nblk, kBlk, 0, st>>>(P->n, alpha_s, p, q, x, r, z, partg, part, state);
    }
    k_pcg_finish<1><<<1, kBlk, 0, st>>>(part, nblk, state, host_dev);
  }

  // FP64 residual of x against rhs (rms_true, and epol from x.rhs), queued
  // behind the iterations; its kernels run only once the solver has stopped.
  void queue_true_residual(const double* rhs) {
    if (fused && prec == TK_FP64) {
      MvArgs<double> a = mv_args<double>();
      a.v = x;
      a.rhs = rhs;
      a.part = part;
      {
        ProfScope ps(ctx, st, "pcg_mv_residual_fp64");
        k_pcg_mv<double, 2><<<ncells, kMvThreads, mv_lds, st>>>(a);
      }
      k_pcg_finish<2><<<1, kBlk, 0, st>>>(part, ncells, state, host_dev);
      return;
    }
    if (prec == TK_MIXED) {
      TmatPh<double> ph = tmat<double>(x, &state->done, false);
      ph.run_when_done = 1;
      ProfScope ps(ctx, st, "units_tmat_fp64");
      k_units<TmatPh<double>><<<P->nunits, 64, unit_lds_bytes<TmatPh<double>>(*P), st>>>(
          P->view(), ph, partial, pstride, nullptr);
    } else {
      TmatCachedPh<double> ph = tmat_cached<double>(x, &state->done, false);
      ph.run_when_done = 1;
      ProfScope ps(ctx, st, "units_tmatc_fp64");
      k_units<TmatCachedPh<double>><<<P->nunits, 64, unit_lds_bytes<TmatCachedPh<double>>(*P),
                                      st>>>(P->view(), ph, partial, pstride, nullptr);
    }
    k_pcg_apply<2><<<nblk, kBlk, 0, st>>>(P->view(), partial, pstride, cself, alpha_s, x, rhs,
                                          nullptr, nullptr, nullptr, nullptr, part, state);
    k_pcg_finish<2><<<1, kBlk, 0, st>>>(part, nblk, state, host_dev);
  }

  template <class R>
  MvArgs<R> mv_args() const {
    MvArgs<R> a = {};
    a.pv = P->view();
    a.gc = (const R*)gc;
    a.gcs = gcs;
    a.box = sys->box;
    a.inv_box = 1.0 / sys->box;
    a.cself = cself;
    a.pos = gathered;
    a.pstride = pstride;
    a.alpha_s = alpha_s;
    a.stage_cap = P->max_nbhd;
    a.own_cap = P->max_occ;
    a.st = state;
    a.host = host_dev;
    return a;
  }

  int npz(int k) const { return k == 0 ? ncells : nblk; }

  // iteration k, first half: convergence test, p_k, q = A p_k
  template <class R>
  void queue_mv(int k) {
    MvArgs<R> a = mv_args<R>();
    a.v = z;
    a.pold = pbuf[(k + 1) & 1];
    a.pnew = pbuf[k & 1];
    a.q = q;
    a.part = pg;
    a.pz_cur = pz[k & 1];
    a.npz_cur = npz(k);
    a.pz_prev = pz[(k + 1) & 1];
    a.npz_prev = k >= 1 ? npz(k - 1) : 0;
    a.k = k;
    ProfScope ps(ctx, st, std::string("pcg_mv") + prec_tag<R>());
    k_pcg_mv<R, 1><<<ncells, kMvThreads, mv_lds, st>>>(a);
  }

  // iteration k, second half: update x, r, z
  void queue_update(int k) {
    ProfScope ps(ctx, st, "pcg_update");
    k_pcg_update_fused<<<nblk, kBlk, 0, st>>>(P->n, alpha_s, pbuf[k & 1], q, x, r, z, pg, ncells,
                                              pz[k & 1], npz(k), pz[(k + 1) & 1], k, state,
                                              host_dev);
  }

  template <class R>
  tk_status run_fused(const double* rhs, double tol, int maxiter, int first_chunk, bool residual) {
    k_pcg_init<<<1, 1, 0, st>>>(state, tol, maxiter);
    {
      MvArgs<R> a = mv_args<R>();
      a.v = x;
      a.rhs = rhs;
      a.r = r;
      a.z = z;
      a.part = pz[0];
      ProfScope ps(ctx, st, std::string("pcg_mv0") + prec_tag<R>());
      k_pcg_mv<R, 0><<<ncells, kMvThreads, mv_lds, st>>>(a);
    }
    queue_mv<R>(0);
    int k = 0;   // index of the last queued first half
    int chunk = first_chunk > 0 ? first_chunk : kChunk;
    for (;;) {
      if (chunk > maxiter - k) chunk = maxiter - k;
      for (int c = 0; c < chunk; ++c) {
        queue_update(k);
        queue_mv<R>(++k);
      }
      if (residual) queue_true_residual(rhs);
      tk_status s = sync_state();
      if (s) return s;
      if (host->done || k >= maxiter) break;
      chunk = predict_chunk(tol);
    }
    return TK_OK;
  }

  // geometric convergence: rms_k ~ rms_0 q^k
  int predict_chunk(double tol) const {
    int chunk = kChunk;
    const double r0 = host->rms0, rk = host->rms;
    if (host->iters > 0 && r0 > 0.0 && rk > 0.0 && rk < r0 && tol > 0.0) {
      const double lq = std::log(rk / r0) / host->iters;
      const double need = std::ceil(std::log(tol / rk) / lq);
      chunk = need < 1.0 ? 1 : need > 4.0 * kChunk ? 4 * kChunk : (int)need;
    }
    return chunk;
  }

  template <class R>
  tk_status run(const double* rhs, double tol, int maxiter, int first_chunk, bool residual) {
    return fused ? run_fused<R>(rhs, tol, maxiter, first_chunk, residual)
                 : run_tiles<R>(rhs, tol, maxiter, first_chunk, residual);
  }

  // PCG on A x = rhs, x holding the initial guess; leaves the result in x.
  // Iterations are queued in chunks with one host synchronisation per chunk:
  // the first chunk has first_chunk iterations (the previous solve's count),
  // later ones the count that the observed convergence rate predicts.
  // Iterations queued past convergence return at once.  With residual set,
  // the FP64 true residual of the final x is queued behind every chunk (it
  // runs once), so a converged solve costs one synchronisation.
  template <class R>
  tk_status run_tiles(const double* rhs, double tol, int maxiter, int first_chunk, bool residual) {
    k_pcg_init<<<1, 1, 0, st>>>(state, tol, maxiter);
    matvec_units<R>(x, nullptr);
    k_pcg_apply<0><<<nblk, kBlk, 0, st>>>(P->view(), partial, pstride, cself, alpha_s, x, rhs, q, r,
                                          z, p, part, state);
    k_pcg_finish<0><<<1, kBlk, 0, st>>>(part, nblk, state, host_dev);
    int queued = 0;
    int chunk = first_chunk > 0 ? first_chunk : kChunk;
    for (;;) {
      if (chunk > maxiter - queued) chunk = maxiter - queued;
      for (int c = 0; c < chunk; ++c) iteration<R>();
      queued += chunk;
      if (residual) queue_true_residual(rhs);
      tk_status s = sync_state();
      if (s) return s;
      if (host->done || queued >= maxiter) break;
      chunk = predict_chunk(tol);
    }
    return TK_OK;
  }

  // FP64 residual of the current x (solver already stopped).
  tk_status true_residual(const double* rhs) {
    queue_true_residual(rhs);
    return sync_state();
  }
};

// Dynamic LDS above the default limit must be allowed per kernel.
tk_status mv_attributes(size_t lds) {
  static size_t done = 0;
  if (lds <= done) return TK_OK;
  const int b = (int)lds;
  TK_HIP(hipFuncSetAttribute((const void*)k_pcg_mv<double, 0>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, b));
  TK_HIP(hipFuncSetAttribute((const void*)k_pcg_mv<double, 1>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, b));
  TK_HIP(hipFuncSetAttribute((const void*)k_pcg_mv<double, 2>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, b));
  TK_HIP(hipFuncSetAttribute((const void*)k_pcg_mv<float, 0>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, b));
  TK_HIP(hipFuncSetAttribute((const void*)k_pcg_mv<float, 1>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, b));
  done = lds;
  return TK_OK;
}

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
  S.prec = prec;
  S.gcs = (long)(P->codes.bytes / sizeof(uint32_t));
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
      (s = scratch(ctx, "pcg_state", sizeof(PcgState), &state)) ||
      (s = scratch(ctx, "pcg_gc", (prec == TK_FP64 ? sizeof(double) : sizeof(float)) * 2 * S.gcs,
                   &S.gc)))
    return s;
  // per-cell fused path: needs the cell's neighbourhood staged in LDS
  S.ncells = P->ncells;
  S.mv_lds = sizeof(double) * (6 * (size_t)P->max_nbhd + (size_t)kMvWaves * 3 * P->max_occ);
  S.fused = P->ncells > 0 && S.mv_lds + 8192 <= kMaxLds;   // + static LDS
  if (S.fused) {
    const size_t npart = sizeof(double) * 2 * (size_t)std::max(S.ncells, S.nblk);
    void *pb0, *pb1, *pz0, *pz1, *pgb;
    if ((s = scratch(ctx, "pcg_pb0", v3, &pb0)) || (s = scratch(ctx, "pcg_pb1", v3, &pb1)) ||
        (s = scratch(ctx, "pcg_pz0", npart, &pz0)) || (s = scratch(ctx, "pcg_pz1", npart, &pz1)) ||
        (s = scratch(ctx, "pcg_pg", npart, &pgb)) ||
        (s = scratch(ctx, "pcg_part2", npart, &part)))
      return s;
    S.pbuf[0] = (double*)pb0;
    S.pbuf[1] = (double*)pb1;
    S.pz[0] = (double*)pz0;
    S.pz[1] = (double*)pz1;
    S.pg = (double*)pgb;
    if ((s = mv_attributes(S.mv_lds))) return s;
  }
  S.alpha_s = (double*)alpha_s; S.b = (double*)b; S.x = (double*)x; S.r = (double*)r;
  S.z = (double*)z; S.p = (double*)p; S.q = (double*)q; S.part = (double*)part;
  S.partg = (double*)partg; S.partial = (double*)partial; S.state = (PcgState*)state;
  S.gathered = (double*)gath;
  if (unit_lds_bytes<EfieldPh<double>>(*P) > kMaxLds) return TK_E_CAPACITY;
  void *hbase, *hdev;
  if ((s = pinned(ctx, 4096, &hbase, &hdev))) return s;
  S.host = (PcgState*)((char*)hbase + 1024);
  S.host_dev = (PcgState*)((char*)hdev + 1024);

  // right-hand side: permanent field (sorted order); the same pass caches the
  // mat-vec's radial factors
  s = prec == TK_FP64 ? launch_efield<double>(ctx, st, *P, sys, mpole, polarity, thole, ewald_beta,
                                              cutoff, S.b, 1, (double*)S.gc, S.gcs)
                      : launch_efield<float>(ctx, st, *P, sys, mpole, polarity, thole, ewald_beta,
                                             cutoff, S.b, 1, (float*)S.gc, S.gcs);
  if (s) return s;
  S.gather_geometry();
  k_pcg_setup<<<S.nblk, kBlk, 0, st>>>(n, (const int32_t*)P->perm.p, polarity, mu_guess, S.b,
                                        S.alpha_s, S.x, S.part);
  k_pcg_count<<<1, kBlk, 0, st>>>(S.part, S.nblk, S.state);
  const int slot = (int)(P - ctx->plans);
  int& hint = ctx->pcg_hint[slot][prec == TK_FP64 ? 0 : 1];
  s = prec == TK_FP64 ? S.run<double>(S.b, tol_debye, maxiter, hint, true)
                      : S.run<float>(S.b, tol_debye, maxiter, hint, true);
  if (s) return s;
  const int done = S.host->done;
  hint = S.host->iters;
  info->iters = S.host->iters;
  info->rms_debye = S.host->rms;
  info->converged = done == 1;
  info->status = done == 1 ? TK_OK : done == 3 ? TK_E_BREAKDOWN : TK_E_NOCONV;
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
      if ((s = S.run<float>((double*)rt, tol_debye, maxiter, 0, false))) return s;
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
