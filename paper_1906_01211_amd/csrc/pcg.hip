// Induced dipoles by preconditioned conjugate gradient, resident on the device
// (the polarization solver of section "Hotspots": its mat-vec is the paper's
// largest hotspot and is called up to 12 times per step).
//
// A plan holds one system or a batch of independent systems; every system
// runs its own PCG (own scalars, own convergence), all of them in the same
// launches.  All solver vectors live in the plan's sorted atom order, where
// each system's cells and atoms are contiguous.
//
// The right-hand-side pass (permanent field) also stores each listed pair's
// two mutual-field radial factors, so the mat-vec only recomputes the pair
// vector and contracts it with the dipoles.  One iteration is two kernels,
// each with one workgroup per cell:
//   k_pcg_mv:     sum the system's r.z and z.z partials (fixed order, in every
//                 workgroup, so all of them take the same decisions), test
//                 convergence, beta, p = z + beta p, q = A p, partials of p.q;
//   k_cs_update:  gamma = p.q, alpha = rho/gamma, x += alpha p, r -= alpha q,
//                 z = alpha_i r, partials of r.z and z.z.
// No grid-wide fences (a device-scope fence writes back the L2 of every XCD);
// kernel boundaries order the reductions.  Every sum runs in a fixed order, so
// iterates are bitwise reproducible and do not depend on the other systems of
// a batch.  The host queues iterations in chunks and reads the mirrored
// states once per chunk; launches queued after a system has stopped return at
// once for its cells.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <vector>

#include <hip/hip_ext.h>

#include "terms.hpp"

namespace tk {
namespace {

constexpr int kChunk = 6;
constexpr int kCellThreads = 256;   // per-cell workgroups

struct PcgState {
  double rho, gamma, alpha, beta, zz, rms, rms0, rms_true, epol, tol;
  int32_t iters, done, npol, maxiter;
};
// done: 0 running, 1 converged (or not part of this solve), 2 iteration limit,
// 3 breakdown, 4 the list's build failed (nothing runs)

// Workgroup sums of N values: wave shuffles, then the waves in order.  Every
// thread gets the sums.  sh holds 16 entries per value.
template <int N>
__device__ __forceinline__ void wg_sum(double* v, double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k)
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) sh[k * 16 + w] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < N; ++k) {
    double t = 0.0;
    for (int ww = 0; ww < nw; ++ww) t += sh[k * 16 + ww];
    v[k] = t;
  }
  __syncthreads();
}

struct CellSys {   // a cell's system: index and cell range
  int sy, c0, c1;
};
__device__ __forceinline__ CellSys cell_sys_of(const PlanView& pv, int c) {
  const int sy = cell_system(pv, c);
  return CellSys{sy, pv.sys[sy].cell0, pv.sys[sy + 1].cell0};
}

// Per-cell tables of the iteration kernels, indexed by XCD position (the
// workgroup's slot in xcd_pos order), so that a workgroup starts with one
// round of independent loads instead of a chain of dependent ones.
constexpr int kEntRow = 32;   // entries per cell row: up to 27 units plus the terminator
static_assert(kCellUnitStride <= kEntRow, "cell entry rows hold every unit and the terminator");
struct MvHdr {                // 48 bytes
  int32_t c, ne, self_j, hs, nown, sy, c0, c1;   // cell, units, self entry, atoms, system range
  double box, inv_box;
};
// A cell's part in one unit: role (0 H side, 1 K side, 2 self), first sorted
// atom of the other cell, that cell's offset in the staged neighbourhood,
// codes before this unit (among the cell's units) and the unit's first code.
// Entry ne is the terminator: off = staged atoms, pre = the cell's codes.
struct MvEnt {
  int32_t role, src, off, pre;
  int64_t uoff;
};

// Per cell: alpha and the initial guesses (caller's, or alpha * b) of the nv
// right-hand sides in sorted order (vector v at offset v * 3n, the caller's
// guess in atom order likewise); count of polarizable atoms into npart[c];
// the cell's header and unit entries.
__global__ __launch_bounds__(kCellThreads) void k_cs_setup(PlanView pv, const double* __restrict__ pol,
                                                           const double* __restrict__ guess,
                                                           const int32_t* __restrict__ guess_on,
                                                           const double* __restrict__ b,
                                                           double* __restrict__ alpha_s,
                                                           double* __restrict__ x,
                                                           double* __restrict__ npart,
                                                           MvHdr* __restrict__ hdr,
                                                           MvEnt* __restrict__ ent, int nv,
                                                           DeferredSums sums, int g0) {
  __shared__ double sh[16];
  if ((int)blockIdx.x >= g0) {   // blocks past the cells: the fused pass's energy sums
    sum_finish_sys<11>(sums.cpart, pv.sys, sums.energy, sums.virial, blockIdx.x - g0);
    return;
  }
  const int pos = xcd_pos(pv.ncells, blockIdx.x);
  if (pos < 0) return;
  const int c = pv.cell_order[pos];
  const int hs = pv.cell_start[c], he = pv.cell_start[c + 1];
  const int sy = cell_system(pv, c);
  const bool use = guess && (!guess_on || guess_on[sy]);
  double cnt[1] = {0.0};
  const long vs = 3L * pv.n;
  for (int s = hs + threadIdx.x; s < he; s += kCellThreads) {
    const int i = pv.perm[s];
    const double a = pol[i];
    alpha_s[s] = a;
    cnt[0] += a > 0.0 ? 1.0 : 0.0;
    for (int v = 0; v < nv; ++v)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        x[v * vs + 3 * s + k] =
            use ? (a > 0.0 ? guess[v * vs + 3 * i + k] : 0.0) : a * b[v * vs + 3 * s + k];
  }
  if (threadIdx.x < 64) {   // wave 0: the unit entries (exclusive prefixes over the cell's units)
    const int lane = threadIdx.x;
    const int32_t* cu = pv.cell_units + (long)c * kCellUnitStride;
    const int ne = cu[0];
    int no = 0, cn = 0, role = -1, ocs = 0;
    long uoff = 0;
    if (lane < ne) {
      const int e = cu[1 + lane];
      const int u = e >> 2;
      role = e & 3;
      const Unit un = pv.units[u];
      const int oc = role == 1 ? un.h : un.k;
      ocs = pv.cell_start[oc];
      no = pv.cell_start[oc + 1] - ocs;
      cn = pv.unit_cnt[u];
      uoff = pv.unit_off[u];
    }
    int io = no, ic = cn;
    for (int o = 1; o < 64; o <<= 1) {
      const int t1 = __shfl_up(io, o), t2 = __shfl_up(ic, o);
      if (lane >= o) {
        io += t1;
        ic += t2;
      }
    }
    if (lane < kEntRow) ent[(long)pos * kEntRow + lane] = MvEnt{role, ocs, io - no, ic - cn, uoff};
    const uint64_t sm = __ballot(lane < ne && role == 2);
    if (lane == 0) {
      const SysDev& sd = pv.sys[sy];
      hdr[pos] = MvHdr{c, ne, sm ? __ffsll((long long)sm) - 1 : 0, hs, he - hs, sy,
                       sd.cell0, pv.sys[sy + 1].cell0, sd.box, sd.inv_box};
    }
  }
  wg_sum<1>(cnt, sh);
  if (threadIdx.x == 0) npart[c] = cnt[0];
}

// One block per system and right-hand side (state sy * nv + v): fresh state.
// active (device, nullable): systems outside the solve start as done.
__global__ __launch_bounds__(64) void k_cs_init(PlanView pv, const double* __restrict__ npart,
                                                PcgState* st, double tol, int maxiter,
                                                const int32_t* __restrict__ active, int nv) {
  __shared__ double sh[16];
  const int sy = blockIdx.x / nv;
  double np[1] = {0.0};
  for (int c = pv.sys[sy].cell0 + threadIdx.x; c < pv.sys[sy + 1].cell0; c += 64) np[0] += npart[c];
  wg_sum<1>(np, sh);
  if (threadIdx.x != 0) return;
  PcgState s0 = {};
  s0.npol = (int)np[0];
  s0.tol = tol;
  s0.maxiter = maxiter;
  s0.done = *pv.status != 0 ? 4 : active && !active[sy] ? 1 : 0;
  st[blockIdx.x] = s0;
}

// ---------------------------------------------------------------------------
// Per-cell mat-vec with the iteration's bookkeeping folded in.
//
// One workgroup per cell C owns C's atoms (cells in the XCD-local order of
// xcd_pos).  It walks the pair codes of all units C takes part in (each
// unordered pair is therefore visited from both of its cells) and
// accumulates only C's side.  With kStage the coordinates
// and operand of all of C's neighbour cells are staged in LDS first;
// otherwise (neighbourhoods too large for LDS) they are read from the sorted
// arrays.  Each wave keeps its own accumulator copy in LDS, summed in wave
// order, so sums are reproducible.  The epilogue applies A to C's atoms
// directly: no partial slots, no separate per-atom pass.
//
// Latency: the workgroup's global reads come in three rounds: (1) the cell
// table, the system state and the partial sums; (2) the staged
// neighbourhood, the first batch of pair codes and factors and the cell's
// own alpha and right-hand side, all issued before any of them is waited
// for; (3) the remaining pair batches.  kMulti: plans holding several
// systems (the system's state and cell range come from the cell table; with
// one system they are known without a read).
//
// kMode 0: v = x:  r = b - A x, z = alpha r; partials r.z, z.z.
// kMode 1: iteration k: convergence test on the partials of r.z and z.z
//          (and the previous r.z), beta, p_k = z_k + beta p_{k-1} as the
//          operand; outputs p_k, q = A p_k and partials of p.q.  The first
//          cell of each system records its state and mirrors it to the host.
// kMode 2: v = x (only once the system has stopped): partials of
//          |alpha (b - A x)|^2 and x.b.
//
// NV right-hand sides on the same operator (the two dipole sets): every
// per-atom vector holds NV blocks of 3n values (block v at offset v * vs),
// each with its own state (sy * NV + v), partials (block v of 2 * ncells)
// and recurrence.  A pair's code and radial factors are read once and applied
// to all NV operands; a right-hand side that has stopped keeps being
// multiplied (beta = 0) but its results are not used.  In mode 2 the second
// partial is x_v . b_(NV-1-v), the cross product that the energy of two
// dipole sets takes.
constexpr int kMvThreads = 512;    // mat-vec workgroups: 8 waves per cell
constexpr int kMvWaves = kMvThreads / 64;
// pairs, and staged atoms, per thread whose loads are issued together (two
// pairs measured fastest for one operand: 21.5 us against 22.8 with four and
// 29 with eight on the 23,559-atom water box; two operands keep two
// workgroups per CU in registers)
template <int NV>
constexpr int mv_batch() { return NV == 1 ? 2 : 2; }
template <int NV>
constexpr int mv_stage_batch() { return NV == 1 ? 3 : 2; }

// double2 slots per staged atom: x y z and NV operands, padded to 16 bytes
template <int NV>
constexpr int mv_slots() { return (3 + 3 * NV + 1) / 2; }

template <class R>
struct MvArgs {
  PlanView pv;
  const MvHdr* hdr;    // [ncells] by XCD position
  const MvEnt* ent;    // [ncells][kEntRow] by XCD position
  const R* gc;
  long gcs;
  double cself;
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
  double* part;         // [NV][2][ncells] per-cell partials
  const double* pz_cur;    // [NV][2][ncells] partials of r.z | z.z of iteration k
  const double* pz_prev;   // [NV][2][ncells] of iteration k - 1
  // full Ewald operator (one system, FP64): the PME field of the operand is
  // subtracted from A v (per right-hand side, blocks as the vectors).
  // Modes 0, 2: rz = field of x.  Mode 1: rz = field of z_k, and the field
  // of p_k = z_k + beta p_(k-1) is rz + beta rf_old (the field is linear),
  // stored in rf_new for the next iteration.
  const double* rz;
  const double* rf_old;
  double* rf_new;
  int k;
  int stage_cap, own_cap;
  long vs;              // offset between right-hand-side blocks (3n)
  PcgState* st;
  PcgState* host;
  // mode 2 only: first take the stopping test of iteration k (as mode 1
  // would), then the residual of the systems that stopped
  int check;
};

template <class R, int kMode, bool kStage, bool kMulti, int NV>
__global__ __launch_bounds__(kMvThreads) void k_pcg_mv(MvArgs<R> A) {
  constexpr int SW = mv_slots<NV>();   // double2 per staged atom
  constexpr int SD = 2 * SW;           // doubles per staged atom
  constexpr int kMvStageBatch = mv_stage_batch<NV>();
  constexpr int kMvBatch = mv_batch<NV>();
  extern __shared__ __align__(16) double lds[];
  __shared__ double red[3 * NV * 16];
  __shared__ int e_role[kEntRow], e_src[kEntRow], e_off[kEntRow], e_pre[kEntRow];
  __shared__ long e_uoff[kEntRow];
  __shared__ int s_done[NV];
  const int tid = threadIdx.x, w = tid >> 6;
  const PlanView& pv = A.pv;
  const int ncells = pv.ncells;
  const int pos = xcd_pos(ncells, blockIdx.x);
  if (pos < 0 || *pv.status != 0) return;   // no cell here, or the list's build failed
  // round 1: cell table, state, partials
  const MvHdr hd = A.hdr[pos];
  if (tid < kEntRow) {
    const MvEnt e = A.ent[(long)pos * kEntRow + tid];
    e_role[tid] = e.role;
    e_src[tid] = e.src;
    e_off[tid] = e.off;
    e_pre[tid] = e.pre;
    e_uoff[tid] = e.uoff;
  }
  const int sy = kMulti ? hd.sy : 0;
  const int c0 = kMulti ? hd.c0 : 0, c1 = kMulti ? hd.c1 : ncells;
  PcgState* st = A.st + sy * NV;
  // one read per workgroup: all its waves agree
  if (tid < NV) s_done[tid] = st[tid].done;
  const long vs = NV > 1 ? A.vs : 0;
  const long pb = 2L * ncells;   // partial block of one right-hand side
  double beta[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) beta[v] = 0.0;
  if (kMode == 1 || (kMode == 2 && A.check)) {
    const int npol_i = st->npol, maxiter = st->maxiter;
    const double tol = st->tol;
    double v3[3 * NV];
#pragma unroll
    for (int k = 0; k < 3 * NV; ++k) v3[k] = 0.0;
    for (int cc = c0 + tid; cc < c1; cc += kMvThreads) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        v3[3 * v] += A.pz_cur[v * pb + cc];
        v3[3 * v + 1] += A.pz_cur[v * pb + ncells + cc];
        if (A.k >= 1) v3[3 * v + 2] += A.pz_prev[v * pb + cc];
      }
    }
    wg_sum<3 * NV>(v3, red);   // its barriers also publish the entries and s_done
    bool run = false;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if (s_done[v]) continue;
      const double rz = v3[3 * v], zz = v3[3 * v + 1], rzp = v3[3 * v + 2];
      const double npol = npol_i > 0 ? (double)npol_i : 1.0;
      const double rms = kDebye * sqrt(zz / npol);
      const int stop = rms <= tol ? 1 : A.k >= maxiter ? 2 : 0;
      if (A.k >= 1) beta[v] = rz / rzp;
      if (hd.c == c0 && tid == 0) {
        PcgState* sv = st + v;
        sv->rho = rz;
        sv->zz = zz;
        sv->rms = rms;
        if (A.k == 0) sv->rms0 = rms;
        sv->beta = beta[v];
        sv->iters = A.k;
        if (stop) sv->done = stop;
        A.host[sy * NV + v] = *sv;
      }
      if (stop) beta[v] = 0.0;
      else run = true;
    }
    // mode 1 goes on while a system runs; mode 2 only once all have stopped
    // (its operand is x itself: every beta is zero then)
    if (kMode == 1 ? !run : run) return;
  } else {
    __syncthreads();
    bool all = true;
#pragma unroll
    for (int v = 0; v < NV; ++v) all = all && s_done[v] != 0;
    if (kMode != 2 && all) return;
    if (kMode == 2 && !all) return;
  }
  const int ne = hd.ne, hs = hd.hs, nown = hd.nown;
  const double box = hd.box, inv_box = hd.inv_box;
  const long ps = A.pstride;
  // operand v + beta * pold: for k = 0 (and modes 0, 2) beta = 0 and pold = v
  const double* pold = (kMode == 1 && A.k >= 1) ? A.pold : A.v;
  // LDS: staged atoms, SD doubles each (x y | z v0 | v1 v2 for one
  // right-hand side: 16-byte reads), then [wave][NV][3][OC] accumulators
  const int SC = kStage ? A.stage_cap : A.own_cap, OC = A.own_cap;
  double2* L2 = (double2*)lds;
  double* ACC = lds + SD * SC;
  const int own0 = kStage ? e_off[hd.self_j] : 0;
  const int total = kStage ? e_off[ne] : nown;
  const int T = e_pre[ne];
  if (total > SC || nown > OC) return;   // past the plan's LDS bounds (a failed build reports it)
  // round 2: staging loads, the first pair batch, own alpha and rhs
  int src[kMvStageBatch];
  double f[kMvStageBatch][SD];
  const auto stage_load = [&](int i0) {
#pragma unroll
    for (int m = 0; m < kMvStageBatch; ++m) {
      const int i = i0 + m * kMvThreads;
      int sidx = -1;
      if (i < total) {
        if (kStage) {
          int lo = 0, hi = ne - 1;   // last entry starting at or before i
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (e_off[mid] <= i) lo = mid;
            else hi = mid - 1;
          }
          sidx = e_src[lo] + (i - e_off[lo]);
        } else {
          sidx = hs + i;
        }
      }
      src[m] = sidx;
      if (sidx < 0) continue;
      f[m][0] = A.pos[sidx];
      f[m][1] = A.pos[ps + sidx];
      f[m][2] = A.pos[2 * ps + sidx];
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int d = 0; d < 3; ++d)
          f[m][3 + 3 * v + d] = fma(beta[v], pold[v * vs + 3 * sidx + d], A.v[v * vs + 3 * sidx + d]);
      if (SD > 3 + 3 * NV) f[m][SD - 1] = 0.0;
    }
  };
  const auto stage_store = [&](int i0) {
#pragma unroll
    for (int m = 0; m < kMvStageBatch; ++m) {
      if (src[m] < 0) continue;
      const int i = i0 + m * kMvThreads;
#pragma unroll
      for (int k = 0; k < SW; ++k) L2[SW * i + k] = make_double2(f[m][2 * k], f[m][2 * k + 1]);
    }
  };
  // pair batches: entry index, code and factors of kMvBatch pairs per thread,
  // double-buffered: batch k + 1 is loaded while batch k is processed (its
  // LDS entry reads come before batch k's LDS atomics, so they do not wait
  // for them)
  int ej[2][kMvBatch];
  uint32_t cd[2][kMvBatch];
  R g1s[2][kMvBatch], g2s[2][kMvBatch];
  int j = 0;   // entry of the thread's current pair (pairs are visited in increasing order)
  const auto batch_load = [&](int v0, int buf) {
#pragma unroll
    for (int m = 0; m < kMvBatch; ++m) {
      const int vix = v0 + m * kMvThreads;
      ej[buf][m] = -1;
      if (vix < T) {
        while (vix >= e_pre[j + 1]) ++j;
        ej[buf][m] = j;
        const long p = e_uoff[j] + (vix - e_pre[j]);
        cd[buf][m] = pv.codes[p];
        g1s[buf][m] = A.gc[p];
        g2s[buf][m] = A.gc[A.gcs + p];
      }
    }
  };
  stage_load(tid);
  batch_load(tid, 0);
  double al0 = 0.0, rhs0[NV][3];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int d = 0; d < 3; ++d) rhs0[v][d] = 0.0;
  if (tid < nown) {
    al0 = A.alpha_s[hs + tid];
    if (kMode != 1)
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int d = 0; d < 3; ++d) rhs0[v][d] = A.rhs[v * vs + 3 * (hs + tid) + d];
  }
  stage_store(tid);
  for (int i0 = tid + kMvThreads * kMvStageBatch; i0 < total; i0 += kMvThreads * kMvStageBatch) {
    stage_load(i0);
    stage_store(i0);
  }
  for (int i = tid; i < kMvWaves * 3 * NV * nown; i += kMvThreads) {
    const int ww = i / (3 * NV * nown), rem = i - ww * 3 * NV * nown;
    ACC[ww * 3 * NV * OC + rem] = 0.0;   // [ww][v][d][t] with rem = (3 v + d) * nown + t
  }
  __syncthreads();
  double* MY = ACC + w * 3 * NV * OC;   // this wave's copy: MY[(3 v + d) * nown + t]
  constexpr int kStep = kMvThreads * kMvBatch;
  const auto process = [&](int buf) {
#pragma unroll
    for (int m = 0; m < kMvBatch; ++m) {
      if (ej[buf][m] < 0) continue;
      const int role = e_role[ej[buf][m]];
      const int offs = kStage ? e_off[ej[buf][m]] : e_src[ej[buf][m]];
      const int a = (int)(cd[buf][m] & 0xffffu), b = (int)(cd[buf][m] >> 16);
      const int own = role == 1 ? b : a;
      const int oth = offs + (role == 1 ? a : b);   // LDS index, or sorted index
      const int ownL = own0 + own;
      const R g1 = g1s[buf][m], g2 = g2s[buf][m];
      double ro[SD];   // the other atom: x y z, then the NV operands
      if (kStage) {
#pragma unroll
        for (int k = 0; k < SW; ++k) {
          const double2 qk = L2[SW * oth + k];
          ro[2 * k] = qk.x;
          ro[2 * k + 1] = qk.y;
        }
      } else {
        ro[0] = A.pos[oth];
        ro[1] = A.pos[ps + oth];
        ro[2] = A.pos[2 * ps + oth];
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
          for (int d = 0; d < 3; ++d)
            ro[3 + 3 * v + d] = fma(beta[v], pold[v * vs + 3 * oth + d], A.v[v * vs + 3 * oth + d]);
      }
      const double2 w0 = L2[SW * ownL], w1 = L2[SW * ownL + 1];
      const double xw[3] = {w0.x, w0.y, w1.x};
      R dv[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double t = ro[d] - xw[d];
        dv[d] = R(fma(-box, rint(t * inv_box), t));
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const R vo[3] = {R(ro[3 + 3 * v]), R(ro[4 + 3 * v]), R(ro[5 + 3 * v])};
        const R so = (vo[0] * dv[0] + vo[1] * dv[1] + vo[2] * dv[2]) * g2;
#pragma unroll
        for (int d = 0; d < 3; ++d)
          lds_add(&MY[(3 * v + d) * nown + own], (double)(dv[d] * so - vo[d] * g1));
      }
      if (role == 2) {   // self unit: the other atom is also this cell's
        const double* rw = lds + SD * ownL;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const R va[3] = {R(rw[3 + 3 * v]), R(rw[4 + 3 * v]), R(rw[5 + 3 * v])};
          const R sa = (va[0] * dv[0] + va[1] * dv[1] + va[2] * dv[2]) * g2;
#pragma unroll
          for (int d = 0; d < 3; ++d)
            lds_add(&MY[(3 * v + d) * nown + b], (double)(dv[d] * sa - va[d] * g1));
        }
      }
    }
  };
  // two batches per trip, so that the buffer index is a constant
  for (int v0 = tid; v0 < T; v0 += 2 * kStep) {
    if (v0 + kStep < T) batch_load(v0 + kStep, 1);
    process(0);
    if (v0 + kStep >= T) break;
    if (v0 + 2 * kStep < T) batch_load(v0 + 2 * kStep, 0);
    process(1);
  }
  __syncthreads();
  double sv[2 * NV];
#pragma unroll
  for (int k = 0; k < 2 * NV; ++k) sv[k] = 0.0;
  for (int t = tid; t < nown; t += kMvThreads) {
    const int s = hs + t;
    const bool first = t == tid;   // alpha and rhs already loaded in round 2
    const double al = first ? al0 : A.alpha_s[s];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const long o = v * vs + 3 * s;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        double fs = 0.0;
#pragma unroll
        for (int ww = 0; ww < kMvWaves; ++ww) fs += ACC[ww * 3 * NV * OC + (3 * v + d) * nown + t];
        const double vv = lds[SD * (own0 + t) + 3 + 3 * v + d];
        double av = al > 0.0 ? vv / al - (fs + A.cself * vv) : 0.0;   // (A v)_s
        if (A.rz) {
          double rf = A.rz[o + d];
          if (kMode == 1) {
            if (A.k >= 1) rf = fma(beta[v], A.rf_old[o + d], rf);
            A.rf_new[o + d] = rf;
          }
          if (al > 0.0) av -= rf;
        }
        if (kMode == 1) {
          A.pnew[o + d] = vv;
          A.q[o + d] = av;
          sv[2 * v] += vv * av;
        } else {
          const double bb = first ? rhs0[v][d] : A.rhs[o + d];
          const double rr = al > 0.0 ? bb - av : 0.0;
          const double zz = al * rr;
          if (kMode == 0) {
            A.r[o + d] = rr;
            A.z[o + d] = zz;
            sv[2 * v] += rr * zz;
            sv[2 * v + 1] += zz * zz;
          } else {
            const int u = NV - 1 - v;   // the other right-hand side (itself for NV = 1)
            const double bu = first ? rhs0[u][d] : A.rhs[u * vs + 3 * s + d];
            sv[2 * v] += zz * zz;
            sv[2 * v + 1] += vv * bu;
          }
        }
      }
    }
  }
  wg_sum<2 * NV>(sv, red);
  if (tid == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      A.part[v * pb + hd.c] = sv[2 * v];
      if (kMode != 1) A.part[v * pb + ncells + hd.c] = sv[2 * v + 1];
    }
  }
}

// Iteration k, second half, per cell: gamma = p.q and rho_k from the
// system's partials (fixed order, in every workgroup), alpha = rho/gamma,
// x += alpha p, r -= alpha q, z = alpha_i r; partials of r.z and z.z for
// iteration k + 1.  The cell's atoms are read in the same round as the
// partials (before alpha is known).  NV right-hand sides as in k_pcg_mv;
// one that has stopped is left as it is.
template <bool kMulti, int NV>
__global__ __launch_bounds__(kCellThreads) void k_cs_update(
    PlanView pv, const MvHdr* __restrict__ hdr, const double* __restrict__ alpha_s,
    const double* __restrict__ p, const double* __restrict__ q, double* __restrict__ x,
    double* __restrict__ r, double* __restrict__ z, const double* __restrict__ pg,
    const double* __restrict__ pz_cur, double* __restrict__ pz_next, int k, PcgState* states,
    PcgState* host, long vs_) {
  __shared__ double sh[2 * NV * 16];
  __shared__ int s_done[NV];
  const int ncells = pv.ncells;
  const int pos = xcd_pos(ncells, blockIdx.x);
  if (pos < 0) return;
  const MvHdr hd = hdr[pos];
  const int sy = kMulti ? hd.sy : 0;
  const int c0 = kMulti ? hd.c0 : 0, c1 = kMulti ? hd.c1 : ncells;
  PcgState* st = states + sy * NV;
  const long vs = NV > 1 ? vs_ : 0;
  const long pb = 2L * ncells;
  // one read per workgroup: all its waves agree
  if (threadIdx.x < NV) s_done[threadIdx.x] = st[threadIdx.x].done;
  double g2[2 * NV];
#pragma unroll
  for (int k2 = 0; k2 < 2 * NV; ++k2) g2[k2] = 0.0;
  for (int cc = c0 + threadIdx.x; cc < c1; cc += kCellThreads) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      g2[2 * v] += pg[v * pb + cc];
      g2[2 * v + 1] += pz_cur[v * pb + cc];
    }
  }
  const int hs = hd.hs, nown = hd.nown;
  const int t0 = threadIdx.x;
  double a0 = 0.0, p0[NV][3], q0[NV][3], x0[NV][3], r0[NV][3];
  if (t0 < nown) {
    const int s = hs + t0;
    a0 = alpha_s[s];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const long e = v * vs + 3 * s + d;
        p0[v][d] = p[e];
        q0[v][d] = q[e];
        x0[v][d] = x[e];
        r0[v][d] = r[e];
      }
  }
  wg_sum<2 * NV>(g2, sh);   // its barriers also publish s_done
  const bool lead = hd.c == c0 && threadIdx.x == 0;
  bool on[NV], any = false;
  double al[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    on[v] = !s_done[v];
    al[v] = 0.0;
    if (!on[v]) continue;
    const double gam = g2[2 * v], rho = g2[2 * v + 1];
    if (!(gam > 0.0)) {   // p.Ap <= 0: not positive definite
      if (lead) {
        st[v].gamma = gam;
        st[v].iters = k;
        st[v].done = 3;
        host[sy * NV + v] = st[v];
      }
      on[v] = false;
      continue;
    }
    al[v] = rho / gam;
    if (lead) {
      st[v].gamma = gam;
      st[v].alpha = al[v];
    }
    any = true;
  }
  if (!any) return;
  double sv[2 * NV];
#pragma unroll
  for (int k2 = 0; k2 < 2 * NV; ++k2) sv[k2] = 0.0;
  for (int t = t0; t < nown; t += kCellThreads) {
    const int s = hs + t;
    const bool first = t == t0;
    const double a = first ? a0 : alpha_s[s];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if (!on[v]) continue;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const long e = v * vs + 3 * s + d;
        x[e] = (first ? x0[v][d] : x[e]) + al[v] * (first ? p0[v][d] : p[e]);
        const double rr = (first ? r0[v][d] : r[e]) - al[v] * (first ? q0[v][d] : q[e]);
        r[e] = rr;
        const double zz = a * rr;
        z[e] = zz;
        sv[2 * v] += rr * zz;
        sv[2 * v + 1] += zz * zz;
      }
    }
  }
  wg_sum<2 * NV>(sv, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if (!on[v]) continue;
      pz_next[v * pb + hd.c] = sv[2 * v];
      pz_next[v * pb + ncells + hd.c] = sv[2 * v + 1];
    }
  }
}

// Per cell, from mat-vec partial slots (the FP64 on-the-fly mat-vec of the
// mixed form): the atom's (A v)_s = v_s/alpha_s - (field_s + c v_s).
// kMode 0: r = b - A x, z = alpha r (refinement right-hand side).
// kMode 2: partials |alpha (b - A x)|^2 and x.b (only for stopped systems).
template <int kMode>
__global__ __launch_bounds__(kCellThreads) void k_cs_apply(PlanView pv,
                                                           const double* __restrict__ partial,
                                                           long pstride, double cself,
                                                           const double* __restrict__ alpha_s,
                                                           const double* __restrict__ v,
                                                           const double* __restrict__ b,
                                                           double* __restrict__ r,
                                                           double* __restrict__ z,
                                                           double* __restrict__ part,
                                                           const PcgState* __restrict__ states) {
  __shared__ double sh[2 * 16];
  __shared__ int s_done;
  const int c = blockIdx.x, ncells = gridDim.x;
  const CellSys cs = cell_sys_of(pv, c);
  if (threadIdx.x == 0) s_done = states[cs.sy].done;
  __syncthreads();
  if (kMode == 2 && !s_done) return;
  const int hs = pv.cell_start[c], he = pv.cell_start[c + 1];
  const int ns = pv.cell_nslot[c];
  double sv[2] = {0.0, 0.0};
  for (int s = hs + threadIdx.x; s < he; s += kCellThreads) {
    double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < kMaxSlots; ++k)   // unrolled: all slot loads in flight at once
      if (k < ns)
#pragma unroll
        for (int d = 0; d < 3; ++d) acc[d] += partial[((long)k * 3 + d) * pstride + s];
    const double a = alpha_s[s];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double vv = v[3 * s + d];
      const double av = a > 0.0 ? vv / a - (acc[d] + cself * vv) : 0.0;
      const double rr = a > 0.0 ? b[3 * s + d] - av : 0.0;
      const double zz = a * rr;
      if (kMode == 0) {
        r[3 * s + d] = rr;
        z[3 * s + d] = zz;
      } else {
        sv[0] += zz * zz;
        sv[1] += vv * b[3 * s + d];
      }
    }
  }
  if (kMode == 2) {
    wg_sum<2>(sv, sh);
    if (threadIdx.x == 0) {
      part[c] = sv[0];
      part[ncells + c] = sv[1];
    }
  }
}

// Outcome of a queued solve (tk_polarize_pcg_queued): the same fields and
// rules as the synchronous call's host result; the mixed form's outcome is
// its FP64 check.
__device__ tk_pcg_info pcg_info_of(const PcgState& h, int mixed) {
  tk_pcg_info r{};
  r.iters = h.iters;
  r.refinements = 0;
  r.rms_debye = h.rms;
  r.rms_true_debye = h.rms_true;
  r.epol = h.epol;
  if (h.done == 3 || h.done == 4) {
    r.status = h.done == 3 ? TK_E_BREAKDOWN : TK_E_CAPACITY;
    r.converged = 0;
  } else {
    const bool ok = mixed ? h.done != 0 && h.rms_true <= h.tol : h.done == 1;
    r.status = ok ? TK_OK : TK_E_NOCONV;
    r.converged = ok ? 1 : 0;
  }
  return r;
}

// One block per system and right-hand side (state sy * nv + v): true-residual
// RMS and E_pol = -C/2 x_v.b_(nv-1-v) from the per-cell partials; mirrored to
// the host.  Only once every right-hand side of the system has stopped.
// info (nullable, device): the queued solve's outcome, one per state.
__global__ __launch_bounds__(64) void k_cs_finish_true(PlanView pv, const double* __restrict__ part,
                                                       PcgState* states, PcgState* host, int nv,
                                                       tk_pcg_info* __restrict__ info,
                                                       int mixed) {
  __shared__ double sh[2 * 16];
  __shared__ int s_done;
  const int sy = blockIdx.x / nv, vi = blockIdx.x - sy * nv;
  const int ncells = pv.ncells;
  PcgState* st = states + blockIdx.x;
  if (threadIdx.x == 0) {
    int all = 1;
    for (int u = 0; u < nv; ++u) all &= states[sy * nv + u].done != 0;
    s_done = all;
  }
  __syncthreads();
  if (!s_done) {
    if (info && threadIdx.x == 0) info[blockIdx.x] = pcg_info_of(*st, mixed);
    return;
  }
  const double* pv_part = part + vi * 2L * ncells;
  double v[2] = {0.0, 0.0};
  for (int c = pv.sys[sy].cell0 + threadIdx.x; c < pv.sys[sy + 1].cell0; c += 64) {
    v[0] += pv_part[c];
    v[1] += pv_part[ncells + c];
  }
  wg_sum<2>(v, sh);
  if (threadIdx.x != 0) return;
  const double npol = st->npol > 0 ? (double)st->npol : 1.0;
  st->rms_true = kDebye * sqrt(v[0] / npol);
  st->epol = -0.5 * kCoulomb * v[1];
  host[blockIdx.x] = *st;
  if (info) info[blockIdx.x] = pcg_info_of(*st, mixed);
}

__global__ void k_pcg_info_empty(tk_pcg_info v, tk_pcg_info* __restrict__ out) { *out = v; }

// Refinement: keep x in dx and start the correction from z (= alpha r_t) for
// the systems being refined.
__global__ void k_refine_begin(PlanView pv, const int32_t* __restrict__ active,
                               double* __restrict__ x, double* __restrict__ dx,
                               const double* __restrict__ z) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= pv.n) return;
  const bool on = active[cell_system(pv, pv.scell[s])] != 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    dx[3 * s + d] = x[3 * s + d];
    if (on) x[3 * s + d] = z[3 * s + d];
  }
}

// x = dx + correction (refined systems) or dx (the others).
__global__ void k_refine_end(PlanView pv, const int32_t* __restrict__ active,
                             double* __restrict__ x, const double* __restrict__ dx) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= pv.n) return;
  const bool on = active[cell_system(pv, pv.scell[s])] != 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) x[3 * s + d] = on ? dx[3 * s + d] + x[3 * s + d] : dx[3 * s + d];
}

// (nothing written when the list's build failed: status nonzero)
__global__ void k_scatter_out(int n, const int32_t* __restrict__ perm, const double* __restrict__ x,
                              double* __restrict__ out, const int32_t* __restrict__ status) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n || *status != 0) return;
  const int i = perm[s];
#pragma unroll
  for (int c = 0; c < 3; ++c) out[3 * i + c] = x[3 * s + c];
}

template <class R, int kMode, bool kStage>
tk_status set_lds_attr(size_t lds) {
  TK_HIP(hipFuncSetAttribute((const void*)k_pcg_mv<R, kMode, kStage, false, 1>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  TK_HIP(hipFuncSetAttribute((const void*)k_pcg_mv<R, kMode, kStage, true, 1>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  if constexpr (std::is_same<R, double>::value)   // two right-hand sides: FP64, one system
    TK_HIP(hipFuncSetAttribute((const void*)k_pcg_mv<R, kMode, kStage, false, 2>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  return TK_OK;
}

// Dynamic LDS above the default limit must be allowed per kernel.
// (Process-wide: several contexts on several host threads share it.)
tk_status mv_attributes(size_t lds) {
  static std::mutex m;
  static size_t done = 0;
  std::lock_guard<std::mutex> lk(m);
  if (lds <= done) return TK_OK;
  tk_status s;
  if ((s = set_lds_attr<double, 0, true>(lds)) || (s = set_lds_attr<double, 1, true>(lds)) ||
      (s = set_lds_attr<double, 2, true>(lds)) || (s = set_lds_attr<float, 0, true>(lds)) ||
      (s = set_lds_attr<float, 1, true>(lds)) || (s = set_lds_attr<double, 0, false>(lds)) ||
      (s = set_lds_attr<double, 1, false>(lds)) || (s = set_lds_attr<double, 2, false>(lds)) ||
      (s = set_lds_attr<float, 0, false>(lds)) || (s = set_lds_attr<float, 1, false>(lds)))
    return s;
  done = lds;
  return TK_OK;
}

struct Solver {
  tk_ctx* ctx;
  hipStream_t st;
  const Plan* P;
  PlanView pv;
  const double* xyz;
  const int32_t* molid;
  const double* polarity;
  const double* thole;
  double beta, cutoff, cself;
  int prec, nsys, ncells;
  long pstride;
  double *alpha_s, *b, *x, *r, *z, *q, *partial, *gathered, *npart, *part, *dx, *rt;
  double* pbuf[2];   // search directions p_k (k even, odd)
  double* pz[2];     // partials of r.z | z.z (k even, odd)
  double* pg;        // partials of p.q
  MvHdr* hdr;        // per-cell tables of the iteration kernels
  MvEnt* ent;
  void* gc;          // cached radial factors g1 | g2 per pair code (solver precision)
  long gcs;
  bool stage;
  size_t mv_lds;
  PcgState* state;      // [nsys]
  PcgState* host;       // [nsys] pinned host mirror
  PcgState* host_dev;   // its device address
  int32_t* active;      // [nsys] device copy of the refinement mask
  int32_t* active_h;    // pinned staging of the mask
  int nv = 1;     // right-hand sides (2: FP64, one system, no reciprocal part)
  long vs = 0;    // offset between right-hand-side blocks of a vector (3n)
  int pme_grid = 0, pme_order = 0;   // full Ewald operator (one system, FP64) when set
  double* rz = nullptr;              // PME field of the current operand
  tk_pcg_info* info_out = nullptr;   // queued solve: its outcome (device), by the FP64 residual
  double* rfb[2] = {nullptr, nullptr};   // PME field of p_k (k even, odd)

  // PME field of v (sorted) into rz, per right-hand side; run_when_done as
  // the iteration kernels, on that right-hand side's state: 0 while it
  // runs, 1 for its stopped solve's residual, -1 always
  tk_status queue_pme(const double* v, int run_when_done) {
    if (!pme_grid) return TK_OK;
    const auto done_of = [&](int k) {
      return run_when_done < 0
                 ? nullptr
                 : (const int32_t*)((const char*)(state + k) + offsetof(PcgState, done));
    };
    if (nv == 2)   // both sets through one packed pass
      return pme_prepared_dipole_field2(ctx, st, P->n, P->box, v, v + vs, beta, pme_grid,
                                        pme_order, rz, rz + vs, done_of(0), done_of(1),
                                        run_when_done < 0 ? 0 : run_when_done);
    for (int k = 0; k < nv; ++k) {
      const int32_t* done =
          run_when_done < 0 ? nullptr
                            : (const int32_t*)((const char*)(state + k) + offsetof(PcgState, done));
      const tk_status s = pme_prepared_dipole_field(ctx, st, P->n, P->box, v + k * vs, beta,
                                                    pme_grid, pme_order, rz + k * vs, done,
                                                    run_when_done < 0 ? 0 : run_when_done);
      if (s) return s;
    }
    return TK_OK;
  }

  template <class R>
  MvArgs<R> mv_args() const {
    MvArgs<R> a = {};
    a.pv = pv;
    a.hdr = hdr;
    a.ent = ent;
    a.gc = (const R*)gc;
    a.gcs = gcs;
    a.cself = cself;
    a.pos = gathered;
    a.pstride = pstride;
    a.alpha_s = alpha_s;
    a.stage_cap = P->max_nbhd;
    a.own_cap = P->max_occ;
    a.vs = vs;
    a.st = state;
    a.host = host_dev;
    return a;
  }

  template <class R, int kMode>
  void launch_mv(const MvArgs<R>& a, const char* name) {
    // when profiled, the launch itself records its start and stop events
    ProfScope ps(ctx, st, std::string(name) + prec_tag<R>(), true);
    const dim3 g(xcd_grid(ncells)), b(kMvThreads);
    const auto go = [&](void (*kern)(MvArgs<R>)) {
      if (ps.start())
        hipExtLaunchKernelGGL(kern, g, b, (uint32_t)mv_lds, st, ps.start(), ps.stop(), 0u, a);
      else
        hipLaunchKernelGGL(kern, g, b, mv_lds, st, a);
    };
    if constexpr (std::is_same<R, double>::value) {
      if (nv == 2) {
        go(stage ? k_pcg_mv<R, kMode, true, false, 2> : k_pcg_mv<R, kMode, false, false, 2>);
        return;
      }
    }
    if (nsys > 1)
      go(stage ? k_pcg_mv<R, kMode, true, true, 1> : k_pcg_mv<R, kMode, false, true, 1>);
    else
      go(stage ? k_pcg_mv<R, kMode, true, false, 1> : k_pcg_mv<R, kMode, false, false, 1>);
  }

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
    a.pz_prev = pz[(k + 1) & 1];
    a.k = k;
    if (pme_grid) {
      a.rz = rz;
      a.rf_old = rfb[(k + 1) & 1];
      a.rf_new = rfb[k & 1];
    }
    launch_mv<R, 1>(a, nv == 2 ? "pcg2_mv" : "pcg_mv");
  }

  // iteration k, second half: update x, r, z
  void queue_update(int k) {
    ProfScope ps(ctx, st, nv == 2 ? "pcg2_update" : "pcg_update");
    const int g = xcd_grid(ncells);
    if (nv == 2)
      k_cs_update<false, 2><<<g, kCellThreads, 0, st>>>(pv, hdr, alpha_s, pbuf[k & 1], q, x, r, z,
                                                        pg, pz[k & 1], pz[(k + 1) & 1], k, state,
                                                        host_dev, vs);
    else if (nsys > 1)
      k_cs_update<true, 1><<<g, kCellThreads, 0, st>>>(pv, hdr, alpha_s, pbuf[k & 1], q, x, r, z,
                                                       pg, pz[k & 1], pz[(k + 1) & 1], k, state,
                                                       host_dev, vs);
    else
      k_cs_update<false, 1><<<g, kCellThreads, 0, st>>>(pv, hdr, alpha_s, pbuf[k & 1], q, x, r, z,
                                                        pg, pz[k & 1], pz[(k + 1) & 1], k, state,
                                                        host_dev, vs);
  }

  // TmatPh for the on-the-fly FP64 mat-vec of the mixed form
  TmatPh<double> tmat64(const double* v) const {
    TmatPh<double> ph;
    ph.xyz = xyz;
    ph.mu = v;
    ph.mu_sorted = 1;
    ph.polarity = polarity;
    ph.thole = thole;
    ph.molid = molid;
    ph.g.set(P->box, cutoff, beta);
    ph.sorted = gathered;
    ph.gstride = pstride;
    ph.perm_ = (const int32_t*)P->perm.p;
    return ph;
  }

  // Static per-atom fields of the mixed form's mat-vecs, gathered once per
  // solve: the coordinates and the damping fields of the on-the-fly FP64
  // mat-vec.  (The FP64 form reuses the coordinates that the permanent-field
  // pass gathered: fields 0-2 of its sorted SoA rows, same stride.)
  void gather_geometry() {
    TmatPh<double> ph = tmat64(nullptr);
    k_gather<TmatPh<double>><<<ceil_div(P->n, 256), 256, 0, st>>>(pv, ph, gathered, pstride);
  }

  // FP64 mat-vec of v on the fly into the partial slots (mixed form)
  void matvec64_tiles(const double* v) {
    TmatPh<double> ph = tmat64(v);
    ProfScope ps(ctx, st, "units_tmat_fp64");
    launch_units(*P, ph, partial, pstride, nullptr, st);
  }

  // FP64 residual of x against rhs (rms_true, and epol from x.rhs), queued
  // behind the iterations; its kernels run only for stopped systems.  With
  // check_k >= 0 (FP64 path, no PME), the residual launch first takes the
  // stopping test of iteration check_k, in place of that iteration's own
  // mat-vec launch (which would only find the stop).
  void queue_true_residual(const double* rhs, int check_k = -1) {
    if (prec == TK_FP64) {
      MvArgs<double> a = mv_args<double>();
      a.v = x;
      a.pold = x;
      a.rhs = rhs;
      a.part = part;
      if (check_k >= 0) {
        a.check = 1;
        a.k = check_k;
        a.pz_cur = pz[check_k & 1];
        a.pz_prev = pz[(check_k + 1) & 1];
      }
      if (pme_grid) {
        queue_pme(x, 1);
        a.rz = rz;
      }
      launch_mv<double, 2>(a, nv == 2 ? "pcg2_mv_residual" : "pcg_mv_residual");
    } else {
      matvec64_tiles(x);
      k_cs_apply<2><<<ncells, kCellThreads, 0, st>>>(pv, partial, pstride, cself, alpha_s, x, rhs,
                                                     nullptr, nullptr, part, state);
    }
    k_cs_finish_true<<<nsys * nv, 64, 0, st>>>(pv, part, state, host_dev, nv, info_out,
                                                prec == TK_MIXED ? 1 : 0);
  }

  tk_status sync_state() {
    TK_HIP(hipGetLastError());
    TK_HIP(hipStreamSynchronize(st));
    return TK_OK;
  }

  bool all_stopped() const {
    for (int k = 0; k < nsys * nv; ++k)
      if (!host[k].done) return false;
    return true;
  }

  // geometric convergence of the slowest running system: rms_k ~ rms_0 q^k
  int predict_chunk(double tol) const {
    int chunk = 1;
    for (int k = 0; k < nsys * nv; ++k) {
      const PcgState& h = host[k];
      if (h.done) continue;
      int c = kChunk;
      if (h.iters > 0 && h.rms0 > 0.0 && h.rms > 0.0 && h.rms < h.rms0 && tol > 0.0) {
        const double lq = std::log(h.rms / h.rms0) / h.iters;
        const double need = std::ceil(std::log(tol / h.rms) / lq);
        c = need < 1.0 ? 1 : need > 4.0 * kChunk ? 4 * kChunk : (int)need;
      }
      chunk = std::max(chunk, c);
    }
    return chunk;
  }

  // PCG on A x = rhs for every system (or the active ones), x holding the
  // initial guess; leaves the result in x.  Iterations are queued in chunks
  // with one host synchronisation per chunk: the first chunk has
  // first_chunk iterations (the previous solve's count), later ones the
  // count that the observed convergence rates predict.  With residual set,
  // the FP64 true residual is queued behind every chunk (it runs once per
  // system), so a converged solve costs one synchronisation.
  template <class R>
  tk_status run(const double* rhs, double tol, int maxiter, int first_chunk, bool residual,
                const int32_t* act) {
    k_cs_init<<<nsys * nv, 64, 0, st>>>(pv, npart, state, tol, maxiter, act, nv);
    tk_status s0;
    {
      MvArgs<R> a = mv_args<R>();
      a.v = x;
      a.pold = x;
      a.rhs = rhs;
      a.r = r;
      a.z = z;
      a.part = pz[0];
      if (pme_grid) {
        if ((s0 = queue_pme(x, -1))) return s0;
        a.rz = rz;
      }
      launch_mv<R, 0>(a, nv == 2 ? "pcg2_mv0" : "pcg_mv0");
    }
    if ((s0 = queue_pme(z, 0))) return s0;
    queue_mv<R>(0);
    int k = 0;   // index of the last queued first half
    int chunk = first_chunk > 0 ? first_chunk : kChunk;
    for (;;) {
      if (chunk > maxiter - k) chunk = maxiter - k;
      for (int c = 0; c < chunk; ++c) {
        queue_update(k);
        if ((s0 = queue_pme(z, 0))) return s0;
        queue_mv<R>(++k);
      }
      if (residual) queue_true_residual(rhs);
      tk_status s = sync_state();
      if (s) return s;
      if (all_stopped() || k >= maxiter) break;
      chunk = predict_chunk(tol);
    }
    return TK_OK;
  }

  // The same iteration, `iters` updates queued with no host synchronisation
  // (launches after convergence return at once), then the FP64 true
  // residual.  The state stays on the device.
  template <class R>
  void run_queued(const double* rhs, double tol, int iters) {
    k_cs_init<<<nsys * nv, 64, 0, st>>>(pv, npart, state, tol, iters, nullptr, nv);
    {
      MvArgs<R> a = mv_args<R>();
      a.v = x;
      a.pold = x;
      a.rhs = rhs;
      a.r = r;
      a.z = z;
      a.part = pz[0];
      launch_mv<R, 0>(a, "pcg_mv0");
    }
    queue_mv<R>(0);
    // FP64: the last stopping test rides on the residual launch
    const bool fold = prec == TK_FP64 && !pme_grid && nv == 1;
    for (int k = 0; k < iters;) {
      queue_update(k);
      if (++k < iters || !fold) queue_mv<R>(k);
    }
    queue_true_residual(rhs, fold ? iters : -1);
  }
};

}  // namespace

tk_status solve_dipoles(tk_ctx* ctx, hipStream_t st, const Plan* P, const double* xyz,
                        const int32_t* molid, const double* mpole, const double* polarity,
                        const double* thole, double ewald_beta, double cutoff, double tol_debye,
                        int32_t maxiter, int prec, const double* mu_guess,
                        const int32_t* guess_on, double* mu_out, tk_pcg_info* info,
                        int pme_grid, int pme_order, int nv, double pscale, double* mp_energy,
                        double* mp_force, double* mp_virial, int32_t queued,
                        tk_pcg_info* info_dev) {
  const int nsys = P->nsys;
  if (pme_grid && (prec != TK_FP64 || nsys != 1 || !pme_args_ok(pme_grid, pme_order)))
    return TK_E_ARG;
  if (nv != 1 && (nv != 2 || prec != TK_FP64 || nsys != 1)) return TK_E_ARG;
  if (queued && (nv != 1 || pme_grid || nsys != 1 || !info_dev)) return TK_E_ARG;
  if (!queued)
    for (int k = 0; k < nsys * nv; ++k) info[k] = tk_pcg_info{};
  const int n = P->n;
  if (n == 0) {
    if (!queued)
      for (int k = 0; k < nsys * nv; ++k) info[k].converged = 1;
    return TK_OK;   // (the queued entry point writes the empty system's outcome itself)
  }
  Solver S;
  S.ctx = ctx;
  S.st = st;
  S.P = P;
  S.pv = P->view();
  S.xyz = xyz;
  S.molid = molid;
  S.polarity = polarity;
  S.thole = thole;
  S.beta = ewald_beta;
  S.cutoff = cutoff;
  S.cself = 4.0 * ewald_beta * ewald_beta * ewald_beta / (3.0 * kSqrtPi);
  S.prec = prec;
  S.nsys = nsys;
  S.ncells = P->ncells;
  S.nv = nv;
  S.vs = 3L * n;
  S.pstride = pad64(n);
  S.gcs = (long)(P->codes.bytes / sizeof(uint32_t));
  // stage whole neighbourhoods in LDS when they fit, else only the own cell
  const size_t acc = (size_t)kMvWaves * 3 * nv * P->max_occ;
  const size_t sd = nv == 2 ? 2 * mv_slots<2>() : 2 * mv_slots<1>();   // doubles per staged atom
  S.stage = sizeof(double) * (sd * (size_t)P->max_nbhd + acc) + 4096 <= kMaxLds;
  S.mv_lds = sizeof(double) * (sd * (size_t)(S.stage ? P->max_nbhd : P->max_occ) + acc);
  if (S.mv_lds + 4096 > kMaxLds) return TK_E_CAPACITY;   // a cell beyond the LDS limit
  const size_t v3 = sizeof(double) * 3 * (size_t)n * nv;
  const size_t npc = sizeof(double) * 2 * (size_t)S.ncells * nv;
  tk_status s;
  void *alpha_s, *b, *x, *r, *z, *q, *partial = nullptr, *gath, *npart, *part, *dx, *rt, *pb0,
       *pb1, *pz0, *pz1, *pg, *state, *act, *hdr, *ent;
  if ((s = scratch(ctx, "pcg_alpha", sizeof(double) * n, &alpha_s)) ||
      (s = scratch(ctx, "pcg_b", v3, &b)) || (s = scratch(ctx, "pcg_x", v3, &x)) ||
      (s = scratch(ctx, "pcg_r", v3, &r)) || (s = scratch(ctx, "pcg_z", v3, &z)) ||
      (s = scratch(ctx, "pcg_q", v3, &q)) || (s = scratch(ctx, "pcg_dx", v3, &dx)) ||
      (s = scratch(ctx, "pcg_rt", v3, &rt)) || (s = scratch(ctx, "pcg_pb0", v3, &pb0)) ||
      (s = scratch(ctx, "pcg_pb1", v3, &pb1)) ||
      (s = scratch(ctx, "pcg_npart", sizeof(double) * S.ncells, &npart)) ||
      (s = scratch(ctx, "pcg_part", npc, &part)) || (s = scratch(ctx, "pcg_pz0", npc, &pz0)) ||
      (s = scratch(ctx, "pcg_pz1", npc, &pz1)) || (s = scratch(ctx, "pcg_pg", npc, &pg)) ||
      (s = scratch(ctx, "pcg_gathered", sizeof(double) * TmatPh<double>::NG * S.pstride, &gath)) ||
      (s = scratch(ctx, "pcg_state", sizeof(PcgState) * nsys * nv, &state)) ||
      (s = scratch(ctx, "pcg_hdr", sizeof(MvHdr) * S.ncells, &hdr)) ||
      (s = scratch(ctx, "pcg_ent", sizeof(MvEnt) * kEntRow * S.ncells, &ent)) ||
      (s = scratch(ctx, "pcg_active", sizeof(int32_t) * nsys, &act)) ||
      (s = scratch(ctx, "pcg_gc", (prec == TK_FP64 ? sizeof(double) : sizeof(float)) * 2 * S.gcs,
                   &S.gc)))
    return s;
  S.alpha_s = (double*)alpha_s; S.b = (double*)b; S.x = (double*)x; S.r = (double*)r;
  S.z = (double*)z; S.q = (double*)q; S.dx = (double*)dx; S.rt = (double*)rt;
  S.gathered = (double*)gath; S.npart = (double*)npart; S.part = (double*)part;
  S.pbuf[0] = (double*)pb0; S.pbuf[1] = (double*)pb1;
  S.pz[0] = (double*)pz0; S.pz[1] = (double*)pz1; S.pg = (double*)pg;
  S.state = (PcgState*)state;
  S.active = (int32_t*)act;
  S.hdr = (MvHdr*)hdr;
  S.ent = (MvEnt*)ent;
  if (pme_grid) {
    void *rz, *rf0, *rf1;
    if ((s = scratch(ctx, "pcg_rz", v3, &rz)) || (s = scratch(ctx, "pcg_rf0", v3, &rf0)) ||
        (s = scratch(ctx, "pcg_rf1", v3, &rf1)))
      return s;
    S.pme_grid = pme_grid;
    S.pme_order = pme_order;
    S.rz = (double*)rz;
    S.rfb[0] = (double*)rf0;
    S.rfb[1] = (double*)rf1;
  }
  if (unit_lds_bytes<EfieldPh<double>>(*P, 1) > kMaxLds) return TK_E_CAPACITY;
  if ((s = mv_attributes(S.mv_lds))) return s;
  const size_t mirror = sizeof(PcgState) * nsys * nv;
  if (queued) {
    // no host reads: the kernels' state mirror goes to device scratch (the
    // context's pinned buffer may be reallocated by a later call while these
    // kernels are still queued)
    void* m;
    if ((s = scratch(ctx, "pcg_mirror", mirror, &m))) return s;
    S.host = nullptr;
    S.host_dev = (PcgState*)m;
    S.active_h = nullptr;
  } else {
    // pinned: [1024, ...) host state mirrors, then the refinement mask
    void *hbase, *hdev;
    if ((s = pinned(ctx, 1024 + mirror + sizeof(int32_t) * nsys + 64, &hbase, &hdev))) return s;
    S.host = (PcgState*)((char*)hbase + 1024);
    S.host_dev = (PcgState*)((char*)hdev + 1024);
    S.active_h = (int32_t*)((char*)hbase + 1024 + mirror);
  }

  // right-hand side: permanent field (sorted order); the same pass caches
  // the mat-vec's radial factors
  const tk_system sys1{n, xyz, P->box, molid};
  // (the multipole pass's energy and virial sums are finished by the setup
  // kernel below, one launch fewer)
  DeferredSums sums;
  if (mp_energy)   // with the multipole energy, forces and virial from the same pass
    s = prec == TK_FP64
            ? launch_mpole_field<double>(ctx, st, *P, &sys1, mpole, polarity, thole, ewald_beta,
                                         cutoff, mp_energy, mp_force, mp_virial, S.b,
                                         (double*)S.gc, S.gcs, &sums)
            : launch_mpole_field<float>(ctx, st, *P, &sys1, mpole, polarity, thole, ewald_beta,
                                        cutoff, mp_energy, mp_force, mp_virial, S.b,
                                        (float*)S.gc, S.gcs, &sums);
  else
    s = prec == TK_FP64 ? launch_efield<double>(ctx, st, *P, &sys1, mpole, polarity, thole,
                                                ewald_beta, cutoff, S.b, 1, (double*)S.gc, S.gcs)
                        : launch_efield<float>(ctx, st, *P, &sys1, mpole, polarity, thole,
                                               ewald_beta, cutoff, S.b, 1, (float*)S.gc, S.gcs);
  if (s) return s;
  // the second right-hand side: same-molecule pairs scaled by pscale
  if (nv == 2 && (s = launch_efield<double>(ctx, st, *P, &sys1, mpole, polarity, thole, ewald_beta,
                                            cutoff, S.b + S.vs, 1, nullptr, 0, pscale)))
    return s;
  // Buffers that the pair-term passes share per stream are taken only now:
  // a pass above may have grown (reallocated) them, the multipole pass
  // needing six accumulators per slot where the mat-vec needs three.
  if (prec == TK_FP64) {   // the FP64 mat-vec reads only coordinates: the ones the field pass gathered
    S.gathered = (double*)ctx->scratch[per_stream("gathered", st)].p;
  } else {
    if ((s = scratch(ctx, per_stream("partial", st).c_str(),
                     sizeof(double) * kMaxSlots * 3 * S.pstride, &partial)))
      return s;
    S.partial = (double*)partial;
    S.gather_geometry();
  }
  // full Ewald: the reciprocal permanent field joins the right-hand side (the
  // PME scratch is separate from the gathered coordinates above)
  for (int v = 0; v < nv && pme_grid; ++v)
    if ((s = pme_perm_field_add(ctx, st, &sys1, mpole, ewald_beta, pme_grid, pme_order,
                                (const int32_t*)P->perm.p, S.b + v * S.vs)))
      return s;
  // the sites of every iteration's dipole field: sorted and tabulated once
  if (pme_grid && (s = pme_prepare_sites(ctx, st, n, P->box, S.gathered, S.pstride, pme_grid,
                                         pme_order)))
    return s;
  const int g0 = xcd_grid(S.ncells);
  k_cs_setup<<<g0 + (sums.cpart ? sums.nsys : 0), kCellThreads, 0, st>>>(
      S.pv, polarity, mu_guess, guess_on, S.b, S.alpha_s, S.x, S.npart, S.hdr, S.ent, nv, sums,
      g0);
  if (queued) {
    S.info_out = info_dev;
    if (prec == TK_FP64) S.run_queued<double>(S.b, tol_debye, queued);
    else S.run_queued<float>(S.b, tol_debye, queued);
    k_scatter_out<<<ceil_div(n, 256), 256, 0, st>>>(n, (const int32_t*)P->perm.p, S.x, mu_out,
                                                    S.pv.status);
    TK_HIP(hipGetLastError());
    return TK_OK;
  }
  const int slot = (int)(P - ctx->plans);
  int& hint = ctx->pcg_hint[slot][prec == TK_FP64 ? 0 : 1];
  s = prec == TK_FP64 ? S.run<double>(S.b, tol_debye, maxiter, hint, true, nullptr)
                      : S.run<float>(S.b, tol_debye, maxiter, hint, true, nullptr);
  if (s) return s;
  int most = 0;
  bool failed_list = false;
  std::vector<int> done(nsys * nv);
  for (int k = 0; k < nsys * nv; ++k) {
    const PcgState& h = S.host[k];
    done[k] = h.done;
    most = std::max(most, h.iters);
    info[k].iters = h.iters;
    info[k].rms_debye = h.rms;
    info[k].converged = h.done == 1;
    info[k].status = h.done == 1   ? TK_OK
                     : h.done == 3 ? TK_E_BREAKDOWN
                     : h.done == 4 ? TK_E_CAPACITY
                                   : TK_E_NOCONV;
    info[k].rms_true_debye = h.rms_true;
    info[k].epol = h.epol;
    failed_list |= h.done == 4;
  }
  // a list whose build went past its bounds: nothing was solved
  if (failed_list) return TK_E_CAPACITY;
  hint = most;
  if (prec == TK_MIXED) {
    // FP64-residual refinement of the systems whose true residual is above
    // the tolerance: solve A d = b - A x with the mixed solver, x += d
    for (int ref = 0; ref < 3; ++ref) {
      int any = 0;
      for (int k = 0; k < nsys; ++k) {
        S.active_h[k] = done[k] != 3 && S.host[k].rms_true > tol_debye ? 1 : 0;
        any |= S.active_h[k];
      }
      if (!any) break;
      TK_HIP(hipMemcpyAsync(S.active, S.active_h, sizeof(int32_t) * nsys, hipMemcpyHostToDevice,
                            st));
      // r_t = b - A x in FP64 (sorted); d0 = alpha r_t into z
      S.matvec64_tiles(S.x);
      k_cs_apply<0><<<S.ncells, kCellThreads, 0, st>>>(S.pv, S.partial, S.pstride, S.cself,
                                                       S.alpha_s, S.x, S.b, S.rt, S.z, nullptr,
                                                       S.state);
      k_refine_begin<<<ceil_div(n, 256), 256, 0, st>>>(S.pv, S.active, S.x, S.dx, S.z);
      if ((s = S.run<float>(S.rt, tol_debye, maxiter, 0, false, S.active))) return s;
      std::vector<int> sub_iters(nsys);
      for (int k = 0; k < nsys; ++k) sub_iters[k] = S.host[k].iters;
      k_refine_end<<<ceil_div(n, 256), 256, 0, st>>>(S.pv, S.active, S.x, S.dx);
      S.queue_true_residual(S.b);
      if ((s = S.sync_state())) return s;
      for (int k = 0; k < nsys; ++k) {
        if (!S.active_h[k]) continue;
        info[k].iters += sub_iters[k];
        info[k].refinements = ref + 1;
        info[k].rms_true_debye = S.host[k].rms_true;
        info[k].epol = S.host[k].epol;
      }
    }
    // the mixed form's outcome is its FP64 check: converged only when the
    // true residual meets the tolerance after refinement, whatever the FP32
    // recurrence reported (a breakdown stays a breakdown)
    for (int k = 0; k < nsys; ++k) {
      if (done[k] == 3) continue;
      const bool ok = info[k].rms_true_debye <= tol_debye;
      info[k].converged = ok ? 1 : 0;
      info[k].status = ok ? TK_OK : TK_E_NOCONV;
    }
  }
  // the dipoles reach mu_out in stream order; the host already has the
  // solve's outcome, so no further synchronisation
  for (int v = 0; v < nv; ++v)
    k_scatter_out<<<ceil_div(n, 256), 256, 0, st>>>(n, (const int32_t*)P->perm.p, S.x + v * S.vs,
                                                    mu_out + v * S.vs, S.pv.status);
  TK_HIP(hipGetLastError());
  return TK_OK;
}

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
  if (sys->n == 0) {
    info->converged = 1;
    return TK_OK;
  }
  if (!mpole || !polarity || !thole || !mu_out) return TK_E_ARG;
  if ((s = solve_dipoles(ctx, (hipStream_t)stream, P, sys->xyz, sys->molid, mpole, polarity, thole,
                         ewald_beta, cutoff, tol_debye, maxiter, prec, mu_guess, nullptr, mu_out,
                         info, 0, 0)))
    return s;
  return info->status;
}

extern "C" tk_status tk_polarize_pcg_queued(tk_ctx* ctx, void* stream, const tk_system* sys,
                                            const tk_nblist* list, const double* mpole,
                                            const double* polarity, const double* thole,
                                            double ewald_beta, double cutoff, double tol_debye,
                                            int32_t iterations, int prec,
                                            const double* mu_guess, double* mu_out,
                                            tk_pcg_info* info_dev) {
  if (!ctx || !info_dev) return TK_E_ARG;
  tk_status s = check_system(sys);
  if (s) return s;
  if (prec != TK_FP64 && prec != TK_MIXED) return TK_E_ARG;
  if (!(ewald_beta >= 0.0) || !std::isfinite(ewald_beta) || !(tol_debye >= 0.0) ||
      iterations < 1 || iterations > 10000)
    return TK_E_ARG;
  const Plan* P;
  if ((s = get_plan(ctx, sys, list, cutoff, &P))) return s;
  hipStream_t st = (hipStream_t)stream;
  if (sys->n == 0) {   // nothing to solve: converged, written in stream order
    tk_pcg_info e{};
    e.converged = 1;
    k_pcg_info_empty<<<1, 1, 0, st>>>(e, info_dev);
    TK_HIP(hipGetLastError());
    return TK_OK;
  }
  if (!mpole || !polarity || !thole || !mu_out) return TK_E_ARG;
  return solve_dipoles(ctx, st, P, sys->xyz, sys->molid, mpole, polarity, thole, ewald_beta,
                       cutoff, tol_debye, iterations, prec, mu_guess, nullptr, mu_out, nullptr,
                       0, 0, 1, 0.0, nullptr, nullptr, nullptr, iterations, info_dev);
}

extern "C" tk_status tk_empole_polarize(tk_ctx* ctx, void* stream, const tk_system* sys,
                                        const tk_nblist* list, const double* mpole,
                                        const double* polarity, const double* thole,
                                        double ewald_beta, double cutoff, double tol_debye,
                                        int32_t maxiter, int prec, const double* mu_guess,
                                        double* mu_out, tk_pcg_info* info, double* energy,
                                        double* force, double* virial) {
  if (!ctx || !info) return TK_E_ARG;
  tk_status s = check_system(sys);
  if (s) return s;
  if (prec != TK_FP64 && prec != TK_MIXED) return TK_E_ARG;
  if (!(ewald_beta >= 0.0) || !std::isfinite(ewald_beta) || !(tol_debye >= 0.0) || maxiter < 0 ||
      !energy || !virial)
    return TK_E_ARG;
  const Plan* P;
  if ((s = get_plan(ctx, sys, list, cutoff, &P))) return s;
  *info = tk_pcg_info{};
  hipStream_t st = (hipStream_t)stream;
  if (sys->n == 0) {
    info->converged = 1;
    TK_HIP(hipMemsetAsync(energy, 0, 3 * sizeof(double), st));
    TK_HIP(hipMemsetAsync(virial, 0, 9 * sizeof(double), st));
    return TK_OK;
  }
  if (!mpole || !polarity || !thole || !mu_out || !force) return TK_E_ARG;
  if ((s = solve_dipoles(ctx, st, P, sys->xyz, sys->molid, mpole, polarity, thole, ewald_beta,
                         cutoff, tol_debye, maxiter, prec, mu_guess, nullptr, mu_out, info, 0, 0,
                         1, 0.0, energy, force, virial)))
    return s;
  return info->status;
}

extern "C" tk_status tk_empole_polarize_queued(tk_ctx* ctx, void* stream, const tk_system* sys,
                                               const tk_nblist* list, const double* mpole,
                                               const double* polarity, const double* thole,
                                               double ewald_beta, double cutoff,
                                               double tol_debye, int32_t iterations, int prec,
                                               const double* mu_guess, double* mu_out,
                                               tk_pcg_info* info_dev, double* energy,
                                               double* force, double* virial) {
  if (!ctx || !info_dev) return TK_E_ARG;
  tk_status s = check_system(sys);
  if (s) return s;
  if (prec != TK_FP64 && prec != TK_MIXED) return TK_E_ARG;
  if (!(ewald_beta >= 0.0) || !std::isfinite(ewald_beta) || !(tol_debye >= 0.0) ||
      iterations < 1 || iterations > 10000 || !energy || !virial)
    return TK_E_ARG;
  const Plan* P;
  if ((s = get_plan(ctx, sys, list, cutoff, &P))) return s;
  hipStream_t st = (hipStream_t)stream;
  if (sys->n == 0) {
    tk_pcg_info e{};
    e.converged = 1;
    k_pcg_info_empty<<<1, 1, 0, st>>>(e, info_dev);
    TK_HIP(hipGetLastError());
    TK_HIP(hipMemsetAsync(energy, 0, 3 * sizeof(double), st));
    TK_HIP(hipMemsetAsync(virial, 0, 9 * sizeof(double), st));
    return TK_OK;
  }
  if (!mpole || !polarity || !thole || !mu_out || !force) return TK_E_ARG;
  return solve_dipoles(ctx, st, P, sys->xyz, sys->molid, mpole, polarity, thole, ewald_beta,
                       cutoff, tol_debye, iterations, prec, mu_guess, nullptr, mu_out, nullptr,
                       0, 0, 1, 0.0, energy, force, virial, iterations, info_dev);
}

extern "C" tk_status tk_polarize_pcg_ewald(tk_ctx* ctx, void* stream, const tk_system* sys,
                                           const tk_nblist* list, const double* mpole,
                                           const double* polarity, const double* thole,
                                           double ewald_beta, double cutoff, int32_t grid,
                                           int32_t order, double tol_debye, int32_t maxiter,
                                           const double* mu_guess, double* mu_out,
                                           tk_pcg_info* info) {
  if (!ctx || !info) return TK_E_ARG;
  tk_status s = check_system(sys);
  if (s) return s;
  if (!(ewald_beta > 0.0) || !std::isfinite(ewald_beta) || !(tol_debye >= 0.0) || maxiter < 0 ||
      !pme_args_ok(grid, order))
    return TK_E_ARG;
  const Plan* P;
  if ((s = get_plan(ctx, sys, list, cutoff, &P))) return s;
  *info = tk_pcg_info{};
  if (sys->n == 0) {
    info->converged = 1;
    return TK_OK;
  }
  if (!mpole || !polarity || !thole || !mu_out) return TK_E_ARG;
  if ((s = solve_dipoles(ctx, (hipStream_t)stream, P, sys->xyz, sys->molid, mpole, polarity, thole,
                         ewald_beta, cutoff, tol_debye, maxiter, TK_FP64, mu_guess, nullptr,
                         mu_out, info, grid, order)))
    return s;
  return info->status;
}

extern "C" tk_status tk_polarize_pcg2(tk_ctx* ctx, void* stream, const tk_system* sys,
                                      const tk_nblist* list, const double* mpole,
                                      const double* polarity, const double* thole,
                                      double ewald_beta, double cutoff, double pscale,
                                      double tol_debye, int32_t maxiter, const double* mu_guess,
                                      double* mu_out, tk_pcg_info* info) {
  if (!ctx || !info) return TK_E_ARG;
  tk_status s = check_system(sys);
  if (s) return s;
  if (!(ewald_beta >= 0.0) || !std::isfinite(ewald_beta) || !(tol_debye >= 0.0) || maxiter < 0 ||
      !(pscale >= 0.0 && pscale <= 1.0))
    return TK_E_ARG;
  const Plan* P;
  if ((s = get_plan(ctx, sys, list, cutoff, &P))) return s;
  info[0] = info[1] = tk_pcg_info{};
  if (sys->n == 0) {
    info[0].converged = info[1].converged = 1;
    return TK_OK;
  }
  if (!mpole || !polarity || !thole || !mu_out) return TK_E_ARG;
  if ((s = solve_dipoles(ctx, (hipStream_t)stream, P, sys->xyz, sys->molid, mpole, polarity, thole,
                         ewald_beta, cutoff, tol_debye, maxiter, TK_FP64, mu_guess, nullptr,
                         mu_out, info, 0, 0, 2, pscale)))
    return s;
  return info[0].status ? info[0].status : info[1].status;
}

extern "C" tk_status tk_polarize_pcg2_ewald(tk_ctx* ctx, void* stream, const tk_system* sys,
                                            const tk_nblist* list, const double* mpole,
                                            const double* polarity, const double* thole,
                                            double ewald_beta, double cutoff, int32_t grid,
                                            int32_t order, double pscale, double tol_debye,
                                            int32_t maxiter, const double* mu_guess,
                                            double* mu_out, tk_pcg_info* info) {
  if (!ctx || !info) return TK_E_ARG;
  tk_status s = check_system(sys);
  if (s) return s;
  if (!(ewald_beta > 0.0) || !std::isfinite(ewald_beta) || !(tol_debye >= 0.0) || maxiter < 0 ||
      !(pscale >= 0.0 && pscale <= 1.0) || !pme_args_ok(grid, order))
    return TK_E_ARG;
  const Plan* P;
  if ((s = get_plan(ctx, sys, list, cutoff, &P))) return s;
  info[0] = info[1] = tk_pcg_info{};
  if (sys->n == 0) {
    info[0].converged = info[1].converged = 1;
    return TK_OK;
  }
  if (!mpole || !polarity || !thole || !mu_out) return TK_E_ARG;
  if ((s = solve_dipoles(ctx, (hipStream_t)stream, P, sys->xyz, sys->molid, mpole, polarity, thole,
                         ewald_beta, cutoff, tol_debye, maxiter, TK_FP64, mu_guess, nullptr,
                         mu_out, info, grid, order, 2, pscale)))
    return s;
  return info[0].status ? info[0].status : info[1].status;
}
