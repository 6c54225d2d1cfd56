// Cell-pair tile skeleton shared by every pair kernel.
//
// One workgroup of W waves per work unit (an unordered pair of neighbouring
// cells H, K):
//   1. stage the current data of H's and K's atoms into LDS (field-major, so
//      consecutive atoms sit in consecutive banks);
//   2. walk the unit's listed pairs (64 W per step, one per lane); each lane
//      evaluates its pair and adds both atoms' contributions to its wave's
//      own LDS accumulators with LDS atomics (the plan orders pairs so that
//      lanes of a step mostly touch distinct atoms);
//   3. sum the wave copies in wave order and write them to the partial-result
//      slots the unit owns for H and for K (no global atomics; each (slot,
//      atom) has one writer);
//   4. reduce per-lane scalars (energies, virial) across each wave, then the
//      waves in order, and write one record per unit.
// A second kernel sums each atom's slots in a fixed order, so results are
// bitwise reproducible run to run.
#pragma once

#include "tk_internal.hpp"

namespace tk {

__device__ __forceinline__ void lds_add(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ double wave_sum_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Minimum-image pair vector d = x_j - x_i and r^2 (the same operation order
// as the reference: one fused multiply-add per component, then
// r^2 = fma(dx,dx, fma(dy,dy, dz*dz))).
__device__ __forceinline__ double image3(const double* LH, const double* LK, int cap, int a, int b,
                                         double box, double inv_box, double d[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double t = LK[c * cap + b] - LH[c * cap + a];
    d[c] = fma(-box, rint(t * inv_box), t);
  }
  return fma(d[0], d[0], fma(d[1], d[1], d[2] * d[2]));
}

template <class Ph, int W>
__global__ __launch_bounds__(64 * W) void k_units(PlanView pv, Ph ph, double* __restrict__ partial,
                                                  long pstride, double* __restrict__ uscal) {
  constexpr int NS1 = Ph::NS > 0 ? Ph::NS : 1;
  constexpr int NT = 64 * W;
  extern __shared__ double lds[];
  __shared__ double red[W * NS1];
  if (ph.skip()) return;   // solver finished: nothing to do
  if (*pv.status != 0) return;   // the list's build failed: its unit records are not valid
  const int u = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const UnitRec un = pv.urec[u];   // one read: cells, slots, system, pairs
  if (pv.nsys > 1) ph.set_sys(pv.sys[un.sy], un.sy);   // batch: this unit's system geometry
  const int hs = un.hs, nh = un.nh;
  const int ks = un.ks, nk = un.nk;
  const int cap = pv.max_occ;
  if (nh > cap || nk > cap) return;   // past the staging bound (a failed build reports it)
  ph.prologue(tid, NT);
  double* LH = lds;
  double* LK = LH + Ph::NF * cap;
  double* AH = LK + Ph::NF * cap;        // [W][NA][cap]: one copy per wave
  double* AK = AH + W * Ph::NA * cap;
  for (int t = tid; t < nh; t += NT) {
#pragma unroll
    for (int f = 0; f < Ph::NG; ++f) LH[f * cap + t] = ph.sorted[f * ph.gstride + hs + t];
    ph.stage_dyn(LH, cap, t, hs + t);
  }
  for (int t = tid; t < nk; t += NT) {
#pragma unroll
    for (int f = 0; f < Ph::NG; ++f) LK[f * cap + t] = ph.sorted[f * ph.gstride + ks + t];
    ph.stage_dyn(LK, cap, t, ks + t);
  }
  for (int t = tid; t < W * Ph::NA * cap; t += NT) {
    AH[t] = 0.0;
    AK[t] = 0.0;
  }
  __syncthreads();
  double sc[NS1];
#pragma unroll
  for (int k = 0; k < NS1; ++k) sc[k] = 0.0;
  double* MH = AH + w * Ph::NA * cap;
  double* MK = AK + w * Ph::NA * cap;
  const long p0 = un.off, p1 = p0 + un.cnt;
  for (long p = p0 + tid; p < p1; p += NT) {
    const uint32_t code = pv.codes[p];
    ph.pair(LH, LK, cap, (int)(code & 0xffffu), (int)(code >> 16), MH, MK, sc, p);
  }
  __syncthreads();
  // the wave copies summed in wave order
  for (int t = tid; t < nh; t += NT)
#pragma unroll
    for (int f = 0; f < Ph::NA; ++f) {
      double v = 0.0;
#pragma unroll
      for (int ww = 0; ww < W; ++ww) v += AH[(ww * Ph::NA + f) * cap + t];
      partial[((long)un.slot_h * Ph::NA + f) * pstride + hs + t] = v;
    }
  for (int t = tid; t < nk; t += NT)
#pragma unroll
    for (int f = 0; f < Ph::NA; ++f) {
      double v = 0.0;
#pragma unroll
      for (int ww = 0; ww < W; ++ww) v += AK[(ww * Ph::NA + f) * cap + t];
      partial[((long)un.slot_k * Ph::NA + f) * pstride + ks + t] = v;
    }
  if (Ph::NS > 0) {
#pragma unroll
    for (int k = 0; k < NS1; ++k) {
      const double v = wave_sum_d(sc[k]);
      if (lane == 0) red[w * NS1 + k] = v;
    }
    __syncthreads();
    if (tid < NS1) {
      double v = 0.0;
#pragma unroll
      for (int ww = 0; ww < W; ++ww) v += red[ww * NS1 + tid];
      uscal[(long)u * NS1 + tid] = v;
    }
  }
}

// Per-call gather of a functor's static per-atom fields into sorted SoA order
// (so tile staging reads contiguous, coalesced rows).
template <class Ph>
__global__ __launch_bounds__(256) void k_gather(PlanView pv, Ph ph, double* __restrict__ out,
                                                long gstride) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= pv.n) return;
  double g[Ph::NG];
  ph.gather(pv.perm[s], g);
#pragma unroll
  for (int f = 0; f < Ph::NG; ++f) out[f * gstride + s] = g[f];
}

// Unit-scalar chunks: each system's units are cut into chunks of kChunkUnits
// (relative to the system's first unit, so a system is cut the same way alone
// or in a batch); chunks are numbered system by system.
constexpr int kChunkUnits = 256;
__device__ __forceinline__ int sys_chunk0(const SysDev* __restrict__ sys, int sy) {
  int c = 0;
  for (int k = 0; k < sy; ++k) c += (sys[k + 1].unit0 - sys[k].unit0 + kChunkUnits - 1) / kChunkUnits;
  return c;
}
inline int total_chunks(const Plan& P) {
  int c = 0;
  for (int k = 0; k < P.nsys; ++k)
    c += (P.h_sys[k + 1].unit0 - P.h_sys[k].unit0 + kChunkUnits - 1) / kChunkUnits;
  return c;
}

// Sum each atom's partial slots and hand the NA sums to Epi.  kRedLanes
// lanes per atom (more waves in flight than one thread per atom): lane q
// sums slots q, q + kRedLanes, ...; the lanes' sums are combined by two
// butterfly steps, which give every lane of the group the same value (IEEE
// addition is commutative), so the order is fixed.
// With NS > 0 and uscal set, block b also sums unit-scalar chunk b (if there
// is one) into cpart[b][NS], threads in unit order, waves in order.
constexpr int kRedLanes = 4;
template <int NA, int NS, class Epi>
__global__ __launch_bounds__(256) void k_reduce(PlanView pv, const double* __restrict__ partial,
                                                long pstride, Epi epi,
                                                const double* __restrict__ uscal,
                                                double* __restrict__ cpart) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int s0 = g / kRedLanes, q = g % kRedLanes;
  const bool valid = s0 < pv.n;
  const int s = valid ? s0 : pv.n - 1;   // lanes past the end repeat the last atom, write nothing
  const int ns = pv.cell_nslot[pv.scell[s]];
  double acc[NA];
#pragma unroll
  for (int f = 0; f < NA; ++f) acc[f] = 0.0;
#pragma unroll
  for (int k0 = 0; k0 < kMaxSlots; k0 += kRedLanes) {   // unrolled: all slot loads in flight
    const int k = k0 + q;
    if (k < ns)
#pragma unroll
      for (int f = 0; f < NA; ++f) acc[f] += partial[((long)k * NA + f) * pstride + s];
  }
#pragma unroll
  for (int f = 0; f < NA; ++f) {
    acc[f] += __shfl_xor(acc[f], 1);
    acc[f] += __shfl_xor(acc[f], 2);
  }
  if (valid && q == 0) epi(s, pv.perm[s], acc);
  if constexpr (NS > 0) {
    if (!uscal) return;
    // this block's chunk: system sy, chunk c of it (uniform over the block)
    int b = blockIdx.x, sy = 0, u0 = 0, u1 = 0;
    for (; sy < pv.nsys; ++sy) {
      u0 = pv.sys[sy].unit0;
      u1 = pv.sys[sy + 1].unit0;
      const int nch = (u1 - u0 + kChunkUnits - 1) / kChunkUnits;
      if (b < nch) break;
      b -= nch;
    }
    if (sy >= pv.nsys) return;
    __shared__ double sh[NS][4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int u = u0 + b * kChunkUnits + tid;
    double v[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) v[k] = u < u1 ? uscal[(long)u * NS + k] : 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o);
      if (lane == 0) sh[k][w] = v[k];
    }
    __syncthreads();
    if (tid < NS) cpart[(long)blockIdx.x * NS + tid] = ((sh[tid][0] + sh[tid][1]) + sh[tid][2]) + sh[tid][3];
  }
}
static_assert(kRedLanes == 4, "the butterfly above has two steps");

// Per system: sum its chunk partials in order and write the energies and
// virial.  Record layout: NS = 11: E_a, E_b, W[9] -> energy {E_a + E_b, E_a,
// E_b}; NS = 10: E, W[9] -> energy {E}.  One wave per system.
// The body is shared with the solver's setup kernel, which takes over this
// launch for the fused multipole pass (every thread of the block calls it).
template <int NS>
__device__ __forceinline__ void sum_finish_sys(const double* __restrict__ cpart,
                                               const SysDev* __restrict__ sys,
                                               double* __restrict__ energy,
                                               double* __restrict__ virial, int sy) {
  static_assert(NS == 10 || NS == 11, "energy records");
  __shared__ double sh[NS];
  const int tid = threadIdx.x;
  const int c0 = sys_chunk0(sys, sy);
  const int nch = (sys[sy + 1].unit0 - sys[sy].unit0 + kChunkUnits - 1) / kChunkUnits;
  if (tid < NS) {
    double t = 0.0;
    for (int c = 0; c < nch; ++c) t += cpart[(long)(c0 + c) * NS + tid];
    constexpr int ne = NS - 9;   // energies in the record
    if (tid >= ne) virial[9 * sy + tid - ne] = t;
    else if (NS == 10) energy[sy] = t;
    else energy[3 * sy + 1 + tid] = t;
    sh[tid] = t;
  }
  if (NS == 11) {
    __syncthreads();
    if (tid == 0) energy[3 * sy] = sh[0] + sh[1];
  }
}

template <int NS>
__global__ __launch_bounds__(64) void k_sum_finish(const double* __restrict__ cpart,
                                                   const SysDev* __restrict__ sys,
                                                   double* __restrict__ energy,
                                                   double* __restrict__ virial) {
  sum_finish_sys<NS>(cpart, sys, energy, virial, blockIdx.x);
}

// A pass's energy and virial sums left to a later kernel on the same stream
// (the solver's setup kernel, for the fused multipole pass of NS = 11).
struct DeferredSums {
  const double* cpart = nullptr;   // null: nothing deferred
  double* energy = nullptr;
  double* virial = nullptr;
  int nsys = 0;
};

// LDS of k_units<Ph, W>: both cells' fields and W accumulator copies each.
template <class Ph>
inline size_t unit_lds_bytes(const Plan& p, int W) {
  return sizeof(double) * (size_t)(2 * (Ph::NF + W * Ph::NA)) *
         (size_t)(p.max_occ > 0 ? p.max_occ : 1);
}

// Ph::kWaves waves per unit when their LDS fits (two workgroups per CU at
// least), else one.  Several waves per unit pay where the pair loop is long
// next to the staging (many pairs per unit, few fields per atom); a term with
// heavy staging and a short loop keeps more units in flight with one wave.
template <class Ph>
inline void launch_units(const Plan& P, const Ph& ph, double* partial, long pstride,
                         double* uscal, hipStream_t st) {
  constexpr int W = Ph::kWaves;
  const size_t lw = unit_lds_bytes<Ph>(P, W);
  if (W > 1 && 2 * (lw + 4096) <= kMaxLds)
    k_units<Ph, W><<<P.nunits, 64 * W, lw, st>>>(P.view(), ph, partial, pstride, uscal);
  else
    k_units<Ph, 1><<<P.nunits, 64, unit_lds_bytes<Ph>(P, 1), st>>>(P.view(), ph, partial, pstride,
                                                                   uscal);
}

inline long pad64(long n) { return (n + 63) / 64 * 64; }

// Device buffers of one pair-term call, when the caller supplies them (the
// allocation-free entry points): partial slots [kMaxSlots][NA][pad64(n)],
// gathered fields [NG][pad64(n)], unit scalars [nunits][NS] and chunk sums
// [chunks][NS] (the last two only for terms with energies).
struct TermWs {
  double* partial = nullptr;
  double* gathered = nullptr;
  double* uscal = nullptr;
  double* cpart = nullptr;
};

}  // namespace tk
