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
  const int u = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const Unit un = pv.units[u];
  if (pv.nsys > 1) {   // batch: this unit's system geometry
    const int sy = pv.cell_sys[un.h];
    ph.set_sys(pv.sys[sy], sy);
  }
  const int hs = pv.cell_start[un.h], nh = pv.cell_start[un.h + 1] - hs;
  const int ks = pv.cell_start[un.k], nk = pv.cell_start[un.k + 1] - ks;
  const int cap = pv.max_occ;
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
  const long p0 = pv.unit_off[u], p1 = p0 + pv.unit_cnt[u];
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

// Sum each atom's partial slots (fixed order) and hand the NA sums to Epi.
template <int NA, class Epi>
__global__ __launch_bounds__(256) void k_reduce(PlanView pv, const double* __restrict__ partial,
                                                long pstride, Epi epi) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= pv.n) return;
  const int ns = pv.cell_nslot[pv.scell[s]];
  double acc[NA];
#pragma unroll
  for (int f = 0; f < NA; ++f) acc[f] = 0.0;
#pragma unroll
  for (int k = 0; k < kMaxSlots; ++k)   // unrolled: all slot loads in flight at once
    if (k < ns)
#pragma unroll
      for (int f = 0; f < NA; ++f) acc[f] += partial[((long)k * NA + f) * pstride + s];
  epi(s, pv.perm[s], acc);
}

// Sum per-unit scalar records in a fixed order, per system:
// out[s][k] = sum over the units u of system s of uscal[u][k]; one block per
// (scalar, system).
template <int NS>
__global__ __launch_bounds__(256) void k_sum_units(const double* __restrict__ uscal,
                                                   const SysDev* __restrict__ sys,
                                                   double* __restrict__ out) {
  __shared__ double sh[256];
  const int k = blockIdx.x, sy = blockIdx.y;
  const int u0 = sys[sy].unit0, u1 = sys[sy + 1].unit0;
  double v = 0.0;
  for (int u = u0 + threadIdx.x; u < u1; u += 256) v += uscal[(long)u * NS + k];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(long)sy * NS + k] = sh[0];
}

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

}  // namespace tk
