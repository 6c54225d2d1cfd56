// Cell-pair tile skeleton shared by every pair kernel.
//
// One wavefront per work unit (an unordered pair of neighbouring cells H, K):
//   1. stage the current data of H's and K's atoms into LDS (field-major, so
//      consecutive atoms sit in consecutive banks);
//   2. walk the unit's listed pairs (64 per step, one per lane); each lane
//      evaluates its pair and adds both atoms' contributions to LDS
//      accumulators with LDS atomics (the plan orders pairs so that lanes of a
//      step touch distinct atoms);
//   3. write the accumulators to the partial-result slots the unit owns for
//      H and for K (no global atomics; each (slot, atom) has one writer);
//   4. reduce per-lane scalars (energies, virial) across the wave and write one
//      record per unit.
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

template <class Ph>
__global__ __launch_bounds__(64) void k_units(PlanView pv, Ph ph, double* __restrict__ partial,
                                              long pstride, double* __restrict__ uscal) {
  extern __shared__ double lds[];
  if (ph.skip()) return;   // solver finished: nothing to do
  const int u = blockIdx.x;
  const int lane = threadIdx.x;
  const Unit un = pv.units[u];
  if (pv.nsys > 1) {   // batch: this unit's system geometry
    const int sy = pv.cell_sys[un.h];
    ph.set_sys(pv.sys[sy], sy);
  }
  const int hs = pv.cell_start[un.h], nh = pv.cell_start[un.h + 1] - hs;
  const int ks = pv.cell_start[un.k], nk = pv.cell_start[un.k + 1] - ks;
  const int cap = pv.max_occ;
  ph.prologue(lane);
  double* LH = lds;
  double* LK = LH + Ph::NF * cap;
  double* AH = LK + Ph::NF * cap;
  double* AK = AH + Ph::NA * cap;
  for (int t = lane; t < nh; t += 64) {
#pragma unroll
    for (int f = 0; f < Ph::NG; ++f) LH[f * cap + t] = ph.sorted[f * ph.gstride + hs + t];
    ph.stage_dyn(LH, cap, t, hs + t);
#pragma unroll
    for (int f = 0; f < Ph::NA; ++f) AH[f * cap + t] = 0.0;
  }
  for (int t = lane; t < nk; t += 64) {
#pragma unroll
    for (int f = 0; f < Ph::NG; ++f) LK[f * cap + t] = ph.sorted[f * ph.gstride + ks + t];
    ph.stage_dyn(LK, cap, t, ks + t);
#pragma unroll
    for (int f = 0; f < Ph::NA; ++f) AK[f * cap + t] = 0.0;
  }
  __syncthreads();
  double sc[Ph::NS > 0 ? Ph::NS : 1];
#pragma unroll
  for (int k = 0; k < (Ph::NS > 0 ? Ph::NS : 1); ++k) sc[k] = 0.0;
  const long p0 = pv.unit_off[u], p1 = p0 + pv.unit_cnt[u];
  for (long p = p0 + lane; p < p1; p += 64) {
    const uint32_t code = pv.codes[p];
    ph.pair(LH, LK, cap, (int)(code & 0xffffu), (int)(code >> 16), AH, AK, sc, p);
  }
  __syncthreads();
  for (int t = lane; t < nh; t += 64)
#pragma unroll
    for (int f = 0; f < Ph::NA; ++f)
      partial[((long)un.slot_h * Ph::NA + f) * pstride + hs + t] = AH[f * cap + t];
  for (int t = lane; t < nk; t += 64)
#pragma unroll
    for (int f = 0; f < Ph::NA; ++f)
      partial[((long)un.slot_k * Ph::NA + f) * pstride + ks + t] = AK[f * cap + t];
  if (Ph::NS > 0) {
#pragma unroll
    for (int k = 0; k < Ph::NS; ++k) {
      double v = wave_sum_d(sc[k]);
      if (lane == 0) uscal[(long)u * Ph::NS + k] = v;
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

template <class Ph>
inline size_t unit_lds_bytes(const Plan& p) {
  return sizeof(double) * (size_t)(2 * (Ph::NF + Ph::NA)) * (size_t)(p.max_occ > 0 ? p.max_occ : 1);
}

inline long pad64(long n) { return (n + 63) / 64 * 64; }

}  // namespace tk
