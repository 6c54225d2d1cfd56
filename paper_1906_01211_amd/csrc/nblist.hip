// Neighbour lists on the GPU, integer and exact (the cell-list builders of the
// paper's Rel profile, with the selection-mask + compress pattern of its
// section "Typical selection loop" mapped to wavefront ballots).
//
// Pipeline:
//   quantize -> cell histogram -> scan -> scatter -> per-cell stable order
//   -> candidate windows (one per cell-pair unit) -> ONE enumeration that
//      writes each unit's listed pairs into its window and counts, per
//      (unit role, atom), the pairs whose CSR row is that atom's
//   -> row lengths + role offsets -> scan  [one host synchronisation]
//   -> dense pair codes, with the canonical CSR entries written from them in
//      the same pass -> rows ordered by j.
// Every pair decision is the same exact test, so the plan (what the pair
// kernels read) and the CSR (what the caller reads) hold the same pair set.
#include <cmath>
#include <cstring>

#include <mutex>

#include "tk_internal.hpp"

namespace tk {
namespace {

constexpr int kBuckets = 1024;

__device__ __forceinline__ bool pair_in(const uint4& a, const uint4& b, uint64_t rq2) {
  int64_t dx = (int32_t)(b.x - a.x), dy = (int32_t)(b.y - a.y), dz = (int32_t)(b.z - a.z);
  uint64_t d2 = (uint64_t)(dx * dx) + (uint64_t)(dy * dy) + (uint64_t)(dz * dz);
  return d2 <= rq2;
}

// Fast form of the exact test: the FP64 sum of squares of the (exact) integer
// differences is within 3 ulp of the true value, so outside a +-2^-50 band
// around rq^2 it decides; inside the band the exact 64-bit test decides.  The
// exact test runs only when some lane of the wave is in the band (a
// wave-uniform branch, almost never taken); every lane of the wave must call.
struct PairTest {
  uint64_t rq2;
  double lo, hi;
  __device__ __forceinline__ PairTest(const SysDev& d) : rq2(d.rq2), lo(d.lo), hi(d.hi) {}
  __device__ __forceinline__ bool operator()(const uint4& a, const uint4& b) const {
    const double dx = (double)(int32_t)(b.x - a.x), dy = (double)(int32_t)(b.y - a.y),
                 dz = (double)(int32_t)(b.z - a.z);
    const double d2 = fma(dx, dx, fma(dy, dy, dz * dz));
    bool in = d2 < lo;
    const bool band = !in && d2 <= hi;
    if (__builtin_expect(__ballot(band) != 0, 0))
      if (band) in = pair_in(a, b, rq2);
    return in;
  }
};

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

__device__ __forceinline__ int lanes_below(uint64_t mask) {
  return __popcll(mask & ((1ull << lane_id()) - 1ull));
}

__device__ __forceinline__ int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

// info: [0] status, [1] max cell occupancy, [2] max CSR row, [3] unused,
//       [4] 1 if the candidate windows (or k_plan's staging bound) did not fit,
//       [5] max atoms over a cell's neighbour cells
// System of atom i: the last system whose first atom is <= i.
__device__ __forceinline__ int atom_system(const SysDev* sys, int nsys, int i) {
  int lo = 0, hi = nsys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sys[mid].atom0 <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// u = floor(frac(x/L) * 2^32) per coordinate; cell = (u * nc) >> 32 per axis,
// offset by the system's first cell.
__device__ __forceinline__ int quantize_atom(const double* __restrict__ xyz, int i,
                                             const SysDev& sd, uint32_t* __restrict__ u,
                                             int32_t* __restrict__ info) {
  int c[3];
  for (int a = 0; a < 3; ++a) {
    const double x = xyz[3 * i + a];
    uint32_t q = 0;
    if (isfinite(x)) {
      const double t = x / sd.box;
      double f = t - floor(t);
      if (f >= 1.0) f = 0.0;
      q = (uint32_t)(f * kTwo32);
    } else {
      atomicMin(&info[0], (int)TK_E_ARG);
    }
    u[3 * i + a] = q;
    c[a] = (int)(((uint64_t)q * (uint64_t)sd.nc) >> 32);
  }
  return sd.cell0 + (c[0] * sd.nc + c[1]) * sd.nc + c[2];
}

__global__ void k_quantize(int n, const double* __restrict__ xyz, const SysDev* __restrict__ sys,
                           int nsys, uint32_t* __restrict__ u, int32_t* __restrict__ cell,
                           int32_t* __restrict__ cell_count, int32_t* __restrict__ info) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int cc = quantize_atom(xyz, i, sys[atom_system(sys, nsys, i)], u, info);
  cell[i] = cc;
  atomicAdd(&cell_count[cc], 1);
}

// Stable counting sort by cell without global atomics (plans with at most
// kMaxHistCells cells): per-block LDS histograms H[c][b], one exclusive scan
// over H in cell-major order, then each atom's slot is its (cell, block)
// offset plus its rank among the block's earlier atoms of the same cell.
// Slots come out ordered by (cell, caller index).
constexpr int kHistBlock = 256;
constexpr int kMaxHistCells = 4096;

__global__ __launch_bounds__(kHistBlock) void k_quantize_hist(int n, const double* __restrict__ xyz,
                                                              const SysDev* __restrict__ sys,
                                                              int nsys, int ncells,
                                                              uint32_t* __restrict__ u,
                                                              int32_t* __restrict__ cell,
                                                              int32_t* __restrict__ H,
                                                              int32_t* __restrict__ info) {
  __shared__ int hist[kMaxHistCells];
  for (int c = threadIdx.x; c < ncells; c += kHistBlock) hist[c] = 0;
  __syncthreads();
  const int i = blockIdx.x * kHistBlock + threadIdx.x;
  if (i < n) {
    const int cc = quantize_atom(xyz, i, sys[atom_system(sys, nsys, i)], u, info);
    cell[i] = cc;
    atomicAdd(&hist[cc], 1);
  }
  __syncthreads();
  const int nblk = gridDim.x;
  for (int c = threadIdx.x; c < ncells; c += kHistBlock) H[(long)c * nblk + blockIdx.x] = hist[c];
}

// off = exclusive scan of H (cell-major).  Block 0 also writes cell_start,
// the largest occupancy and the capacity check.
__global__ __launch_bounds__(kHistBlock) void k_scatter_stable(
    int n, int ncells, const int32_t* __restrict__ cell, const int32_t* __restrict__ off,
    const uint32_t* __restrict__ u, int32_t* __restrict__ perm, int32_t* __restrict__ scell,
    uint4* __restrict__ us, int32_t* __restrict__ cstart, int32_t* __restrict__ info) {
  __shared__ int cl[kHistBlock];
  const int nblk = gridDim.x;
  const int i = blockIdx.x * kHistBlock + threadIdx.x;
  const int c = i < n ? cell[i] : -1;
  cl[threadIdx.x] = c;
  __syncthreads();
  if (i < n) {
    int rank = 0;
    for (int t = 0; t < (int)threadIdx.x; ++t) rank += cl[t] == c;
    const int slot = off[(long)c * nblk + blockIdx.x] + rank;
    perm[slot] = i;
    scell[slot] = c;
    us[slot] = make_uint4(u[3 * i], u[3 * i + 1], u[3 * i + 2], (uint32_t)i);
  }
  if (blockIdx.x == 0) {
    int occ = 0;
    for (int cc = threadIdx.x; cc < ncells; cc += kHistBlock) {
      const int s0 = off[(long)cc * nblk];
      const int s1 = cc + 1 < ncells ? off[(long)(cc + 1) * nblk] : n;
      cstart[cc] = s0;
      occ = max(occ, s1 - s0);
    }
    for (int o = 32; o > 0; o >>= 1) occ = max(occ, __shfl_xor(occ, o));
    if ((threadIdx.x & 63) == 0) {   // one atomic per wave
      atomicMax(&info[1], occ);
      if (occ > kMaxCellAtoms) atomicMin(&info[0], (int)TK_E_CAPACITY);
    }
    if (threadIdx.x == 0) cstart[ncells] = n;
  }
}

__global__ void k_scatter(int n, const int32_t* __restrict__ cell, const int32_t* __restrict__ cstart,
                          int32_t* __restrict__ cursor, int32_t* __restrict__ tmp) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = cell[i];
  tmp[cstart[c] + atomicAdd(&cursor[c], 1)] = i;
}

// One wave per cell: order the cell's atoms by caller index (rank by count).
__global__ __launch_bounds__(64) void k_cellsort(const int32_t* __restrict__ cstart,
                                                 const int32_t* __restrict__ tmp,
                                                 const uint32_t* __restrict__ u,
                                                 int32_t* __restrict__ perm, int32_t* __restrict__ scell,
                                                 uint4* __restrict__ us, int32_t* __restrict__ info) {
  __shared__ int idx[kMaxCellAtoms];
  int c = blockIdx.x, start = cstart[c], m = cstart[c + 1] - start;
  if (threadIdx.x == 0) atomicMax(&info[1], m);
  if (m > kMaxCellAtoms) {
    // the build fails; the cell's slots still get its atoms (unsorted), so
    // the plan's permutation stays one for the kernels that gather through it
    if (threadIdx.x == 0) atomicMin(&info[0], (int)TK_E_CAPACITY);
    for (int t = threadIdx.x; t < m; t += 64) {
      const int e = tmp[start + t];
      perm[start + t] = e;
      scell[start + t] = c;
      us[start + t] = make_uint4(u[3 * e], u[3 * e + 1], u[3 * e + 2], (uint32_t)e);
    }
    return;
  }
  for (int t = threadIdx.x; t < m; t += 64) idx[t] = tmp[start + t];
  __syncthreads();
  for (int t = threadIdx.x; t < m; t += 64) {
    int e = idx[t], rank = 0;
    for (int k = 0; k < m; ++k) rank += idx[k] < e;
    int s = start + rank;
    perm[s] = e;
    scell[s] = c;
    us[s] = make_uint4(u[3 * e], u[3 * e + 1], u[3 * e + 2], (uint32_t)e);
  }
}

// Fixed-point span [lo, hi] of cell index ci along one axis: the u with
// (u * nc) >> 32 == ci, i.e. lo = ceil(ci 2^32 / nc), hi = ceil((ci + 1)
// 2^32 / nc) - 1.  In FP64 the quotient (below 2^33) is within 2^-21 of the
// exact one while a non-integer quotient is at least 1/nc from an integer,
// so the ceilings are exact.
__device__ __forceinline__ void cell_span(int ci, int nc, uint32_t& lo, uint32_t& hi) {
  lo = (uint32_t)ceil((double)ci * 4294967296.0 / (double)nc);
  hi = (uint32_t)((uint64_t)ceil((double)(ci + 1) * 4294967296.0 / (double)nc) - 1u);
}

// Square of the periodic fixed-point distance from u to the span [lo, hi]:
// 0 inside; else the shorter of the wrapping steps forward to lo and back
// to hi (at most 2^31, so three squares fit in 64 bits).
__device__ __forceinline__ uint64_t span_d2(uint32_t u, uint32_t lo, uint32_t hi) {
  if (u >= lo && u <= hi) return 0;
  const uint32_t d1 = lo - u, d2 = u - hi;
  const uint64_t d = d1 < d2 ? d1 : d2;
  return d * d;
}

// Reach filter: an atom whose squared distance to a cell's box exceeds rq^2
// has no partner in that cell.  Every b in the cell lies in the box, and the
// per-axis distance to the box is at most |int32(u_b - u_a)|, so the box
// distance never exceeds the exact pair distance: the filter drops no pair.
struct CellBox {
  uint32_t lo[3], hi[3];
  __device__ __forceinline__ CellBox(int local, int nc) {
    const int ci[3] = {local / (nc * nc), (local / nc) % nc, local % nc};
#pragma unroll
    for (int a = 0; a < 3; ++a) cell_span(ci[a], nc, lo[a], hi[a]);
  }
  __device__ __forceinline__ bool reach(const uint4& v, uint64_t rq2) const {
    return span_d2(v.x, lo[0], hi[0]) + span_d2(v.y, lo[1], hi[1]) + span_d2(v.z, lo[2], hi[2]) <=
           rq2;
  }
};

constexpr int kPlanMaxWaves = 4;   // waves per unit: 1, 2 or 4 (host's choice by cell size)
constexpr int kPlanRegions = (kMaxCellAtoms / 64) * kPlanMaxWaves;   // (H chunk, wave) regions

// One workgroup of W = blockDim.x / 64 waves per cell-pair unit (H, K).
//  1. Reach filter: the atoms of H that can reach K's box and those of K
//     that can reach H's box are staged in LDS, in cell order (a self unit
//     keeps all).  Corner and edge neighbours lose most of their atoms.
//  2. Candidates (a, b) of the survivors are visited in "diagonal" order
//     b = (m + k) mod |K'| for the survivor m of H on each lane (chunks of
//     64), so consecutive listed pairs touch distinct atoms on both sides
//     (conflict-free LDS accumulation in the pair kernels).  Wave w takes
//     its part of the k range; each (chunk, wave) region of the unit's window
//     receives its passing codes a | b << 16 (cell-local indices) in visit
//     order and its count goes to rcnt; the compaction concatenates regions
//     in (chunk, wave) order.
//  3. Per (unit role, atom): the number of pairs whose CSR row is that
//     atom's (the smaller caller index owns the pair).
__global__ __launch_bounds__(64 * kPlanMaxWaves) void k_plan(
    int nunits, const Unit* __restrict__ units, const int32_t* __restrict__ cstart,
    const uint4* __restrict__ us, const SysDev* __restrict__ sys,
    const int32_t* __restrict__ cell_sys, long pstride, const int64_t* __restrict__ unit_off,
    long code_cap, uint32_t* __restrict__ codes, int32_t* __restrict__ unit_cnt,
    int64_t* __restrict__ cnt64, int32_t* __restrict__ rcnt, int2* __restrict__ nfilt,
    int32_t* __restrict__ slot_cnt, int32_t* __restrict__ info, int occ_cap) {
  // dynamic LDS: sH sK (uint4), then iH iK cH cK (int), occ_cap entries each;
  // occ_cap is the host's bound on the cell occupancy (a larger cell makes
  // the host rerun with kMaxCellAtoms)
  extern __shared__ uint4 plan_lds[];
  uint4* sH = plan_lds;
  uint4* sK = sH + occ_cap;
  int* iH = (int*)(sK + occ_cap);
  int* iK = iH + occ_cap;
  int* cH = iK + occ_cap;
  int* cK = cH + occ_cap;
  __shared__ int wc[2][2][kPlanMaxWaves];
  __shared__ int rc[kPlanRegions];
  const int uidx = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int NT = blockDim.x, W = NT >> 6;
  if (unit_off[nunits] > code_cap) {   // windows do not fit: host grows the buffer, reruns
    if (uidx == 0 && tid == 0) info[4] = 1;
    return;
  }
  const Unit un = units[uidx];
  const int hs = cstart[un.h], nh = cstart[un.h + 1] - hs;
  const int ks = cstart[un.k], nk = cstart[un.k + 1] - ks;
  if (nh > kMaxCellAtoms || nk > kMaxCellAtoms) return;
  if (nh > occ_cap || nk > occ_cap) {   // staging bound too small: host reruns with kMaxCellAtoms
    if (tid == 0) info[4] = 1;
    return;
  }
  const SysDev sd = sys[cell_sys ? cell_sys[un.h] : 0];
  const PairTest test(sd);
  const bool self = un.h == un.k;
  const uint4 z4 = make_uint4(0, 0, 0, 0);
  const CellBox bh(un.h - sd.cell0, sd.nc), bk(un.k - sd.cell0, sd.nc);
  for (int t = tid; t < nh; t += NT) cH[t] = 0;
  for (int t = tid; t < nk; t += NT) cK[t] = 0;
  // 1. stable compaction of the survivors of both cells, one pass per NT
  //    atoms (wave counts double-buffered: one barrier per pass)
  int nhf = 0, nkf = 0;
  const int nmax = nh > nk ? nh : nk;
  for (int r0 = 0, par = 0; r0 < nmax; r0 += NT, par ^= 1) {
    const int t = r0 + tid;
    uint4 vh = z4, vk = z4;
    bool kh = false, kk = false;
    if (t < nh) {
      vh = us[hs + t];
      kh = self || bk.reach(vh, sd.rq2);
    }
    if (t < nk) {
      vk = us[ks + t];
      kk = self || bh.reach(vk, sd.rq2);
    }
    const uint64_t mh = __ballot(kh), mk = __ballot(kk);
    if (lane == 0) {
      wc[par][0][w] = __popcll(mh);
      wc[par][1][w] = __popcll(mk);
    }
    __syncthreads();
    int ph = nhf, pk = nkf;
    for (int ww = 0; ww < W; ++ww) {
      const int ch = wc[par][0][ww], ck = wc[par][1][ww];
      ph += ww < w ? ch : 0;
      pk += ww < w ? ck : 0;
      nhf += ch;
      nkf += ck;
    }
    if (kh) {
      const int p = ph + lanes_below(mh);
      sH[p] = vh;
      iH[p] = t;
    }
    if (kk) {
      const int p = pk + lanes_below(mk);
      sK[p] = vk;
      iK[p] = t;
    }
  }
  __syncthreads();
  // 2. enumeration
  const int nch = (nhf + 63) >> 6;
  const int kp = (nkf + W - 1) / W;
  const int kk0 = min(w * kp, nkf), kk1 = min(kk0 + kp, nkf);
  uint32_t* win = codes + unit_off[uidx];
  constexpr int kPlanUnroll = 4;
  for (int ch = 0; ch < nch; ++ch) {
    const int m = ch * 64 + lane;
    const int la = min(64, nhf - ch * 64);
    const bool av = m < nhf;
    const uint4 ua = av ? sH[m] : z4;
    const int a = av ? iH[m] : 0;
    uint32_t* out = win + (long)64 * ch * nkf + (long)la * kk0;   // region (ch, w)
    int bp = nkf > 0 ? (m + kk0) % nkf : 0;   // b position, advanced incrementally
    int cnt = 0, own = 0;
    for (int kq = kk0; kq < kk1; kq += kPlanUnroll) {
      int bj[kPlanUnroll];
      uint4 kj[kPlanUnroll];
      bool pj[kPlanUnroll];
#pragma unroll
      for (int j = 0; j < kPlanUnroll; ++j) {
        bj[j] = bp;
        if (++bp == nkf) bp = 0;
      }
#pragma unroll
      for (int j = 0; j < kPlanUnroll; ++j) kj[j] = sK[bj[j]];
#pragma unroll
      for (int j = 0; j < kPlanUnroll; ++j) {   // branch-free except the rare band test
        // a self unit keeps every atom, so positions are cell indices there
        const bool ok = av & (kq + j < kk1) & (!self | (m < bj[j]));
        pj[j] = ok & test(ua, kj[j]);
      }
#pragma unroll
      for (int j = 0; j < kPlanUnroll; ++j) {
        const uint64_t mask = __ballot(pj[j]);
        if (pj[j]) {
          const int b = iK[bj[j]];
          out[cnt + lanes_below(mask)] = (uint32_t)a | ((uint32_t)b << 16);
          if (ua.w < kj[j].w) ++own;
          else atomicAdd(&cK[b], 1);
        }
        cnt += __popcll(mask);
      }
    }
    if (av && own) atomicAdd(&cH[a], own);
    if (lane == 0) rc[ch * W + w] = cnt;
  }
  __syncthreads();
  // 3. counts
  const int nr = nch * W;
  if (tid < nr) rcnt[(long)uidx * kPlanRegions + tid] = rc[tid];
  if (tid == 0) {
    int tot = 0;
    for (int r = 0; r < nr; ++r) tot += rc[r];
    unit_cnt[uidx] = tot;
    cnt64[uidx] = tot;
    nfilt[uidx] = make_int2(nhf, nkf);
  }
  for (int t = tid; t < nh; t += NT) slot_cnt[(long)un.slot_h * pstride + hs + t] = cH[t];
  for (int t = tid; t < nk; t += NT) slot_cnt[(long)un.slot_k * pstride + ks + t] = cK[t];
}

// Per unit: move the unit's pair codes from the regions of its candidate
// window to its place in the dense code array (windows are sized by
// candidates, the dense array by listed pairs), regions in (chunk, wave)
// order; write the unit's record for the pair kernels (see UnitRec); and,
// when the caller asked for the CSR (col set), put each pair's j into its
// row at the owner atom's role offset (order inside a role is fixed by the
// row sort that follows).
struct CsrOut {
  const int32_t* perm;
  const int32_t* slot_off;   // per (role, sorted atom): offset inside the owner's row
  const int32_t* row_ptr;
  int32_t* col;              // nullptr: no CSR
  long col_cap;              // entries col holds
  long pstride;
  int occ;                   // dynamic LDS: 4 * occ ints
};
template <int kCompactThreads>   // threads per unit: compact_launch picks them
__global__ __launch_bounds__(kCompactThreads) void k_compact(const int64_t* __restrict__ woff,
                                                 const uint32_t* __restrict__ windows,
                                                 const int64_t* __restrict__ doff,
                                                 const int32_t* __restrict__ rcnt,
                                                 const int2* __restrict__ nfilt, int W,
                                                 uint32_t* __restrict__ codes,
                                                 const Unit* __restrict__ units,
                                                 const int32_t* __restrict__ cstart,
                                                 const int32_t* __restrict__ unit_cnt,
                                                 const int32_t* __restrict__ cell_sys,
                                                 UnitRec* __restrict__ rec, CsrOut csr,
                                                 long code_cap,
                                                 const int32_t* __restrict__ status) {
  __shared__ int rs[kPlanRegions], rd[kPlanRegions + 1];
  extern __shared__ int csr_lds[];   // pH pK | bH bK (occ each); cursors reuse nothing
  __shared__ int cH[kMaxCellAtoms], cK[kMaxCellAtoms];
  const int u = blockIdx.x, tid = threadIdx.x;
  // a build past its bounds (status set) or codes past the array: nothing
  // here is safe to follow, and the plan's users skip it
  if (*status != 0 || doff[gridDim.x] > code_cap) return;
  const Unit un = units[u];
  const int hs = cstart[un.h], nh = cstart[un.h + 1] - hs;
  const int ks = cstart[un.k], nk = cstart[un.k + 1] - ks;
  if (tid == 64)   // a lane of the second wave: the record, beside wave 0's prefix
    rec[u] = UnitRec{hs, nh, ks, nk, un.slot_h, un.slot_k, cell_sys ? cell_sys[un.h] : 0,
                     unit_cnt[u], doff[u]};
  const bool fill = csr.col != nullptr && nh <= csr.occ && nk <= csr.occ &&
                    doff[gridDim.x] <= csr.col_cap;
  int* pH = csr_lds;
  int* pK = pH + csr.occ;
  int* bH = pK + csr.occ;
  int* bK = bH + csr.occ;
  if (fill) {
    for (int t = tid; t < nh; t += kCompactThreads) {
      const int i = csr.perm[hs + t];
      pH[t] = i;
      cH[t] = 0;
      bH[t] = csr.row_ptr[i] + csr.slot_off[(long)un.slot_h * csr.pstride + hs + t];
    }
    for (int t = tid; t < nk; t += kCompactThreads) {
      const int i = csr.perm[ks + t];
      pK[t] = i;
      cK[t] = 0;
      bK[t] = csr.row_ptr[i] + csr.slot_off[(long)un.slot_k * csr.pstride + ks + t];
    }
  }
  const int2 nf = nfilt[u];
  const int nhf = nf.x, nkf = nf.y;
  const int nr = ((nhf + 63) >> 6) * W;
  const int kp = (nkf + W - 1) / W;
  if (tid < 64) {   // wave 0: region starts (window) and dense prefix
    int c = 0;
    if (tid < nr) {
      const int ch = tid / W, w = tid % W;
      const int la = min(64, nhf - ch * 64);
      rs[tid] = 64 * ch * nkf + la * min(w * kp, nkf);
      c = rcnt[(long)u * kPlanRegions + tid];
    }
    int incl = c;
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl, o);
      if (tid >= o) incl += t;
    }
    if (tid < nr) rd[tid] = incl - c;
    if (tid == nr - 1) rd[nr] = incl;
    if (nr == 0 && tid == 0) rd[0] = 0;
  }
  __syncthreads();
  const uint32_t* src = windows + woff[u];
  uint32_t* dst = codes + doff[u];
  const int m = rd[nr];
  for (int t0 = tid; t0 < m; t0 += 4 * kCompactThreads) {   // four loads in flight per thread
    uint32_t v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int t = t0 + k * kCompactThreads;
      v[k] = 0u;
      if (t < m) {
        int lo = 0, hi = nr - 1;   // last region starting at or before t
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (rd[mid] <= t) lo = mid;
          else hi = mid - 1;
        }
        v[k] = src[rs[lo] + (t - rd[lo])];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (t0 + k * kCompactThreads < m) {
        dst[t0 + k * kCompactThreads] = v[k];
        if (fill) {
          const int a = (int)(v[k] & 0xffffu), b = (int)(v[k] >> 16);
          const int ia = pH[a], ib = pK[b];
          if (ia < ib) csr.col[bH[a] + atomicAdd(&cH[a], 1)] = ib;
          else csr.col[bK[b] + atomicAdd(&cK[b], 1)] = ia;
        }
      }
  }
}

// Threads per unit of the compaction: the largest of 128..1024 that still
// gives each thread four codes on average (measured on the 7, 9 and 12 A
// lists, about 230, 1,100 and 4,800 codes per unit: 128, 256 and 1024
// threads, 18.0, 28.0 and 236 us against 21.5, 28.0 and 260 us with 256 for
// all three).
template <class... A>
static void compact_launch(double codes_per_unit, int nunits, size_t lds, hipStream_t st,
                           A... args) {
  if (codes_per_unit >= 4.0 * 1024)
    k_compact<1024><<<nunits, 1024, lds, st>>>(args...);
  else if (codes_per_unit >= 4.0 * 512)
    k_compact<512><<<nunits, 512, lds, st>>>(args...);
  else if (codes_per_unit >= 4.0 * 256)
    k_compact<256><<<nunits, 256, lds, st>>>(args...);
  else
    k_compact<128><<<nunits, 128, lds, st>>>(args...);
}

// Per sorted atom: the CSR row length (sum over its unit roles, written in
// caller order) and, in place, the exclusive prefix of its per-role counts.
constexpr int kRowSlotsThreads = 1024;
__global__ __launch_bounds__(kRowSlotsThreads) void k_row_slots(int n, const int32_t* __restrict__ perm, const int32_t* __restrict__ scell,
                            const int32_t* __restrict__ cell_nslot, long pstride,
                            int32_t* __restrict__ slot_cnt, int32_t* __restrict__ row_cnt,
                            int32_t* __restrict__ info) {
  const int s0 = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = s0 < n;
  const int s = valid ? s0 : n - 1;   // lanes past the end repeat the last atom, write nothing
  const int ns = cell_nslot[scell[s]];
  int c[kMaxSlots];
#pragma unroll
  for (int k = 0; k < kMaxSlots; ++k) c[k] = k < ns ? slot_cnt[(long)k * pstride + s] : 0;
  int run = 0;
#pragma unroll
  for (int k = 0; k < kMaxSlots; ++k) {
    if (valid && k < ns) slot_cnt[(long)k * pstride + s] = run;
    run += c[k];
  }
  if (valid) row_cnt[perm[s]] = run;
  // longest row: wave maximum, then the workgroup's, then one atomic per
  // workgroup (atomics on one word from every XCD serialise)
  __shared__ int wmax[kRowSlotsThreads / 64];
  int m = run;
  for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kRowSlotsThreads / 64; ++w) m = max(m, wmax[w]);
    atomicMax(&info[2], m);
  }
}

// Batch plans: the unit and cell tables of every system, from the per-nc
// templates, with cell and unit indices offset by the system's first ones.
struct TplPtrs {
  const Unit* units;
  const int32_t* nslot;
  const int32_t* cu;
  const int32_t* order;
};

__global__ void k_batch_units(int nunits, int nsys, const SysDev* __restrict__ sys,
                              const TplPtrs* __restrict__ tpl, Unit* __restrict__ out) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= nunits) return;
  int lo = 0, hi = nsys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sys[mid].unit0 <= u) lo = mid;
    else hi = mid - 1;
  }
  const SysDev& d = sys[lo];
  const Unit t = tpl[lo].units[u - d.unit0];
  out[u] = Unit{t.h + d.cell0, t.k + d.cell0, t.slot_h, t.slot_k};
}

__global__ void k_batch_cells(int ncells, int nsys, const SysDev* __restrict__ sys,
                              const TplPtrs* __restrict__ tpl, int32_t* __restrict__ nslot,
                              int32_t* __restrict__ cu, int32_t* __restrict__ cell_sys,
                              int32_t* __restrict__ order) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  int lo = 0, hi = nsys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sys[mid].cell0 <= c) lo = mid;
    else hi = mid - 1;
  }
  const SysDev& d = sys[lo];
  const int lc = c - d.cell0;
  nslot[c] = tpl[lo].nslot[lc];
  cell_sys[c] = lo;
  order[c] = d.cell0 + tpl[lo].order[lc];   // systems in turn, each octant-grouped
  const int32_t* e = tpl[lo].cu + (long)lc * kCellUnitStride;
  int32_t* o = cu + (long)c * kCellUnitStride;
  o[0] = e[0];
  for (int j = 0; j < e[0]; ++j) o[1 + j] = ((e[1 + j] >> 2) + d.unit0) * 4 + (e[1 + j] & 3);
}

// One launch, two jobs (both need only the cell starts):
//  - blocks [0, nbu): candidate window of each unit, |H| * |K| slots;
//  - the rest: one wave per cell, atoms in its neighbour cells (itself
//    included); the maximum goes to info[5] (staging size of the per-cell
//    mat-vec).
__global__ __launch_bounds__(256) void k_cand_nbhd(int nunits, int ncells, int nbu,
                                                   const int32_t* __restrict__ cu,
                                                   const Unit* __restrict__ units,
                                                   const int32_t* __restrict__ cstart,
                                                   int64_t* __restrict__ cand,
                                                   int32_t* __restrict__ info) {
  __shared__ int wmax[4];
  if ((int)blockIdx.x < nbu) {
    const int u = blockIdx.x * 256 + threadIdx.x;
    if (u >= nunits) return;
    const Unit un = units[u];
    cand[u] =
        (int64_t)(cstart[un.h + 1] - cstart[un.h]) * (int64_t)(cstart[un.k + 1] - cstart[un.k]);
    return;
  }
  const int c = ((int)blockIdx.x - nbu) * 4 + (threadIdx.x >> 6);   // one wave per cell
  const int lane = lane_id();
  int cnt = 0;
  if (c < ncells) {
    const int32_t* e = cu + (long)c * kCellUnitStride;
    if (lane < e[0]) {
      const int u = e[1 + lane] >> 2, role = e[1 + lane] & 3;
      const int oc = role == 1 ? units[u].h : units[u].k;
      cnt = cstart[oc + 1] - cstart[oc];
    }
  }
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
  if (lane == 0) wmax[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0)
    atomicMax(&info[5], max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3])));
}

// Gathers the build's outcome into pinned host memory (one kernel instead of
// several small copies).
// info is left zeroed for the next build.
__global__ void k_readback(int32_t* __restrict__ info, const int32_t* __restrict__ rp_end,
                           const int64_t* __restrict__ off_end, const int64_t* __restrict__ pairs,
                           int32_t* __restrict__ host, int32_t* __restrict__ dstat) {
  dstat[0] = 0;   // the host checks this build before any kernel uses the plan
  for (int k = 0; k < 6; ++k) host[k] = info[k];
  for (int k = 0; k < 8; ++k) info[k] = 0;
  host[3] = (int32_t)*pairs;   // listed pairs, summed over the units
  host[6] = *rp_end;
  *(int64_t*)(host + 8) = *off_end;
}

// Stream-ordered builds: the system table through a kernel argument (no
// host staging buffer that a later call could overwrite before the copy
// runs), the status words cleared, and the outcome checked against the
// caller's bounds on the device.
struct SysPair {
  SysDev s[2];
};
__global__ void k_put_sys(SysPair v, SysDev* __restrict__ out, int32_t* __restrict__ info) {
  if (threadIdx.x < 2) out[threadIdx.x] = v.s[threadIdx.x];
  if (threadIdx.x < 8) info[threadIdx.x] = 0;
}

struct AsyncBounds {
  int32_t max_occ, max_row, max_nbhd;
  int64_t windows, cap;
};
// info: [0] error, [1] max occupancy, [2] max row, [4] enumeration did not
// fit (windows or staging bound), [5] max neighbourhood.
__global__ void k_build_status(const int32_t* __restrict__ info, const int32_t* __restrict__ rp_end,
                               const int64_t* __restrict__ win_end,
                               const int64_t* __restrict__ pairs, AsyncBounds b,
                               int64_t* __restrict__ npairs_dev, int32_t* __restrict__ status_dev,
                               int32_t* __restrict__ dstat, tk_nblist_bounds* __restrict__ report) {
  const bool fit = info[4] == 0;   // else the unit counts (and rows) were not formed
  const int64_t np = *pairs;
  int32_t st = info[0];
  if (st == 0 && (!fit || info[1] > b.max_occ || info[5] > b.max_nbhd || *win_end > b.windows ||
                  np > b.cap || info[2] > b.max_row))
    st = TK_E_CAPACITY;
  if (st == 0 && (int64_t)*rp_end != np) st = TK_E_HIP;   // rows and units disagree
  *npairs_dev = fit ? np : -1;
  *status_dev = st;
  dstat[0] = st;
  if (report) {
    report->max_occ = info[1];
    report->max_row = fit ? info[2] : -1;
    report->max_nbhd = info[5];
    report->reserved = 0;
    report->windows = *win_end;
    report->npairs = fit ? np : -1;
  }
}

// One wave per CSR row, blockDim.x / 64 rows per workgroup (up to
// kRowsPerBlock): order the row by j (monotone buckets over [jmin, jmax],
// then rank inside a bucket).  LDS per wave: A[max_row], G[max_row], cnt,
// off.  One row per workgroup measured fastest at every list size (7, 9 and
// 12 A rows: 22.7, 32.5 and 440 us against 23.2-24.0, 34.1 and 479 us with
// four rows, whose waves wait at each barrier for the block's longest row).
constexpr int kRowsPerBlock = 1;
__global__ __launch_bounds__(64 * kRowsPerBlock) void k_rowsort(int n,
                                                                const int32_t* __restrict__ row_ptr,
                                                                int32_t* __restrict__ col,
                                                                int max_row,
                                                                const int32_t* __restrict__ status) {
  extern __shared__ int lds[];
  if (*status != 0) return;   // the build failed: row_ptr and col are not a list
  const int w = threadIdx.x >> 6;
  const int i = blockIdx.x * (blockDim.x >> 6) + w;
  const int lane = lane_id();
  const int nbmax = max_row < kBuckets ? max_row : kBuckets;
  int* A = lds + (size_t)w * (2 * max_row + 2 * nbmax);
  int* G = A + max_row;
  int* cnt = G + max_row;
  int* off = cnt + nbmax;
  int start = 0, m = 0;
  if (i < n) {
    start = row_ptr[i];
    m = row_ptr[i + 1] - start;
  }
  // every wave takes part in the barriers; rows of 0 or 1 entries do no work
  // (nor a row longer than the LDS bound, which the build reports)
  if (m <= 1 || m > max_row) m = 0;
  int jmin = 0x7fffffff, jmax = -1;
  for (int e = lane; e < m; e += 64) {
    const int v = col[start + e];
    A[e] = v;
    jmin = min(jmin, v);
    jmax = max(jmax, v);
  }
  jmin = wave_min(jmin);
  jmax = wave_max(jmax);
  const int nb = m < kBuckets ? m : kBuckets;
  const double scale = m > 0 ? (double)nb / (double)(jmax - jmin + 1) : 0.0;
  for (int b = lane; b < nb; b += 64) cnt[b] = 0;
  __syncthreads();
  for (int e = lane; e < m; e += 64) {
    const int b = min(nb - 1, (int)((double)(A[e] - jmin) * scale));
    atomicAdd(&cnt[b], 1);
  }
  __syncthreads();
  const int per = (nb + 63) / 64, b0 = lane * per, b1 = min(nb, b0 + per);
  int sum = 0;
  for (int b = b0; b < b1; ++b) sum += cnt[b];
  int incl = sum;
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  int run = incl - sum;
  for (int b = b0; b < b1; ++b) {
    off[b] = run;
    run += cnt[b];
  }
  __syncthreads();
  for (int b = lane; b < nb; b += 64) cnt[b] = 0;   // reuse as fill cursor
  __syncthreads();
  for (int e = lane; e < m; e += 64) {
    const int b = min(nb - 1, (int)((double)(A[e] - jmin) * scale));
    G[off[b] + atomicAdd(&cnt[b], 1)] = A[e];
  }
  __syncthreads();
  for (int e = lane; e < m; e += 64) {
    const int j = A[e];
    const int b = min(nb - 1, (int)((double)(j - jmin) * scale));
    const int k0 = off[b], k1 = k0 + cnt[b];
    int rank = k0;
    for (int k = k0; k < k1; ++k) rank += G[k] < j;
    col[start + rank] = j;
  }
}

// Rows of up to kNetMax entries: one wave per row sorts it in registers
// with a bitonic network (Batcher's merge network on the next power of two,
// padded with INT_MAX).  Element e of the row sits in lane e % 64, register
// e / 64, so loads and stores are coalesced; partners 1-32 apart are
// exchanged by lane shuffles, partners 64 or more apart within the lane.
// Waves are independent (no LDS, no barriers).
constexpr int kNetMax = 1024;
constexpr int kNetRows = 4;   // rows (waves) per workgroup

template <int K>   // registers per lane: the row is padded to 64 K entries
__device__ __forceinline__ void net_sort_row(int32_t* __restrict__ c, int m) {
  const int lane = lane_id();
  int v[K];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const int e = q * 64 + lane;
    v[q] = e < m ? c[e] : 0x7fffffff;
  }
#pragma unroll
  for (int k = 2; k <= 64 * K; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j >= 64) {   // partner in register q ^ (j / 64) of the same lane
        const int jq = j >> 6;
#pragma unroll
        for (int q = 0; q < K; ++q) {
          if (q & jq) continue;
          const int p = q | jq;
          const bool up = (((q << 6) | lane) & k) == 0;
          const int lo = min(v[q], v[p]), hi = max(v[q], v[p]);
          v[q] = up ? lo : hi;
          v[p] = up ? hi : lo;
        }
      } else {         // partner in lane ^ j, same register
        const bool lower = (lane & j) == 0;
#pragma unroll
        for (int q = 0; q < K; ++q) {
          const int o = __shfl_xor(v[q], j);
          const bool up = (((q << 6) | lane) & k) == 0;
          v[q] = (lower == up) ? min(v[q], o) : max(v[q], o);
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const int e = q * 64 + lane;
    if (e < m) c[e] = v[q];
  }
}

__global__ __launch_bounds__(64 * kNetRows) void k_rowsort_net(int n,
                                                               const int32_t* __restrict__ row_ptr,
                                                               int32_t* __restrict__ col,
                                                               const int32_t* __restrict__ status) {
  if (*status != 0) return;   // the build failed: row_ptr and col are not a list
  const int i = blockIdx.x * kNetRows + (int)(threadIdx.x >> 6);
  if (i >= n) return;         // wave-uniform: the whole wave leaves
  const int start = row_ptr[i], m = row_ptr[i + 1] - start;
  int32_t* c = col + start;
  if (m <= 1) return;
  if (m <= 64) net_sort_row<1>(c, m);
  else if (m <= 128) net_sort_row<2>(c, m);
  else if (m <= 256) net_sort_row<4>(c, m);
  else if (m <= 512) net_sort_row<8>(c, m);
  else if (m <= kNetMax) net_sort_row<16>(c, m);
  // (longer rows never reach this kernel: the host takes k_rowsort when the
  // row bound exceeds kNetMax, and a longer row fails the build)
}

// The row sort for a list whose rows hold at most max_row entries.
tk_status launch_rowsort(hipStream_t st, int n, const int32_t* row_ptr, int32_t* col, int max_row,
                         size_t lds1, const int32_t* status);

// Dynamic LDS above the default limit must be allowed per kernel.
// (Process-wide: several contexts on several host threads share it.)
tk_status rowsort_attribute(size_t lds) {
  static std::mutex m;
  static size_t done = 0;
  std::lock_guard<std::mutex> lk(m);
  if (lds <= done) return TK_OK;
  TK_HIP(hipFuncSetAttribute((const void*)k_rowsort, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds));
  done = lds;
  return TK_OK;
}

tk_status launch_rowsort(hipStream_t st, int n, const int32_t* row_ptr, int32_t* col, int max_row,
                         size_t lds1, const int32_t* status) {
  if (max_row <= kNetMax) {
    k_rowsort_net<<<ceil_div(n, kNetRows), 64 * kNetRows, 0, st>>>(n, row_ptr, col, status);
    return TK_OK;
  }
  // several rows per workgroup while they fit the default LDS limit
  const int rpb = lds1 * kRowsPerBlock <= 65536 ? kRowsPerBlock : 1;
  const size_t lds = lds1 * rpb;
  tk_status s;
  if (lds > 65536 && (s = rowsort_attribute(lds))) return s;
  k_rowsort<<<ceil_div(n, rpb), 64 * rpb, lds, st>>>(n, row_ptr, col, max_row, status);
  return TK_OK;
}

}  // namespace

// Upload a cells-per-edge template table once.
static tk_status upload_tables(tk_ctx* ctx, CellTables& T) {
  if (T.uploaded) return TK_OK;
  tk_status s;
  if ((s = ensure(ctx, T.units_d, sizeof(Unit) * T.nunits)) ||
      (s = ensure(ctx, T.nslot_d, sizeof(int32_t) * T.ncells)) ||
      (s = ensure(ctx, T.cu_d, sizeof(int32_t) * T.cu.size())) ||
      (s = ensure(ctx, T.order_d, sizeof(int32_t) * T.order.size())))
    return s;
  TK_HIP(hipMemcpy(T.cu_d.p, T.cu.data(), sizeof(int32_t) * T.cu.size(), hipMemcpyHostToDevice));
  TK_HIP(hipMemcpy(T.order_d.p, T.order.data(), sizeof(int32_t) * T.order.size(),
                   hipMemcpyHostToDevice));
  TK_HIP(hipMemcpy(T.units_d.p, T.units.data(), sizeof(Unit) * T.nunits, hipMemcpyHostToDevice));
  TK_HIP(hipMemcpy(T.nslot_d.p, T.nslot.data(), sizeof(int32_t) * T.ncells, hipMemcpyHostToDevice));
  T.uploaded = true;
  return TK_OK;
}

// One list build, split at its host synchronisation so that several builds
// (on one or several streams) share it: begin() queues everything up to the
// readback, finish() checks the readback (rerunning the enumeration in the
// rare case that a bound was short), then queues the compaction and the CSR.
// Each build of a group has its own scratch (names suffixed by its index) and
// its own pinned readback and staging regions.
constexpr int kMaxBuildJobs = 4;
constexpr size_t kStageBase = 4096;   // pinned: [64 k, 64 k + 64) readback of build k; staging after

struct BuildJob {
  // request
  int slot = 0, n = 0, job = 0;
  const double* xyz = nullptr;
  PlanSpec spec{};
  int32_t* row_ptr = nullptr;
  int32_t* col = nullptr;
  int64_t cap = 0;
  int64_t* npairs_out = nullptr;
  hipStream_t st = nullptr;
  // stream-ordered form (tk_nblist_build_async): sizes from the caller's
  // bounds, outcome to device memory, no host synchronisation
  bool async = false;
  tk_nblist_bounds bd{};
  int64_t* npairs_dev = nullptr;
  int32_t* status_dev = nullptr;
  tk_nblist_bounds* report_dev = nullptr;
  // state between the phases
  Plan* P = nullptr;
  std::vector<SysDev> sd;
  std::vector<CellTables*> tabs;
  int nsys = 0, ncells = 0, nunits = 0, occ_cap = 0, plan_waves = 1;
  long pstride = 0;
  double est = 0.0;
  DevBuf* wb = nullptr;
  void *u = nullptr, *cell = nullptr, *ccount = nullptr, *cursor = nullptr, *tmp = nullptr,
       *info = nullptr, *cand = nullptr, *rcnt = nullptr, *rptr = nullptr, *woff = nullptr,
       *cnt64 = nullptr, *regcnt = nullptr, *nfilt = nullptr;
  int32_t *h = nullptr, *hd = nullptr, *rp = nullptr;
  char *stage = nullptr;   // pinned staging of the system table (and batch template pointers)
  const SysDev* sysd = nullptr;
  const Unit* units = nullptr;
  const int32_t *nslot = nullptr, *cu = nullptr, *order = nullptr, *cell_sys = nullptr;

  std::string nm(const char* base) const {
    return job ? std::string(base) + "." + std::to_string(job) : std::string(base);
  }
  size_t stage_bytes() const {   // 256-byte aligned
    const size_t b = sizeof(SysDev) * (spec.nsys + 1) + sizeof(TplPtrs) * spec.nsys;
    return (b + 255) / 256 * 256;
  }
};

// Checks, per-system cell grids and the window estimate.
static tk_status build_check(tk_ctx* ctx, BuildJob& J) {
  if (!J.npairs_out) return TK_E_ARG;
  *J.npairs_out = 0;
  const PlanSpec& spec = J.spec;
  const int nsys = spec.nsys, n = J.n;
  if (nsys < 1 || J.slot < 0 || J.slot >= kNumPlans || J.cap < 0 || n < 0) return TK_E_ARG;
  if (J.col && !J.row_ptr) return TK_E_ARG;
  if (n > 0 && !J.xyz) return TK_E_ARG;
  if (spec.atom0[0] != 0 || spec.atom0[nsys] != n) return TK_E_ARG;
  J.P = &ctx->plans[J.slot];
  J.P->valid = false;
  J.nsys = nsys;
  J.sd.assign(nsys + 1, SysDev{});
  J.tabs.assign(nsys, nullptr);
  J.ncells = J.nunits = 0;
  J.est = 16.0 * n + 65536.0;
  tk_status s;
  for (int k = 0; k < nsys; ++k) {
    const double box = spec.box[k], cut = spec.cutoff[k];
    const int na = spec.atom0[k + 1] - spec.atom0[k];
    if (!(box > 0.0) || !std::isfinite(box) || !(cut > 0.0) || !std::isfinite(cut) || na < 0)
      return TK_E_ARG;
    if (cut > 0.5 * box) return TK_E_CUTOFF;
    int nc = (int)std::floor(box / cut);
    if (nc < 1) nc = 1;
    CellTables& T = cell_tables(ctx, nc);
    if ((s = upload_tables(ctx, T))) return s;
    J.tabs[k] = &T;
    const uint64_t rq = (uint64_t)std::floor((cut / box) * kTwo32);
    SysDev& d = J.sd[k];
    d.box = box;
    d.inv_box = 1.0 / box;
    d.rq2 = rq * rq;
    d.lo = (double)d.rq2 * (1.0 - 0x1p-50);
    d.hi = (double)d.rq2 * (1.0 + 0x1p-50);
    d.nc = nc;
    d.cell0 = J.ncells;
    d.unit0 = J.nunits;
    d.atom0 = spec.atom0[k];
    J.ncells += T.ncells;
    J.nunits += T.nunits;
    // candidate windows: sum over units of |H||K|, estimated from the density
    // (the buffer grows, and the enumeration reruns, if the estimate is short)
    const double mean = (double)na / T.ncells;
    J.est += 1.15 * (double)T.nunits * mean * mean;
  }
  SysDev& t = J.sd[nsys];
  t.cell0 = J.ncells;
  t.unit0 = J.nunits;
  t.atom0 = n;
  return TK_OK;
}

// The enumeration and everything that depends on it up to the readback.
static tk_status enqueue_enumeration(tk_ctx* ctx, BuildJob& J) {
  Plan& P = *J.P;
  const hipStream_t st = J.st;
  const int n = J.n, nunits = J.nunits;
  tk_status s;
  const int32_t* cstart = (const int32_t*)P.cell_start.p;
  if (n > 0) {
    {
      ProfScope ps(ctx, st, "nblist_plan");
      const size_t plds = (2 * sizeof(uint4) + 4 * sizeof(int)) * (size_t)J.occ_cap;
      k_plan<<<nunits, 64 * J.plan_waves, plds, st>>>(
          nunits, J.units, cstart, (uint4*)P.us.p, J.sysd, J.cell_sys, J.pstride,
          (int64_t*)J.woff, (long)(J.wb->bytes / 4), (uint32_t*)J.wb->p, (int32_t*)P.unit_cnt.p,
          (int64_t*)J.cnt64, (int32_t*)J.regcnt, (int2*)J.nfilt, (int32_t*)P.slots.p,
          (int32_t*)J.info, J.occ_cap);
    }
    k_row_slots<<<ceil_div(n, kRowSlotsThreads), kRowSlotsThreads, 0, st>>>(
        n, (int32_t*)P.perm.p, (int32_t*)P.scell.p,
                                                   J.nslot, J.pstride, (int32_t*)P.slots.p,
                                                   (int32_t*)J.rcnt, (int32_t*)J.info);
    // row pointers, and the dense code offsets (with the unit-based pair
    // total for the readback)
    if ((s = scan_pair(ctx, st, (int32_t*)J.rcnt, J.rp, n, (int64_t*)J.cnt64,
                       (int64_t*)P.unit_off.p, nunits, J.job)))
      return s;
  } else {
    TK_HIP(hipMemsetAsync(P.unit_cnt.p, 0, sizeof(int32_t) * nunits, st));
    TK_HIP(hipMemsetAsync(P.unit_off.p, 0, sizeof(int64_t) * (nunits + 1), st));
    TK_HIP(hipMemsetAsync(J.woff, 0, sizeof(int64_t) * (nunits + 1), st));
    TK_HIP(hipMemsetAsync(J.rp, 0, sizeof(int32_t), st));
  }
  if (J.async) {
    const AsyncBounds b{std::min(J.bd.max_occ, kMaxCellAtoms), J.bd.max_row, J.bd.max_nbhd,
                        J.bd.windows, J.cap};
    k_build_status<<<1, 1, 0, st>>>((const int32_t*)J.info, J.rp + n,
                                    (const int64_t*)J.woff + nunits,
                                    (const int64_t*)P.unit_off.p + nunits, b, J.npairs_dev,
                                    J.status_dev, (int32_t*)P.dstat.p, J.report_dev);
    TK_HIP(hipGetLastError());
    return TK_OK;
  }
  // one readback: status, max occupancy, max row, pairs, window overflow,
  // max neighbourhood, list total
  k_readback<<<1, 1, 0, st>>>((int32_t*)J.info, J.rp + n, (int64_t*)J.woff + nunits,
                              (int64_t*)P.unit_off.p + nunits, J.hd, (int32_t*)P.dstat.p);
  TK_HIP(hipGetLastError());
  return TK_OK;
}

// Everything up to the readback, queued on J.st (no synchronisation).
// hb/hdb: the group's pinned buffer (host and device addresses).
static tk_status build_begin(tk_ctx* ctx, BuildJob& J, char* hb, char* hdb) {
  Plan& P = *J.P;
  const hipStream_t st = J.st;
  const int n = J.n, nsys = J.nsys, ncells = J.ncells, nunits = J.nunits;
  const std::vector<SysDev>& sd = J.sd;
  const int nn = n > 0 ? n : 1;
  J.pstride = (nn + 63) / 64 * 64;
  tk_status s;
  if ((s = ensure(ctx, P.perm, sizeof(int32_t) * nn)) || (s = ensure(ctx, P.scell, sizeof(int32_t) * nn)) ||
      (s = ensure(ctx, P.cell_start, sizeof(int32_t) * (ncells + 1))) ||
      (s = ensure(ctx, P.unit_off, sizeof(int64_t) * (nunits + 1))) ||
      (s = ensure(ctx, P.unit_cnt, sizeof(int32_t) * nunits)) ||
      (s = ensure(ctx, P.us, sizeof(uint4) * nn)) ||
      (s = ensure(ctx, P.slots, sizeof(int32_t) * kMaxSlots * J.pstride)) ||
      (s = ensure(ctx, P.dstat, 2 * sizeof(int32_t))))
    return s;
  const void* sysd_was = P.sysd.p;
  if ((s = ensure(ctx, P.sysd, sizeof(SysDev) * (nsys + 1)))) return s;
  // candidate windows: scratch of the build (the plan keeps the dense
  // codes); grown to the exact size and rerun if the estimate is short
  J.wb = &ctx->scratch[J.nm("nb_windows")];
  if (J.wb->bytes < sizeof(uint32_t) * (size_t)J.est &&
      (s = ensure(ctx, *J.wb, sizeof(uint32_t) * (size_t)J.est)))
    return s;
  if ((s = scratch(ctx, J.nm("nb_u").c_str(), sizeof(uint32_t) * 3 * nn, &J.u)) ||
      (s = scratch(ctx, J.nm("nb_cell").c_str(), sizeof(int32_t) * nn, &J.cell)) ||
      (s = scratch(ctx, J.nm("nb_ccount").c_str(), sizeof(int32_t) * (ncells + 1), &J.ccount)) ||
      (s = scratch(ctx, J.nm("nb_cursor").c_str(), sizeof(int32_t) * ncells, &J.cursor)) ||
      (s = scratch(ctx, J.nm("nb_tmp").c_str(), sizeof(int32_t) * nn, &J.tmp)) ||
      (s = scratch(ctx, J.nm("nb_info").c_str(), sizeof(int32_t) * 8, &J.info)) ||
      (s = scratch(ctx, J.nm("nb_cand").c_str(), sizeof(int64_t) * (nunits + 1), &J.cand)) ||
      (s = scratch(ctx, J.nm("nb_woff").c_str(), sizeof(int64_t) * (nunits + 1), &J.woff)) ||
      (s = scratch(ctx, J.nm("nb_cnt64").c_str(), sizeof(int64_t) * (nunits + 1), &J.cnt64)) ||
      (s = scratch(ctx, J.nm("nb_rcnt").c_str(), sizeof(int32_t) * (nn + 1), &J.rcnt)) ||
      (s = scratch(ctx, J.nm("nb_rptr").c_str(), sizeof(int32_t) * (nn + 1), &J.rptr)) ||
      (s = scratch(ctx, J.nm("nb_regcnt").c_str(), sizeof(int32_t) * kPlanRegions * (size_t)nunits,
                   &J.regcnt)) ||
      (s = scratch(ctx, J.nm("nb_nfilt").c_str(), sizeof(int2) * (size_t)nunits, &J.nfilt)))
    return s;
  const size_t sys_bytes = sizeof(SysDev) * (nsys + 1);
  if (J.async) {   // one system (checked by the caller): table and status words by one kernel
    SysPair v;
    v.s[0] = sd[0];
    v.s[1] = sd[1];
    k_put_sys<<<1, 64, 0, st>>>(v, (SysDev*)P.sysd.p, (int32_t*)J.info);
    P.h_sys = sd;
  }
  // pinned (synchronous builds): this build's readback slot, then its
  // staging region
  J.h = J.async ? nullptr : (int32_t*)(hb + 64 * J.job);
  J.hd = J.async ? nullptr : (int32_t*)(hdb + 64 * J.job);
  char* stage = J.stage;
  // the previous readback and staging of this context have been consumed
  // (every group synchronises before it returns).  The system table is
  // uploaded only when it differs from the plan's copy.
  if (!J.async && (P.sysd.p != sysd_was || P.h_sys.size() != sd.size() ||
                   std::memcmp(P.h_sys.data(), sd.data(), sys_bytes) != 0)) {
    std::memcpy(stage, sd.data(), sys_bytes);
    TK_HIP(hipMemcpyAsync(P.sysd.p, stage, sys_bytes, hipMemcpyHostToDevice, st));
    P.h_sys = sd;
  }
  J.sysd = (const SysDev*)P.sysd.p;
  J.cell_sys = nullptr;
  if (nsys == 1) {
    J.units = (const Unit*)J.tabs[0]->units_d.p;
    J.nslot = (const int32_t*)J.tabs[0]->nslot_d.p;
    J.cu = (const int32_t*)J.tabs[0]->cu_d.p;
    J.order = (const int32_t*)J.tabs[0]->order_d.p;
  } else {
    TplPtrs* tp = (TplPtrs*)(stage + sys_bytes);
    for (int k = 0; k < nsys; ++k)
      tp[k] = TplPtrs{(const Unit*)J.tabs[k]->units_d.p, (const int32_t*)J.tabs[k]->nslot_d.p,
                      (const int32_t*)J.tabs[k]->cu_d.p, (const int32_t*)J.tabs[k]->order_d.p};
    if ((s = ensure(ctx, P.tplp, sizeof(TplPtrs) * nsys)) ||
        (s = ensure(ctx, P.bunits, sizeof(Unit) * nunits)) ||
        (s = ensure(ctx, P.bnslot, sizeof(int32_t) * ncells)) ||
        (s = ensure(ctx, P.bcu, sizeof(int32_t) * kCellUnitStride * (size_t)ncells)) ||
        (s = ensure(ctx, P.cell_sys, sizeof(int32_t) * ncells)) ||
        (s = ensure(ctx, P.border, sizeof(int32_t) * ncells)))
      return s;
    TK_HIP(hipMemcpyAsync(P.tplp.p, tp, sizeof(TplPtrs) * nsys, hipMemcpyHostToDevice, st));
    k_batch_units<<<ceil_div(nunits, 256), 256, 0, st>>>(nunits, nsys, J.sysd,
                                                         (const TplPtrs*)P.tplp.p,
                                                         (Unit*)P.bunits.p);
    k_batch_cells<<<ceil_div(ncells, 256), 256, 0, st>>>(ncells, nsys, J.sysd,
                                                         (const TplPtrs*)P.tplp.p,
                                                         (int32_t*)P.bnslot.p, (int32_t*)P.bcu.p,
                                                         (int32_t*)P.cell_sys.p,
                                                         (int32_t*)P.border.p);
    J.units = (const Unit*)P.bunits.p;
    J.nslot = (const int32_t*)P.bnslot.p;
    J.cu = (const int32_t*)P.bcu.p;
    J.order = (const int32_t*)P.border.p;
    J.cell_sys = (const int32_t*)P.cell_sys.p;
  }
  // status words: zero after every completed build (the readback clears them;
  // a stream-ordered build clears them with its system table)
  if (!J.async) {
    if (!ctx->nb_info_zero[J.job]) TK_HIP(hipMemsetAsync(J.info, 0, sizeof(int32_t) * 8, st));
    ctx->nb_info_zero[J.job] = false;
  }
  const int32_t* cstart = (const int32_t*)P.cell_start.p;
  J.rp = J.row_ptr ? J.row_ptr : (int32_t*)J.rptr;
  int32_t* info = (int32_t*)J.info;
  if (n > 0 && ncells <= kMaxHistCells) {
    const int nblk = ceil_div(n, kHistBlock);
    const long hl = (long)ncells * nblk;
    void *H, *Hoff;
    if ((s = scratch(ctx, J.nm("nb_hist").c_str(), sizeof(int32_t) * hl, &H)) ||
        (s = scratch(ctx, J.nm("nb_hist_off").c_str(), sizeof(int32_t) * (hl + 1), &Hoff)))
      return s;
    {
      ProfScope ps(ctx, st, "nblist_quantize");
      k_quantize_hist<<<nblk, kHistBlock, 0, st>>>(n, J.xyz, J.sysd, nsys, ncells,
                                                    (uint32_t*)J.u, (int32_t*)J.cell,
                                                    (int32_t*)H, info);
    }
    if ((s = scan_i32(ctx, st, (int32_t*)H, (int32_t*)Hoff, (int)hl, J.job))) return s;
    {
      ProfScope ps(ctx, st, "nblist_cellsort");
      k_scatter_stable<<<nblk, kHistBlock, 0, st>>>(n, ncells, (int32_t*)J.cell, (int32_t*)Hoff,
                                                     (uint32_t*)J.u, (int32_t*)P.perm.p,
                                                     (int32_t*)P.scell.p, (uint4*)P.us.p,
                                                     (int32_t*)P.cell_start.p, info);
    }
  } else if (n > 0) {
    TK_HIP(hipMemsetAsync(J.ccount, 0, sizeof(int32_t) * (ncells + 1), st));
    TK_HIP(hipMemsetAsync(J.cursor, 0, sizeof(int32_t) * ncells, st));
    {
      ProfScope ps(ctx, st, "nblist_quantize");
      k_quantize<<<ceil_div(n, 256), 256, 0, st>>>(n, J.xyz, J.sysd, nsys, (uint32_t*)J.u,
                                                    (int32_t*)J.cell, (int32_t*)J.ccount, info);
    }
    if ((s = scan_i32(ctx, st, (int32_t*)J.ccount, (int32_t*)P.cell_start.p, ncells, J.job)))
      return s;
    k_scatter<<<ceil_div(n, 256), 256, 0, st>>>(n, (int32_t*)J.cell, cstart, (int32_t*)J.cursor,
                                                 (int32_t*)J.tmp);
    {
      ProfScope ps(ctx, st, "nblist_cellsort");
      k_cellsort<<<ncells, 64, 0, st>>>(cstart, (int32_t*)J.tmp, (uint32_t*)J.u,
                                        (int32_t*)P.perm.p, (int32_t*)P.scell.p, (uint4*)P.us.p,
                                        info);
    }
  } else {
    TK_HIP(hipMemsetAsync(P.cell_start.p, 0, sizeof(int32_t) * (ncells + 1), st));
  }
  if (n > 0) {
    const int nbu = ceil_div(nunits, 256);
    k_cand_nbhd<<<nbu + ceil_div(ncells, 4), 256, 0, st>>>(nunits, ncells, nbu, J.cu, J.units,
                                                         cstart, (int64_t*)J.cand, info);
    if ((s = scan_i64(ctx, st, (int64_t*)J.cand, (int64_t*)J.woff, nunits, J.job))) return s;
  }
  // staging bound of k_plan: three times the largest mean cell occupancy
  // (at least 64); a denser cell makes the build rerun with kMaxCellAtoms
  double max_mean = 0.0;
  for (int k = 0; k < nsys; ++k) {
    const int cells = sd[k + 1].cell0 - sd[k].cell0;
    max_mean = std::fmax(max_mean, (double)(J.spec.atom0[k + 1] - J.spec.atom0[k]) / cells);
  }
  int occ_cap = (int)std::ceil(3.0 * max_mean);
  J.occ_cap = occ_cap < 64 ? 64 : occ_cap > kMaxCellAtoms ? kMaxCellAtoms : occ_cap;
  if (J.async) J.occ_cap = std::min(J.bd.max_occ, kMaxCellAtoms);   // the caller's bound
  // waves per unit of the enumeration: more for larger cells
  J.plan_waves = max_mean > 96.0 ? 4 : max_mean > 48.0 ? 2 : 1;
  return enqueue_enumeration(ctx, J);
}

// After the stream has reached the readback: checks (and the rare rerun),
// then the compaction and the CSR, queued (no further synchronisation).
static tk_status build_finish(tk_ctx* ctx, BuildJob& J) {
  Plan& P = *J.P;
  const hipStream_t st = J.st;
  const int n = J.n, nunits = J.nunits;
  int32_t* h = J.h;
  tk_status s;
  ctx->nb_info_zero[J.job] = true;
  if (h[0] != 0) return h[0];
  if (h[4] != 0) {
    // windows or staging bound did not fit: exact sizes, enumerate again (the
    // rerun repeats neither the cell sort nor the neighbourhood sizes)
    const int first_occ = h[1], first_nbhd = h[5];
    const int64_t need = *(int64_t*)(h + 8);
    if ((s = ensure(ctx, *J.wb, sizeof(uint32_t) * (size_t)need))) return s;
    J.occ_cap = kMaxCellAtoms;
    ctx->nb_info_zero[J.job] = false;
    if ((s = enqueue_enumeration(ctx, J))) return s;
    TK_HIP(hipStreamSynchronize(st));
    ctx->nb_info_zero[J.job] = true;
    h[1] = first_occ;
    h[5] = first_nbhd;
    if (h[0] != 0) return h[0];
    if (h[4] != 0) return TK_E_HIP;
  }
  const int64_t list_pairs = h[6];
  *J.npairs_out = list_pairs;
  if (list_pairs != (int64_t)h[3]) {
    std::fprintf(stderr, "libtk: plan/list pair count mismatch %d vs %d\n", h[3], h[6]);
    return TK_E_HIP;
  }
  const int max_row = h[2];
  // dense codes at unit_off (the exclusive scan of the unit counts), and the
  // per-unit records of the pair kernels
  if ((s = ensure(ctx, P.codes, sizeof(uint32_t) * (size_t)(list_pairs > 0 ? list_pairs : 1))) ||
      (s = ensure(ctx, P.urec, sizeof(UnitRec) * (size_t)(nunits > 0 ? nunits : 1))))
    return s;
  const int32_t* cstart = (const int32_t*)P.cell_start.p;
  if (J.row_ptr && list_pairs > J.cap) return TK_E_CAPACITY;
  const int occ = h[1] > 0 ? h[1] : 1;
  if (n > 0) {
    // the dense codes, the unit records and (when asked for) the CSR entries
    ProfScope ps(ctx, st, "nblist_compact");
    CsrOut csr{(const int32_t*)P.perm.p, (const int32_t*)P.slots.p, J.rp,
               J.row_ptr && list_pairs > 0 ? J.col : nullptr, (long)J.cap, J.pstride, occ};
    compact_launch((double)list_pairs / std::max(nunits, 1), nunits, sizeof(int) * 4 * (size_t)occ,
                   st, (const int64_t*)J.woff, (const uint32_t*)J.wb->p,
                   (const int64_t*)P.unit_off.p, (const int32_t*)J.regcnt, (const int2*)J.nfilt,
                   J.plan_waves, (uint32_t*)P.codes.p, J.units, cstart,
                   (const int32_t*)P.unit_cnt.p, J.cell_sys, (UnitRec*)P.urec.p, csr,
                   (long)(P.codes.bytes / sizeof(uint32_t)), (const int32_t*)P.dstat.p);
  }
  if (J.row_ptr) {
    const int nb = max_row < kBuckets ? max_row : kBuckets;
    const size_t lds1 = sizeof(int) * (2 * (size_t)max_row + 2 * (size_t)nb);
    if (max_row > kNetMax && lds1 > kMaxLds) return TK_E_CAPACITY;
    if (n > 0 && list_pairs > 0) {
      ProfScope ps(ctx, st, "nblist_rowsort");
      if ((s = launch_rowsort(st, n, J.rp, J.col, max_row, lds1, (const int32_t*)P.dstat.p)))
        return s;
    }
  }
  TK_HIP(hipGetLastError());
  P.valid = true;
  P.n = n;
  P.nsys = J.nsys;
  P.box = J.spec.box[0];
  P.cutoff = J.spec.cutoff[0];
  P.nc = J.sd[0].nc;
  P.ncells = J.ncells;
  P.nunits = nunits;
  P.max_occ = h[1];
  P.max_row = max_row;
  P.max_nbhd = h[5];
  P.npairs = list_pairs;
  P.windows = *(int64_t*)(h + 8);
  P.measured = true;
  P.units_p = J.units;
  P.nslot_p = J.nslot;
  P.cu_p = J.cu;
  P.order_p = J.order;
  return TK_OK;
}

// A group of builds sharing one host synchronisation per distinct stream.
static tk_status build_group(tk_ctx* ctx, BuildJob* jobs, int nj) {
  if (nj < 1 || nj > kMaxBuildJobs) return TK_E_ARG;
  tk_status s;
  for (int k = 0; k < nj; ++k) {
    jobs[k].job = k;
    for (int m = 0; m < k; ++m)   // two builds of a group may not share a plan slot
      if (jobs[m].slot == jobs[k].slot) return TK_E_ARG;
    if ((s = build_check(ctx, jobs[k]))) return s;
  }
  // pinned buffer for the whole group, taken before anything is queued
  size_t bytes = kStageBase;
  for (int k = 0; k < nj; ++k) bytes += jobs[k].stage_bytes();
  char *hb, *hdb;
  if ((s = pinned(ctx, bytes, (void**)&hb, (void**)&hdb))) return s;
  size_t off = kStageBase;
  for (int k = 0; k < nj; ++k) {
    jobs[k].stage = hb + off;
    off += jobs[k].stage_bytes();
  }
  // queue every build; on a failure the builds already queued are waited for
  // (they write the pinned buffer) before the error is returned
  int queued = 0;
  for (; queued < nj; ++queued)
    if ((s = build_begin(ctx, jobs[queued], hb, hdb))) break;
  // builds to wait for: all, or those queued (in full or in part) before a failure
  const int nwait = s ? queued + 1 : nj;
  for (int k = 0; k < nwait; ++k) {
    bool seen = false;
    for (int m = 0; m < k; ++m) seen |= jobs[m].st == jobs[k].st;
    if (!seen) {
      const hipError_t e = hipStreamSynchronize(jobs[k].st);
      if (!s && e != hipSuccess) return hip_status(e, "hipStreamSynchronize");
    }
  }
  if (s) return s;
  for (int k = 0; k < nj; ++k)
    if ((s = build_finish(ctx, jobs[k]))) return s;
  return TK_OK;
}

// Stream-ordered build, after the enumeration has been queued: the dense
// codes, unit records and CSR sized from the caller's capacity and bounds.
// The kernels check the device status that k_build_status wrote (a build
// past its bounds writes nothing), so nothing here waits for the host.
static tk_status build_finish_async(tk_ctx* ctx, BuildJob& J) {
  Plan& P = *J.P;
  const hipStream_t st = J.st;
  const int n = J.n, nunits = J.nunits;
  tk_status s;
  const int occ = std::max(1, std::min(J.bd.max_occ, kMaxCellAtoms));
  const int max_row = J.bd.max_row;
  const int nb = max_row < kBuckets ? max_row : kBuckets;
  const size_t lds1 = sizeof(int) * (2 * (size_t)max_row + 2 * (size_t)nb);
  if (J.row_ptr && max_row > kNetMax && lds1 > kMaxLds) return TK_E_CAPACITY;
  if ((s = ensure(ctx, P.codes, sizeof(uint32_t) * (size_t)std::max<int64_t>(J.cap, 1))) ||
      (s = ensure(ctx, P.urec, sizeof(UnitRec) * (size_t)(nunits > 0 ? nunits : 1))))
    return s;
  const int32_t* cstart = (const int32_t*)P.cell_start.p;
  if (n > 0) {
    ProfScope ps(ctx, st, "nblist_compact");
    CsrOut csr{(const int32_t*)P.perm.p, (const int32_t*)P.slots.p, J.rp, J.row_ptr ? J.col : nullptr,
               (long)J.cap, J.pstride, occ};
    // the pair capacity stands in for the count, which only the device knows
    compact_launch((double)J.cap / std::max(nunits, 1), nunits, sizeof(int) * 4 * (size_t)occ, st,
                   (const int64_t*)J.woff, (const uint32_t*)J.wb->p,
                   (const int64_t*)P.unit_off.p, (const int32_t*)J.regcnt, (const int2*)J.nfilt,
                   J.plan_waves, (uint32_t*)P.codes.p, J.units, cstart,
                   (const int32_t*)P.unit_cnt.p, J.cell_sys, (UnitRec*)P.urec.p, csr,
                   (long)(P.codes.bytes / sizeof(uint32_t)), (const int32_t*)P.dstat.p);
  }
  if (J.row_ptr && n > 0) {
    ProfScope ps(ctx, st, "nblist_rowsort");
    if ((s = launch_rowsort(st, n, J.rp, J.col, max_row, lds1, (const int32_t*)P.dstat.p)))
      return s;
  }
  TK_HIP(hipGetLastError());
  P.valid = true;
  P.n = n;
  P.nsys = J.nsys;
  P.box = J.spec.box[0];
  P.cutoff = J.spec.cutoff[0];
  P.nc = J.sd[0].nc;
  P.ncells = J.ncells;
  P.nunits = nunits;
  P.max_occ = occ;
  P.max_row = max_row;
  P.max_nbhd = J.bd.max_nbhd;
  P.npairs = -1;
  P.measured = false;
  P.units_p = J.units;
  P.nslot_p = J.nslot;
  P.cu_p = J.cu;
  P.order_p = J.order;
  return TK_OK;
}

tk_status build_plans(tk_ctx* ctx, hipStream_t st, int nj, const int* slots, int n,
                      const double* xyz, const PlanSpec* specs, int64_t* npairs_out) {
  if (nj < 1 || nj > kMaxBuildJobs) return TK_E_ARG;
  BuildJob J[kMaxBuildJobs];
  for (int k = 0; k < nj; ++k) {
    J[k].slot = slots[k];
    J[k].n = n;
    J[k].xyz = xyz;
    J[k].spec = specs[k];
    J[k].npairs_out = &npairs_out[k];
    J[k].st = st;
  }
  return build_group(ctx, J, nj);
}

tk_status build_plan(tk_ctx* ctx, hipStream_t st, int slot, int n, const double* xyz,
                     const PlanSpec& spec, int32_t* row_ptr, int32_t* col, int64_t cap,
                     int64_t* npairs_out) {
  BuildJob J;
  J.slot = slot;
  J.n = n;
  J.xyz = xyz;
  J.spec = spec;
  J.row_ptr = row_ptr;
  J.col = col;
  J.cap = cap;
  J.npairs_out = npairs_out;
  J.st = st;
  return build_group(ctx, &J, 1);
}

static tk_status nblist_build_impl(tk_ctx* ctx, hipStream_t st, const tk_system* sys,
                                   double cutoff, int slot, int32_t* row_ptr, int32_t* col,
                                   int64_t cap, int64_t* npairs_out) {
  if (!npairs_out) return TK_E_ARG;
  *npairs_out = 0;
  tk_status s = check_system(sys);
  if (s) return s;
  if (!(cutoff > 0.0) || !std::isfinite(cutoff)) return TK_E_ARG;
  if (slot < 0 || slot >= TK_MAX_PLANS) return TK_E_ARG;
  const int32_t atom0[2] = {0, sys->n};
  PlanSpec spec{1, atom0, &sys->box, &cutoff};
  return build_plan(ctx, st, slot, sys->n, sys->xyz, spec, row_ptr, col, cap, npairs_out);
}

static tk_status nblist_build_multi_impl(tk_ctx* ctx, int nl, void* const* streams,
                                         const tk_system* sys, const double* cutoffs,
                                         const int32_t* slots, int32_t* const* row_ptrs,
                                         int32_t* const* cols, const int64_t* caps,
                                         int64_t* npairs) {
  if (nl < 1 || nl > kMaxBuildJobs || !cutoffs || !slots || !npairs) return TK_E_ARG;
  for (int k = 0; k < nl; ++k) npairs[k] = 0;
  tk_status s = check_system(sys);
  if (s) return s;
  const int32_t atom0[2] = {0, sys->n};
  BuildJob J[kMaxBuildJobs];
  for (int k = 0; k < nl; ++k) {
    if (!(cutoffs[k] > 0.0) || !std::isfinite(cutoffs[k])) return TK_E_ARG;
    if (slots[k] < 0 || slots[k] >= TK_MAX_PLANS) return TK_E_ARG;
    J[k].slot = slots[k];
    J[k].n = sys->n;
    J[k].xyz = sys->xyz;
    J[k].spec = PlanSpec{1, atom0, &sys->box, &cutoffs[k]};
    J[k].row_ptr = row_ptrs ? row_ptrs[k] : nullptr;
    J[k].col = cols ? cols[k] : nullptr;
    J[k].cap = caps ? caps[k] : 0;
    J[k].npairs_out = &npairs[k];
    J[k].st = streams ? (hipStream_t)streams[k] : nullptr;
  }
  return build_group(ctx, J, nl);
}

static tk_status nblist_build_async_impl(tk_ctx* ctx, hipStream_t st, const tk_system* sys,
                                         double cutoff, int slot, const tk_nblist_bounds* bd,
                                         int32_t* row_ptr, int32_t* col, int64_t cap,
                                         int64_t* npairs_dev, int32_t* status_dev,
                                         tk_nblist_bounds* report) {
  if (!bd || !npairs_dev || !status_dev || cap < 0) return TK_E_ARG;
  if (bd->windows < 1 || bd->max_occ < 1 || bd->max_row < 1 || bd->max_nbhd < 1 || bd->npairs < 0)
    return TK_E_ARG;
  tk_status s = check_system(sys);
  if (s) return s;
  if (!(cutoff > 0.0) || !std::isfinite(cutoff)) return TK_E_ARG;
  if (slot < 0 || slot >= TK_MAX_PLANS) return TK_E_ARG;
  const int32_t atom0[2] = {0, sys->n};
  int64_t host_np = 0;   // build_check's host count (unused here)
  BuildJob J;
  J.slot = slot;
  J.job = kMaxBuildJobs + slot;   // scratch of its own per slot: slots build concurrently
  J.n = sys->n;
  J.xyz = sys->xyz;
  J.spec = PlanSpec{1, atom0, &sys->box, &cutoff};
  J.row_ptr = row_ptr;
  J.col = col;
  J.cap = cap;
  J.npairs_out = &host_np;
  J.st = st;
  J.async = true;
  J.bd = *bd;
  J.npairs_dev = npairs_dev;
  J.status_dev = status_dev;
  J.report_dev = report;
  if ((s = build_check(ctx, J))) return s;
  J.est = (double)bd->windows;   // the candidate windows: the caller's bound
  if ((s = build_begin(ctx, J, nullptr, nullptr))) return s;
  return build_finish_async(ctx, J);
}

static tk_status nblist_bounds_get_impl(tk_ctx* ctx, int slot, double headroom,
                                        tk_nblist_bounds* out) {
  if (!out || slot < 0 || slot >= TK_MAX_PLANS || !(headroom >= 0.0) || !std::isfinite(headroom))
    return TK_E_ARG;
  const Plan& P = ctx->plans[slot];
  if (!P.valid || !P.measured || P.nsys != 1) return TK_E_PLAN;
  const double f = 1.0 + headroom;
  auto up32 = [f](int32_t v) { return (int32_t)std::min(std::ceil(f * std::max(v, 1)), 2.0e9); };
  auto up64 = [f](int64_t v) { return (int64_t)std::ceil(f * (double)std::max<int64_t>(v, 1)); };
  out->max_occ = std::min(up32(P.max_occ), kMaxCellAtoms);
  out->max_row = up32(P.max_row);
  out->max_nbhd = up32(P.max_nbhd);
  out->reserved = 0;
  out->windows = up64(P.windows);
  out->npairs = up64(P.npairs);
  return TK_OK;
}

}  // namespace tk

extern "C" tk_status tk_nblist_bounds_get(tk_ctx* ctx, int32_t plan_slot, double headroom,
                                          tk_nblist_bounds* out) {
  if (!ctx) return TK_E_ARG;
  return tk::nblist_bounds_get_impl(ctx, plan_slot, headroom, out);
}

extern "C" tk_status tk_nblist_build_async(tk_ctx* ctx, void* stream, const tk_system* sys,
                                           double cutoff, int32_t plan_slot,
                                           const tk_nblist_bounds* bounds, int32_t* row_ptr,
                                           int32_t* col, int64_t cap, int64_t* npairs_dev,
                                           int32_t* status_dev, tk_nblist_bounds* report_dev) {
  if (!ctx) return TK_E_ARG;
  return tk::nblist_build_async_impl(ctx, (hipStream_t)stream, sys, cutoff, plan_slot, bounds,
                                     row_ptr, col, cap, npairs_dev, status_dev, report_dev);
}

extern "C" tk_status tk_nblist_build(tk_ctx* ctx, void* stream, const tk_system* sys, double cutoff,
                                     int32_t plan_slot, int32_t* row_ptr, int32_t* col, int64_t cap,
                                     int64_t* npairs) {
  if (!ctx) return TK_E_ARG;
  return tk::nblist_build_impl(ctx, (hipStream_t)stream, sys, cutoff, plan_slot, row_ptr, col, cap,
                               npairs);
}

extern "C" tk_status tk_nblist_build_multi(tk_ctx* ctx, int32_t nlists, void* const* streams,
                                           const tk_system* sys, const double* cutoffs,
                                           const int32_t* plan_slots, int32_t* const* row_ptrs,
                                           int32_t* const* cols, const int64_t* caps,
                                           int64_t* npairs) {
  if (!ctx) return TK_E_ARG;
  return tk::nblist_build_multi_impl(ctx, nlists, streams, sys, cutoffs, plan_slots, row_ptrs,
                                     cols, caps, npairs);
}
