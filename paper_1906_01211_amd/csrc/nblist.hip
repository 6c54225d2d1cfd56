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
//   -> canonical CSR written from the pair codes -> rows ordered by j.
// Every pair decision is the same exact test, so the plan (what the pair
// kernels read) and the CSR (what the caller reads) hold the same pair set.
#include <cmath>

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
// around rq^2 it decides; inside the band the exact 64-bit test decides.
struct PairTest {
  uint64_t rq2;
  double lo, hi;
  __device__ __forceinline__ bool operator()(const uint4& a, const uint4& b) const {
    const double dx = (double)(int32_t)(b.x - a.x), dy = (double)(int32_t)(b.y - a.y),
                 dz = (double)(int32_t)(b.z - a.z);
    const double d2 = fma(dx, dx, fma(dy, dy, dz * dz));
    if (d2 < lo) return true;
    if (d2 > hi) return false;
    return pair_in(a, b, rq2);
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

// info: [0] status, [1] max cell occupancy, [2] max CSR row, [3] listed pairs,
//       [4] 1 if the candidate windows did not fit the plan buffer,
//       [5] max atoms over a cell's neighbour cells
// u = floor(frac(x/L) * 2^32) per coordinate; cell = (u * nc) >> 32 per axis.
__global__ void k_quantize(int n, const double* __restrict__ xyz, double box, int nc,
                           uint32_t* __restrict__ u, int32_t* __restrict__ cell,
                           int32_t* __restrict__ cell_count, int32_t* __restrict__ info) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c[3];
  for (int a = 0; a < 3; ++a) {
    double x = xyz[3 * i + a];
    uint32_t q = 0;
    if (isfinite(x)) {
      double t = x / box;
      double f = t - floor(t);
      if (f >= 1.0) f = 0.0;
      q = (uint32_t)(f * kTwo32);
    } else {
      atomicMin(&info[0], (int)TK_E_ARG);
    }
    u[3 * i + a] = q;
    c[a] = (int)(((uint64_t)q * (uint64_t)nc) >> 32);
  }
  int cc = (c[0] * nc + c[1]) * nc + c[2];
  cell[i] = cc;
  atomicAdd(&cell_count[cc], 1);
}

// Stable counting sort by cell without global atomics (boxes with at most
// kMaxHistCells cells): per-block LDS histograms H[c][b], one exclusive scan
// over H in cell-major order, then each atom's slot is its (cell, block)
// offset plus its rank among the block's earlier atoms of the same cell.
// Slots come out ordered by (cell, caller index).
constexpr int kHistBlock = 256;
constexpr int kMaxHistCells = 4096;

__global__ __launch_bounds__(kHistBlock) void k_quantize_hist(int n, const double* __restrict__ xyz,
                                                              double box, int nc, int ncells,
                                                              uint32_t* __restrict__ u,
                                                              int32_t* __restrict__ cell,
                                                              int32_t* __restrict__ H,
                                                              int32_t* __restrict__ info) {
  __shared__ int hist[kMaxHistCells];
  for (int c = threadIdx.x; c < ncells; c += kHistBlock) hist[c] = 0;
  __syncthreads();
  const int i = blockIdx.x * kHistBlock + threadIdx.x;
  if (i < n) {
    int c[3];
    for (int a = 0; a < 3; ++a) {
      const double x = xyz[3 * i + a];
      uint32_t q = 0;
      if (isfinite(x)) {
        const double t = x / box;
        double f = t - floor(t);
        if (f >= 1.0) f = 0.0;
        q = (uint32_t)(f * kTwo32);
      } else {
        atomicMin(&info[0], (int)TK_E_ARG);
      }
      u[3 * i + a] = q;
      c[a] = (int)(((uint64_t)q * (uint64_t)nc) >> 32);
    }
    const int cc = (c[0] * nc + c[1]) * nc + c[2];
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
    for (int cc = threadIdx.x; cc < ncells; cc += kHistBlock) {
      const int s0 = off[(long)cc * nblk];
      const int s1 = cc + 1 < ncells ? off[(long)(cc + 1) * nblk] : n;
      cstart[cc] = s0;
      atomicMax(&info[1], s1 - s0);
      if (s1 - s0 > kMaxCellAtoms) atomicMin(&info[0], (int)TK_E_CAPACITY);
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
    if (threadIdx.x == 0) atomicMin(&info[0], (int)TK_E_CAPACITY);
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

// Candidate window of each unit: |H| * |K| slots.
__global__ void k_cand(int nunits, const Unit* __restrict__ units, const int32_t* __restrict__ cstart,
                       int64_t* __restrict__ cand) {
  int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= nunits) return;
  Unit un = units[u];
  cand[u] = (int64_t)(cstart[un.h + 1] - cstart[un.h]) * (int64_t)(cstart[un.k + 1] - cstart[un.k]);
}

// One wave per cell-pair unit (H, K), both cells staged in LDS.  Candidates
// (a in H, b in K) are visited in "diagonal" order b = (a + k) mod |K|, so
// consecutive listed pairs touch distinct atoms on both sides (conflict-free
// LDS accumulation in the pair kernels).  Writes the unit's pair codes
// a | b << 16 into its window, the unit's pair count, and per (unit role,
// atom) the number of pairs whose CSR row is that atom's (the smaller caller
// index owns the pair).
__global__ __launch_bounds__(64) void k_plan(int nunits, const Unit* __restrict__ units,
                                             const int32_t* __restrict__ cstart,
                                             const uint4* __restrict__ us, PairTest test,
                                             long pstride, const int64_t* __restrict__ unit_off,
                                             long code_cap, uint32_t* __restrict__ codes,
                                             int32_t* __restrict__ unit_cnt,
                                             int32_t* __restrict__ slot_cnt,
                                             int32_t* __restrict__ info) {
  __shared__ uint4 sK[kMaxCellAtoms];
  __shared__ int cH[kMaxCellAtoms], cK[kMaxCellAtoms];
  const int uidx = blockIdx.x;
  const int lane = lane_id();
  if (unit_off[nunits] > code_cap) {   // windows do not fit: host grows the buffer, reruns
    if (uidx == 0 && lane == 0) info[4] = 1;
    return;
  }
  const Unit un = units[uidx];
  const int hs = cstart[un.h], nh = cstart[un.h + 1] - hs;
  const int ks = cstart[un.k], nk = cstart[un.k + 1] - ks;
  if (nh > kMaxCellAtoms || nk > kMaxCellAtoms) return;
  const bool self = un.h == un.k;
  for (int t = lane; t < nh; t += 64) cH[t] = 0;
  for (int t = lane; t < nk; t += 64) {
    sK[t] = us[ks + t];
    cK[t] = 0;
  }
  __syncthreads();
  uint32_t* out = codes + unit_off[uidx];
  int cnt = 0;
  // visit order: (k, a) with a fastest; each lane keeps its own H atom in
  // registers for a whole chunk of 64 a's.
  for (int a0 = 0; a0 < nh; a0 += 64) {
    const int a = a0 + lane;
    const uint4 ua = a < nh ? us[hs + a] : make_uint4(0, 0, 0, 0);
    int b = a;   // b = (a + kk) mod nk, advanced incrementally
    while (b >= nk && nk > 0) b -= nk;
    for (int kk = 0; kk < nk; ++kk) {
      bool pass = false;
      if (a < nh && (!self || a < b)) pass = test(ua, sK[b]);
      const uint64_t mask = __ballot(pass);
      if (pass) {
        out[cnt + lanes_below(mask)] = (uint32_t)a | ((uint32_t)b << 16);
        atomicAdd(ua.w < sK[b].w ? &cH[a] : &cK[b], 1);
      }
      cnt += __popcll(mask);
      if (++b == nk) b = 0;
    }
  }
  __syncthreads();
  if (lane == 0) {
    unit_cnt[uidx] = cnt;
    atomicAdd(&info[3], cnt);
  }
  for (int t = lane; t < nh; t += 64) slot_cnt[(long)un.slot_h * pstride + hs + t] = cH[t];
  for (int t = lane; t < nk; t += 64) slot_cnt[(long)un.slot_k * pstride + ks + t] = cK[t];
}

// Per sorted atom: the CSR row length (sum over its unit roles, written in
// caller order) and, in place, the exclusive prefix of its per-role counts.
__global__ void k_row_slots(int n, const int32_t* __restrict__ perm, const int32_t* __restrict__ scell,
                            const int32_t* __restrict__ cell_nslot, long pstride,
                            int32_t* __restrict__ slot_cnt, int32_t* __restrict__ row_cnt,
                            int32_t* __restrict__ info) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int ns = cell_nslot[scell[s]];
  int c[kMaxSlots];
#pragma unroll
  for (int k = 0; k < kMaxSlots; ++k) c[k] = k < ns ? slot_cnt[(long)k * pstride + s] : 0;
  int run = 0;
#pragma unroll
  for (int k = 0; k < kMaxSlots; ++k) {
    if (k < ns) slot_cnt[(long)k * pstride + s] = run;
    run += c[k];
  }
  row_cnt[perm[s]] = run;
  atomicMax(&info[2], run);
}

// One wave per unit: each listed pair's j goes into its CSR row, at the
// owner atom's role offset (order inside a role is fixed by the row sort).
__global__ __launch_bounds__(64) void k_csr_fill(const Unit* __restrict__ units,
                                                 const int32_t* __restrict__ cstart,
                                                 const int32_t* __restrict__ perm, long pstride,
                                                 const int64_t* __restrict__ unit_off,
                                                 const int32_t* __restrict__ unit_cnt,
                                                 const uint32_t* __restrict__ codes,
                                                 const int32_t* __restrict__ slot_off,
                                                 const int32_t* __restrict__ row_ptr,
                                                 int32_t* __restrict__ col) {
  __shared__ int pH[kMaxCellAtoms], pK[kMaxCellAtoms], cH[kMaxCellAtoms], cK[kMaxCellAtoms];
  __shared__ int bH[kMaxCellAtoms], bK[kMaxCellAtoms];
  const int uidx = blockIdx.x, lane = lane_id();
  const Unit un = units[uidx];
  const int hs = cstart[un.h], nh = cstart[un.h + 1] - hs;
  const int ks = cstart[un.k], nk = cstart[un.k + 1] - ks;
  if (nh > kMaxCellAtoms || nk > kMaxCellAtoms) return;
  for (int t = lane; t < nh; t += 64) {
    const int i = perm[hs + t];
    pH[t] = i;
    cH[t] = 0;
    bH[t] = row_ptr[i] + slot_off[(long)un.slot_h * pstride + hs + t];
  }
  for (int t = lane; t < nk; t += 64) {
    const int i = perm[ks + t];
    pK[t] = i;
    cK[t] = 0;
    bK[t] = row_ptr[i] + slot_off[(long)un.slot_k * pstride + ks + t];
  }
  __syncthreads();
  const uint32_t* src = codes + unit_off[uidx];
  const int m = unit_cnt[uidx];
  for (int p = lane; p < m; p += 64) {
    const uint32_t code = src[p];
    const int a = (int)(code & 0xffffu), b = (int)(code >> 16);
    const int ia = pH[a], ib = pK[b];
    if (ia < ib) col[bH[a] + atomicAdd(&cH[a], 1)] = ib;
    else col[bK[b] + atomicAdd(&cK[b], 1)] = ia;
  }
}

// One wave per cell: atoms in its neighbour cells (itself included); the
// maximum goes to info[5] (staging size of the per-cell mat-vec).
__global__ __launch_bounds__(64) void k_nbhd(const int32_t* __restrict__ cu,
                                             const Unit* __restrict__ units,
                                             const int32_t* __restrict__ cstart,
                                             int32_t* __restrict__ info) {
  const int32_t* e = cu + (long)blockIdx.x * kCellUnitStride;
  const int lane = lane_id();
  int cnt = 0;
  if (lane < e[0]) {
    const int u = e[1 + lane] >> 2, role = e[1 + lane] & 3;
    const int oc = role == 1 ? units[u].h : units[u].k;
    cnt = cstart[oc + 1] - cstart[oc];
  }
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
  if (lane == 0) atomicMax(&info[5], cnt);
}

// Gathers the build's outcome into pinned host memory (one kernel instead of
// several small copies).
__global__ void k_readback(const int32_t* __restrict__ info, const int32_t* __restrict__ rp_end,
                           const int64_t* __restrict__ off_end, int32_t* __restrict__ host) {
  for (int k = 0; k < 6; ++k) host[k] = info[k];
  host[6] = *rp_end;
  *(int64_t*)(host + 8) = *off_end;
}

// One wave per CSR row: order the row by j (monotone buckets over [jmin, jmax],
// then rank inside a bucket).  LDS: A[max_row], G[max_row], cnt, off.
__global__ __launch_bounds__(64) void k_rowsort(int n, const int32_t* __restrict__ row_ptr,
                                                int32_t* __restrict__ col, int max_row) {
  extern __shared__ int lds[];
  const int i = blockIdx.x;
  const int lane = lane_id();
  const int start = row_ptr[i], m = row_ptr[i + 1] - start;
  if (m <= 1) return;
  const int nbmax = max_row < kBuckets ? max_row : kBuckets;
  int* A = lds;
  int* G = A + max_row;
  int* cnt = G + max_row;
  int* off = cnt + nbmax;
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
  const double scale = (double)nb / (double)(jmax - jmin + 1);
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

}  // namespace

static tk_status nblist_build_impl(tk_ctx* ctx, hipStream_t st, const tk_system* sys,
                                   double cutoff, int slot, int32_t* row_ptr, int32_t* col,
                                   int64_t cap, int64_t* npairs_out) {
  if (!npairs_out) return TK_E_ARG;
  *npairs_out = 0;
  tk_status s = check_system(sys);
  if (s) return s;
  if (!(cutoff > 0.0) || !std::isfinite(cutoff)) return TK_E_ARG;
  if (cutoff > 0.5 * sys->box) return TK_E_CUTOFF;
  if (slot < 0 || slot >= TK_MAX_PLANS || cap < 0) return TK_E_ARG;
  if (col && !row_ptr) return TK_E_ARG;
  Plan& P = ctx->plans[slot];
  P.valid = false;
  const int n = sys->n;
  int nc = (int)std::floor(sys->box / cutoff);
  if (nc < 1) nc = 1;
  CellTables& T = cell_tables(ctx, nc);
  const uint64_t rq = (uint64_t)std::floor((cutoff / sys->box) * kTwo32);
  PairTest test;
  test.rq2 = rq * rq;
  test.lo = (double)test.rq2 * (1.0 - 0x1p-50);
  test.hi = (double)test.rq2 * (1.0 + 0x1p-50);
  const int nn = n > 0 ? n : 1;
  const long pstride = (nn + 63) / 64 * 64;
  const bool want_csr = row_ptr != nullptr;

  // device copies of the cell tables (uploaded once per cells-per-edge value)
  if (!T.uploaded) {
    if ((s = ensure(T.units_d, sizeof(Unit) * T.nunits)) ||
        (s = ensure(T.nslot_d, sizeof(int32_t) * T.ncells)) ||
        (s = ensure(T.cu_d, sizeof(int32_t) * T.cu.size())))
      return s;
    TK_HIP(hipMemcpy(T.cu_d.p, T.cu.data(), sizeof(int32_t) * T.cu.size(), hipMemcpyHostToDevice));
    TK_HIP(hipMemcpy(T.units_d.p, T.units.data(), sizeof(Unit) * T.nunits, hipMemcpyHostToDevice));
    TK_HIP(hipMemcpy(T.nslot_d.p, T.nslot.data(), sizeof(int32_t) * T.ncells, hipMemcpyHostToDevice));
    T.uploaded = true;
  }
  if ((s = ensure(P.perm, sizeof(int32_t) * nn)) || (s = ensure(P.scell, sizeof(int32_t) * nn)) ||
      (s = ensure(P.cell_start, sizeof(int32_t) * (T.ncells + 1))) ||
      (s = ensure(P.unit_off, sizeof(int64_t) * (T.nunits + 1))) ||
      (s = ensure(P.unit_cnt, sizeof(int32_t) * T.nunits)) ||
      (s = ensure(P.us, sizeof(uint4) * nn)) ||
      (s = ensure(P.slots, sizeof(int32_t) * kMaxSlots * pstride)))
    return s;
  // candidate windows: sum over units of |H||K|, estimated from the density
  // (the buffer grows, and the enumeration reruns, if the estimate is short)
  const double mean = (double)n / T.ncells;
  const double est = 1.15 * (double)T.nunits * mean * mean + 16.0 * n + 65536.0;
  if (P.codes.bytes < sizeof(uint32_t) * (size_t)est &&
      (s = ensure(P.codes, sizeof(uint32_t) * (size_t)est)))
    return s;
  void *u, *cell, *ccount, *cursor, *tmp, *info, *cand, *rcnt, *rptr;
  if ((s = scratch(ctx, "nb_u", sizeof(uint32_t) * 3 * nn, &u)) ||
      (s = scratch(ctx, "nb_cell", sizeof(int32_t) * nn, &cell)) ||
      (s = scratch(ctx, "nb_ccount", sizeof(int32_t) * (T.ncells + 1), &ccount)) ||
      (s = scratch(ctx, "nb_cursor", sizeof(int32_t) * T.ncells, &cursor)) ||
      (s = scratch(ctx, "nb_tmp", sizeof(int32_t) * nn, &tmp)) ||
      (s = scratch(ctx, "nb_info", sizeof(int32_t) * 8, &info)) ||
      (s = scratch(ctx, "nb_cand", sizeof(int64_t) * (T.nunits + 1), &cand)) ||
      (s = scratch(ctx, "nb_rcnt", sizeof(int32_t) * (nn + 1), &rcnt)) ||
      (s = scratch(ctx, "nb_rptr", sizeof(int32_t) * (nn + 1), &rptr)))
    return s;
  TK_HIP(hipMemsetAsync(info, 0, sizeof(int32_t) * 8, st));
  const int32_t* cstart = (const int32_t*)P.cell_start.p;
  const Unit* units = (const Unit*)T.units_d.p;
  int32_t* rp = want_csr ? row_ptr : (int32_t*)rptr;
  int32_t *h, *hd;
  if ((s = pinned(ctx, 4096, (void**)&h, (void**)&hd))) return s;
  if (n > 0 && T.ncells <= kMaxHistCells) {
    const int nblk = ceil_div(n, kHistBlock);
    const long hl = (long)T.ncells * nblk;
    void *H, *Hoff;
    if ((s = scratch(ctx, "nb_hist", sizeof(int32_t) * hl, &H)) ||
        (s = scratch(ctx, "nb_hist_off", sizeof(int32_t) * (hl + 1), &Hoff)))
      return s;
    {
      ProfScope ps(ctx, st, "nblist_quantize");
      k_quantize_hist<<<nblk, kHistBlock, 0, st>>>(n, sys->xyz, sys->box, nc, T.ncells,
                                                    (uint32_t*)u, (int32_t*)cell, (int32_t*)H,
                                                    (int32_t*)info);
    }
    if ((s = scan_i32(ctx, st, (int32_t*)H, (int32_t*)Hoff, (int)hl))) return s;
    {
      ProfScope ps(ctx, st, "nblist_cellsort");
      k_scatter_stable<<<nblk, kHistBlock, 0, st>>>(n, T.ncells, (int32_t*)cell, (int32_t*)Hoff,
                                                     (uint32_t*)u, (int32_t*)P.perm.p,
                                                     (int32_t*)P.scell.p, (uint4*)P.us.p,
                                                     (int32_t*)P.cell_start.p, (int32_t*)info);
    }
  } else if (n > 0) {
    TK_HIP(hipMemsetAsync(ccount, 0, sizeof(int32_t) * (T.ncells + 1), st));
    TK_HIP(hipMemsetAsync(cursor, 0, sizeof(int32_t) * T.ncells, st));
    {
      ProfScope ps(ctx, st, "nblist_quantize");
      k_quantize<<<ceil_div(n, 256), 256, 0, st>>>(n, sys->xyz, sys->box, nc, (uint32_t*)u,
                                                    (int32_t*)cell, (int32_t*)ccount, (int32_t*)info);
    }
    if ((s = scan_i32(ctx, st, (int32_t*)ccount, (int32_t*)P.cell_start.p, T.ncells))) return s;
    k_scatter<<<ceil_div(n, 256), 256, 0, st>>>(n, (int32_t*)cell, cstart, (int32_t*)cursor,
                                                 (int32_t*)tmp);
    {
      ProfScope ps(ctx, st, "nblist_cellsort");
      k_cellsort<<<T.ncells, 64, 0, st>>>(cstart, (int32_t*)tmp, (uint32_t*)u, (int32_t*)P.perm.p,
                                          (int32_t*)P.scell.p, (uint4*)P.us.p, (int32_t*)info);
    }
  } else {
    TK_HIP(hipMemsetAsync(P.cell_start.p, 0, sizeof(int32_t) * (T.ncells + 1), st));
  }
  if (n > 0) {
    k_cand<<<ceil_div(T.nunits, 256), 256, 0, st>>>(T.nunits, units, cstart, (int64_t*)cand);
    if ((s = scan_i64(ctx, st, (int64_t*)cand, (int64_t*)P.unit_off.p, T.nunits))) return s;
  }
  for (int attempt = 0; attempt < 2; ++attempt) {
    if (n > 0) {
      k_nbhd<<<T.ncells, 64, 0, st>>>((const int32_t*)T.cu_d.p, units, cstart, (int32_t*)info);
      {
        ProfScope ps(ctx, st, "nblist_plan");
        k_plan<<<T.nunits, 64, 0, st>>>(T.nunits, units, cstart, (uint4*)P.us.p, test, pstride,
                                        (int64_t*)P.unit_off.p, (long)(P.codes.bytes / 4),
                                        (uint32_t*)P.codes.p, (int32_t*)P.unit_cnt.p,
                                        (int32_t*)P.slots.p, (int32_t*)info);
      }
      k_row_slots<<<ceil_div(n, 256), 256, 0, st>>>(n, (int32_t*)P.perm.p, (int32_t*)P.scell.p,
                                                     (int32_t*)T.nslot_d.p, pstride,
                                                     (int32_t*)P.slots.p, (int32_t*)rcnt,
                                                     (int32_t*)info);
      if ((s = scan_i32(ctx, st, (int32_t*)rcnt, rp, n))) return s;
    } else {
      TK_HIP(hipMemsetAsync(P.unit_cnt.p, 0, sizeof(int32_t) * T.nunits, st));
      TK_HIP(hipMemsetAsync(P.unit_off.p, 0, sizeof(int64_t) * (T.nunits + 1), st));
      TK_HIP(hipMemsetAsync(rp, 0, sizeof(int32_t), st));
    }
    // one readback: status, max occupancy, max row, pairs, window overflow, list total
    k_readback<<<1, 1, 0, st>>>((int32_t*)info, rp + n, (int64_t*)P.unit_off.p + T.nunits, hd);
    TK_HIP(hipGetLastError());
    TK_HIP(hipStreamSynchronize(st));
    if (h[0] != 0) return h[0];
    if (h[4] == 0) break;
    if (attempt == 1) return TK_E_HIP;
    // windows did not fit: grow to the exact size and enumerate again
    const int64_t need = *(int64_t*)(h + 8);
    if ((s = ensure(P.codes, sizeof(uint32_t) * (size_t)need))) return s;
    TK_HIP(hipMemsetAsync(info, 0, sizeof(int32_t) * 8, st));
  }
  const int64_t list_pairs = h[6];
  *npairs_out = list_pairs;
  if (list_pairs != (int64_t)h[3]) {
    std::fprintf(stderr, "libtk: plan/list pair count mismatch %d vs %d\n", h[3], h[6]);
    return TK_E_HIP;
  }
  const int max_row = h[2];
  if (want_csr) {
    if (list_pairs > cap) return TK_E_CAPACITY;
    const int nb = max_row < kBuckets ? max_row : kBuckets;
    const size_t lds = sizeof(int) * (2 * (size_t)max_row + 2 * (size_t)nb);
    if (lds > kMaxLds) return TK_E_CAPACITY;
    if (n > 0 && list_pairs > 0) {
      {
        ProfScope ps(ctx, st, "nblist_csr_fill");
        k_csr_fill<<<T.nunits, 64, 0, st>>>(units, cstart, (int32_t*)P.perm.p, pstride,
                                            (int64_t*)P.unit_off.p, (int32_t*)P.unit_cnt.p,
                                            (uint32_t*)P.codes.p, (int32_t*)P.slots.p, rp, col);
      }
      {
        ProfScope ps(ctx, st, "nblist_rowsort");
        k_rowsort<<<n, 64, lds, st>>>(n, rp, col, max_row);
      }
    }
  }
  TK_HIP(hipGetLastError());
  P.valid = true;
  P.n = n;
  P.box = sys->box;
  P.cutoff = cutoff;
  P.nc = nc;
  P.ncells = T.ncells;
  P.nunits = T.nunits;
  P.max_occ = h[1];
  P.max_row = max_row;
  P.max_nbhd = h[5];
  P.cu_p = (const int32_t*)T.cu_d.p;
  P.npairs = list_pairs;
  P.units_p = units;
  P.nslot_p = (const int32_t*)T.nslot_d.p;
  return TK_OK;
}

}  // namespace tk

extern "C" tk_status tk_nblist_build(tk_ctx* ctx, void* stream, const tk_system* sys, double cutoff,
                                     int32_t plan_slot, int32_t* row_ptr, int32_t* col, int64_t cap,
                                     int64_t* npairs) {
  if (!ctx) return TK_E_ARG;
  return tk::nblist_build_impl(ctx, (hipStream_t)stream, sys, cutoff, plan_slot, row_ptr, col, cap,
                               npairs);
}
