// Neighbour lists on the GPU, integer and exact (the cell-list builders of the
// paper's Rel profile, with the selection-mask + compress pattern of its
// section "Typical selection loop" mapped to wavefront ballots).
//
// Steps:  quantize -> cell histogram -> scan -> scatter -> per-cell stable order
//         -> cell-pair plan (count, scan, fill)
//         -> canonical CSR rows (count, scan, fill with an in-LDS ordering by j).
// Every pair decision is the same exact 64-bit integer test, so the plan and
// the CSR hold the same pair set, bit for bit, whatever the launch order.
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

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

__device__ __forceinline__ int lanes_below(uint64_t mask) {
  return __popcll(mask & ((1ull << lane_id()) - 1ull));
}

__device__ __forceinline__ int wave_sum(int v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

// u = floor(frac(x/L) * 2^32) per coordinate; cell = (u * nc) >> 32 per axis.
__global__ void k_quantize(int n, const double* __restrict__ xyz, double box, int nc,
                           uint32_t* __restrict__ u, int32_t* __restrict__ cell,
                           int32_t* __restrict__ cell_count, int32_t* __restrict__ status) {
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
      atomicMin(status, (int)TK_E_ARG);
    }
    u[3 * i + a] = q;
    c[a] = (int)(((uint64_t)q * (uint64_t)nc) >> 32);
  }
  int cc = (c[0] * nc + c[1]) * nc + c[2];
  cell[i] = cc;
  atomicAdd(&cell_count[cc], 1);
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

// One wave per cell-pair unit.  Candidates (a in H, b in K) are visited in
// "diagonal" order b = (a + k) mod |K|, so consecutive listed pairs touch
// distinct atoms on both sides (conflict-free LDS accumulation later).
template <bool kFill>
__global__ __launch_bounds__(64) void k_plan(int nunits, const Unit* __restrict__ units,
                                             const int32_t* __restrict__ cstart,
                                             const uint4* __restrict__ us, uint64_t rq2,
                                             int32_t* __restrict__ unit_cnt,
                                             const int32_t* __restrict__ unit_ptr,
                                             uint32_t* __restrict__ codes) {
  int uidx = blockIdx.x;
  if (uidx >= nunits) return;
  Unit un = units[uidx];
  int hs = cstart[un.h], nh = cstart[un.h + 1] - hs;
  int ks = cstart[un.k], nk = cstart[un.k + 1] - ks;
  if (nh > kMaxCellAtoms || nk > kMaxCellAtoms) return;
  bool self = un.h == un.k;
  int base = kFill ? unit_ptr[uidx] : 0, cnt = 0;
  int lane = lane_id();
  for (int kk = 0; kk < nk; ++kk) {
    for (int a0 = 0; a0 < nh; a0 += 64) {
      int a = a0 + lane;
      bool pass = false;
      int b = 0;
      if (a < nh) {
        b = (a + kk) % nk;
        if (!self || a < b) pass = pair_in(us[hs + a], us[ks + b], rq2);
      }
      uint64_t mask = __ballot(pass);
      if (kFill && pass) codes[base + lanes_below(mask)] = (uint32_t)a | ((uint32_t)b << 16);
      int pc = __popcll(mask);
      base += pc;
      cnt += pc;
    }
  }
  if (!kFill && lane == 0) unit_cnt[uidx] = cnt;
}

// One wave per caller row i: visit the atoms of the (unique) neighbour cells
// of cell(i), keep j > i inside the cutoff.  Count mode writes the row length;
// fill mode collects the row in LDS, orders it by j and writes it.
template <bool kFill>
__global__ __launch_bounds__(64) void k_rows(int n, const int32_t* __restrict__ cell,
                                             const uint32_t* __restrict__ u,
                                             const int32_t* __restrict__ nbr,
                                             const int32_t* __restrict__ cstart,
                                             const uint4* __restrict__ us, uint64_t rq2,
                                             int32_t* __restrict__ row_cnt,
                                             const int32_t* __restrict__ row_ptr,
                                             int32_t* __restrict__ col, int32_t* __restrict__ info) {
  extern __shared__ int lds[];
  int i = blockIdx.x;
  if (i >= n) return;
  int lane = lane_id();
  uint4 ui = make_uint4(u[3 * i], u[3 * i + 1], u[3 * i + 2], (uint32_t)i);
  int c = cell[i];
  int nn = nbr[c * 28];
  int m = 0;
  int* A = lds;   // [max_row] row entries in visit order
  for (int q = 0; q < nn; ++q) {
    int cc = nbr[c * 28 + 1 + q];
    int t0 = cstart[cc], t1 = cstart[cc + 1];
    for (int t = t0; t < t1; t += 64) {
      int tt = t + lane;
      bool pass = false;
      uint4 uj;
      if (tt < t1) {
        uj = us[tt];
        pass = uj.w > (uint32_t)i && pair_in(ui, uj, rq2);
      }
      uint64_t mask = __ballot(pass);
      if (kFill && pass) A[m + lanes_below(mask)] = (int)uj.w;
      m += __popcll(mask);
    }
  }
  if (!kFill) {
    if (lane == 0) {
      row_cnt[i] = m;
      atomicMax(&info[2], m);
    }
    return;
  }
  __syncthreads();
  int start = row_ptr[i];
  if (m == 0) return;
  // order the row by j: monotone buckets over [jmin, jmax], then rank inside a bucket
  int jmin = 0x7fffffff, jmax = -1;
  for (int e = lane; e < m; e += 64) {
    jmin = min(jmin, A[e]);
    jmax = max(jmax, A[e]);
  }
  jmin = wave_min(jmin);
  jmax = wave_max(jmax);
  int nb = m < kBuckets ? m : kBuckets;
  double scale = (double)nb / (double)(jmax - jmin + 1);
  int* G = A + m;          // [m] entries grouped by bucket
  int* cnt = G + m;        // [nb]
  int* off = cnt + nb;     // [nb]
  for (int b = lane; b < nb; b += 64) {
    cnt[b] = 0;
    off[b] = 0;
  }
  __syncthreads();
  for (int e = lane; e < m; e += 64) {
    int b = min(nb - 1, (int)((double)(A[e] - jmin) * scale));
    atomicAdd(&cnt[b], 1);
  }
  __syncthreads();
  // exclusive scan of cnt (one wave: each lane scans a contiguous chunk)
  int per = (nb + 63) / 64, b0 = lane * per, b1 = min(nb, b0 + per), s = 0;
  for (int b = b0; b < b1; ++b) s += cnt[b];
  int incl = s;
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  int run = incl - s;
  for (int b = b0; b < b1; ++b) {
    off[b] = run;
    run += cnt[b];
  }
  __syncthreads();
  for (int b = lane; b < nb; b += 64) cnt[b] = 0;   // reuse as fill cursor
  __syncthreads();
  for (int e = lane; e < m; e += 64) {
    int b = min(nb - 1, (int)((double)(A[e] - jmin) * scale));
    G[off[b] + atomicAdd(&cnt[b], 1)] = A[e];
  }
  __syncthreads();
  for (int e = lane; e < m; e += 64) {
    int j = A[e];
    int b = min(nb - 1, (int)((double)(j - jmin) * scale));
    int k0 = off[b], k1 = k0 + cnt[b], rank = k0;
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
  if ((row_ptr == nullptr) != (col == nullptr) && !(row_ptr && cap == 0)) return TK_E_ARG;
  Plan& P = ctx->plans[slot];
  P.valid = false;
  const int n = sys->n;
  int nc = (int)std::floor(sys->box / cutoff);
  if (nc < 1) nc = 1;
  const CellTables& T = cell_tables(ctx, nc);
  const uint64_t rq = (uint64_t)std::floor((cutoff / sys->box) * kTwo32);
  const uint64_t rq2 = rq * rq;
  const int nn = n > 0 ? n : 1;

  // plan buffers (device) and the host-built cell tables
  if ((s = ensure(P.perm, sizeof(int32_t) * nn)) || (s = ensure(P.scell, sizeof(int32_t) * nn)) ||
      (s = ensure(P.cell_start, sizeof(int32_t) * (T.ncells + 1))) ||
      (s = ensure(P.cell_nslot, sizeof(int32_t) * T.ncells)) ||
      (s = ensure(P.units, sizeof(Unit) * T.nunits)) ||
      (s = ensure(P.unit_ptr, sizeof(int32_t) * (T.nunits + 1))) ||
      (s = ensure(P.us, sizeof(uint4) * nn)) || (s = ensure(P.nbr, sizeof(int32_t) * T.ncells * 28)))
    return s;
  TK_HIP(hipMemcpyAsync(P.units.p, T.units.data(), sizeof(Unit) * T.nunits, hipMemcpyHostToDevice, st));
  TK_HIP(hipMemcpyAsync(P.cell_nslot.p, T.nslot.data(), sizeof(int32_t) * T.ncells,
                        hipMemcpyHostToDevice, st));
  TK_HIP(hipMemcpyAsync(P.nbr.p, T.nbr.data(), sizeof(int32_t) * T.ncells * 28,
                        hipMemcpyHostToDevice, st));
  void *u, *cell, *ccount, *cursor, *tmp, *info, *ucnt, *rcnt, *rptr;
  if ((s = scratch(ctx, "nb_u", sizeof(uint32_t) * 3 * nn, &u)) ||
      (s = scratch(ctx, "nb_cell", sizeof(int32_t) * nn, &cell)) ||
      (s = scratch(ctx, "nb_ccount", sizeof(int32_t) * (T.ncells + 1), &ccount)) ||
      (s = scratch(ctx, "nb_cursor", sizeof(int32_t) * T.ncells, &cursor)) ||
      (s = scratch(ctx, "nb_tmp", sizeof(int32_t) * nn, &tmp)) ||
      (s = scratch(ctx, "nb_info", sizeof(int32_t) * 8, &info)) ||
      (s = scratch(ctx, "nb_ucnt", sizeof(int32_t) * (T.nunits + 1), &ucnt)) ||
      (s = scratch(ctx, "nb_rcnt", sizeof(int32_t) * (nn + 1), &rcnt)) ||
      (s = scratch(ctx, "nb_rptr", sizeof(int32_t) * (nn + 1), &rptr)))
    return s;
  TK_HIP(hipMemsetAsync(ccount, 0, sizeof(int32_t) * (T.ncells + 1), st));
  TK_HIP(hipMemsetAsync(cursor, 0, sizeof(int32_t) * T.ncells, st));
  TK_HIP(hipMemsetAsync(info, 0, sizeof(int32_t) * 8, st));
  const int32_t* cstart = (const int32_t*)P.cell_start.p;
  if (n > 0) {
    k_quantize<<<ceil_div(n, 256), 256, 0, st>>>(n, sys->xyz, sys->box, nc, (uint32_t*)u,
                                                  (int32_t*)cell, (int32_t*)ccount, (int32_t*)info);
  }
  if ((s = scan_i32(ctx, st, (int32_t*)ccount, (int32_t*)P.cell_start.p, T.ncells))) return s;
  if (n > 0) {
    k_scatter<<<ceil_div(n, 256), 256, 0, st>>>(n, (int32_t*)cell, cstart, (int32_t*)cursor,
                                                 (int32_t*)tmp);
    k_cellsort<<<T.ncells, 64, 0, st>>>(cstart, (int32_t*)tmp, (uint32_t*)u, (int32_t*)P.perm.p,
                                        (int32_t*)P.scell.p, (uint4*)P.us.p, (int32_t*)info);
    k_plan<false><<<T.nunits, 64, 0, st>>>(T.nunits, (Unit*)P.units.p, cstart, (uint4*)P.us.p, rq2,
                                           (int32_t*)ucnt, nullptr, nullptr);
    k_rows<false><<<n, 64, 0, st>>>(n, (int32_t*)cell, (uint32_t*)u, (int32_t*)P.nbr.p, cstart,
                                    (uint4*)P.us.p, rq2, (int32_t*)rcnt, nullptr, nullptr,
                                    (int32_t*)info);
  } else {
    TK_HIP(hipMemsetAsync(ucnt, 0, sizeof(int32_t) * (T.nunits + 1), st));
  }
  if ((s = scan_i32(ctx, st, (int32_t*)ucnt, (int32_t*)P.unit_ptr.p, T.nunits))) return s;
  int32_t* rp = row_ptr ? row_ptr : (int32_t*)rptr;
  if (n > 0) {
    if ((s = scan_i32(ctx, st, (int32_t*)rcnt, rp, n))) return s;
  } else {
    TK_HIP(hipMemsetAsync(rp, 0, sizeof(int32_t), st));
  }
  // one readback: status, max cell occupancy, max row, plan total, list total
  int32_t* h;
  if ((s = pinned(ctx, 64, (void**)&h))) return s;
  TK_HIP(hipMemcpyAsync(h, info, sizeof(int32_t) * 4, hipMemcpyDeviceToHost, st));
  TK_HIP(hipMemcpyAsync(h + 4, (int32_t*)P.unit_ptr.p + T.nunits, sizeof(int32_t),
                        hipMemcpyDeviceToHost, st));
  TK_HIP(hipMemcpyAsync(h + 5, rp + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  TK_HIP(hipStreamSynchronize(st));
  if (h[0] != 0) return h[0];
  int64_t plan_pairs = h[4], list_pairs = h[5];
  *npairs_out = list_pairs;
  if (plan_pairs != list_pairs) {
    std::fprintf(stderr, "libtk: plan/list pair count mismatch %lld vs %lld\n",
                 (long long)plan_pairs, (long long)list_pairs);
    return TK_E_HIP;
  }
  if (row_ptr && list_pairs > cap) return TK_E_CAPACITY;
  if ((s = ensure(P.codes, sizeof(uint32_t) * (plan_pairs > 0 ? plan_pairs : 1)))) return s;
  if (n > 0) {
    k_plan<true><<<T.nunits, 64, 0, st>>>(T.nunits, (Unit*)P.units.p, cstart, (uint4*)P.us.p, rq2,
                                          nullptr, (int32_t*)P.unit_ptr.p, (uint32_t*)P.codes.p);
    if (row_ptr && list_pairs > 0) {
      int max_row = h[2];
      int nb = max_row < kBuckets ? max_row : kBuckets;
      size_t lds = sizeof(int) * (2 * (size_t)max_row + 2 * (size_t)nb);
      if (lds > 160 * 1024) return TK_E_CAPACITY;
      k_rows<true><<<n, 64, lds, st>>>(n, (int32_t*)cell, (uint32_t*)u, (int32_t*)P.nbr.p, cstart,
                                       (uint4*)P.us.p, rq2, nullptr, rp, col, (int32_t*)info);
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
  P.max_row = h[2];
  P.npairs = list_pairs;
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
