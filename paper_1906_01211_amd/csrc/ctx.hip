// Host runtime of libtk: context, grow-only device buffers, cell tables, a
// device exclusive scan, and argument checks shared by the entry points.
#include <cmath>
#include <cstring>
#include <iterator>

#include "tk_internal.hpp"

namespace tk {

tk_status hip_status(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) return TK_E_NOMEM;
  std::fprintf(stderr, "libtk: %s failed: %s\n", what, hipGetErrorString(e));
  return TK_E_HIP;
}

tk_status ensure(tk_ctx* ctx, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.bytes >= bytes) return TK_OK;
  size_t want = bytes + bytes / 4;   // headroom so slightly larger inputs reuse it
  want = (want + 255) & ~size_t(255);
  // the context's device budget (the old buffer is kept when it refuses)
  const size_t total = ctx->arena_bytes - b.bytes + want;
  if (ctx->arena_budget && total > ctx->arena_budget) {
    if (ctx->arena_budget >= ctx->arena_bytes - b.bytes + bytes) want = bytes;   // no headroom
    else return TK_E_NOMEM;
  }
  if (b.p) {
    TK_HIP(hipDeviceSynchronize());   // queued kernels may still use the old buffer
    TK_HIP(hipFree(b.p));
    ctx->arena_bytes -= b.bytes;
    b.p = nullptr;
    b.bytes = 0;
  }
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    b.p = nullptr;
    return hip_status(e, "hipMalloc");
  }
  b.bytes = want;
  ctx->arena_bytes += want;
  return TK_OK;
}

tk_status scratch(tk_ctx* ctx, const char* name, size_t bytes, void** out) {
  DevBuf& b = ctx->scratch[name];
  tk_status s = ensure(ctx, b, bytes);
  *out = b.p;
  return s;
}

tk_status pinned(tk_ctx* ctx, size_t bytes, void** out, void** dev) {
  if (ctx->pinned_bytes < bytes) {
    if (ctx->pinned) TK_HIP(hipHostFree(ctx->pinned));
    ctx->pinned = nullptr;
    ctx->pinned_dev = nullptr;
    ctx->pinned_bytes = 0;
    size_t want = bytes < 4096 ? 4096 : bytes;
    TK_HIP(hipHostMalloc(&ctx->pinned, want, hipHostMallocCoherent));   // fine-grained: kernels write it directly
    TK_HIP(hipHostGetDevicePointer(&ctx->pinned_dev, ctx->pinned, 0));
    ctx->pinned_bytes = want;
  }
  *out = ctx->pinned;
  if (dev) *dev = ctx->pinned_dev;
  return TK_OK;
}

CellTables& cell_tables(tk_ctx* ctx, int nc) {
  auto it = ctx->tables.find(nc);
  if (it != ctx->tables.end()) return it->second;
  CellTables t;
  t.nc = nc;
  t.ncells = nc * nc * nc;
  t.nbr.assign((size_t)t.ncells * 28, -1);
  std::vector<int32_t> cnt(t.ncells, 0);
  for (int c = 0; c < t.ncells; ++c) {
    int ci[3] = {c / (nc * nc), (c / nc) % nc, c % nc};
    int nb[3][3], m[3];
    for (int a = 0; a < 3; ++a) {   // unique neighbour cells per dimension
      m[a] = 0;
      for (int o = -1; o <= 1; ++o) {
        int v = ((ci[a] + o) % nc + nc) % nc;
        bool dup = false;
        for (int q = 0; q < m[a]; ++q) dup |= nb[a][q] == v;
        if (!dup) nb[a][m[a]++] = v;
      }
    }
    int k = 0;
    for (int x = 0; x < m[0]; ++x)
      for (int y = 0; y < m[1]; ++y)
        for (int z = 0; z < m[2]; ++z) t.nbr[(size_t)c * 28 + 1 + k++] = (nb[0][x] * nc + nb[1][y]) * nc + nb[2][z];
    t.nbr[(size_t)c * 28] = k;
  }
  for (int h = 0; h < t.ncells; ++h) {
    int k = t.nbr[(size_t)h * 28];
    for (int q = 0; q < k; ++q) {
      int kc = t.nbr[(size_t)h * 28 + 1 + q];
      if (kc < h) continue;
      Unit u;
      u.h = h;
      u.k = kc;
      u.slot_h = cnt[h]++;
      u.slot_k = cnt[kc]++;
      t.units.push_back(u);
    }
  }
  t.nunits = (int32_t)t.units.size();
  t.nslot = cnt;
  // Dispatch order of the units: by the number of axes on which the two
  // cells differ (self, face, edge, corner neighbours), cell order inside.
  // The expected pair count falls steeply along that sequence, so the heavy
  // units start first and the light ones fill the end of a launch.  Slots
  // were assigned above, so every atom's partial results (summed in slot
  // order) do not depend on this order.
  std::vector<int32_t> rank(t.nunits);   // creation index -> dispatch index
  {
    auto axes = [nc](int a, int b) {
      const int da[3] = {a / (nc * nc), (a / nc) % nc, a % nc};
      const int db[3] = {b / (nc * nc), (b / nc) % nc, b % nc};
      return (da[0] != db[0]) + (da[1] != db[1]) + (da[2] != db[2]);
    };
    std::vector<Unit> by_type;
    by_type.reserve(t.nunits);
    for (int ty = 0; ty <= 3; ++ty)
      for (int u = 0; u < t.nunits; ++u)
        if (axes(t.units[u].h, t.units[u].k) == ty) {
          rank[u] = (int32_t)by_type.size();
          by_type.push_back(t.units[u]);
        }
    // per cell: the units it takes part in (each unique neighbour cell once),
    // in creation order, encoded dispatch index * 4 + role (0: the cell is
    // the unit's H, 1: its K, 2: both)
    t.cu.assign((size_t)t.ncells * kCellUnitStride, 0);
    for (int u = 0; u < t.nunits; ++u) {
      const Unit& un = t.units[u];
      const int32_t r = rank[u];
      if (un.h == un.k) {
        int32_t* e = &t.cu[(size_t)un.h * kCellUnitStride];
        e[1 + e[0]++] = r * 4 + 2;
      } else {
        int32_t* e = &t.cu[(size_t)un.h * kCellUnitStride];
        e[1 + e[0]++] = r * 4 + 0;
        e = &t.cu[(size_t)un.k * kCellUnitStride];
        e[1 + e[0]++] = r * 4 + 1;
      }
    }
    t.units.swap(by_type);
  }
  // cells grouped by octant (each axis split at ceil(nc/2)), lexicographic inside
  const int half = (nc + 1) / 2;
  for (int oct = 0; oct < 8; ++oct)
    for (int x = 0; x < nc; ++x)
      for (int y = 0; y < nc; ++y)
        for (int z = 0; z < nc; ++z) {
          const int o = (x >= half) * 4 + (y >= half) * 2 + (z >= half);
          if (o == oct) t.order.push_back((x * nc + y) * nc + z);
        }
  return ctx->tables.emplace(nc, std::move(t)).first->second;
}

// ---------------------------------------------------------------------------
// Exclusive scan (three phases: block sums, scan of block sums, block scan).
constexpr int kScanBlock = 256, kScanItems = 4, kScanTile = kScanBlock * kScanItems;

template <class T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* sh, T* total) {
  int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    T t = tid >= off ? sh[tid - off] : T(0);
    __syncthreads();
    sh[tid] += t;
    __syncthreads();
  }
  T incl = sh[tid];
  *total = sh[kScanBlock - 1];
  __syncthreads();
  return incl - v;
}

template <class T>
__device__ __forceinline__ void scan_sums_body(const T* in, long len, T* bsum, int b, T* sh) {
  long base = (long)b * kScanTile + threadIdx.x * kScanItems;
  T s = 0;
  for (int q = 0; q < kScanItems; ++q)
    if (base + q < len) s += in[base + q];
  T tot;
  block_exclusive_scan<T>(s, sh, &tot);
  if (threadIdx.x == 0) bsum[b] = tot;
}

template <class T>
__global__ __launch_bounds__(kScanBlock) void k_scan_sums(const T* in, long len, T* bsum) {
  __shared__ T sh[kScanBlock];
  scan_sums_body<T>(in, len, bsum, blockIdx.x, sh);
}

template <class T>
__global__ __launch_bounds__(kScanBlock) void k_scan_bsum(T* bsum, int nb) {
  __shared__ T sh[kScanBlock];
  T carry = 0;
  for (int b0 = 0; b0 < nb; b0 += kScanBlock) {
    int i = b0 + threadIdx.x;
    T v = i < nb ? bsum[i] : T(0);
    T tot;
    T ex = block_exclusive_scan<T>(v, sh, &tot);
    if (i < nb) bsum[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

template <class T>
__global__ __launch_bounds__(kScanBlock) void k_scan_final(const T* in, long len, const T* bsum,
                                                           T* out) {
  __shared__ T sh[kScanBlock];
  long base = (long)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  T v[kScanItems], s = 0;
  for (int q = 0; q < kScanItems; ++q) {
    v[q] = base + q < len ? in[base + q] : T(0);
    s += v[q];
  }
  T tot;
  T ex = block_exclusive_scan<T>(s, sh, &tot) + bsum[blockIdx.x];
  for (int q = 0; q < kScanItems; ++q) {
    if (base + q < len) out[base + q] = ex;
    ex += v[q];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[len] = bsum[gridDim.x];
}

// One workgroup for arrays up to kScan1Max (one launch instead of two or
// three).  The array is read as kItems tiles of kScan1Threads values, thread
// t holding value t of every tile (coalesced loads, all in flight together);
// the tiles are scanned inside the waves level by level (the kItems shuffles
// of a level are independent); wave 0 scans the (tile, wave) totals in
// tile-major order, which gives every wave of every tile its offset; each
// thread adds its wave's offset.
constexpr int kScan1Threads = 1024;
constexpr long kScan1Max = (long)kScan1Threads * 4;
constexpr int kScan2MaxBlocks = 4096;

template <class T, int kItems>
__global__ __launch_bounds__(kScan1Threads) void k_scan1(const T* __restrict__ in, long len,
                                                         T* __restrict__ out) {
  constexpr int kW = kScan1Threads / 64;
  constexpr int kTot = kItems * kW;      // (tile, wave) totals
  constexpr int kPer = (kTot + 63) / 64;  // per lane of wave 0
  __shared__ T wsum[kTot];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  T v[kItems], incl[kItems];
#pragma unroll
  for (int q = 0; q < kItems; ++q) {
    const long e = (long)q * kScan1Threads + tid;
    v[q] = e < len ? in[e] : T(0);
    incl[q] = v[q];
  }
  for (int o = 1; o < 64; o <<= 1) {   // inclusive scans inside the wave, all tiles per level
#pragma unroll
    for (int q = 0; q < kItems; ++q) {
      const T t = __shfl_up(incl[q], o);
      if (lane >= o) incl[q] += t;
    }
  }
#pragma unroll
  for (int q = 0; q < kItems; ++q) {
    if (lane == 63) wsum[q * kW + w] = incl[q];
    v[q] = incl[q] - v[q];   // exclusive, inside the wave
  }
  __syncthreads();
  if (w == 0) {   // exclusive scan of the totals, tile-major; each lane holds kPer of them
    T x[kPer], s = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int i = lane * kPer + k;
      x[k] = i < kTot ? wsum[i] : T(0);
      s += x[k];
    }
    T inc = s;
    for (int o = 1; o < 64; o <<= 1) {
      const T t = __shfl_up(inc, o);
      if (lane >= o) inc += t;
    }
    T run = inc - s;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int i = lane * kPer + k;
      if (i < kTot) wsum[i] = run;
      run += x[k];
    }
    if (lane == 63) out[len] = inc;   // the total
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kItems; ++q) {
    const long e = (long)q * kScan1Threads + tid;
    if (e < len) out[e] = wsum[q * kW + w] + v[q];
  }
}

// Final pass that finds its own carry: block b sums the tile totals of the
// blocks before it (fixed order), so no separate pass over the totals.
template <class T>
__device__ __forceinline__ void scan_final_carry_body(const T* in, long len, const T* bsum, T* out,
                                                      int b, int nb, T* sh) {
  T c = 0;
  for (int k = threadIdx.x; k < b; k += kScanBlock) c += bsum[k];
  T ctot;
  block_exclusive_scan<T>(c, sh, &ctot);
  long base = (long)b * kScanTile + threadIdx.x * kScanItems;
  T v[kScanItems], s = 0;
  for (int q = 0; q < kScanItems; ++q) {
    v[q] = base + q < len ? in[base + q] : T(0);
    s += v[q];
  }
  T tot;
  T ex = block_exclusive_scan<T>(s, sh, &tot) + ctot;
  for (int q = 0; q < kScanItems; ++q) {
    if (base + q < len) out[base + q] = ex;
    ex += v[q];
  }
  if (b == nb - 1 && threadIdx.x == 0) out[len] = ctot + tot;
}

template <class T>
__global__ __launch_bounds__(kScanBlock) void k_scan_final_carry(const T* in, long len,
                                                                 const T* bsum, T* out) {
  __shared__ T sh[kScanBlock];
  scan_final_carry_body<T>(in, len, bsum, out, blockIdx.x, gridDim.x, sh);
}

// Two independent scans in the same two launches (blocks [0, nb1) scan the
// first array, the rest the second).
template <class T1, class T2>
__global__ __launch_bounds__(kScanBlock) void k_scan_sums2(const T1* in1, long len1, T1* bs1,
                                                           int nb1, const T2* in2, long len2,
                                                           T2* bs2) {
  __shared__ T1 sh1[kScanBlock];
  __shared__ T2 sh2[kScanBlock];
  if ((int)blockIdx.x < nb1) scan_sums_body<T1>(in1, len1, bs1, blockIdx.x, sh1);
  else scan_sums_body<T2>(in2, len2, bs2, blockIdx.x - nb1, sh2);
}

template <class T1, class T2>
__global__ __launch_bounds__(kScanBlock) void k_scan_final2(const T1* in1, long len1, const T1* bs1,
                                                            T1* out1, int nb1, const T2* in2,
                                                            long len2, const T2* bs2, T2* out2) {
  __shared__ T1 sh1[kScanBlock];
  __shared__ T2 sh2[kScanBlock];
  const int nb2 = gridDim.x - nb1;
  if ((int)blockIdx.x < nb1) scan_final_carry_body<T1>(in1, len1, bs1, out1, blockIdx.x, nb1, sh1);
  else scan_final_carry_body<T2>(in2, len2, bs2, out2, blockIdx.x - nb1, nb2, sh2);
}

template <class T>
static tk_status scan_t(tk_ctx* ctx, hipStream_t st, const T* in, T* out, long len,
                        const char* name) {
  // one workgroup up to four tiles (measured: beyond that the two-launch
  // scan over many workgroups is as fast or faster)
  if (len <= kScan1Max) {
    k_scan1<T, 4><<<1, kScan1Threads, 0, st>>>(in, len, out);
    TK_HIP(hipGetLastError());
    return TK_OK;
  }
  int nb = ceil_div(len, kScanTile);
  if (nb < 1) nb = 1;
  void* bs;
  tk_status s = scratch(ctx, name, sizeof(T) * (nb + 1), &bs);
  if (s) return s;
  if (nb <= kScan2MaxBlocks) {
    k_scan_sums<T><<<nb, kScanBlock, 0, st>>>(in, len, (T*)bs);
    k_scan_final_carry<T><<<nb, kScanBlock, 0, st>>>(in, len, (T*)bs, out);
    TK_HIP(hipGetLastError());
    return TK_OK;
  }
  k_scan_sums<T><<<nb, kScanBlock, 0, st>>>(in, len, (T*)bs);
  k_scan_bsum<T><<<1, kScanBlock, 0, st>>>((T*)bs, nb);
  k_scan_final<T><<<nb, kScanBlock, 0, st>>>(in, len, (T*)bs, out);
  TK_HIP(hipGetLastError());
  return TK_OK;
}

static std::string scan_name(const char* base, int job) {
  return job ? std::string(base) + "." + std::to_string(job) : std::string(base);
}

tk_status scan_i32(tk_ctx* ctx, hipStream_t st, const int32_t* in, int32_t* out, int len, int job) {
  return scan_t<int32_t>(ctx, st, in, out, len, scan_name("scan_bsum32", job).c_str());
}

tk_status scan_i64(tk_ctx* ctx, hipStream_t st, const int64_t* in, int64_t* out, long len,
                   int job) {
  return scan_t<int64_t>(ctx, st, in, out, len, scan_name("scan_bsum64", job).c_str());
}

tk_status scan_pair(tk_ctx* ctx, hipStream_t st, const int32_t* in1, int32_t* out1, int len1,
                    const int64_t* in2, int64_t* out2, long len2, int job) {
  const int nb1 = ceil_div(len1 > 0 ? len1 : 1, kScanTile);
  const int nb2 = ceil_div(len2 > 0 ? len2 : 1, kScanTile);
  if (nb1 > kScan2MaxBlocks || nb2 > kScan2MaxBlocks) {
    tk_status s = scan_i32(ctx, st, in1, out1, len1, job);
    return s ? s : scan_i64(ctx, st, in2, out2, len2, job);
  }
  void *b1, *b2;
  tk_status s;
  if ((s = scratch(ctx, scan_name("scan_bsum32", job).c_str(), sizeof(int32_t) * (nb1 + 1), &b1)) ||
      (s = scratch(ctx, scan_name("scan_bsum64", job).c_str(), sizeof(int64_t) * (nb2 + 1), &b2)))
    return s;
  k_scan_sums2<int32_t, int64_t><<<nb1 + nb2, kScanBlock, 0, st>>>(in1, len1, (int32_t*)b1, nb1,
                                                                   in2, len2, (int64_t*)b2);
  k_scan_final2<int32_t, int64_t><<<nb1 + nb2, kScanBlock, 0, st>>>(
      in1, len1, (const int32_t*)b1, out1, nb1, in2, len2, (const int64_t*)b2, out2);
  TK_HIP(hipGetLastError());
  return TK_OK;
}

static hipEvent_t take_event(tk_ctx* ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

ProfScope::ProfScope(tk_ctx* c, hipStream_t s, const std::string& name, bool kernel_events)
    : ctx(c), st(s) {
  // an empty name is never timed
  if (!ctx->prof_on || name.empty() || (!ctx->prof_only.empty() && ctx->prof_only != name)) return;
  a = take_event(ctx);
  if (!a) return;
  if (kernel_events) {
    b = take_event(ctx);
    if (!b) {
      ctx->event_pool.push_back(a);
      a = nullptr;
      return;
    }
    on_kernel = true;
  } else {
    (void)hipEventRecord(a, st);
  }
  e = &ctx->prof[name];
}

ProfScope::~ProfScope() {
  if (!e) return;
  if (!on_kernel) {
    b = take_event(ctx);
    if (!b) return;
    (void)hipEventRecord(b, st);
  }
  e->pending.emplace_back(a, b);
}

static void prof_drain(tk_ctx* ctx) {
  for (auto& kv : ctx->prof) {
    for (auto& ev : kv.second.pending) {
      float ms = 0.f;
      if (hipEventSynchronize(ev.second) == hipSuccess &&
          hipEventElapsedTime(&ms, ev.first, ev.second) == hipSuccess) {
        kv.second.ms += ms;
        kv.second.launches += 1;
      }
      ctx->event_pool.push_back(ev.first);
      ctx->event_pool.push_back(ev.second);
    }
    kv.second.pending.clear();
  }
}

tk_status check_system(const tk_system* sys) {
  if (!sys || sys->n < 0 || !(sys->box > 0.0) || !std::isfinite(sys->box)) return TK_E_ARG;
  if (sys->n > 0 && (!sys->xyz || !sys->molid)) return TK_E_ARG;
  return TK_OK;
}

tk_status get_plan(tk_ctx* ctx, const tk_system* sys, const tk_nblist* list, double cutoff,
                   const Plan** out) {
  if (!list || !(cutoff > 0.0)) return TK_E_ARG;
  if (cutoff > 0.5 * sys->box) return TK_E_CUTOFF;
  if (list->plan < 0 || list->plan >= TK_MAX_PLANS) return TK_E_PLAN;
  const Plan& p = ctx->plans[list->plan];
  if (!p.valid || p.nsys != 1 || p.n != sys->n || p.box != sys->box || p.cutoff != list->cutoff ||
      p.npairs != list->npairs)
    return TK_E_PLAN;
  if (cutoff > p.cutoff) return TK_E_ARG;   // the list must cover the kernel cutoff
  *out = &p;
  return TK_OK;
}

}  // namespace tk

extern "C" {

tk_status tk_create(int device, tk_ctx** out) {
  if (!out) return TK_E_ARG;
  *out = nullptr;
  int ndev = 0;
  TK_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return TK_E_ARG;
  TK_HIP(hipSetDevice(device));
  void* fixed = nullptr;   // this device's copy of the allocation-free entry point's scratch
  tk_status s = tk::noalloc_setup(device, &fixed);
  if (s) return s;
  tk_ctx* c = new tk_ctx();
  c->device = device;
  c->noalloc_scratch = fixed;
  *out = c;
  return TK_OK;
}

tk_status tk_set_arena_budget(tk_ctx* ctx, size_t bytes) {
  if (!ctx) return TK_E_ARG;
  ctx->arena_budget = bytes;
  return TK_OK;
}

size_t tk_arena_bytes(const tk_ctx* ctx) { return ctx ? ctx->arena_bytes : 0; }

tk_status tk_profile_enable(tk_ctx* ctx, int on, const char* only) {
  if (!ctx) return TK_E_ARG;
  ctx->prof_on = on != 0;
  ctx->prof_only = only ? only : "";
  // the events come from a pool: fill it now, so that timed launches do not
  // create events on the host between them
  constexpr size_t kPrefill = 4096;
  if (ctx->prof_on && ctx->event_pool.size() < kPrefill / 4) {
    TK_HIP(hipSetDevice(ctx->device));
    while (ctx->event_pool.size() < kPrefill) {
      hipEvent_t e = nullptr;
      TK_HIP(hipEventCreate(&e));
      ctx->event_pool.push_back(e);
    }
  }
  return TK_OK;
}

tk_status tk_profile_read(tk_ctx* ctx, int32_t idx, char* name, int32_t name_len,
                          int64_t* launches, double* total_ms) {
  if (!ctx || idx < 0) return TK_E_ARG;
  tk::prof_drain(ctx);
  if (idx >= (int32_t)ctx->prof.size()) return TK_E_ARG;
  auto it = ctx->prof.begin();
  std::advance(it, idx);
  if (name && name_len > 0) {
    std::strncpy(name, it->first.c_str(), (size_t)name_len - 1);
    name[name_len - 1] = 0;
  }
  if (launches) *launches = it->second.launches;
  if (total_ms) *total_ms = it->second.ms;
  return TK_OK;
}

tk_status tk_profile_reset(tk_ctx* ctx) {
  if (!ctx) return TK_E_ARG;
  tk::prof_drain(ctx);
  ctx->prof.clear();
  return TK_OK;
}

void tk_destroy(tk_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  tk::prof_drain(ctx);
  for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
  auto freeb = [](tk::DevBuf& b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  };
  for (auto& p : ctx->plans) {
    freeb(p.perm); freeb(p.scell); freeb(p.cell_start); freeb(p.unit_off); freeb(p.unit_cnt);
    freeb(p.codes); freeb(p.us); freeb(p.slots); freeb(p.urec); freeb(p.sysd);
    freeb(p.cell_sys); freeb(p.bunits); freeb(p.bnslot); freeb(p.bcu); freeb(p.border);
    freeb(p.tplp); freeb(p.dstat);
  }
  for (auto& kv : ctx->tables) {
    freeb(kv.second.units_d);
    freeb(kv.second.nslot_d);
    freeb(kv.second.cu_d);
    freeb(kv.second.order_d);
  }
  for (auto& kv : ctx->scratch) freeb(kv.second);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  delete ctx;
}

const char* tk_strerror(tk_status s) {
  switch (s) {
    case TK_OK: return "ok";
    case TK_E_ARG: return "invalid argument";
    case TK_E_CUTOFF: return "cutoff exceeds half the box edge";
    case TK_E_CAPACITY: return "output capacity too small (required size reported)";
    case TK_E_NOCONV: return "polarization solver did not converge within maxiter";
    case TK_E_BREAKDOWN: return "polarization operator not positive definite (p.Ap <= 0)";
    case TK_E_NOMEM: return "device memory allocation failed";
    case TK_E_HIP: return "HIP runtime error";
    case TK_E_BUSY: return "result not ready";
    case TK_E_PLAN: return "neighbour-list plan missing or built for another system";
    case TK_E_TOOBIG:
      return "system too large for the fixed scratch of the allocation-free entry point";
    default: return "unknown status";
  }
}

}  // extern "C"
