// Host runtime of libtk: context, grow-only device buffers, cell tables, a
// device exclusive scan, and argument checks shared by the entry points.
#include <cmath>
#include <cstring>

#include "tk_internal.hpp"

namespace tk {

tk_status hip_status(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) return TK_E_NOMEM;
  std::fprintf(stderr, "libtk: %s failed: %s\n", what, hipGetErrorString(e));
  return TK_E_HIP;
}

tk_status ensure(DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.bytes >= bytes) return TK_OK;
  if (b.p) {
    TK_HIP(hipDeviceSynchronize());   // queued kernels may still use the old buffer
    TK_HIP(hipFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
  }
  size_t want = bytes + bytes / 4;   // headroom so slightly larger inputs reuse it
  want = (want + 255) & ~size_t(255);
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    b.p = nullptr;
    return hip_status(e, "hipMalloc");
  }
  b.bytes = want;
  return TK_OK;
}

tk_status scratch(tk_ctx* ctx, const char* name, size_t bytes, void** out) {
  DevBuf& b = ctx->scratch[name];
  tk_status s = ensure(b, bytes);
  *out = b.p;
  return s;
}

tk_status pinned(tk_ctx* ctx, size_t bytes, void** out) {
  if (ctx->pinned_bytes < bytes) {
    if (ctx->pinned) TK_HIP(hipHostFree(ctx->pinned));
    ctx->pinned = nullptr;
    ctx->pinned_bytes = 0;
    size_t want = bytes < 4096 ? 4096 : bytes;
    TK_HIP(hipHostMalloc(&ctx->pinned, want, hipHostMallocDefault));
    ctx->pinned_bytes = want;
  }
  *out = ctx->pinned;
  return TK_OK;
}

const CellTables& cell_tables(tk_ctx* ctx, int nc) {
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
  return ctx->tables.emplace(nc, std::move(t)).first->second;
}

// ---------------------------------------------------------------------------
// Exclusive scan (three phases: block sums, scan of block sums, block scan).
constexpr int kScanBlock = 256, kScanItems = 4, kScanTile = kScanBlock * kScanItems;

__device__ __forceinline__ int block_exclusive_scan(int v, int* sh, int* total) {
  int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    int t = tid >= off ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += t;
    __syncthreads();
  }
  int incl = sh[tid];
  *total = sh[kScanBlock - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_sums(const int32_t* in, int len, int32_t* bsum) {
  __shared__ int sh[kScanBlock];
  long base = (long)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int s = 0;
  for (int q = 0; q < kScanItems; ++q)
    if (base + q < len) s += in[base + q];
  int tot;
  block_exclusive_scan(s, sh, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_bsum(int32_t* bsum, int nb) {
  __shared__ int sh[kScanBlock];
  int carry = 0;
  for (int b0 = 0; b0 < nb; b0 += kScanBlock) {
    int i = b0 + threadIdx.x;
    int v = i < nb ? bsum[i] : 0;
    int tot;
    int ex = block_exclusive_scan(v, sh, &tot);
    if (i < nb) bsum[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_final(const int32_t* in, int len,
                                                           const int32_t* bsum, int32_t* out) {
  __shared__ int sh[kScanBlock];
  long base = (long)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int v[kScanItems], s = 0;
  for (int q = 0; q < kScanItems; ++q) {
    v[q] = base + q < len ? in[base + q] : 0;
    s += v[q];
  }
  int tot;
  int ex = block_exclusive_scan(s, sh, &tot) + bsum[blockIdx.x];
  for (int q = 0; q < kScanItems; ++q) {
    if (base + q < len) out[base + q] = ex;
    ex += v[q];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[len] = bsum[gridDim.x];
}

tk_status scan_i32(tk_ctx* ctx, hipStream_t st, const int32_t* in, int32_t* out, int len) {
  int nb = ceil_div(len, kScanTile);
  if (nb < 1) nb = 1;
  void* bs;
  tk_status s = scratch(ctx, "scan_bsum", sizeof(int32_t) * (nb + 1), &bs);
  if (s) return s;
  k_scan_sums<<<nb, kScanBlock, 0, st>>>(in, len, (int32_t*)bs);
  k_scan_bsum<<<1, kScanBlock, 0, st>>>((int32_t*)bs, nb);
  k_scan_final<<<nb, kScanBlock, 0, st>>>(in, len, (int32_t*)bs, out);
  TK_HIP(hipGetLastError());
  return TK_OK;
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
  if (!p.valid || p.n != sys->n || p.box != sys->box || p.cutoff != list->cutoff ||
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
  tk_ctx* c = new tk_ctx();
  c->device = device;
  *out = c;
  return TK_OK;
}

void tk_destroy(tk_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  auto freeb = [](tk::DevBuf& b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  };
  for (auto& p : ctx->plans) {
    freeb(p.perm); freeb(p.scell); freeb(p.cell_start); freeb(p.cell_nslot); freeb(p.units);
    freeb(p.unit_ptr); freeb(p.codes); freeb(p.us); freeb(p.nbr);
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
    default: return "unknown status";
  }
}

}  // extern "C"
