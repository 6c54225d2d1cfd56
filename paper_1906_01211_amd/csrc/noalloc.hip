// The allocation-free form of the induced-dipole field mat-vec, for callers
// that may not allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).
//
// Its device buffers (the per-atom partial slots and the gathered per-atom
// fields of the cell-pair kernels) live in one fixed file-scope array; each
// device that loads the library holds its own copy until the process ends.
// The host never uses the array's name as a device address: tk_create looks
// up this device's address of it once (hipGetSymbolAddress, with the device
// current) and every launch takes that address.  Every call on a device
// shares that device's copy, so calls that overlap on one device (two streams,
// two contexts) race on it and must be ordered by the caller.  Nothing in the
// array has to start at zero: every slot that a call reads back was written
// earlier in the same call.
#include <mutex>

#include "pairs.hpp"

namespace {
// 32 MiB: the mat-vec takes 720 bytes per atom (28 partial slots of three
// components and six gathered fields, rows padded to 64 atoms), so systems of
// up to 46,592 atoms fit.
constexpr size_t kNoAllocBytes = size_t(32) << 20;
}  // namespace

static __device__ __align__(256) double scratch[kNoAllocBytes / sizeof(double)];

namespace tk {
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};
}  // namespace

tk_status noalloc_setup(int device, void** addr) {
  if (device < 0 || device >= kMaxDevices) return TK_E_ARG;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_addr[device]) {
    void* p = nullptr;
    // "::": inside namespace tk the bare name is the scratch-buffer function
    TK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(::scratch)));
    if (!p) return TK_E_HIP;
    g_addr[device] = p;
  }
  *addr = g_addr[device];
  return TK_OK;
}

}  // namespace tk

extern "C" {

int32_t tk_tmatvec_noalloc_max_atoms(void) {
  const size_t per64 = tk::tmatvec_ws_doubles_n(64) * sizeof(double);   // bytes per 64 atoms
  return (int32_t)(kNoAllocBytes / per64 * 64);
}

tk_status tk_tmatvec_noalloc(tk_ctx* ctx, void* stream, const tk_system* sys,
                             const tk_nblist* list, const double* polarity, const double* thole,
                             double ewald_beta, double cutoff, int include_diag, int prec,
                             const double* mu, double* out) {
  if (!ctx || !ctx->noalloc_scratch) return TK_E_ARG;
  if (sys && sys->n > tk_tmatvec_noalloc_max_atoms()) return TK_E_TOOBIG;
  const long n = sys ? (sys->n > 0 ? sys->n : 0) : 0;
  double* base = (double*)ctx->noalloc_scratch;
  tk::TermWs ws;
  ws.partial = base;   // [kMaxSlots][3][pad64(n)], then the gathered fields
  ws.gathered = base + (size_t)tk::kMaxSlots * 3 * tk::pad64(n);
  return tk::tmatvec_checked(ctx, (hipStream_t)stream, sys, list, polarity, thole, ewald_beta,
                             cutoff, include_diag, prec, mu, out, &ws,
                             kNoAllocBytes / sizeof(double));
}

}  // extern "C"
