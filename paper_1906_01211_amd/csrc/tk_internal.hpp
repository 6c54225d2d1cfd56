// Internal declarations of libtk: context, plan slots, device-buffer arena,
// launch helpers.  Host and device code include this header; it is not part of
// the C-ABI (include/tk.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "tk.h"

namespace tk {

// Readings where the paper is silent (Coulomb constant, Debye factor).
constexpr double kCoulomb = 332.0637;
constexpr double kDebye = 4.80320;
constexpr double kSqrtPi = 1.7724538509055160273;
constexpr double kTwo32 = 4294967296.0;

// Cell-pair work decomposition.  Cells are at least one list cutoff wide, so
// every listed pair joins a cell to one of its (at most 27) neighbours.  A
// work unit is an unordered neighbouring cell pair (H, K), H <= K; each cell
// takes part in at most 28 unit roles (27 neighbours, the self pair twice),
// and each role owns one partial-result slot for the cell's atoms.
constexpr int kMaxSlots = 28;
// Plan slots beyond the caller's TK_MAX_PLANS, used by the batch step.
constexpr int kBatchPlan7 = TK_MAX_PLANS, kBatchPlan9 = TK_MAX_PLANS + 1;
constexpr int kNumPlans = TK_MAX_PLANS + 2;
constexpr int kCellUnitStride = 28;  // per-cell unit list: count + up to 27 entries
constexpr int kMaxCellAtoms = 512;   // LDS staging limit per cell
constexpr int kWave = 64;
constexpr size_t kMaxLds = 160 * 1024;   // LDS per workgroup on gfx950

struct Unit {
  int32_t h, k, slot_h, slot_k;
};

// Everything a pair kernel's workgroup needs about its unit, in one record
// (built once per list): the two cells' first sorted atom and size, the
// partial-result slots, the system, and the unit's listed pairs.
struct UnitRec {
  int32_t hs, nh, ks, nk, slot_h, slot_k, sy, cnt;
  int64_t off;
};

// One system of a plan.  A plan holds one system (the single-system entry
// points) or a batch of independent systems (the serving path): each system
// has its own box, cell grid and list cutoff; its cells, units and atoms are
// contiguous ranges of the plan's.
struct SysDev {
  double box, inv_box;
  uint64_t rq2;            // quantised list cutoff squared (exact test)
  double lo, hi;           // band of the FP64 pre-test around rq2
  int32_t nc, cell0, unit0, atom0;
};

// Device views of a plan (the pair set of one neighbour list, in cell-pair
// order).  Sorted position s = rank of an atom by (cell, caller index).
struct PlanView {
  int32_t n, ncells, nunits, max_occ;
  const int32_t* perm;        // [n] sorted position -> caller index
  const int32_t* scell;       // [n] cell of sorted position
  const int32_t* cell_start;  // [ncells+1]
  const int32_t* cell_nslot;  // [ncells] number of unit roles of the cell
  const Unit* units;          // [nunits]
  const int64_t* unit_off;    // [nunits+1] start of each unit's window in codes
  const int32_t* unit_cnt;    // [nunits] listed pairs of the unit (window prefix)
  const uint32_t* codes;      // pair codes: a | b << 16 (local indices in H, K)
  const int32_t* cell_units;  // [ncells][28]: count, then unit * 4 + role
  const int32_t* cell_order;  // [ncells] cells grouped by octant of their system's box
  int32_t nsys;
  const SysDev* sys;          // [nsys]
  const int32_t* cell_sys;    // [ncells] system of each cell; nullptr when nsys == 1
  const UnitRec* urec;        // [nunits]
  // build outcome on the device: 0 when the plan is whole.  A build queued
  // without a host synchronisation (tk_nblist_build_async) can exceed the
  // caller's bounds; kernels that index plan tables skip their work then.
  const int32_t* status;
};

// Workgroups are dispatched to the 8 XCDs round-robin.  Per-cell kernels
// launch 8 * ceil(ncells / 8) workgroups and map workgroup i to position
// (i % 8) * ceil(ncells / 8) + i / 8 of the octant-grouped cell order, so
// each XCD (with its own L2) works on one spatially compact block of cells
// and most neighbour cells share an L2.  Both return -1 for the padding.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_pos(int ncells, int wg) {
  const int per = (ncells + kXcds - 1) / kXcds;
  const int pos = (wg % kXcds) * per + wg / kXcds;
  return pos < ncells ? pos : -1;
}
__device__ __forceinline__ int xcd_cell(const PlanView& pv, int wg) {
  const int pos = xcd_pos(pv.ncells, wg);
  return pos >= 0 ? pv.cell_order[pos] : -1;
}
inline int xcd_grid(int ncells) { return (ncells + kXcds - 1) / kXcds * kXcds; }

// System of a cell (0 for single-system plans).
__device__ __forceinline__ int cell_system(const PlanView& pv, int c) {
  return pv.cell_sys ? pv.cell_sys[c] : 0;
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct Plan {
  bool valid = false;
  int32_t n = 0;
  double box = 0.0, cutoff = 0.0;
  int32_t nc = 0, ncells = 0, nunits = 0, max_occ = 0, max_row = 0;
  int32_t max_nbhd = 0;   // max over cells of the atoms in the cell's neighbour cells (itself included)
  int64_t npairs = 0;      // -1: built by tk_nblist_build_async (the count is on the device)
  int64_t windows = 0;     // candidate pairs of the last synchronous build (sum |H| |K|)
  bool measured = false;   // the sizes above were measured by a synchronous build
  DevBuf perm, scell, cell_start, unit_off, unit_cnt, codes, us, slots, urec;
  const Unit* units_p = nullptr;       // device cell tables (shared by plans with the same
  const int32_t* nslot_p = nullptr;    // nc for one system; built per batch otherwise)
  const int32_t* cu_p = nullptr;
  const int32_t* order_p = nullptr;
  int32_t nsys = 1;
  std::vector<SysDev> h_sys;           // host copy of sysd (as uploaded), with a final entry holding the totals
  DevBuf sysd, cell_sys, bunits, bnslot, bcu, border, tplp;
  DevBuf dstat;                        // int32 [2]: build outcome (PlanView::status), spare
  PlanView view() const {
    PlanView v;
    v.nsys = nsys;
    v.sys = (const SysDev*)sysd.p;
    v.cell_sys = nsys > 1 ? (const int32_t*)cell_sys.p : nullptr;
    v.n = n; v.ncells = ncells; v.nunits = nunits; v.max_occ = max_occ;
    v.perm = (const int32_t*)perm.p; v.scell = (const int32_t*)scell.p;
    v.cell_start = (const int32_t*)cell_start.p; v.cell_nslot = nslot_p;
    v.units = units_p; v.unit_off = (const int64_t*)unit_off.p;
    v.unit_cnt = (const int32_t*)unit_cnt.p;
    v.codes = (const uint32_t*)codes.p;
    v.cell_units = cu_p;
    v.cell_order = order_p;
    v.status = (const int32_t*)dstat.p;
    v.urec = (const UnitRec*)urec.p;
    return v;
  }
};

struct CellTables {   // host-built tables for one cells-per-edge value
  int32_t nc = 0, ncells = 0, nunits = 0;
  std::vector<Unit> units;
  std::vector<int32_t> nslot;     // per cell
  std::vector<int32_t> nbr;       // per cell: count, then up to 27 neighbour cells
  std::vector<int32_t> cu;        // per cell: count, then unit * 4 + role (kCellUnitStride)
  std::vector<int32_t> order;     // cells grouped by octant of the box (XCD-local workgroups)
  bool uploaded = false;
  DevBuf units_d, nslot_d, cu_d, order_d;  // device copies
};

}  // namespace tk

namespace tk {
struct ProfEntry {
  int64_t launches = 0;
  double ms = 0.0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
};
}  // namespace tk

struct tk_ctx {
  int device = 0;
  bool prof_on = false;
  std::string prof_only;
  std::map<std::string, tk::ProfEntry> prof;
  std::vector<hipEvent_t> event_pool;
  tk::Plan plans[tk::kNumPlans];
  std::map<std::string, tk::DevBuf> scratch;   // grow-only named device buffers
  std::map<int, tk::CellTables> tables;        // by cells per edge
  void* pinned = nullptr;                      // host readback buffer (device-writable)
  void* pinned_dev = nullptr;                  // its device address
  size_t pinned_bytes = 0;
  int pcg_hint[tk::kNumPlans][2] = {};         // last solve's iteration count per plan slot, precision
  bool nb_info_zero[4] = {};                   // per build of a group: its status words are zero
  void* noalloc_scratch = nullptr;             // device address of the fixed scratch array
  size_t arena_budget = 0;                     // device bytes the context may hold (0: any)
  size_t arena_bytes = 0;                      // device bytes it holds (grow-only buffers)
};

namespace tk {

tk_status hip_status(hipError_t e, const char* what);
#define TK_HIP(call)                                     \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return tk::hip_status(e_, #call); \
  } while (0)

// Grow-only buffers: the first call with a given size allocates, later calls
// reuse.  Never freed before tk_destroy.
// The context's budget, when set, bounds the sum of all its buffers
// (TK_E_NOMEM beyond it, the old buffer kept).
tk_status ensure(tk_ctx* ctx, DevBuf& b, size_t bytes);
tk_status scratch(tk_ctx* ctx, const char* name, size_t bytes, void** out);
// Pinned host memory that kernels write directly (zero-copy readback).
tk_status pinned(tk_ctx* ctx, size_t bytes, void** out, void** dev = nullptr);
CellTables& cell_tables(tk_ctx* ctx, int nc);

// Exclusive scan of int32 counts: out[0..len] with out[len] = total.
// Scratch of work that may run on several streams of one context at the
// same time (the pair terms): one buffer set per stream.
inline std::string per_stream(const char* base, hipStream_t st) {
  if (!st) return base;
  char buf[40];
  std::snprintf(buf, sizeof buf, "@%p", (void*)st);
  return std::string(base) + buf;
}
// job: index of the list build in a group (separate scratch per build).
tk_status scan_i32(tk_ctx* ctx, hipStream_t st, const int32_t* in, int32_t* out, int len,
                   int job = 0);
tk_status scan_i64(tk_ctx* ctx, hipStream_t st, const int64_t* in, int64_t* out, long len,
                   int job = 0);
// Both exclusive scans (out[len] = total) in two launches.
tk_status scan_pair(tk_ctx* ctx, hipStream_t st, const int32_t* in1, int32_t* out1, int len1,
                    const int64_t* in2, int64_t* out2, long len2, int job = 0);

// Systems of a plan (host arrays): atom0[nsys+1] offsets, box[nsys],
// list cutoff[nsys].
struct PlanSpec {
  int nsys;
  const int32_t* atom0;
  const double* box;
  const double* cutoff;
};
// Builds plan slot `slot` for the atoms xyz[n][3] (and the caller's CSR when
// row_ptr is given); synchronises the stream once.
tk_status build_plan(tk_ctx* ctx, hipStream_t st, int slot, int n, const double* xyz,
                     const PlanSpec& spec, int32_t* row_ptr, int32_t* col, int64_t cap,
                     int64_t* npairs_out);
// Several plans of the same atoms (no CSR), queued on one stream with one
// synchronisation.
tk_status build_plans(tk_ctx* ctx, hipStream_t st, int nj, const int* slots, int n,
                      const double* xyz, const PlanSpec* specs, int64_t* npairs_out);

// Induced dipoles of every system of plan P (right-hand side, PCG, FP64 true
// residual and, in the mixed form, refinement).  xyz, molid and the
// parameters are in caller order for the plan's atoms; mu_guess is used for
// the systems whose guess_on entry (device [nsys], nullable: all) is nonzero;
// info[P->nsys] is host memory.  Synchronises the stream while solving;
// mu_out is written in stream order after the return.
// Reciprocal space (smooth PME, pme.hip).  grid: 16, 32, 64 or 128; order 5..8.
bool pme_args_ok(int grid, int order);
// -grad phi of dipoles v ([n][3], the sites' own order) for a solve whose
// sites (positions pos[a * ps + j]) do not move: pme_prepare_sites sorts
// the sites and tabulates their spline weights once (this stream's scratch);
// pme_prepared_dipole_field then takes only the dipoles; with done set, its
// launches return at once while *done != 0 (run_when_done 0) or while
// *done == 0 (run_when_done 1).  A contribution
// refused by the fixed-point spread makes this and every later field of the
// solve NaN.
tk_status pme_prepare_sites(tk_ctx* ctx, hipStream_t st, int n, double box, const double* pos,
                            long ps, int grid, int order);
tk_status pme_prepared_dipole_field(tk_ctx* ctx, hipStream_t st, int n, double box,
                                    const double* v, double beta, int grid, int order,
                                    double* out, const int32_t* done, int run_when_done);
// The fields of two dipole sets in one pass over the mesh (the two meshes
// packed into one complex FFT), each set spread and gathered under its own
// done flag (done2 for v2), the FFT passes while either runs.
tk_status pme_prepared_dipole_field2(tk_ctx* ctx, hipStream_t st, int n, double box,
                                     const double* v, const double* v2, double beta, int grid,
                                     int order, double* out, double* out2, const int32_t* done,
                                     const int32_t* done2, int run_when_done);
// PME energies and forces of two multipole sets of the same sites in one
// pass over the mesh (the two meshes packed into one complex FFT).  e1, e2:
// device [1]; f1, f2: device [n][3].
tk_status pme_mpole_pair(tk_ctx* ctx, hipStream_t st, const tk_system* sys, const double* m1,
                         const double* m2, double beta, int grid, int order, double* e1,
                         double* f1, double* e2, double* f2);
// b_sorted[3 s + a] += reciprocal field of the permanent multipoles at site perm[s].
tk_status pme_perm_field_add(tk_ctx* ctx, hipStream_t st, const tk_system* sys,
                             const double* mpole, double beta, int grid, int order,
                             const int32_t* perm, double* b_sorted);
// With mp_energy set, the permanent multipoles' energy [3], forces (caller
// order) and virial [9] come out of the same pass as the right-hand side.
tk_status solve_dipoles(tk_ctx* ctx, hipStream_t st, const Plan* P, const double* xyz,
                        const int32_t* molid, const double* mpole, const double* polarity,
                        const double* thole, double ewald_beta, double cutoff, double tol_debye,
                        int32_t maxiter, int prec, const double* mu_guess,
                        const int32_t* guess_on, double* mu_out, tk_pcg_info* info,
                        int pme_grid = 0, int pme_order = 0, int nv = 1, double pscale = 0.0,
                        double* mp_energy = nullptr, double* mp_force = nullptr,
                        double* mp_virial = nullptr, int32_t queued = 0,
                        tk_pcg_info* info_dev = nullptr);

// The allocation-free entry point's fixed scratch (noalloc.hip): resolves
// the device address of this device's copy of the array (once per device;
// the device must be current) into *addr.
tk_status noalloc_setup(int device, void** addr);
struct TermWs;
// Mutual-field mat-vec with its argument checks (tk_tmatvec); with ws set,
// every device buffer comes from ws and the call fails with TK_E_TOOBIG when
// they would need more than ws_limit_doubles doubles.
tk_status tmatvec_checked(tk_ctx* ctx, hipStream_t st, const tk_system* sys,
                          const tk_nblist* list, const double* polarity, const double* thole,
                          double ewald_beta, double cutoff, int include_diag, int prec,
                          const double* mu, double* out, const TermWs* ws,
                          size_t ws_limit_doubles);
// Doubles of scratch the mat-vec takes for n atoms (partial slots and
// gathered fields, each padded to a multiple of 64 atoms).
size_t tmatvec_ws_doubles_n(long n);

// Checks shared by the pair entry points.
tk_status check_system(const tk_system* sys);
tk_status get_plan(tk_ctx* ctx, const tk_system* sys, const tk_nblist* list, double cutoff,
                   const Plan** out);

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

// Brackets one kernel launch with events when kernel timing is on.
// on_kernel: the scope times one kernel launched with hipExtLaunchKernelGGL
// and the events start()/stop() (recorded by the dispatch itself, so no
// marker gaps); otherwise markers are recorded around the scope.  start() is
// null when the scope is not being timed.
struct ProfScope {
  tk_ctx* ctx;
  hipStream_t st;
  ProfEntry* e = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  bool on_kernel = false;
  ProfScope(tk_ctx* c, hipStream_t s, const std::string& name, bool kernel_events = false);
  ~ProfScope();
  hipEvent_t start() const { return on_kernel ? a : nullptr; }
  hipEvent_t stop() const { return on_kernel ? b : nullptr; }
};

}  // namespace tk
