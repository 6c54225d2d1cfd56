// Serving runtime: continuous batching of AMOEBA step requests on one GPU.
//
// The server runs up to kMaxLanes lanes (three unless the caller asks for
// fewer).  A lane is a host thread with its own
// context (plans and scratch), HIP stream and pinned staging.  An idle lane
// takes the requests queued at that moment, in arrival order, into a batch
// and runs one multi-system step for the whole batch (tk_batch_step) on its
// stream; a request that arrives while batches are on the GPU is taken at
// once by the next idle lane, so its work overlaps theirs on the device (the
// solver's host synchronisations of one lane leave the GPU to the others).
// A system's results do not depend on the batch it runs in (every per-system
// sum has a fixed order), so a request returns the same numbers alone or in
// the mix.
//
// Admission is by measured device memory.  Every lane reports what its
// context and staging hold after each batch (grow-only buffers: what its
// largest batch needed).  A batch is admitted to a lane when its
// reservation, the lane's projected holdings, plus what the other lanes hold
// or have reserved stays within the budget.  The projection uses the
// measured bytes per atom (the largest rate any lane has reported on a batch
// of 4,096 atoms or more, a fixed allowance set apart; a fixed per-atom
// estimate before that).  The lane's context is bounded by its reservation
// (tk_set_arena_budget): a batch that would need more fails with TK_E_NOMEM
// before it launches, and the lane runs its first request alone and returns
// the others to the head of the queue; a request refused alone goes back to
// the head of the queue, known to need half as much again, and fails only
// when refused with the whole budget to itself.  An idle lane whose holdings
// keep the head request out frees its context (the others keep theirs).  The
// lanes' device bytes never exceed the budget.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "tk.h"

namespace {

constexpr int kMaxLanes = 3;

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Req {
  uint64_t id = 0;
  int32_t n = 0;
  double box = 0.0;
  uint64_t session = 0;
  std::vector<double> xyz, mpole, pol, thole, rad, eps;
  std::vector<int32_t> molid;
  size_t footprint = 0;
  size_t need = 0;   // device bytes it is known to need (0: not known)
  tk_timing timing{};
  bool done = false;
  tk_status status = TK_OK;
  tk_step_result res{};
  std::vector<double> f_mpole, mu, f_vdw;
};

// Grow-only pinned host buffer.
struct Pinned {
  void* p = nullptr;
  size_t bytes = 0;
  tk_status ensure(size_t want) {
    if (want <= bytes) return TK_OK;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) return TK_E_NOMEM;
    bytes = want;
    return TK_OK;
  }
  ~Pinned() {
    if (p) (void)hipHostFree(p);
  }
};

// Grow-only device buffer.
struct Dev {
  void* p = nullptr;
  size_t bytes = 0;
  tk_status ensure(size_t want) {
    if (want <= bytes) return TK_OK;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    if (hipMalloc(&p, want) != hipSuccess) return TK_E_NOMEM;
    bytes = want;
    return TK_OK;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  ~Dev() { release(); }
};

// Device bytes of a batch's staging (inputs 20 doubles and a molecule id per
// atom, outputs 9 doubles per atom).
size_t staging_bytes(size_t n) {
  return sizeof(double) * (20 * n + 1) + sizeof(int32_t) * (n + 1) + sizeof(double) * (9 * n + 1);
}

// Device bytes of a lane's staging once it has run a batch of n atoms (its
// buffers only grow: each keeps the larger of its size and what n needs).
struct Lane;
size_t staging_after(const Lane& L, size_t n);

struct Lane {
  int index = 0;
  tk_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  Pinned h_in, h_mol, h_out;
  Dev d_in, d_mol, d_out;
  size_t held = 0;       // device bytes the lane holds (context + staging), as last measured
  size_t reserved = 0;   // projected bytes of its running batch (>= held while it runs)
  int64_t max_atoms = 0; // atoms of the largest batch it has run
  std::thread th;
  size_t device_bytes() const {
    return (ctx ? tk_arena_bytes(ctx) : 0) + d_in.bytes + d_mol.bytes + d_out.bytes;
  }
};

// Drops the lane's context and staging and starts a new context: after a
// refused batch the buffers it grew part of the way are given back, so what
// the lane holds is always what its successful batches needed.
tk_status reset_lane(Lane& L, int device) {
  if (L.ctx) tk_destroy(L.ctx);
  L.ctx = nullptr;
  L.d_in.release();
  L.d_mol.release();
  L.d_out.release();
  return tk_create(device, &L.ctx);
}

size_t staging_after(const Lane& L, size_t n) {
  return std::max(L.d_in.bytes, sizeof(double) * (20 * n + 1)) +
         std::max(L.d_mol.bytes, sizeof(int32_t) * (n + 1)) +
         std::max(L.d_out.bytes, sizeof(double) * (9 * n + 1));
}

}  // namespace

struct tk_server {
  int device = 0;
  tk_step_params prm{};
  size_t budget = 0;
  int32_t max_batch = 0;
  std::mutex m;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Req>> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Req>> reqs;
  std::unordered_map<uint64_t, std::vector<double>> session_mu;   // last dipoles per session
  uint64_t next_id = 1;
  int32_t batches = 0;
  double bytes_per_atom = 0.0;   // measured (0: none yet)
  size_t peak = 0;               // largest sum of the lanes' measured holdings
  bool stop = false;
  int nlanes = kMaxLanes;
  int alive = 0;   // lanes still taking work
  Lane lanes[kMaxLanes];   // lanes past nlanes stay empty (no context, nothing held)

  void loop(Lane& L);
  // A lane that cannot make a context stops (called with m held); when it
  // was the last one, the queued requests fail rather than wait for ever.
  void lane_lost();
  // projected device bytes of a batch of `atoms` atoms on a lane
  size_t project(const Lane& L, int64_t atoms) const;
  size_t others(const Lane& L) const;
  tk_status run(Lane& L, std::vector<std::shared_ptr<Req>>& batch,
                const std::vector<std::vector<double>>& guesses);
};

extern "C" size_t tk_server_footprint(int32_t n) {
  // the estimate before any batch has been measured, from what lanes measure
  // on water-density systems (17-22 KB per atom for a whole step): candidate
  // windows of both list builds ~10 KB, pair codes of both lists ~1.1 KB,
  // cached mat-vec factors ~1.4 KB, the pair terms' partial slots (six
  // accumulators per slot) ~1.7 KB, gathered fields ~0.7 KB, solver vectors
  // and their mirrors ~1 KB, staging and per-cell tables the rest.  Plus
  // fixed per-system tables.
  return (size_t)(n > 0 ? n : 0) * 20480 + 256 * 1024;
}

// Per-context memory that does not scale with the atoms (cell tables, plan
// records of small batches, event pools): allowed for beside the measured
// per-atom rate, which is taken only from batches of kRateAtoms atoms or more.
constexpr size_t kFixedBytes = size_t(8) << 20;
constexpr int64_t kRateAtoms = 4096;

size_t tk_server::project(const Lane& L, int64_t atoms) const {
  // a lane sized for a larger batch already holds what this one needs
  if (atoms <= L.max_atoms) return L.held;
  size_t est = kFixedBytes + tk_server_footprint((int32_t)atoms);
  if (bytes_per_atom > 0.0)   // measured, with 10 % headroom
    est = kFixedBytes + (size_t)(1.1 * bytes_per_atom * (double)atoms);
  // buffers only grow: a lane never holds less than it does now
  return std::max(est, L.held);
}

size_t tk_server::others(const Lane& L) const {
  size_t s = 0;
  for (const Lane& o : lanes)
    if (&o != &L) s += std::max(o.held, o.reserved);
  return s;
}

tk_status tk_server::run(Lane& L, std::vector<std::shared_ptr<Req>>& batch,
                         const std::vector<std::vector<double>>& guesses) {
  const int nsys = (int)batch.size();
  std::vector<int32_t> off(nsys + 1, 0);
  std::vector<double> box(nsys);
  std::vector<int32_t> use_guess(nsys, 0);
  bool any_guess = false;
  for (int k = 0; k < nsys; ++k) {
    off[k + 1] = off[k] + batch[k]->n;
    box[k] = batch[k]->box;
    use_guess[k] = !guesses[k].empty();
    any_guess |= use_guess[k] != 0;
  }
  const size_t n = (size_t)off[nsys];
  // field offsets (doubles) in the input block
  const size_t o_xyz = 0, o_mp = 3 * n, o_pol = 13 * n, o_th = 14 * n, o_rad = 15 * n,
               o_eps = 16 * n, o_g = 17 * n, nin = 20 * n;
  tk_status s;
  if ((s = L.h_in.ensure(sizeof(double) * (nin + 1))) ||
      (s = L.d_in.ensure(sizeof(double) * (nin + 1))) ||
      (s = L.h_mol.ensure(sizeof(int32_t) * (n + 1))) ||
      (s = L.d_mol.ensure(sizeof(int32_t) * (n + 1))) ||
      (s = L.h_out.ensure(sizeof(double) * (9 * n + 1))) ||
      (s = L.d_out.ensure(sizeof(double) * (9 * n + 1))))
    return s;
  double* hi = (double*)L.h_in.p;
  int32_t* hm = (int32_t*)L.h_mol.p;
  for (int k = 0; k < nsys; ++k) {
    const Req& r = *batch[k];
    const size_t a = (size_t)off[k], na = (size_t)r.n;
    std::memcpy(hi + o_xyz + 3 * a, r.xyz.data(), sizeof(double) * 3 * na);
    std::memcpy(hi + o_mp + 10 * a, r.mpole.data(), sizeof(double) * 10 * na);
    std::memcpy(hi + o_pol + a, r.pol.data(), sizeof(double) * na);
    std::memcpy(hi + o_th + a, r.thole.data(), sizeof(double) * na);
    std::memcpy(hi + o_rad + a, r.rad.data(), sizeof(double) * na);
    std::memcpy(hi + o_eps + a, r.eps.data(), sizeof(double) * na);
    if (!guesses[k].empty())
      std::memcpy(hi + o_g + 3 * a, guesses[k].data(), sizeof(double) * 3 * na);
    else std::memset(hi + o_g + 3 * a, 0, sizeof(double) * 3 * na);
    std::memcpy(hm + a, r.molid.data(), sizeof(int32_t) * na);
  }
  if (hipMemcpyAsync(L.d_in.p, L.h_in.p, sizeof(double) * nin, hipMemcpyHostToDevice, L.stream) ||
      hipMemcpyAsync(L.d_mol.p, L.h_mol.p, sizeof(int32_t) * n, hipMemcpyHostToDevice, L.stream))
    return TK_E_HIP;
  const double* di = (const double*)L.d_in.p;
  double* dout = (double*)L.d_out.p;
  tk_batch b{nsys, off.data(), box.data(), di + o_xyz, (const int32_t*)L.d_mol.p};
  std::vector<tk_step_result> res(nsys);
  s = tk_batch_step(L.ctx, L.stream, &b, &prm, di + o_mp, di + o_pol, di + o_th, di + o_rad,
                    di + o_eps, any_guess ? di + o_g : nullptr,
                    any_guess ? use_guess.data() : nullptr, dout, dout + 3 * n, dout + 6 * n,
                    res.data());
  if (s) {
    (void)hipStreamSynchronize(L.stream);   // nothing of the batch is left in flight
    return s;
  }
  if (hipMemcpyAsync(L.h_out.p, L.d_out.p, sizeof(double) * 9 * n, hipMemcpyDeviceToHost,
                     L.stream) ||
      hipStreamSynchronize(L.stream))
    return TK_E_HIP;
  const double* ho = (const double*)L.h_out.p;
  for (int k = 0; k < nsys; ++k) {
    Req& r = *batch[k];
    const size_t a = (size_t)off[k], na = (size_t)r.n;
    r.res = res[k];
    r.f_mpole.assign(ho + 3 * a, ho + 3 * (a + na));
    r.mu.assign(ho + 3 * n + 3 * a, ho + 3 * n + 3 * (a + na));
    r.f_vdw.assign(ho + 6 * n + 3 * a, ho + 6 * n + 3 * (a + na));
  }
  return TK_OK;
}

void tk_server::lane_lost() {
  if (--alive > 0) return;
  for (auto& r : queue) {
    r->status = TK_E_NOMEM;
    r->done = true;
  }
  queue.clear();
  cv_done.notify_all();
}

void tk_server::loop(Lane& L) {
  (void)hipSetDevice(device);   // the lane thread's device (checked at creation)
  for (;;) {
    std::vector<std::shared_ptr<Req>> batch;
    std::vector<std::vector<double>> guesses;
    size_t limit = 0;
    {
      std::unique_lock<std::mutex> lk(m);
      for (;;) {
        if (stop && queue.empty()) return;   // stop requested and nothing left
        if (!queue.empty()) {
          // requests in arrival order while the projection fits
          const size_t held_elsewhere = others(L);
          const size_t room = budget - std::min(budget, held_elsewhere);
          int64_t atoms = 0;
          for (const auto& r : queue) {
            if ((int)batch.size() >= max_batch) break;
            // nothing held anywhere: the head request runs alone whatever the
            // projection says (its context stays bounded by the budget)
            const bool alone = batch.empty() && L.held == 0 && held_elsewhere == 0;
            const size_t want = std::max(project(L, atoms + r->n), r->need) +
                                staging_bytes((size_t)(atoms + r->n));
            if (!alone && want > room) break;
            atoms += r->n;
            batch.push_back(r);
          }
          if (!batch.empty()) {
            queue.erase(queue.begin(), queue.begin() + (long)batch.size());
            size_t need = project(L, atoms);
            for (auto& r : batch) need = std::max(need, r->need);
            L.reserved = need + staging_bytes((size_t)atoms);
            limit = room;
            break;
          }
          // the head request does not fit beside what this idle lane holds:
          // give the memory back (another lane, or this one next time, fits it)
          if (L.held > 0 && L.ctx) {
            lk.unlock();
            const tk_status cs = reset_lane(L, device);
            lk.lock();
            L.held = 0;
            L.max_atoms = 0;
            if (cs) {   // no context: this lane stops taking work
              L.ctx = nullptr;
              lane_lost();
              return;
            }
            cv_work.notify_all();   // the other lanes see the room this made
            continue;
          }
        }
        cv_work.wait(lk);
      }
      for (auto& r : batch) {
        std::vector<double> g;
        if (r->session) {
          auto it = session_mu.find(r->session);
          if (it != session_mu.end() && it->second.size() == 3 * (size_t)r->n) g = it->second;
        }
        guesses.push_back(std::move(g));
      }
    }
    // the context may not grow beyond the lane's reservation (the sum of the
    // reservations stays within the budget, so their holdings do too)
    int64_t batch_atoms = 0;
    for (auto& r : batch) batch_atoms += r->n;
    const size_t stage = staging_after(L, (size_t)batch_atoms);
    const size_t cap = std::min(L.reserved, limit);
    (void)tk_set_arena_budget(L.ctx, cap > stage ? cap - stage : 1);
    const int64_t t0 = now_ns();
    int32_t index;
    {
      std::lock_guard<std::mutex> lk(m);
      index = batches++;
    }
    for (auto& r : batch) {
      r->timing.t_start = t0;
      r->timing.batch_size = (int32_t)batch.size();
      r->timing.batch_index = index;
      r->timing.lane = L.index;
    }
    tk_status s = run(L, batch, guesses);
    if (s == TK_E_NOMEM && batch.size() > 1) {
      // the batch needs more than the admission allowed: run its first
      // request alone (on a new context: the refused batch's partly grown
      // buffers are given back) and return the others to the head of the
      // queue
      {
        std::lock_guard<std::mutex> lk(m);
        for (size_t k = batch.size(); k-- > 1;) queue.push_front(batch[k]);
      }
      cv_work.notify_all();
      batch.resize(1);
      guesses.resize(1);
      batch[0]->timing.batch_size = 1;
      s = reset_lane(L, device);
      L.max_atoms = 0;
      if (s == TK_OK) {
        const size_t stage1 = staging_after(L, (size_t)batch[0]->n);
        (void)tk_set_arena_budget(L.ctx, cap > stage1 ? cap - stage1 : 1);
        s = run(L, batch, guesses);
      }
    }
    if (s == TK_E_NOMEM) {
      // refused alone within its reservation: unless that was the whole
      // budget with nothing held elsewhere, it goes back to the head of the
      // queue, known to need half as much again (and 16 MiB) more, and waits
      // for that room
      std::unique_lock<std::mutex> lk(m);
      if (others(L) > 0 || cap < budget) {
        batch[0]->need = std::min(budget, std::max(batch[0]->need, cap + cap / 2 + (16u << 20)));
        queue.push_front(batch[0]);
        lk.unlock();
        const tk_status cs = reset_lane(L, device);   // give the partly grown buffers back
        lk.lock();
        L.held = L.device_bytes();
        L.max_atoms = 0;
        L.reserved = 0;
        if (cs) {   // no context: this lane stops taking work
          L.ctx = nullptr;
          L.held = 0;
          lane_lost();
          lk.unlock();
          cv_work.notify_all();
          return;
        }
        lk.unlock();
        cv_work.notify_all();
        continue;
      }
    }
    const int64_t t1 = now_ns();
    int64_t atoms = 0;
    for (auto& r : batch) atoms += r->n;
    {
      std::lock_guard<std::mutex> lk(m);
      L.max_atoms = std::max(L.max_atoms, atoms);
      L.held = L.device_bytes();
      L.reserved = 0;
      if (s == TK_OK && L.max_atoms >= kRateAtoms && L.held > kFixedBytes)
        bytes_per_atom =
            std::max(bytes_per_atom, (double)(L.held - kFixedBytes) / (double)L.max_atoms);
      size_t tot = 0;
      for (const Lane& o : lanes) tot += o.held;
      peak = std::max(peak, tot);
      for (auto& r : batch) {
        r->status = s;
        r->timing.t_done = t1;
        r->done = true;
        if (s == TK_OK && r->session) session_mu[r->session] = r->mu;
      }
    }
    cv_done.notify_all();
    cv_work.notify_all();   // memory and a lane are free again
    if (!L.ctx) {           // a new context could not be made: this lane stops
      std::lock_guard<std::mutex> lk(m);
      lane_lost();
      return;
    }
  }
}

extern "C" {

tk_status tk_server_create_lanes(int device, const tk_step_params* params, size_t hbm_budget,
                                 int32_t max_batch, int32_t lanes, tk_server** out) {
  if (!out || !params || max_batch < 1 || hbm_budget == 0 || lanes < 1 || lanes > kMaxLanes)
    return TK_E_ARG;
  *out = nullptr;
  tk_server* srv = new tk_server();
  srv->device = device;
  srv->prm = *params;
  srv->budget = hbm_budget;
  srv->max_batch = max_batch;
  srv->nlanes = lanes;
  for (int k = 0; k < lanes; ++k) {
    Lane& L = srv->lanes[k];
    L.index = k;
    tk_status s = tk_create(device, &L.ctx);
    if (!s && hipStreamCreate(&L.stream) != hipSuccess) s = TK_E_HIP;
    if (s) {
      for (int j = 0; j <= k; ++j) {
        if (srv->lanes[j].stream) (void)hipStreamDestroy(srv->lanes[j].stream);
        if (srv->lanes[j].ctx) tk_destroy(srv->lanes[j].ctx);
      }
      delete srv;
      return s;
    }
  }
  srv->alive = lanes;
  for (int k = 0; k < lanes; ++k) {
    Lane& L = srv->lanes[k];
    L.th = std::thread([srv, &L] { srv->loop(L); });
  }
  *out = srv;
  return TK_OK;
}

tk_status tk_server_create(int device, const tk_step_params* params, size_t hbm_budget,
                           int32_t max_batch, tk_server** out) {
  return tk_server_create_lanes(device, params, hbm_budget, max_batch, kMaxLanes, out);
}

tk_status tk_server_submit(tk_server* srv, const tk_request* q, uint64_t* id) {
  if (!srv || !q || !id || q->n < 0 || !(q->box > 0.0)) return TK_E_ARG;
  if (q->n > 0 && (!q->xyz || !q->molid || !q->mpole || !q->polarity || !q->thole ||
                   !q->vdw_rad || !q->vdw_eps))
    return TK_E_ARG;
  const double need = srv->prm.rc_ewald + srv->prm.skin;
  if (need > 0.5 * q->box) return TK_E_CUTOFF;
  auto r = std::make_shared<Req>();
  r->n = q->n;
  r->box = q->box;
  r->session = q->session;
  r->footprint = tk_server_footprint(q->n);
  {   // one request alone must be able to fit the budget: rejected here only
      // when even the estimate without headroom (the measured rate once there
      // is one) exceeds it; a request that passes and still needs more fails
      // when it is refused with the whole budget to itself
    std::lock_guard<std::mutex> lk(srv->m);
    size_t fp = r->footprint;
    if (srv->bytes_per_atom > 0.0)
      fp = kFixedBytes + (size_t)(srv->bytes_per_atom * (double)q->n);
    if (fp + staging_bytes((size_t)q->n) > srv->budget) return TK_E_CAPACITY;
  }
  const size_t n = (size_t)q->n;
  r->xyz.assign(q->xyz, q->xyz + 3 * n);
  r->molid.assign(q->molid, q->molid + n);
  r->mpole.assign(q->mpole, q->mpole + 10 * n);
  r->pol.assign(q->polarity, q->polarity + n);
  r->thole.assign(q->thole, q->thole + n);
  r->rad.assign(q->vdw_rad, q->vdw_rad + n);
  r->eps.assign(q->vdw_eps, q->vdw_eps + n);
  r->timing.t_submit = now_ns();
  r->timing.lane = -1;
  {
    std::lock_guard<std::mutex> lk(srv->m);
    if (srv->stop) return TK_E_ARG;
    if (srv->alive == 0) return TK_E_NOMEM;   // no lane could keep a context
    r->id = srv->next_id++;
    srv->reqs[r->id] = r;
    srv->queue.push_back(r);
  }
  srv->cv_work.notify_all();
  *id = r->id;
  return TK_OK;
}

tk_status tk_server_poll(tk_server* srv, uint64_t id, tk_step_result* result, tk_timing* timing,
                         double* force_mpole, double* mu, double* force_vdw) {
  if (!srv) return TK_E_ARG;
  std::shared_ptr<Req> r;
  {
    std::lock_guard<std::mutex> lk(srv->m);
    auto it = srv->reqs.find(id);
    if (it == srv->reqs.end()) return TK_E_ARG;
    r = it->second;
    if (!r->done) return TK_E_BUSY;
  }
  if (timing) *timing = r->timing;
  if (r->status) return r->status;
  if (result) *result = r->res;
  const size_t b = sizeof(double) * 3 * (size_t)r->n;
  if (force_mpole) std::memcpy(force_mpole, r->f_mpole.data(), b);
  if (mu) std::memcpy(mu, r->mu.data(), b);
  if (force_vdw) std::memcpy(force_vdw, r->f_vdw.data(), b);
  return TK_OK;
}

tk_status tk_server_release(tk_server* srv, uint64_t id) {
  if (!srv) return TK_E_ARG;
  std::lock_guard<std::mutex> lk(srv->m);
  auto it = srv->reqs.find(id);
  if (it == srv->reqs.end() || !it->second->done) return TK_E_ARG;
  srv->reqs.erase(it);
  return TK_OK;
}

tk_status tk_server_stats(tk_server* srv, tk_server_usage* out) {
  if (!srv || !out) return TK_E_ARG;
  std::lock_guard<std::mutex> lk(srv->m);
  out->lanes = srv->nlanes;
  out->batches = srv->batches;
  out->budget = srv->budget;
  out->peak_device_bytes = srv->peak;
  size_t held = 0;
  for (const Lane& L : srv->lanes) held += L.held;
  out->device_bytes = held;
  out->bytes_per_atom = srv->bytes_per_atom;
  return TK_OK;
}

void tk_server_destroy(tk_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->m);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  for (Lane& L : srv->lanes)
    if (L.th.joinable()) L.th.join();
  for (Lane& L : srv->lanes) {
    if (L.stream) (void)hipStreamDestroy(L.stream);
    L.d_in.release();
    L.d_mol.release();
    L.d_out.release();
    if (L.ctx) tk_destroy(L.ctx);
  }
  delete srv;
}

}  // extern "C"
