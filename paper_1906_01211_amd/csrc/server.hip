// Serving runtime: continuous batching of AMOEBA step requests on one GPU.
//
// A worker thread owns a context and a stream.  It takes requests from the
// queue in arrival order into a batch while the batch's estimated device
// footprint stays within the budget, runs one multi-system step for the whole
// batch (tk_batch_step), publishes the results, and starts the next batch
// with whatever has arrived meanwhile.  Host staging is pinned and grow-only.
#include <hip/hip_runtime.h>

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
  ~Dev() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

struct tk_server {
  int device = 0;
  tk_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
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
  int inflight = 0;
  bool stop = false;
  std::thread worker;
  // staging: inputs (xyz | mpole | pol | thole | rad | eps | guess), molid, outputs
  Pinned h_in, h_mol, h_out;
  Dev d_in, d_mol, d_out;

  void loop();
  tk_status run(std::vector<std::shared_ptr<Req>>& batch,
                const std::vector<const std::vector<double>*>& guesses);
};

extern "C" size_t tk_server_footprint(int32_t n) {
  // per atom: inputs 164 B (coordinates, molecule id, multipoles, four
  // parameters, guess) and outputs 72 B; candidate windows of the 9 A list
  // build ~7.2 KB (transient, shared by both builds); pair codes of both
  // lists ~1.1 KB; cached mat-vec factors ~1.4 KB; partial-result slots
  // 0.7 KB; sorted fields and solver vectors ~0.5 KB.  Plus fixed per-system
  // tables.
  return (size_t)(n > 0 ? n : 0) * 11264 + 256 * 1024;
}

tk_status tk_server::run(std::vector<std::shared_ptr<Req>>& batch,
                         const std::vector<const std::vector<double>*>& guesses) {
  const int nsys = (int)batch.size();
  std::vector<int32_t> off(nsys + 1, 0);
  std::vector<double> box(nsys);
  std::vector<int32_t> use_guess(nsys, 0);
  bool any_guess = false;
  for (int k = 0; k < nsys; ++k) {
    off[k + 1] = off[k] + batch[k]->n;
    box[k] = batch[k]->box;
    use_guess[k] = guesses[k] != nullptr;
    any_guess |= use_guess[k] != 0;
  }
  const size_t n = (size_t)off[nsys];
  // field offsets (doubles) in the input block
  const size_t o_xyz = 0, o_mp = 3 * n, o_pol = 13 * n, o_th = 14 * n, o_rad = 15 * n,
               o_eps = 16 * n, o_g = 17 * n, nin = 20 * n;
  tk_status s;
  if ((s = h_in.ensure(sizeof(double) * (nin + 1))) || (s = d_in.ensure(sizeof(double) * (nin + 1))) ||
      (s = h_mol.ensure(sizeof(int32_t) * (n + 1))) || (s = d_mol.ensure(sizeof(int32_t) * (n + 1))) ||
      (s = h_out.ensure(sizeof(double) * (9 * n + 1))) ||
      (s = d_out.ensure(sizeof(double) * (9 * n + 1))))
    return s;
  double* hi = (double*)h_in.p;
  int32_t* hm = (int32_t*)h_mol.p;
  for (int k = 0; k < nsys; ++k) {
    const Req& r = *batch[k];
    const size_t a = (size_t)off[k], na = (size_t)r.n;
    std::memcpy(hi + o_xyz + 3 * a, r.xyz.data(), sizeof(double) * 3 * na);
    std::memcpy(hi + o_mp + 10 * a, r.mpole.data(), sizeof(double) * 10 * na);
    std::memcpy(hi + o_pol + a, r.pol.data(), sizeof(double) * na);
    std::memcpy(hi + o_th + a, r.thole.data(), sizeof(double) * na);
    std::memcpy(hi + o_rad + a, r.rad.data(), sizeof(double) * na);
    std::memcpy(hi + o_eps + a, r.eps.data(), sizeof(double) * na);
    if (guesses[k]) std::memcpy(hi + o_g + 3 * a, guesses[k]->data(), sizeof(double) * 3 * na);
    else std::memset(hi + o_g + 3 * a, 0, sizeof(double) * 3 * na);
    std::memcpy(hm + a, r.molid.data(), sizeof(int32_t) * na);
  }
  if (hipMemcpyAsync(d_in.p, h_in.p, sizeof(double) * nin, hipMemcpyHostToDevice, stream) ||
      hipMemcpyAsync(d_mol.p, h_mol.p, sizeof(int32_t) * n, hipMemcpyHostToDevice, stream))
    return TK_E_HIP;
  const double* di = (const double*)d_in.p;
  double* dout = (double*)d_out.p;
  tk_batch b{nsys, off.data(), box.data(), di + o_xyz, (const int32_t*)d_mol.p};
  std::vector<tk_step_result> res(nsys);
  s = tk_batch_step(ctx, stream, &b, &prm, di + o_mp, di + o_pol, di + o_th, di + o_rad,
                          di + o_eps, any_guess ? di + o_g : nullptr,
                          any_guess ? use_guess.data() : nullptr, dout, dout + 3 * n,
                          dout + 6 * n, res.data());
  if (s) return s;
  if (hipMemcpyAsync(h_out.p, d_out.p, sizeof(double) * 9 * n, hipMemcpyDeviceToHost, stream) ||
      hipStreamSynchronize(stream))
    return TK_E_HIP;
  const double* ho = (const double*)h_out.p;
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

void tk_server::loop() {
  (void)hipSetDevice(device);   // the worker thread's device (checked at creation)
  for (;;) {
    std::vector<std::shared_ptr<Req>> batch;
    std::vector<const std::vector<double>*> guesses;
    {
      std::unique_lock<std::mutex> lk(m);
      cv_work.wait(lk, [&] { return stop || !queue.empty(); });
      if (queue.empty()) return;   // stop requested and nothing left
      size_t fp = 0;
      while (!queue.empty() && (int)batch.size() < max_batch) {
        const std::shared_ptr<Req>& r = queue.front();
        if (!batch.empty() && fp + r->footprint > budget) break;
        fp += r->footprint;
        batch.push_back(r);
        queue.pop_front();
      }
      for (auto& r : batch) {
        const std::vector<double>* g = nullptr;
        if (r->session) {
          auto it = session_mu.find(r->session);
          if (it != session_mu.end() && it->second.size() == 3 * (size_t)r->n) g = &it->second;
        }
        guesses.push_back(g);
      }
      inflight = (int)batch.size();
    }
    // the session guesses are only replaced by this thread, so the pointers
    // stay valid while the batch runs
    const int64_t t0 = now_ns();
    const int32_t index = batches++;
    for (auto& r : batch) {
      r->timing.t_start = t0;
      r->timing.batch_size = (int32_t)batch.size();
      r->timing.batch_index = index;
    }
    const tk_status s = run(batch, guesses);
    const int64_t t1 = now_ns();
    {
      std::lock_guard<std::mutex> lk(m);
      for (auto& r : batch) {
        r->status = s;
        r->timing.t_done = t1;
        r->done = true;
        if (s == TK_OK && r->session) session_mu[r->session] = r->mu;
      }
      inflight = 0;
    }
    cv_done.notify_all();
  }
}

extern "C" {

tk_status tk_server_create(int device, const tk_step_params* params, size_t hbm_budget,
                           int32_t max_batch, tk_server** out) {
  if (!out || !params || max_batch < 1 || hbm_budget == 0) return TK_E_ARG;
  *out = nullptr;
  tk_ctx* ctx = nullptr;
  tk_status s = tk_create(device, &ctx);
  if (s) return s;
  tk_server* srv = new tk_server();
  srv->device = device;
  srv->ctx = ctx;
  srv->prm = *params;
  srv->budget = hbm_budget;
  srv->max_batch = max_batch;
  if (hipStreamCreate(&srv->stream) != hipSuccess) {
    tk_destroy(ctx);
    delete srv;
    return TK_E_HIP;
  }
  srv->worker = std::thread([srv] { srv->loop(); });
  *out = srv;
  return TK_OK;
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
  if (r->footprint > srv->budget) return TK_E_CAPACITY;
  const size_t n = (size_t)q->n;
  r->xyz.assign(q->xyz, q->xyz + 3 * n);
  r->molid.assign(q->molid, q->molid + n);
  r->mpole.assign(q->mpole, q->mpole + 10 * n);
  r->pol.assign(q->polarity, q->polarity + n);
  r->thole.assign(q->thole, q->thole + n);
  r->rad.assign(q->vdw_rad, q->vdw_rad + n);
  r->eps.assign(q->vdw_eps, q->vdw_eps + n);
  r->timing.t_submit = now_ns();
  {
    std::lock_guard<std::mutex> lk(srv->m);
    if (srv->stop) return TK_E_ARG;
    r->id = srv->next_id++;
    srv->reqs[r->id] = r;
    srv->queue.push_back(r);
  }
  srv->cv_work.notify_one();
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

void tk_server_destroy(tk_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->m);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  (void)hipStreamDestroy(srv->stream);
  tk_destroy(srv->ctx);
  delete srv;
}

}  // extern "C"
