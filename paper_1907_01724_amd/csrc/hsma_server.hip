// Request server over resident systems: continuous batching of single-ion-move energy
// changes and full-energy evaluations, admission of systems by device memory, per-request
// timestamps.  Host code only; the device work is the batched single-ion-move pipeline
// (launch_delta) and the FP64 full evaluation of a system.
//
// Scheduling: a host thread keeps a FIFO of pending requests.  Whenever a batch slot is free
// it takes, in arrival order, every pending single-ion-move request whose system has no move
// on the device and no earlier request still waiting, up to max_batch, and launches them as
// one batch on that slot's stream.  Full-energy requests take energy slots (their own streams
// and workspaces); a full energy first copies its system's state, and holds back the system's
// later committed moves and energies until that copy is done.  Queries (moves that are not
// committed) and full energies only read a system, so a query may pass a full energy of its
// system that waits for a slot or for its copy; nothing passes a committed move.  Each
// system's results are therefore those of its requests run one by one in arrival order.  Several slots let new
// batches start while earlier ones are still running, so work that arrives while the device
// is busy overlaps with it.  A request's result is independent of the batch it lands in:
// every request of a batch runs on its own grid row with its system's own reduction order.
#include <string.h>

#include <atomic>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>
#include <vector>

#include "hsma_internal.h"

using namespace hsma;

namespace {

// A stream with a hardware queue of its own.  The runtime gives a process a few hardware queues
// (four by default) and maps further streams onto them, so a server stream could share a queue
// with a stream used before it (the caller's, a graph capture's, another server's), and a move
// batch would then wait behind whatever that queue holds; both were measured (move latencies ten
// times longer, or the two energy streams on one queue).  A stream created with a CU mask always
// gets a new queue; the mask here enables every CU.  Such streams synchronise with the legacy
// default stream.
hipError_t own_queue_stream(int device, hipStream_t *st) {
  int ncu = 0;
  hipError_t e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return e;
  if (ncu < 1 || ncu > 32 * 64) return hipErrorInvalidValue;
  uint32_t mask[64] = {};
  for (int i = 0; i < ncu; ++i) mask[i / 32] |= 1u << (i % 32);
  return hipExtStreamCreateWithCUMask(st, (uint32_t)((ncu + 31) / 32), mask);
}

struct Pending {
  hsma_request r;
  double t_submit;
};

struct DeltaSlot {
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  DeReq *h_reqs = nullptr;  // pinned
  DeReq *d_reqs = nullptr;
  double *d_dE = nullptr;
  double *h_dE = nullptr;   // pinned
  std::vector<Pending> reqs;
  double t_start = 0.0;
  bool busy = false;
};

// A full energy runs on a snapshot of its system's positions and charges, taken at its start
// (the copy ends at event snap); its system takes further requests once the copy is done,
// while the energy itself still runs.
struct EnergySlot {
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  hipEvent_t snap = nullptr;
  bool snapped = false;
  void *ws = nullptr;  // the energy's workspace, then the snapshot (x, y, z, q)
  size_t ws_bytes = 0;
  double *d_E = nullptr;
  double *h_E = nullptr;  // pinned
  Pending req;
  double t_start = 0.0;
  bool busy = false;
};

}  // namespace

struct hsma_server_s {
  int device = 0;
  hsma_server_opts opts;
  std::mutex mu;
  std::condition_variable wake;  // signalled on submit and stop: the idle scheduler sleeps on it
  std::deque<Pending> pending;
  std::vector<hsma_result> done;
  std::vector<hsma_system_s *> systems;  // by id; nullptr once removed
  std::vector<int> busy;                 // 1 while a move of the system is on the device
  std::vector<int> snapping;             // 1 while a full energy copies the system's state
  SysDev *d_sys = nullptr;               // descriptors by id
  size_t used = 0, budget = 0;
  std::vector<DeltaSlot> dslots;
  std::vector<EnergySlot> eslots;
  std::thread th;
  std::atomic<bool> stop{false};
  bool failed = false;  // a device error was seen: every later request completes with HSMA_EDEVICE
  std::chrono::steady_clock::time_point t0;
  // (system creation runs on the first move slot's stream: every stream beyond the device's
  // hardware queues shares one with another, and an energy stream sharing one with a move or
  // energy stream serialises behind it)
  // statistics
  uint64_t n_done = 0, n_batches = 0, n_batched_reqs = 0;
  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

void finish(hsma_server_s *S, const Pending &p, int status, double value, double t_start, double t_done) {
  hsma_result r;
  r.tag = p.r.tag;
  r.type = p.r.type;
  r.sys = p.r.sys;
  r.status = status;
  r.value = value;
  r.t_submit = p.t_submit;
  r.t_start = t_start;
  r.t_done = t_done;
  S->done.push_back(r);
  S->n_done++;
}

bool valid_request(hsma_server_s *S, const hsma_request &r) {
  if (r.sys < 0 || r.sys >= (int)S->systems.size() || !S->systems[r.sys]) return false;
  if (r.type == HSMA_REQ_ENERGY) return true;
  if (r.type != HSMA_REQ_DELTA) return false;
  const hsma_system_s *sys = S->systems[r.sys];
  if (r.k < 0 || r.k >= sys->n) return false;
  if (!(std::isfinite(r.x) && std::isfinite(r.y) && std::isfinite(r.z))) return false;
  return std::sqrt(r.x * r.x + r.y * r.y + r.z * r.z) < sys->h.pl.a;
}

// One pass of the scheduler; returns true when anything happened.  Called with S->mu held.
// Only hipErrorNotReady means that a slot's work is still running; any other error from the
// event completes the slot's requests with HSMA_EDEVICE and marks the server failed, after which
// every waiting and every new request completes at once with HSMA_EDEVICE.
// Workspace of an energy slot for a system: the full energy's workspace and the snapshot.
size_t energy_slot_bytes(const hsma_system_s *sys) {
  return system_workspace_bytes(sys) + (4 * sizeof(double) * (size_t)sys->n + 255) / 256 * 256;
}

bool schedule_once(hsma_server_s *S) {
  bool did = false;
  // completions
  for (DeltaSlot &d : S->dslots) {
    if (!d.busy) continue;
    const hipError_t q = hipEventQuery(d.ev);
    if (q == hipErrorNotReady) continue;
    const int status = q == hipSuccess ? HSMA_OK : HSMA_EDEVICE;
    if (status != HSMA_OK) S->failed = true;
    const double t = S->now();
    for (size_t i = 0; i < d.reqs.size(); ++i) {
      finish(S, d.reqs[i], status, status == HSMA_OK ? d.h_dE[i] : 0.0, d.t_start, t);
      S->busy[d.reqs[i].r.sys] = 0;
    }
    d.reqs.clear();
    d.busy = false;
    did = true;
  }
  for (EnergySlot &e : S->eslots) {
    if (!e.busy) continue;
    if (!e.snapped) {
      const hipError_t qs = hipEventQuery(e.snap);
      if (qs == hipSuccess) {  // the system may take its next requests
        e.snapped = true;
        S->snapping[e.req.r.sys] = 0;
        did = true;
      } else if (qs != hipErrorNotReady) {
        S->failed = true;
      }
    }
    const hipError_t q = hipEventQuery(e.ev);
    if (q == hipErrorNotReady) continue;
    const int status = q == hipSuccess ? HSMA_OK : HSMA_EDEVICE;
    if (status != HSMA_OK) S->failed = true;
    finish(S, e.req, status, status == HSMA_OK ? *e.h_E : 0.0, e.t_start, S->now());
    if (!e.snapped) S->snapping[e.req.r.sys] = 0;
    e.busy = false;
    did = true;
  }
  if (S->pending.empty()) return did;
  if (S->failed) {
    const double t = S->now();
    for (const Pending &p : S->pending) finish(S, p, HSMA_EDEVICE, 0.0, t, t);
    S->pending.clear();
    return true;
  }
  // A scan in arrival order.  blocked[b]: 2 once a move of system b is left waiting or taken
  // in this pass (nothing later of b may start); 1 once only full energies of b are left
  // waiting (later queries of b may start, nothing else).
  std::vector<char> blocked(S->systems.size(), 0);
  DeltaSlot *ds = nullptr;
  for (DeltaSlot &d : S->dslots)
    if (!d.busy) {
      ds = &d;
      break;
    }
  int64_t max_n = 0;
  int max_M = 0, max_P = 0, max_K = 0;
  auto free_eslot = [S]() {
    for (const EnergySlot &e : S->eslots)
      if (!e.busy) return true;
    return false;
  };
  bool eslot = free_eslot();
  for (auto it = S->pending.begin(); it != S->pending.end();) {
    // nothing more can start in this pass: the move batch is full (or no slot) and no energy slot is free
    if (!eslot && (!ds || (int)ds->reqs.size() >= S->opts.max_batch)) break;
    const hsma_request &r = it->r;
    const bool query = r.type == HSMA_REQ_DELTA && !r.commit;
    const int held = blocked[r.sys] > S->snapping[r.sys] ? blocked[r.sys] : S->snapping[r.sys];
    const int level = S->busy[r.sys] ? 2 : held;
    if (level == 2 || (level == 1 && !query)) {
      const char mine = r.type == HSMA_REQ_ENERGY ? 1 : 2;
      if (blocked[r.sys] < mine) blocked[r.sys] = mine;
      ++it;
      continue;
    }
    if (r.type == HSMA_REQ_ENERGY) {
      EnergySlot *es = nullptr;
      for (EnergySlot &e : S->eslots)
        if (!e.busy) {
          es = &e;
          break;
        }
      if (!es) {
        if (blocked[r.sys] < 1) blocked[r.sys] = 1;
        ++it;
        continue;
      }
      hsma_system_s *sys = S->systems[r.sys];
      const size_t need = energy_slot_bytes(sys);
      bool ok = true;
      if (es->ws_bytes < need) {
        (void)hipFree(es->ws);
        S->used -= es->ws_bytes;
        es->ws = nullptr;
        es->ws_bytes = 0;
        if (hipMalloc(&es->ws, need) == hipSuccess) {
          es->ws_bytes = need;
          S->used += need;
        } else {
          ok = false;
        }
      }
      const Pending p = *it;
      it = S->pending.erase(it);
      if (!ok) {
        finish(S, p, HSMA_ENOMEM, 0.0, S->now(), S->now());
        continue;
      }
      es->req = p;
      es->t_start = S->now();
      S->snapping[p.r.sys] = 1;  // (r referred to the erased element)
      if (blocked[p.r.sys] < 1) blocked[p.r.sys] = 1;
      // the snapshot: the system's x, y, z, q after its workspace
      const size_t wsb = system_workspace_bytes(sys), nb = sizeof(double) * (size_t)sys->n;
      double *snap = (double *)((char *)es->ws + wsb);
      const double *src[4] = {sys->h.x, sys->h.y, sys->h.z, sys->h.q};
      hsma_status rc = HSMA_OK;
      for (int c = 0; c < 4 && rc == HSMA_OK; ++c)
        if (nb && hipMemcpyAsync(snap + c * sys->n, src[c], nb, hipMemcpyDeviceToDevice, es->st) != hipSuccess)
          rc = HSMA_EDEVICE;
      if (rc == HSMA_OK && hipEventRecord(es->snap, es->st) != hipSuccess) rc = HSMA_EDEVICE;
      es->snapped = false;
      if (rc == HSMA_OK)
        rc = system_full_energy_at(sys, snap, snap + sys->n, snap + 2 * sys->n, snap + 3 * sys->n, es->d_E, es->ws,
                                   wsb, es->st);
      if (rc == HSMA_OK && hipMemcpyAsync(es->h_E, es->d_E, sizeof(double), hipMemcpyDeviceToHost, es->st) != hipSuccess)
        rc = HSMA_EDEVICE;
      if (rc == HSMA_OK && hipEventRecord(es->ev, es->st) != hipSuccess) rc = HSMA_EDEVICE;
      if (rc != HSMA_OK) {
        (void)hipStreamSynchronize(es->st);
        S->snapping[p.r.sys] = 0;
        finish(S, p, rc, 0.0, es->t_start, S->now());
        continue;
      }
      es->busy = true;
      eslot = free_eslot();
      did = true;
      continue;
    }
    // single-ion move
    if (!ds || (int)ds->reqs.size() >= S->opts.max_batch) {
      blocked[r.sys] = 2;
      ++it;
      continue;
    }
    const hsma_system_s *sys = S->systems[r.sys];
    DeReq &q = ds->h_reqs[ds->reqs.size()];
    q.sys = r.sys;
    q.commit = r.commit ? 1 : 0;
    q.k = r.k;
    q.x = r.x;
    q.y = r.y;
    q.z = r.z;
    q.dE = ds->d_dE + ds->reqs.size();
    ds->reqs.push_back(*it);
    if (sys->n > max_n) max_n = sys->n;
    if (sys->h.M > max_M) max_M = sys->h.M;
    if (sys->h.P > max_P) max_P = sys->h.P;
    if (sys->h.K > max_K) max_K = sys->h.K;
    S->busy[r.sys] = 1;
    blocked[r.sys] = 2;
    it = S->pending.erase(it);
  }
  if (ds && !ds->reqs.empty()) {
    const int n = (int)ds->reqs.size();
    ds->t_start = S->now();
    hsma_status rc = HSMA_OK;
    if (hipMemcpyAsync(ds->d_reqs, ds->h_reqs, sizeof(DeReq) * n, hipMemcpyHostToDevice, ds->st) != hipSuccess)
      rc = HSMA_EDEVICE;
    if (rc == HSMA_OK) rc = launch_delta(S->d_sys, ds->d_reqs, DeReq(), n, max_n, max_M, max_P, max_K, ds->st,
                                           S->opts.move_priority);
    if (rc == HSMA_OK && hipMemcpyAsync(ds->h_dE, ds->d_dE, sizeof(double) * n, hipMemcpyDeviceToHost, ds->st) !=
                             hipSuccess)
      rc = HSMA_EDEVICE;
    if (rc == HSMA_OK && hipEventRecord(ds->ev, ds->st) != hipSuccess) rc = HSMA_EDEVICE;
    if (rc != HSMA_OK) {
      (void)hipStreamSynchronize(ds->st);
      for (const Pending &p : ds->reqs) {
        S->busy[p.r.sys] = 0;
        finish(S, p, rc, 0.0, ds->t_start, S->now());
      }
      ds->reqs.clear();
    } else {
      ds->busy = true;
      S->n_batches++;
      S->n_batched_reqs += n;
    }
    did = true;
  }
  return did;
}

// The scheduler thread: while requests are pending or on the device it polls (yielding the CPU
// between passes, since timed sleeps are far coarser than a request); with nothing to do it
// sleeps until a submit or stop signals it.
void run_loop(hsma_server_s *S) {
  (void)hipSetDevice(S->device);
  while (!S->stop.load()) {
    std::unique_lock<std::mutex> lk(S->mu);
    const bool did = schedule_once(S);
    bool idle = S->pending.empty();
    if (idle)
      for (const DeltaSlot &d : S->dslots) idle = idle && !d.busy;
    if (idle)
      for (const EnergySlot &e : S->eslots) idle = idle && !e.busy;
    if (idle) {
      S->wake.wait_for(lk, std::chrono::milliseconds(100),
                       [S] { return S->stop.load() || !S->pending.empty(); });
      continue;
    }
    lk.unlock();
    if (!did) std::this_thread::yield();
  }
}

void server_free(hsma_server_s *S) {
  if (S->th.joinable()) {
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->stop.store(true);
    }
    S->wake.notify_all();
    S->th.join();
  }
  for (DeltaSlot &d : S->dslots) {
    if (d.st) (void)hipStreamSynchronize(d.st);
    (void)hipHostFree(d.h_reqs);
    (void)hipHostFree(d.h_dE);
    (void)hipFree(d.d_reqs);
    (void)hipFree(d.d_dE);
    if (d.ev) (void)hipEventDestroy(d.ev);
    if (d.st) (void)hipStreamDestroy(d.st);
  }
  for (EnergySlot &e : S->eslots) {
    if (e.st) (void)hipStreamSynchronize(e.st);
    (void)hipFree(e.ws);
    (void)hipFree(e.d_E);
    (void)hipHostFree(e.h_E);
    if (e.ev) (void)hipEventDestroy(e.ev);
    if (e.snap) (void)hipEventDestroy(e.snap);
    if (e.st) (void)hipStreamDestroy(e.st);
  }
  for (hsma_system_s *s : S->systems)
    if (s) hsma_system_destroy(s);
  (void)hipFree(S->d_sys);
  delete S;
}

// resident bytes of a system of N ions on a plan (the footprint hsma_system_create reports)
size_t footprint_of(hsma_plan_t pl, int64_t N) {
  const Geometry *g = pl->geo;
  const size_t nb = sizeof(double) * (size_t)N;
  const size_t nA = (size_t)((N + 255) / 256);
  return 4 * nb + sizeof(double) * (6 * (size_t)g->P + 2 * (size_t)g->M + 2 * (size_t)g->K + 1 + nA + g->P) +
         sizeof(SysDev);
}

}  // namespace

extern "C" hsma_server_opts hsma_server_opts_default(void) {
  hsma_server_opts o;
  o.memory_budget = 0;
  o.max_systems = 1024;
  o.max_batch = 256;
  o.delta_slots = 1;
  o.energy_slots = 2;
  o.energy_workgroups = 0;
  o.move_priority = 1;
  return o;
}

extern "C" hsma_status hsma_server_create(const hsma_server_opts *opts, hsma_server_t *out) {
  if (!out) return HSMA_EINVAL;
  *out = nullptr;
  hsma_server_opts o = opts ? *opts : hsma_server_opts_default();
  if (o.max_systems < 1 || o.max_batch < 1 || o.max_batch > 65535 || o.delta_slots < 1 || o.energy_slots < 1 ||
      (o.move_priority != 0 && o.move_priority != 1))
    return HSMA_EINVAL;
  hsma_server_s *S = new hsma_server_s();
  S->opts = o;
  S->t0 = std::chrono::steady_clock::now();
  hsma_status rc = HSMA_OK;
  if (hipGetDevice(&S->device) != hipSuccess) rc = HSMA_EDEVICE;
  size_t fre = 0, tot = 0;
  if (rc == HSMA_OK && hipMemGetInfo(&fre, &tot) != hipSuccess) rc = HSMA_EDEVICE;
  S->budget = o.memory_budget ? o.memory_budget : fre / 2;
  if (rc == HSMA_OK && o.energy_workgroups == 0) {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, S->device) != hipSuccess) rc = HSMA_EDEVICE;
    S->opts.energy_workgroups = ncu > 0 ? ncu : 1;
  }
  if (rc == HSMA_OK && hipMalloc(&S->d_sys, sizeof(SysDev) * o.max_systems) != hipSuccess) rc = HSMA_EDEVICE;
  S->dslots.resize(o.delta_slots);
  for (DeltaSlot &d : S->dslots) {
    if (rc != HSMA_OK) break;
    if (own_queue_stream(S->device, &d.st) != hipSuccess ||
        hipEventCreateWithFlags(&d.ev, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void **)&d.h_reqs, sizeof(DeReq) * o.max_batch, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&d.h_dE, sizeof(double) * o.max_batch, hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&d.d_reqs, sizeof(DeReq) * o.max_batch) != hipSuccess ||
        hipMalloc(&d.d_dE, sizeof(double) * o.max_batch) != hipSuccess)
      rc = HSMA_ENOMEM;
  }
  S->eslots.resize(o.energy_slots);
  for (EnergySlot &e : S->eslots) {
    if (rc != HSMA_OK) break;
    if (own_queue_stream(S->device, &e.st) != hipSuccess ||
        hipEventCreateWithFlags(&e.ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&e.snap, hipEventDisableTiming) != hipSuccess ||
        hipMalloc(&e.d_E, sizeof(double)) != hipSuccess ||
        hipHostMalloc((void **)&e.h_E, sizeof(double), hipHostMallocDefault) != hipSuccess)
      rc = HSMA_ENOMEM;
  }
  if (rc != HSMA_OK) {
    server_free(S);
    return rc;
  }
  S->th = std::thread(run_loop, S);
  *out = S;
  return HSMA_OK;
}

extern "C" hsma_status hsma_server_destroy(hsma_server_t S) {
  if (!S) return HSMA_EINVAL;
  server_free(S);
  return HSMA_OK;
}

extern "C" hsma_status hsma_server_add_system(hsma_server_t S, hsma_plan_t pl, int64_t N, const double *x,
                                              const double *y, const double *z, const double *q, int *id) {
  if (!S || !pl || !id || N < 1) return HSMA_EINVAL;
  const size_t fp = footprint_of(pl, N);
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if ((int)S->systems.size() >= S->opts.max_systems) {
      // reuse a removed id if any
      bool free_id = false;
      for (hsma_system_s *s : S->systems) free_id = free_id || !s;
      if (!free_id) return HSMA_EBUSY;
    }
    if (S->used + fp > S->budget) return HSMA_EBUSY;
    S->used += fp;  // reserved while the system is built
  }
  hsma_system_t sys = nullptr;
  hsma_status rc = hsma_system_create(pl, N, x, y, z, q, S->dslots[0].st, &sys);
  std::lock_guard<std::mutex> lk(S->mu);
  if (rc != HSMA_OK) {
    S->used -= fp;
    return rc;
  }
  S->used += sys->footprint;
  S->used -= fp;
  // the full-energy workspaces must grow to this system's size: that memory counts too
  const size_t need = energy_slot_bytes(sys);
  size_t grow = 0;
  for (const EnergySlot &e : S->eslots)
    if (e.ws_bytes < need) grow += need - e.ws_bytes;
  if (S->used + grow > S->budget) {
    S->used -= sys->footprint;
    hsma_system_destroy(sys);
    return HSMA_EBUSY;
  }
  int slot = -1;
  for (size_t i = 0; i < S->systems.size(); ++i)
    if (!S->systems[i]) {
      slot = (int)i;
      break;
    }
  if (slot < 0 && (int)S->systems.size() >= S->opts.max_systems) {
    // another add took the last id while this system was built outside the lock
    S->used -= sys->footprint;
    hsma_system_destroy(sys);
    return HSMA_EBUSY;
  }
  if (slot < 0) {
    slot = (int)S->systems.size();
    S->systems.push_back(nullptr);
    S->busy.push_back(0);
    S->snapping.push_back(0);
  }
  if (hipMemcpy(S->d_sys + slot, &sys->h, sizeof(SysDev), hipMemcpyHostToDevice) != hipSuccess) {
    S->used -= sys->footprint;
    hsma_system_destroy(sys);
    return HSMA_EDEVICE;
  }
  S->systems[slot] = sys;
  S->busy[slot] = 0;
  S->snapping[slot] = 0;
  sys->g64->tune.ewaves = S->opts.energy_workgroups > 0 ? S->opts.energy_workgroups : 0;
  // Full-energy workspaces grow here, at admission, rather than in the scheduler, where freeing
  // device memory would stall every request in flight (a slot busy now grows when next used).
  for (EnergySlot &e : S->eslots) {
    if (e.busy || e.ws_bytes >= need) continue;
    (void)hipFree(e.ws);
    S->used -= e.ws_bytes;
    e.ws = nullptr;
    e.ws_bytes = 0;
    if (hipMalloc(&e.ws, need) == hipSuccess) {
      e.ws_bytes = need;
      S->used += need;
    }
  }
  *id = slot;
  return HSMA_OK;
}

extern "C" hsma_status hsma_server_remove_system(hsma_server_t S, int id) {
  if (!S) return HSMA_EINVAL;
  for (;;) {
    {
      std::lock_guard<std::mutex> lk(S->mu);
      if (id < 0 || id >= (int)S->systems.size() || !S->systems[id]) return HSMA_EINVAL;
      bool waiting = S->busy[id] != 0 || S->snapping[id] != 0;
      for (const Pending &p : S->pending) waiting = waiting || p.r.sys == id;
      // a full energy past its snapshot still runs on the system's plan
      for (const EnergySlot &e : S->eslots) waiting = waiting || (e.busy && e.req.r.sys == id);
      if (!waiting) {
        hsma_system_s *sys = S->systems[id];
        S->systems[id] = nullptr;
        S->used -= sys->footprint;
        hsma_system_destroy(sys);
        return HSMA_OK;
      }
    }
    std::this_thread::sleep_for(std::chrono::microseconds(100));
  }
}

extern "C" hsma_status hsma_server_submit(hsma_server_t S, const hsma_request *reqs, int n) {
  if (!S || (n > 0 && !reqs) || n < 0) return HSMA_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  const double t = S->now();
  for (int i = 0; i < n; ++i) {
    Pending p;
    p.r = reqs[i];
    p.t_submit = t;
    if (!valid_request(S, reqs[i])) {
      finish(S, p, HSMA_EINVAL, 0.0, t, t);
      continue;
    }
    if (S->failed) {
      finish(S, p, HSMA_EDEVICE, 0.0, t, t);
      continue;
    }
    S->pending.push_back(p);
  }
  S->wake.notify_one();
  return HSMA_OK;
}

extern "C" int hsma_server_poll(hsma_server_t S, hsma_result *out, int max) {
  if (!S || !out || max <= 0) return 0;
  std::lock_guard<std::mutex> lk(S->mu);
  const int n = (int)(S->done.size() < (size_t)max ? S->done.size() : (size_t)max);
  for (int i = 0; i < n; ++i) out[i] = S->done[i];
  S->done.erase(S->done.begin(), S->done.begin() + n);
  return n;
}

extern "C" hsma_status hsma_server_stats(hsma_server_t S, hsma_server_info *info) {
  if (!S || !info) return HSMA_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  info->memory_used = S->used;
  info->memory_budget = S->budget;
  info->pending = (int64_t)S->pending.size();
  info->completed = S->n_done;
  info->batches = S->n_batches;
  info->batched_requests = S->n_batched_reqs;
  int live = 0;
  for (hsma_system_s *s : S->systems) live += s != nullptr;
  info->systems = live;
  info->now = S->now();
  return HSMA_OK;
}

// Open-loop load: request i is submitted at arrival[i] seconds after the call starts (a
// busy-waiting injector thread); returns when every request has a result, in out[i]
// (matched by position; tags are overwritten with the request index).  A request that has no
// result RUN_LOAD_GRACE seconds after the last arrival is reported with HSMA_EDEVICE and the call
// returns HSMA_EDEVICE, as it does when any request completed with HSMA_EDEVICE.
constexpr double RUN_LOAD_GRACE = 120.0;
extern "C" hsma_status hsma_server_run_load(hsma_server_t S, const hsma_request *reqs, const double *arrival, int n,
                                            hsma_result *out) {
  if (!S || n < 0 || (n > 0 && (!reqs || !arrival || !out))) return HSMA_EINVAL;
  for (int i = 0; i < n; ++i)
    if (!(arrival[i] >= 0.0 && arrival[i] < 1e6)) return HSMA_EINVAL;
  const double t_begin = S->now();
  double last = 0.0;
  for (int i = 0; i < n; ++i) last = arrival[i] > last ? arrival[i] : last;
  const double deadline = t_begin + last + RUN_LOAD_GRACE;
  std::vector<char> have(n > 0 ? n : 1, 0);
  std::thread inj([&]() {
    for (int i = 0; i < n; ++i) {
      const double due = t_begin + arrival[i];
      while (S->now() < due) {
        const double wait = due - S->now();
        if (wait > 2e-4) std::this_thread::sleep_for(std::chrono::microseconds(50));
      }
      hsma_request r = reqs[i];
      r.tag = (uint64_t)i;
      hsma_server_submit(S, &r, 1);
    }
  });
  int got = 0;
  bool timed_out = false, device_error = false;
  std::vector<hsma_result> buf(1024);
  while (got < n) {
    const int k = hsma_server_poll(S, buf.data(), (int)buf.size());
    for (int i = 0; i < k; ++i) {
      const uint64_t t = buf[i].tag;
      if (t < (uint64_t)n && !have[t]) {
        out[t] = buf[i];
        have[t] = 1;
        device_error = device_error || buf[i].status == HSMA_EDEVICE;
        ++got;
      }
    }
    if (k == 0) {
      if (S->now() > deadline) {
        timed_out = true;
        break;
      }
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  }
  inj.join();
  for (int i = 0; i < n; ++i) {  // times relative to the start of the load
    if (!have[i]) {
      out[i] = hsma_result();
      out[i].tag = (uint64_t)i;
      out[i].type = reqs[i].type;
      out[i].sys = reqs[i].sys;
      out[i].status = HSMA_EDEVICE;
      out[i].t_submit = out[i].t_start = out[i].t_done = S->now();
    }
    out[i].t_submit -= t_begin;
    out[i].t_start -= t_begin;
    out[i].t_done -= t_begin;
  }
  return timed_out || device_error ? HSMA_EDEVICE : HSMA_OK;
}
