// Launch settings of a group, and their choice by timing (hsma_group_autotune).
//
// The settings only change how the same sums are laid out over the device (which kernel, block
// size, item order, chunk length, persistent or one item per block, fit route), so a choice
// changes results only in the summation order.  The tuner times the caller's own call with HIP
// events on the caller's stream, one setting at a time (coordinate descent), and keeps the
// result per call shape in a process-wide cache.
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "hsma_internal.h"

namespace hsma {
namespace {

hsma_launch_settings settings_of(const hsma_group_s *g) {
  hsma_launch_settings s;
  s.persistent = g->tune.persistent;
  s.target_items = g->tune.target_items;
  s.symmetric = g->tune.symmetric;
  s.sym_order = g->tune.sym_order;
  s.fit = g->tune.fit;
  s.energy_block = g->tune.eblock;
  s.energy_workgroups = g->tune.ewaves;
  return s;
}

bool settings_valid(const hsma_launch_settings &s) {
  return (s.persistent == 0 || s.persistent == 1) && s.target_items >= 64 && s.target_items <= (1 << 22) &&
         s.symmetric >= 0 && s.symmetric <= 3 && s.sym_order >= 0 && s.sym_order <= 2 && s.fit >= 0 && s.fit <= 4 &&
         (s.energy_block == 0 || s.energy_block == 128 || s.energy_block == 256 || s.energy_block == 512) &&
         s.energy_workgroups >= 0 &&
         s.energy_workgroups <= (1 << 20);
}

void settings_put(hsma_group_s *g, const hsma_launch_settings &s) {
  g->tune.persistent = s.persistent;
  g->tune.target_items = s.target_items;
  g->tune.symmetric = s.symmetric;
  g->tune.sym_order = s.sym_order;
  g->tune.fit = s.fit;
  g->tune.eblock = s.energy_block;
  g->tune.ewaves = s.energy_workgroups;
}

std::mutex tune_mu;
std::map<std::string, hsma_launch_settings> tune_cache;

int bit_length(int64_t v) {
  int b = 0;
  for (; v > 0; v >>= 1) ++b;
  return b;
}

struct Call {
  hsma_group_s *g;
  int nsys;
  const int64_t *offsets;
  const int32_t *plan_of;
  int64_t total_n, max_n;
  const double *x, *y, *z, *q;
  double *phi, *E;
  void *ws;
  size_t ws_bytes;
  hipStream_t st;
};

// Mean time of one call (ms) over reps calls after one untimed call; < 0 when the call is
// refused with these settings (its workspace exceeds ws_bytes); HSMA_EDEVICE on HIP errors.
hsma_status time_call(const Call &c, hipEvent_t a, hipEvent_t b, int reps, double &ms) {
  const hsma_status rc = run_batched(c.g, c.nsys, c.offsets, c.plan_of, c.total_n, c.max_n, c.x, c.y, c.z, c.q, c.phi,
                                     c.E, c.ws, c.ws_bytes, c.st);
  if (rc == HSMA_EINVAL) {
    ms = -1.0;
    return HSMA_OK;
  }
  if (rc != HSMA_OK) return rc;
  HSMA_HIP(hipEventRecord(a, c.st));
  for (int r = 0; r < reps; ++r) {
    const hsma_status rr = run_batched(c.g, c.nsys, c.offsets, c.plan_of, c.total_n, c.max_n, c.x, c.y, c.z, c.q,
                                       c.phi, c.E, c.ws, c.ws_bytes, c.st);
    if (rr != HSMA_OK) return rr;
  }
  HSMA_HIP(hipEventRecord(b, c.st));
  HSMA_HIP(hipEventSynchronize(b));
  float t = 0.0f;
  HSMA_HIP(hipEventElapsedTime(&t, a, b));
  ms = (double)t / reps;
  return HSMA_OK;
}

using Field = int hsma_launch_settings::*;
using Dims = std::vector<std::pair<Field, std::vector<int>>>;

// The tuned dimensions, in the order they are tuned, with their candidate values.
Dims tune_dims(const hsma_group_s *g, bool pot, bool energy) {
  Dims d;
  if (pot) {
    d.push_back({&hsma_launch_settings::symmetric, {1, 0, 2, 3}});
    d.push_back({&hsma_launch_settings::sym_order, {0, 1, 2}});
    if (g->pair_prec != HSMA_PAIR_FP64) d.push_back({&hsma_launch_settings::fit, {0, 1, 2, 4}});
  }
  if (energy) {
    const int ncu = g->geo->ncu;
    d.push_back({&hsma_launch_settings::energy_block, {0, 128, 256, 512}});
    d.push_back({&hsma_launch_settings::energy_workgroups, {0, ncu, 2 * ncu, 4 * ncu}});
  }
  d.push_back({&hsma_launch_settings::persistent, {0, 1}});
  d.push_back({&hsma_launch_settings::target_items, {65536, 16384, 4096}});
  return d;
}

// The largest workspace over every combination of the candidate values (and s itself).
size_t max_workspace(hsma_group_s *g, const hsma_launch_settings &s, const Dims &d, size_t k, int nsys,
                     int64_t total_n, int64_t max_n) {
  if (k == d.size()) {
    const hsma_launch_settings keep = settings_of(g);
    settings_put(g, s);
    const size_t b = call_workspace_bytes(g, nsys, total_n, max_n, false);
    settings_put(g, keep);
    return b;
  }
  size_t m = max_workspace(g, s, d, k + 1, nsys, total_n, max_n);
  for (int v : d[k].second) {
    hsma_launch_settings c = s;
    c.*(d[k].first) = v;
    const size_t b = max_workspace(g, c, d, k + 1, nsys, total_n, max_n);
    m = b > m ? b : m;
  }
  return m;
}

}  // namespace
}  // namespace hsma

using namespace hsma;

extern "C" size_t hsma_group_autotune_workspace_bytes(hsma_group_t grp, int nsys, int64_t total_n, int64_t max_n) {
  if (!grp || nsys < 1 || total_n < 0 || max_n < 0 || max_n > total_n) return 0;
  return max_workspace(grp, settings_of(grp), tune_dims(grp, true, true), 0, nsys, total_n, max_n);
}

extern "C" hsma_status hsma_group_set_energy_launch(hsma_group_t grp, int block, int workgroups) {
  if (!grp || (block != 0 && block != 128 && block != 256 && block != 512) || workgroups < 0 ||
      workgroups > (1 << 20))
    return HSMA_EINVAL;
  grp->tune.eblock = block;
  grp->tune.ewaves = workgroups;
  return HSMA_OK;
}

extern "C" hsma_status hsma_group_get_settings(hsma_group_t grp, hsma_launch_settings *out) {
  if (!grp || !out) return HSMA_EINVAL;
  *out = settings_of(grp);
  return HSMA_OK;
}

extern "C" hsma_status hsma_group_apply_settings(hsma_group_t grp, const hsma_launch_settings *s) {
  if (!grp || !s || !settings_valid(*s)) return HSMA_EINVAL;
  settings_put(grp, *s);
  return HSMA_OK;
}

extern "C" hsma_status hsma_group_autotune(hsma_group_t grp, int nsys, const int64_t *offsets, const int32_t *plan_of,
                                           int64_t total_n, int64_t max_n, const double *x, const double *y,
                                           const double *z, const double *q, double *phi, double *E, void *ws,
                                           size_t ws_bytes, hipStream_t st, int flags, hsma_tune_result *out) {
  if (!grp || !out || (flags & ~HSMA_TUNE_FORCE) != 0) return HSMA_EINVAL;
  hipDeviceProp_t prop;
  HSMA_HIP(hipGetDeviceProperties(&prop, grp->device));
  const Geometry *geo = grp->geo;
  char key[512];
  std::snprintf(key, sizeof(key), "%s|cu%d|prec%d|dip%d|M%d|P%d|K%d|out%d|s%d|n%d|m%d", prop.gcnArchName, geo->ncu,
                grp->pair_prec, grp->dipole, geo->M, grp->P_ev, geo->K, (phi ? 1 : 0) + (E ? 2 : 0), bit_length(nsys),
                bit_length(total_n), bit_length(max_n));
  *out = hsma_tune_result{};
  if (!(flags & HSMA_TUNE_FORCE)) {
    std::lock_guard<std::mutex> lk(tune_mu);
    auto it = tune_cache.find(key);
    if (it != tune_cache.end()) {
      settings_put(grp, it->second);
      out->chosen = it->second;
      out->cached = 1;
      return HSMA_OK;
    }
  }
  const Call c{grp, nsys, offsets, plan_of, total_n, max_n, x, y, z, q, phi, E, ws, ws_bytes, st};
  hipEvent_t a = nullptr, b = nullptr;
  HSMA_HIP(hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return HSMA_EDEVICE;
  }
  const hsma_launch_settings start = settings_of(grp);
  hsma_launch_settings best = start;
  double best_ms = 0.0;
  hsma_status rc = time_call(c, a, b, 1, best_ms);  // also the first contact: sets the repetition count
  int reps = 2;
  if (rc == HSMA_OK && best_ms < 0.0) rc = HSMA_EINVAL;  // the call as the caller configured it is refused
  if (rc == HSMA_OK) {
    reps = best_ms > 0.0 ? (int)(20.0 / best_ms) : 10;  // about 20 ms of calls per candidate
    reps = reps < 2 ? 2 : (reps > 10 ? 10 : reps);
    rc = time_call(c, a, b, reps, best_ms);
  }
  out->ms_start = best_ms;
  if (rc == HSMA_OK) out->trials[0] = hsma_tune_trial{start, best_ms};
  const Dims dims = tune_dims(grp, phi != nullptr || E == nullptr, E != nullptr);
  int timed = 1;
  for (size_t d = 0; d < dims.size() && rc == HSMA_OK; ++d) {
    const Field f = dims[d].first;
    for (int v : dims[d].second) {
      if (best.*f == v) continue;
      hsma_launch_settings cand = best;
      cand.*f = v;
      settings_put(grp, cand);
      double ms = 0.0;
      rc = time_call(c, a, b, reps, ms);
      if (rc != HSMA_OK) break;
      if (timed < HSMA_TUNE_MAX_TRIALS) out->trials[timed] = hsma_tune_trial{cand, ms};
      ++timed;
      if (ms > 0.0 && ms < 0.98 * best_ms) {
        best = cand;
        best_ms = ms;
      }
    }
  }
  settings_put(grp, rc == HSMA_OK ? best : start);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc != HSMA_OK) return rc;
  out->chosen = best;
  out->ms_tuned = best_ms;
  out->timed = timed;
  std::lock_guard<std::mutex> lk(tune_mu);
  tune_cache[key] = best;
  return HSMA_OK;
}
