// Internal declarations shared by the translation units of libhsma (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/hsma.h"

#define HSMA_PI 3.14159265358979323846

// Return HSMA_EDEVICE from the enclosing function when a HIP call fails.
#define HSMA_HIP(call)                         \
  do {                                         \
    hipError_t e_ = (call);                    \
    if (e_ != hipSuccess) return HSMA_EDEVICE; \
  } while (0)

namespace hsma {

// Dimensionless operators shared by every plan with the same discretisation:
// everything is expressed on the unit sphere and in units of the cavity radius.
struct Geometry {
  int p, K, P, M, F1, F2;
  double tau, rc_over_a;
  int device;
  int ncu;             // compute units of the device (persistent grid size)
  double *unit_check;  // M x 3 unit vectors of the check points
  double *unit_nodes;  // P x 3 unit vectors of the Fibonacci nodes
  double *what;        // P Fibonacci weights on the unit sphere (sum 4 pi)
  double *pinv64;      // K x M: (Yc^T Yc)^{-1} Yc^T, Yc = real SH at the check points
  float *pinv32;       // same, FP32
  double *lhat64;      // P x K: what_s (1 + tau)^n Y_nm(y_s) / (4 pi)
  float *lhat32;       // same, FP32
  // The two operators split into three BF16 terms x ~ b0 + b1 + b2 (b0 = bf16(x),
  // b1 = bf16(x - b0), b2 = bf16(x - b0 - b1)) for the split-BF16 MFMA fits: the b0 plane,
  // then b1, then b2, each row zero-padded to a multiple of 32 columns.
  uint16_t *pinv_bf;   // 3 x K x Mp, Mp = M rounded up to 32
  uint16_t *lhat_bf;   // 3 x P x Kp, Kp = K rounded up to 32
  int Mp, Kp;
  int *nidx;           // K: degree n of each coefficient index
  int refs;
};

// Per-plan scalars and pointers, stored on the device (one per plan of a group) and
// also kept on the host for kernel arguments.
struct PlanDev {
  double a, a2, c0;           // radius, radius^2, 1 / (4 pi eps1)
  double gamma, sigma, dbar;  // constants of eq. "Anuapp"
  double Rtau, rc;            // auxiliary-sphere and check-point radii
  double far, rmin;           // an ion with r < rmin has its image at infinity (distance `far`)
  const double *fg;           // 2K: f_nm then g_nm (the per-plan diagonals of the fit operator)
  const float4 *chk32;        // M check points at radius rc
  const double4 *chk64;
  const float4 *nodes32;      // P surface nodes at radius R_tau
  const double4 *nodes64;
};

// Device descriptor of one resident system (single-ion-move state).
struct SysDev {
  PlanDev pl;
  const double *pinv64, *lhat64;
  const int *nidx;
  int K, M, P;
  int64_t n;
  double *x, *y, *z, *q;
  double *s;      // 2P: Q' then D' (the strengths the evaluation kernel uses)
  double *w;      // 2P: sum_i q_i S(x_i)
  double *E;      // 1: current energy
  double *dc;     // 2M scratch: check-field change (u then v)
  double *ab;     // 2K scratch
  double *ds;     // 2P scratch
  double *dw;     // 2P scratch
  double *partA;  // ceil(n / 256) scratch
  double *partE;  // P scratch
};

// One single-ion-move request.
struct DeReq {
  int sys;      // index into the descriptor array
  int commit;   // apply the move after evaluating it
  int64_t k;
  double x, y, z;
  double *dE;   // [device] output, or nullptr
};

}  // namespace hsma

struct hsma_system_s {
  hsma_plan_t plan;
  hsma_group_s *g64;     // FP64 group over the plan (full evaluations)
  hsma::SysDev h;        // host copy of the descriptor
  hsma::SysDev *d;       // device copy
  int64_t n;
  void *ws;              // workspace of the initial full evaluation (freed after creation)
  size_t ws_bytes;
  size_t footprint;      // resident device bytes
  int device;
};

namespace hsma {
// Single-ion-move pipeline for nreq requests (reqs on the device, or `one` when nreq = 1 and
// reqs is null); max_* bound the systems the requests refer to.  Each system may have at
// most one request in a batch.
hsma_status launch_delta(const SysDev *systems, const DeReq *reqs, DeReq one, int nreq, int64_t max_n, int max_M,
                         int max_P, int max_K, hipStream_t st);
// Resident blocks per compute unit of the check and evaluation kernels for a pair precision.
hsma_status pair_occupancy(int pair_prec, int *occ_check, int *occ_eval);
hsma_status system_full_energy(hsma_system_s *sys, double *E, void *ws, size_t ws_bytes, hipStream_t st);
size_t system_workspace_bytes(const hsma_system_s *sys);
}  // namespace hsma

// Launch-shape parameters of the pair kernels (see hsma_group_tune).
struct hsma_tune_s {
  int persistent;    // 1: persistent blocks taking items from a device counter; 0: one item per block
  int target_items;  // items each pair kernel aims to create (sets the source-chunk sizes)
  int occ_check;     // resident blocks per compute unit of the check and evaluation kernels
  int occ_eval;      // (occupancy API, set when the group is built)
  int symmetric;     // symmetric Kelvin kernel: 0 never, 1 for large launches, 2 / 3 whenever it
                     // applies with ion blocks of 256 / 512
  int fit;           // fit apply in the FP32 pair modes: 0 automatic, 1 GEMV, 2 FP32 MFMA,
                     // 3 split-BF16x3 MFMA, 4 split-BF16x6 MFMA
};

struct hsma_group_s {
  hsma_tune_s tune;
  int nplans;
  hsma::Geometry *geo;   // shared by every plan of the group
  hsma::PlanDev *dev;    // nplans entries on the device
  int pair_prec;
  int device;
  int *flag;             // device-side domain flag
  float4 *nodes32;       // surface nodes of every plan (plan i at i * P), for the evaluation kernel
  double4 *nodes64;
  int prof_on;           // record HIP events around each stage
  void *prof;            // hsma::Profile
  int owned_by_plan;     // the internal one-plan group of a plan
};

struct hsma_plan_s {
  double a, eps1, eps2, kappa;
  hsma_plan_opts opts;
  hsma::Geometry *geo;
  hsma::PlanDev host;    // the same values as the device copy
  double *fg;            // 2K
  float4 *chk32;
  double4 *chk64;
  float4 *nodes32;
  double4 *nodes64;
  hsma_group_s *self;    // one-plan group used by the single-system entry points
  int device;
};

namespace hsma {

hsma_status geometry_acquire(int p, int P, int M, int F1, double tau, double rc_over_a, Geometry **out);
void geometry_release(Geometry *g);
hsma_status group_build(int nplans, const hsma_plan_t *plans, int owned_by_plan, hsma_group_s **out);
void group_free(hsma_group_s *g);

// Workspace layout of one batched call (offsets in bytes from the workspace base).
struct Layout {
  int nsys;
  int64_t total_n, max_n;
  int chc, che;                  // sources per item (check / evaluation), multiples of 128
  int sym_tb, sch;               // symmetric Kelvin kernel: ions per block and surface chunks (0: off)
  int64_t items_c, items_e, fin; // upper bounds of the item and finish-block counts
  int64_t parts_c, parts_e;      // upper bounds of the partial-sum slots
  size_t sched, item_sys_c, item_sys_e, fin_sys;
  size_t img, tgt, srcw, self, wk, rk, chk_part, uv, uv32, ab, h32, gemm2, qd, eval_part, phi, epart, E;
  size_t total;
  bool field;                    // potential and field (one-directional evaluation, 4 values per slot)
  size_t sfield;                 // own-image field per ion (double4), field layouts only
  bool lo;                       // FP32 lo parts of target and image coordinates (field, FP32 pairs)
  size_t tlo, ilo;
  bool mfma;                     // fit applied as MFMA GEMMs
  int bf_terms;                  // ... with products of BF16 splits of 2 (x3) or 3 (x6) terms; 0: FP32
};
Layout layout(const hsma_group_s *g, int nsys, int64_t total_n, int64_t max_n, bool field = false);

// Stage timing with HIP events recorded on the launch stream (off unless enabled).
enum Stage { ST_PACK = 0, ST_CHECK = 1, ST_FIT = 2, ST_EVAL = 3, ST_FINISH = 4, ST_COUNT = 5 };
struct ProfRec {
  int stage;
  hipEvent_t a, b;
};
struct Profile {
  std::mutex mu;
  ProfRec *recs = nullptr;
  int n = 0, cap = 0;
};
// Records the start event of a stage and returns its end event (to pass to prof_end),
// or nullptr when profiling is off.
hipEvent_t prof_begin(hsma_group_s *g, int stage, hipStream_t st);
void prof_end(hipEvent_t end, hipStream_t st);
void prof_free(hsma_group_s *g);

// The batched hot path; offsets is a device array of nsys + 1 entries, or nullptr for
// a single system of total_n ions.  E may be nullptr.
hsma_status run_batched(hsma_group_s *g, int nsys, const int64_t *offsets, const int32_t *plan_of, int64_t total_n,
                        int64_t max_n, const double *x, const double *y, const double *z, const double *q,
                        double *phi, double *E, void *ws, size_t ws_bytes, hipStream_t st, double *ex = nullptr,
                        double *ey = nullptr, double *ez = nullptr);

}  // namespace hsma
