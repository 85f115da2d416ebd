// Internal declarations shared by the translation units of libhsma (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/hsma.h"

#define HSMA_PI 3.14159265358979323846

// Return HSMA_EDEVICE from the enclosing function when a HIP call fails.
#define HSMA_HIP(call)                                        \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) return HSMA_EDEVICE;                \
  } while (0)

namespace hsma {

// Dimensionless operators shared by every plan with the same discretisation:
// everything is expressed on the unit sphere and in units of the cavity radius.
struct Geometry {
  int p, K, P, M, F1, F2;
  double tau, rc_over_a;
  int device;
  double *unit_check;  // M x 3 unit vectors of the check points
  double *unit_nodes;  // P x 3 unit vectors of the Fibonacci nodes
  double *what;        // P Fibonacci weights on the unit sphere (sum 4 pi)
  double *pinv64;      // K x M: (Yc^T Yc)^{-1} Yc^T, Yc = real SH at the check points
  float *pinv32;       // same, FP32
  double *lhat64;      // P x K: what_s (1 + tau)^n Y_nm(y_s) / (4 pi)
  float *lhat32;       // same, FP32
  int *nidx;           // K: degree n of each coefficient index
  int refs;
};

// Scalars of one plan, passed to kernels by value.
struct Consts {
  double a, a2, eps1, gamma, sigma, dbar, Rtau, rc, c0;  // c0 = 1 / (4 pi eps1)
  double far;                                            // distance used for an image at infinity
  double rmin;                                           // below this radius an ion's image is at infinity
};

}  // namespace hsma

struct hsma_plan_s {
  double a, eps1, eps2, kappa;
  hsma_plan_opts opts;
  hsma::Geometry *geo;
  hsma::Consts c;
  double *fg;          // 2K: f_nm then g_nm (the per-plan diagonals of the fit operator)
  float4 *chk32;       // M check points at radius rc (w unused)
  double4 *chk64;
  float4 *nodes32;     // P surface nodes at radius R_tau (w unused)
  double4 *nodes64;
  int *flag;           // device-side domain flag
  int device;
  int prof_on;         // record HIP events around each stage
  void *prof;          // hsma::Profile
};

namespace hsma {

hsma_status geometry_acquire(int p, int P, int M, int F1, double tau, double rc_over_a, Geometry **out);
void geometry_release(Geometry *g);

// Workspace layout for one system of N ions (offsets in bytes from ws).
struct Workspace {
  size_t img, tgt, srcw, self, chk_part, uv, ab, qd, eval_part, phi, e_part, total;
  int chk_chunks, chk_chunk, eval_chunks, eval_chunk, e_blocks;
};
Workspace workspace_layout(const hsma_plan_s *plan, int64_t N);

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
hipEvent_t prof_begin(hsma_plan_s *plan, int stage, hipStream_t st);
void prof_end(hipEvent_t end, hipStream_t st);
void prof_free(hsma_plan_s *plan);

}  // namespace hsma
