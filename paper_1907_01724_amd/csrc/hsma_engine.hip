// Hot path of the HSMA reaction potential (Algorithm 1, steps 2-5) for gfx950, for one
// or many ion configurations ("systems") in one set of launches.
//
//   k_schedule      per-system item counts and prefix sums from the ion offsets
//   k_near_count,   (energy launches) each system's ions with r > 0.995 a placed after its others,
//   k_near_scan     so that the energy sums can take expanded distances on the rest
//   k_pack          item -> system maps; Kelvin images (Sec. 2.4: r_K = (a/r)^2 x, q_K), exact FP64
//                   own-image term, packed sources/targets in the pair precision, domain check
//   k_check         check fields u_k = sum_i q_i G0(c_k, x_i), v_k = sum_i q_i (r_i/a) G0(c_k, x_i)
//                   (Algorithm 1, step 2): items = (system, 64 check points, source chunk)
//   k_check_finish  fixed-order sum of the chunk partials
//   fit             alpha' = pinv u, beta' = pinv v; h = f . alpha' + g . beta';
//                   Q' = Lhat (n . h), D' = -Lhat h (steps 3-4: the fixed least-squares fit and
//                   Green's second identity on the nodes): k_fit_* GEMVs for a few systems,
//                   MFMA GEMMs (k_gemm_nt FP32, k_gemm64_nt FP64, k_gemm_bf split BF16) across many
//   k_kelvin_sym    Phi_i = sum_{j != i} q_K,j / |x_i - r_K,j| + sum_s [Q'_s + D'_s (d.y_s)/|d|^2]/|d|
//                   (eq. "phirffinall", step 5) over block pairs (I, J >= I), one reciprocal root
//                   for both directions of a pair (symmetric image distance), and surface items;
//                   k_kelvin_sym64 in FP64; k_eval the one-directional form for small launches
//   k_eval_field    the potential and the field at the ions
//   k_finish        Phi_i = own-image term + fixed-order sum of the partial slots (k_finish_field)
//   k_energy64      (energy launches) FP64 pair energies of the block pairs and surface items,
//                   one value per item; k_self_energy, k_energy_chunks, k_energy_items: E_b in a
//                   fixed order; k_energy: E_b = 1/2 sum_i q_i Phi_i from the potentials
//
// Pair kernels hold targets in registers and read sources at wave-uniform addresses (scalar
// loads); every sum is reduced in a fixed order, so a call is bitwise reproducible.
#include <math.h>
#include <stdlib.h>

#include "hsma_internal.h"

namespace hsma {
namespace {

constexpr int WAVES = 4;
constexpr int TPB = 64 * WAVES;  // threads per block in the pair kernels
constexpr int GRP = 64;          // targets per item
constexpr int TILE = 32;         // sources per FP32 partial sum before folding into FP64
constexpr int FINB = 256;        // ions per finish block
constexpr int SCHED_T = 1024;    // threads of the schedule kernel
constexpr int SYM_SH = 2;        // surface items per block and chunk (each takes 1/SYM_SH of the block's ions)
// Automatic fit route: the FP32 MFMA GEMMs from this many systems per call, the GEMVs below.
// The GEMMs have K / 64 row tiles (7 at p = 20) and take 0.25-0.4 ms at any batch up to
// about 1000 systems, while the GEMVs grow by 1.2-2.5 us per system (P = 1024-1600): the
// measured crossover lies between 128 and 256 systems.
constexpr int FIT_MFMA_MIN_SYS = 192;
constexpr int64_t SYM_TAIL_ROUNDS = 4;  // launches of at most this many rounds of resident waves
                                        // of block pairs put the surface items last
constexpr int64_t SYM_MAX_BYTES = (int64_t)16 << 30;  // partial-slot bound above which the symmetric
                                                       // Kelvin kernel is not used

template <int MODE>
struct PT {
  using T = float;
  using T2 = float2;
  using T4 = float4;
};
template <>
struct PT<HSMA_PAIR_FP64> {
  using T = double;
  using T2 = double2;
  using T4 = double4;
};

__device__ __forceinline__ float rinv(float r2) { return __builtin_amdgcn_rsqf(r2); }

// 1/sqrt(r2) in FP64: the hardware FP64 estimate (v_rsq_f64, relative error below 6e-8,
// measured) refined by one Newton step y <- y + y (1 - r2 y^2) / 2 (relative error ~4e-15).
__device__ __forceinline__ double rinv(double r2) {
  const double y = __builtin_amdgcn_rsq(r2);
  const double t = r2 * y;
  const double e = fma(-t, y, 1.0);
  return fma(y * 0.5, e, y);
}

// Twice 1/sqrt(r2) in FP64: y (3 - r2 y^2) from the hardware estimate y, the same Newton step
// as rinv with its factor 1/2 left to the caller (one instruction fewer per pair).
__device__ __forceinline__ double rinv2(double r2) {
  const double y = __builtin_amdgcn_rsq(r2);
  return y * fma(-(r2 * y), y, 3.0);
}

template <typename T4>
__device__ __forceinline__ T4 make4(double x, double y, double z, double w);
template <>
__device__ __forceinline__ float4 make4<float4>(double x, double y, double z, double w) {
  return make_float4((float)x, (float)y, (float)z, (float)w);
}
template <>
__device__ __forceinline__ double4 make4<double4>(double x, double y, double z, double w) {
  return make_double4(x, y, z, w);
}

template <int MODE>
__device__ __forceinline__ const typename PT<MODE>::T4 *chk_of(const PlanDev &p) {
  if constexpr (MODE == HSMA_PAIR_FP64) return p.chk64; else return p.chk32;
}
template <int MODE>
inline const typename PT<MODE>::T4 *group_nodes(const hsma_group_s *g) {
  if constexpr (MODE == HSMA_PAIR_FP64)
    return g->nodes64;
  else
    return g->nodes32;
}

__device__ __forceinline__ int64_t cdiv64(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------------
// Schedule.  sched (int64) holds, each with nsys + 1 entries:
//   [0] ion offsets  [1] check-item prefix  [2] eval-item prefix  [3] finish-block prefix
//   [4] check partial-slot prefix  [5] eval partial-slot prefix
//   [6] surface-item prefix of the symmetric kernel.  Its items come in one of two orders: in
//       a launch of few block pairs (one round of the chip's resident waves or less), every
//       system's block pairs, then every system's surface items, so that the shorter surface
//       items fill the end of the launch; otherwise each system's block pairs and then its
//       surface items, so that a system's targets are read while they are still in L2.
//       Either way system b's pairs are items [2][b] .. [6][b] - 1 when interleaved, or start
//       at [2][b] otherwise, and its surface items start at [6][b].
//   [7] prefix of the energy-sum chunks (energy-only launches: EC consecutive item energies of
//       one system, its block pairs first, then its surface items).
// followed by 32 words: [2] schedule valid, [3] launch kind: 1 for the energy-only launch, else 0,
// plus 16 x the pair precision (read back by hsma_debug_intermediates); the persistent kernels'
// item counters, one per die: [8..15] the energy kernel, [16..23] the check sums, [24..31] the
// evaluation kernels.
// ---------------------------------------------------------------------------------
constexpr int64_t EC = 4096;  // item energies per chunk of the energy reduction
// Energy pairs with an ion within r <= NEAR_R a take the expanded form of the squared image
// distance (see energy_item), and so do check sums over such sources (check_range_expanded);
// pairs of two ions nearer the interface, and check sums over them, take the exact form.
constexpr double NEAR_R = 0.995;
// Surface pairs of the energy launch take the expanded squared distance when every node lies on
// the sphere R_tau >= SURF_EXPANDED a (see energy_item).
constexpr double SURF_EXPANDED = 1.05;
constexpr int64_t ETAIL_ROUNDS = 4;  // energy launches: blocks of 128 below this many rounds of wave slots
// One source of the energy launch's check sums in the normalised form (see check_range_expanded):
// w = (r/a)^2 + (rc/a)^2, the position scaled by -2/(a w), and the weights of u and v over sqrt(w).
// One record, so that a run of sources is one stretch of scalar loads.
struct CheckSrc {
  double x, y, z, wu, wv;
};
constexpr int CTR_WORDS = 32, CTR_ENERGY = 8, CTR_CHECK = 16, CTR_EVAL = 24;
struct Sched {
  int64_t *off, *ic, *ie, *fb, *pc, *pe, *is, *ec, *ctr;
  __host__ __device__ Sched(int64_t *base, int nsys) {
    const int64_t s = nsys + 1;
    off = base;
    ic = base + s;
    ie = base + 2 * s;
    fb = base + 3 * s;
    pc = base + 4 * s;
    pe = base + 5 * s;
    is = base + 6 * s;
    ec = base + 7 * s;
    ctr = base + 8 * s;
  }
};

// Bounds the host sized the workspace with; the schedule refuses work beyond them.
struct Bounds {
  int64_t total_n, max_n, items_c, items_e, fin, parts_c, parts_e, echunks;
  int nplans;
};

// Super-tiles of the energy kernel's block pairs: a system of B >= 64 blocks numbers its pairs by
// tiles of ST x ST blocks (the triangle of tiles row by row, a tile's pairs row by row, ST^2
// item numbers per tile, those outside the triangle or beyond B left empty), so that the pairs
// of one tile, 2 ST blocks of data, are neighbours in the item order; smaller systems number the
// triangle of blocks row by row (ST = 1).
constexpr int ST = 16;
__host__ __device__ __forceinline__ int64_t super_of(int64_t B) { return B >= 64 ? ST : 1; }

// Evaluation items of a system: one-directional (items), or for the symmetric kernels its block
// pairs I <= J (items; numbered in super-tiles when tiles is set) and its surface items (surf:
// SYM_SH per block and surface chunk).
__device__ __forceinline__ void eval_counts(int64_t n, int P, int che, int sym_tb, int sch, int64_t &items,
                                            int64_t &surf, int64_t &parts, bool tiles = false) {
  surf = 0;
  if (n <= 0) {
    items = parts = 0;
  } else if (sym_tb > 0) {
    const int64_t B = cdiv64(n, sym_tb);
    const int64_t S = tiles ? super_of(B) : 1, NB = cdiv64(B, S);
    items = NB * (NB + 1) / 2 * S * S;
    surf = B * sch * SYM_SH;
    parts = n * (B + sch);
  } else {
    items = cdiv64(n, GRP) * cdiv64(n + P, che);
    parts = items * GRP;
  }
}

__global__ __launch_bounds__(SCHED_T) void k_schedule(int nsys, const int64_t *__restrict__ offsets,
                                                      const int32_t *__restrict__ plan_of, Bounds bd, int M, int P,
                                                      int chc, int che, int sym_tb, int sch, int64_t sym_tail,
                                                      int kind,
                                                      int64_t *__restrict__ base, int *__restrict__ flag) {
  Sched S(base, nsys);
  __shared__ int64_t sc[7][SCHED_T];
  const int t = threadIdx.x, nt = blockDim.x;  // nt <= SCHED_T, a multiple of 64
  const int seg = (nsys + nt - 1) / nt;
  const int b0 = t * seg, b1 = min(nsys, b0 + seg);
  const int64_t Gc = cdiv64(M, GRP);
  const int64_t n_single = bd.total_n;
  // the device offsets and plan indices must agree with what the host sized the work by
  int bad = 0;
  for (int b = b0; b < b1; ++b) {
    const int64_t lo = offsets ? offsets[b] : 0, hi = offsets ? offsets[b + 1] : n_single;
    if (lo < 0 || hi < lo || hi > bd.total_n || hi - lo > bd.max_n) bad = 1;
    if (b == 0 && lo != 0) bad = 1;
    if (b == nsys - 1 && hi != bd.total_n) bad = 1;
    if (plan_of && (plan_of[b] < 0 || plan_of[b] >= bd.nplans)) bad = 1;
  }
  bad = __syncthreads_or(bad);
  int64_t acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int b = b0; b < b1 && !bad; ++b) {
    const int64_t lo = offsets ? offsets[b] : 0, hi = offsets ? offsets[b + 1] : n_single;
    const int64_t n = hi - lo;
    const int64_t chunks_c = n > 0 ? cdiv64(n, chc) : 0;
    int64_t items_e, surf_e, parts_e;
    eval_counts(n, P, che, sym_tb, sch, items_e, surf_e, parts_e, (kind & 15) == 1);
    acc[0] += Gc * chunks_c;
    acc[1] += items_e;
    acc[2] += cdiv64(n, FINB);
    acc[3] += Gc * chunks_c * GRP;
    acc[4] += parts_e;
    acc[5] += surf_e;
    acc[6] += sym_tb > 0 ? cdiv64(items_e, EC) + cdiv64(surf_e, EC) : 0;
  }
  for (int k = 0; k < 7; ++k) sc[k][t] = acc[k];
  __syncthreads();
  // inclusive Hillis-Steele scan over the thread totals
  for (int o = 1; o < nt; o <<= 1) {
    int64_t v[7];
    for (int k = 0; k < 7; ++k) v[k] = t >= o ? sc[k][t - o] : 0;
    __syncthreads();
    for (int k = 0; k < 7; ++k) sc[k][t] += v[k];
    __syncthreads();
  }
  int64_t run[7];
  for (int k = 0; k < 7; ++k) run[k] = sc[k][t] - acc[k];  // exclusive start of this segment
  // surface items last when the block pairs of the launch are few (sc[1] holds only pairs)
  const bool surf_last = sc[1][nt - 1] <= sym_tail;
  if (surf_last) run[5] += sc[1][nt - 1];
  for (int b = b0; b < b1 && !bad; ++b) {
    const int64_t lo = offsets ? offsets[b] : 0, hi = offsets ? offsets[b + 1] : n_single;
    const int64_t n = hi - lo;
    const int64_t chunks_c = n > 0 ? cdiv64(n, chc) : 0;
    int64_t items_e, surf_e, parts_e;
    eval_counts(n, P, che, sym_tb, sch, items_e, surf_e, parts_e, (kind & 15) == 1);
    S.off[b] = lo;
    S.ic[b] = run[0];
    S.ie[b] = surf_last ? run[1] : run[1] + run[5];
    S.fb[b] = run[2];
    S.pc[b] = run[3];
    S.pe[b] = run[4];
    S.is[b] = surf_last ? run[5] : S.ie[b] + items_e;
    S.ec[b] = run[6];
    run[0] += Gc * chunks_c;
    run[1] += items_e;
    run[2] += cdiv64(n, FINB);
    run[3] += Gc * chunks_c * GRP;
    run[4] += parts_e;
    run[5] += surf_e;
    run[6] += sym_tb > 0 ? cdiv64(items_e, EC) + cdiv64(surf_e, EC) : 0;
  }
  if (t == nt - 1) {
    S.off[nsys] = offsets ? offsets[nsys] : n_single;
    S.ic[nsys] = sc[0][t];
    S.ie[nsys] = surf_last ? sc[1][t] : sc[1][t] + sc[5][t];
    S.fb[nsys] = sc[2][t];
    S.pc[nsys] = sc[3][t];
    S.pe[nsys] = sc[4][t];
    S.is[nsys] = sc[1][t] + sc[5][t];
    S.ec[nsys] = sc[6][t];
    for (int k = 0; k < CTR_WORDS; ++k) S.ctr[k] = 0;
    S.ctr[3] = kind;
    const bool fits = sc[0][t] <= bd.items_c && sc[1][t] + sc[5][t] <= bd.items_e && sc[2][t] <= bd.fin &&
                      sc[3][t] <= bd.parts_c && sc[4][t] <= bd.parts_e && sc[6][t] <= bd.echunks;
    const bool ok = !bad && fits;
    S.ctr[2] = ok ? 1 : 0;  // every later kernel of the call does nothing unless set
    if (!ok) atomicOr(flag, 2);
  }
}

__device__ __forceinline__ bool sched_ok(const Sched &S) { return S.ctr[2] != 0; }

// The system an item belongs to: the last b with pre[b] <= i in a prefix array of nsys + 1
// entries (systems without items share their prefix value with the next one).
__device__ __forceinline__ int system_of(const int64_t *__restrict__ pre, int nsys, int64_t i) {
  int lo = 0, hi = nsys;  // pre[lo] <= i < pre[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= i)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// item -> system maps of the check, evaluation and finish items, grid-stride over all threads
__device__ __forceinline__ void fill_maps(const Sched &S, int nsys, int *__restrict__ sys_c, int *__restrict__ sys_e,
                                          int *__restrict__ sys_f) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = t0; i < S.ic[nsys]; i += stride) sys_c[i] = system_of(S.ic, nsys, i);
  for (int64_t i = t0; i < S.ie[nsys]; i += stride) sys_e[i] = system_of(S.ie, nsys, i);
  for (int64_t i = S.ie[nsys] + t0; i < S.is[nsys]; i += stride) sys_e[i] = system_of(S.is, nsys, i);
  for (int64_t i = t0; i < S.fb[nsys]; i += stride) sys_f[i] = system_of(S.fb, nsys, i);
}

// ---------------------------------------------------------------------------------
// Energy launches place each system's ions with r > NEAR_R a after its other ions, keeping
// the order within each part, so that the energy kernel's ion blocks below the boundary
// hold no ion near the interface (see energy_item).  Per finish block: the count of such ions
// (k_near_count), then per system the start of each block's part of either kind (k_near_scan),
// then each ion's packed position (partition_rank, in k_pack).
// ---------------------------------------------------------------------------------
__device__ __forceinline__ bool near_interface(double x, double y, double z, double a) {
  return x * x + y * y + z * z > (NEAR_R * a) * (NEAR_R * a);  // false for non-finite input
}

__global__ __launch_bounds__(FINB) void k_near_count(int nsys, const int64_t *__restrict__ base,
                                                     const PlanDev *__restrict__ plans,
                                                     const int32_t *__restrict__ plan_of, const double *__restrict__ x,
                                                     const double *__restrict__ y, const double *__restrict__ z,
                                                     int *__restrict__ cnt) {
  Sched S(const_cast<int64_t *>(base), nsys);
  if (!sched_ok(S)) return;
  const int64_t f = blockIdx.x;
  if (f >= S.fb[nsys]) return;  // uniform across the block
  const int b = system_of(S.fb, nsys, f);
  const int64_t lo = S.off[b], n = S.off[b + 1] - lo, il = (f - S.fb[b]) * FINB + threadIdx.x;
  const double a = plans[plan_of ? plan_of[b] : 0].a;
  const bool nr = il < n && near_interface(x[lo + il], y[lo + il], z[lo + il], a);
  const int c = __syncthreads_count(nr);
  if (threadIdx.x == 0) cnt[f] = c;
}

// One block per system: its ions far from the interface first, then the others, each part in
// the order of the finish blocks; block-wide scans over the system's finish blocks, 256 at a time.
__global__ __launch_bounds__(256) void k_near_scan(int nsys, const int64_t *__restrict__ base,
                                                   const int *__restrict__ cnt, int64_t *__restrict__ farst,
                                                   int64_t *__restrict__ nearst, int64_t *__restrict__ nfar) {
  Sched S(const_cast<int64_t *>(base), nsys);
  __shared__ int64_t sn[256], sf[256];
  if (!sched_ok(S)) return;
  const int b = blockIdx.x, t = threadIdx.x;
  const int64_t n = S.off[b + 1] - S.off[b], f0 = S.fb[b], f1 = S.fb[b + 1];
  int64_t tot = 0;
  for (int64_t f = f0 + t; f < f1; f += 256) tot += cnt[f];
  sn[t] = tot;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) sn[t] += sn[t + o];
    __syncthreads();
  }
  const int64_t nf = n - sn[0];
  if (t == 0) nfar[b] = nf;
  __syncthreads();
  int64_t cf = 0, cn = nf;  // starts of the next chunk's far and near parts
  for (int64_t c0 = f0; c0 < f1; c0 += 256) {
    const int64_t f = c0 + t;
    const int64_t m = f < f1 ? ((n - (f - f0) * FINB) < FINB ? n - (f - f0) * FINB : FINB) : 0;  // ions of block f
    const int64_t vn = f < f1 ? cnt[f] : 0, vf = m - vn;
    sn[t] = vn;
    sf[t] = vf;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {  // inclusive scans
      const int64_t an = t >= o ? sn[t - o] : 0, af = t >= o ? sf[t - o] : 0;
      __syncthreads();
      sn[t] += an;
      sf[t] += af;
      __syncthreads();
    }
    if (f < f1) {
      farst[f] = cf + sf[t] - vf;
      nearst[f] = cn + sn[t] - vn;
    }
    cf += sf[255];
    cn += sn[255];
    __syncthreads();
  }
}

// The packed position within its system of an ion of finish block f (all threads of the block
// take part; the valid ions are the block's first threads): its part's start plus the ions of
// the same kind before it in the block.
__device__ __forceinline__ int64_t partition_rank(bool nr, int64_t far0, int64_t near0) {
  __shared__ int wn[FINB / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const unsigned long long bal = __ballot(nr);
  if (lane == 0) wn[wv] = __popcll(bal);
  __syncthreads();
  int below = 0;
  for (int k = 0; k < wv; ++k) below += wn[k];
  below += __popcll(bal & ((1ull << lane) - 1ull));
  return nr ? near0 + below : far0 + ((int)threadIdx.x - below);
}

// ---------------------------------------------------------------------------------
// Kelvin images and packing: one finish block (256 ions of one system) per block.
// ---------------------------------------------------------------------------------
// Also fills the item -> system maps the later kernels of the call read.
template <int MODE>
__global__ __launch_bounds__(256) void k_pack(int nsys, const int64_t *__restrict__ base, int *__restrict__ sys_c,
                                              int *__restrict__ sys_e, int *__restrict__ sys_f,
                                              const PlanDev *__restrict__ plans, const int32_t *__restrict__ plan_of,
                                              const double *__restrict__ x, const double *__restrict__ y,
                                              const double *__restrict__ z, const double *__restrict__ q,
                                              typename PT<MODE>::T4 *__restrict__ img,
                                              typename PT<MODE>::T4 *__restrict__ tgt,
                                              typename PT<MODE>::T *__restrict__ srcw, double *__restrict__ self,
                                              typename PT<MODE>::T *__restrict__ wk, double *__restrict__ rk,
                                              double *__restrict__ qr, double4 *__restrict__ emx,
                                              double2 *__restrict__ ew, CheckSrc *__restrict__ csrc,
                                              const int64_t *__restrict__ farst,
                                              const int64_t *__restrict__ nearst, double *__restrict__ qpk,
                                              double4 *__restrict__ sfield, float4 *__restrict__ tlo,
                                              float4 *__restrict__ ilo, int *__restrict__ flag) {
  using T4 = typename PT<MODE>::T4;
  using T = typename PT<MODE>::T;
  Sched S(const_cast<int64_t *>(base), nsys);
  if (!sched_ok(S)) return;
  fill_maps(S, nsys, sys_c, sys_e, sys_f);
  const int64_t f = blockIdx.x;
  if (f >= S.fb[nsys]) return;  // uniform across the block
  const int b = system_of(S.fb, nsys, f);
  const int64_t il = (f - S.fb[b]) * FINB + threadIdx.x;
  const int64_t lo = S.off[b], n = S.off[b + 1] - lo;
  const bool in = il < n;
  const int64_t i = lo + (in ? il : 0);
  const PlanDev c = plans[plan_of ? plan_of[b] : 0];
  const double xi = x[i], yi = y[i], zi = z[i], qi = q[i];
  // packed position: the ion's own, or after its system's far ions when it lies near the interface
  const int64_t d = farst ? lo + partition_rank(in && near_interface(xi, yi, zi, c.a), farst[f], nearst[f]) : i;
  if (!in) return;
  if (qpk) qpk[d] = qi;
  const double r2 = xi * xi + yi * yi + zi * zi;
  const double r = sqrt(r2);
  const bool ok = isfinite(xi) && isfinite(yi) && isfinite(zi) && isfinite(qi) && r < c.a;
  if (!ok) {
    atomicOr(flag, 1);
    img[d] = make4<T4>(0.0, 0.0, 2.0 * c.far, 0.0);
    tgt[d] = make4<T4>(0.0, 0.0, 0.0, 0.0);
    srcw[d] = (T)0;
    self[d] = 0.0;
    if (wk) {
      wk[d] = (T)0;
      rk[d] = 0.0;
    }
    if (qr) qr[d] = 0.0;
    if (emx) {
      emx[d] = make_double4(0.0, 0.0, 0.0, 0.0);
      ew[d] = make_double2(0.0, 0.0);
      csrc[d] = CheckSrc{0.0, 0.0, 0.0, 0.0, 0.0};  // a unit distance, zero weights
    }
    if (sfield) sfield[d] = make_double4(0.0, 0.0, 0.0, 0.0);
    if (tlo) {
      tlo[d] = make_float4(0.f, 0.f, 0.f, 0.f);
      ilo[d] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    return;
  }
  const double qp = qi * c.c0;  // q / (4 pi eps1)
  double kx, ky, kz, qk, reff;
  if (r >= c.rmin) {
    reff = r;
    const double fk = c.a2 / r2;  // r_K = (a/r)^2 x
    kx = fk * xi;
    ky = fk * yi;
    kz = fk * zi;
    const double rK = c.a2 / r;
    qk = qp / c.a * (c.gamma * rK + c.dbar * (c.Rtau - rK) * 0.5);
  } else {
    // image at infinity: q_K / |x - r_K| -> q (gamma - dbar/2) / a for every target;
    // represented by a point at distance `far` with the matching strength
    const double ux = r > 0.0 ? xi / r : 0.0, uy = r > 0.0 ? yi / r : 0.0, uz = r > 0.0 ? zi / r : 1.0;
    kx = c.far * ux;
    ky = c.far * uy;
    kz = c.far * uz;
    qk = qp * (c.gamma - 0.5 * c.dbar) * c.far / c.a;
    reff = c.a2 / c.far;  // the radius whose Kelvin point is the stand-in at distance `far`
  }
  // own image: q_K / (4 pi eps1 |x - r_K|) with |x - r_K| = (a^2 - r^2) / r, written so that it
  // stays regular at r = 0 and keeps FP64 accuracy as r -> a
  const double sp = qp / c.a * (c.gamma * c.a2 + 0.5 * c.dbar * (c.Rtau * r - c.a2)) / ((c.a - r) * (c.a + r));
  self[d] = sp;
  if (sfield) {
    // its field: q'_K (x - r_K) / |x - r_K|^3 with x - r_K = -x (a^2 - r^2) / r^2, i.e.
    // -x times the own-image potential over (a^2 - r^2); zero at the centre
    const double e = -sp / ((c.a - r) * (c.a + r));
    sfield[d] = make_double4(e * xi, e * yi, e * zi, 0.0);
  }
  img[d] = make4<T4>(kx, ky, kz, qk);
  tgt[d] = make4<T4>(xi, yi, zi, qp);
  if (tlo) {  // what FP32 rounding left of each coordinate, so that pair differences keep ~2^-48 a
    tlo[d] = make_float4((float)(xi - (double)(float)xi), (float)(yi - (double)(float)yi),
                         (float)(zi - (double)(float)zi), 0.f);
    ilo[d] = make_float4((float)(kx - (double)(float)kx), (float)(ky - (double)(float)ky),
                         (float)(kz - (double)(float)kz), 0.f);
  }
  srcw[d] = (T)(qp * r / c.a);
  if (wk) {
    wk[d] = (T)(qk * reff);  // c0 q_K r: the ion's image strength times its radius
    rk[d] = 1.0 / reff;
  }
  if (qr) qr[d] = qi / reff;  // the charge over the radius (energy sums)
  if (emx) {
    // The expanded pair form of the energy kernel (see energy_item): the position whose Kelvin
    // point is the image (x itself, or the stand-in's) scaled by -2/a, and (r/a)^2; the weights
    // c0 q_K r / a^2 and q / a^2 of the two pair sums.
    const double ex = r >= c.rmin ? xi : kx * reff * reff / c.a2, ey = r >= c.rmin ? yi : ky * reff * reff / c.a2,
                 ez = r >= c.rmin ? zi : kz * reff * reff / c.a2;
    const double u = (reff / c.a) * (reff / c.a);
    emx[d] = make_double4(-2.0 * ex / c.a, -2.0 * ey / c.a, -2.0 * ez / c.a, u);
    ew[d] = make_double2(qk * reff / c.a2, qi / c.a2);
    // the normalised form of the check sums (see check_range_expanded), from the ion itself; the
    // weights of u and v as in tgt and srcw
    const double w = r2 / c.a2 + (c.rc / c.a) * (c.rc / c.a), sc = -2.0 / (c.a * w), sw = 1.0 / sqrt(w);
    csrc[d] = CheckSrc{xi * sc, yi * sc, zi * sc, qp * sw, qp * r / c.a * sw};
  }
}

// The device's accelerator dies: gfx950 (MI355X) has 8, each with its own L2, and places
// workgroup w on die w % NXCD.  xcd_item deals the item numbers out in runs of XQ workgroups (one
// super-tile's ST^2 items): die x takes runs x, x + NXCD, x + 2 NXCD, ..., so the pairs of a tile
// run on one die and share its L2, and the dies share the work evenly.  The grid must be a multiple
// of NXCD XQ workgroups.  Only locality depends on the die count: the map is a bijection of
// [0, WAVES grid) whatever it is.
constexpr int NXCD = 8;
constexpr int XQ = ST * ST / WAVES;
__device__ __forceinline__ int64_t xcd_item(int w) {
  const int64_t x = blockIdx.x % NXCD, k = blockIdx.x / NXCD;
  const int64_t run = (k / XQ) * NXCD + x;
  return (run * XQ + k % XQ) * WAVES + w;
}

// Persistent form: die x's items are its runs' items in order, t = 0, 1, ... (run t / (XQ WAVES),
// offset t % (XQ WAVES)); its waves take them EG at a time from the die's own counter, so that the
// dies do not contend for one counter and a run still stays on one die.  Every die index 0..NXCD-1
// has workgroups (the grid is a multiple of NXCD), so every item is taken, wherever the workgroups
// actually run.
constexpr int EG = 4;  // items per claim
__device__ __forceinline__ int64_t die_item(int64_t x, int64_t t) {
  constexpr int64_t RUN = (int64_t)XQ * WAVES;
  return ((t / RUN) * NXCD + x) * RUN + t % RUN;
}

// ---------------------------------------------------------------------------------
// Item loop of the check and evaluation kernels.  One item per block: the block index.  The
// persistent form runs a grid of resident blocks (a multiple of NXCD): die x = blockIdx % NXCD
// takes the items of its runs, IRUN consecutive items dealt out per die as in die_item, IC at a
// time from its own counter, so that the dies do not contend for one address and a claim serves
// several items.  A relaxed read of the counter lets a block that finds its die's items drained
// leave without an atomic.  The item index is made wave-uniform (readfirstlane) so that
// everything derived from it stays in scalar registers and the source loads remain scalar loads.
// ---------------------------------------------------------------------------------
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(uint64_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

constexpr int IC = 2;         // items per claim of a persistent block
constexpr int64_t IRUN = 16;  // consecutive items per run of a die
__device__ __forceinline__ int64_t die_run_item(int64_t x, int64_t t) {
  return ((t / IRUN) * NXCD + x) * IRUN + t % IRUN;
}

struct ItemLoop {
  int64_t t = 0;
  int left = 0;
  bool first = true;
  // dctr: the NXCD per-die counters (zero at the start of the launch); slot: one shared word
  __device__ __forceinline__ bool next(bool persistent, int64_t total, int64_t *dctr, int64_t *slot,
                                       int64_t &item) {
    if (!persistent) {
      if (!first) return false;
      first = false;
      item = (int64_t)blockIdx.x;
      return item < total;
    }
    const int64_t x = blockIdx.x % NXCD;
    if (!first) __syncthreads();  // every wave is done with the previous item's shared data
    first = false;
    if (left == 0) {
      if (threadIdx.x == 0) {
        const int64_t cur = (int64_t)__hip_atomic_load((unsigned long long *)&dctr[x], __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
        *slot = die_run_item(x, cur) >= total ? cur
                                              : (int64_t)atomicAdd((unsigned long long *)&dctr[x], (unsigned long long)IC);
      }
      __syncthreads();
      t = uniform64(*slot);
      left = IC;
    }
    item = die_run_item(x, t);  // increasing in t: once past the end, every later claim is too
    ++t;
    --left;
    return item < total;
  }
};

// The slice of an item's source range [b0, b1) that wave w takes: the range split evenly over
// the waves in whole 32-source tiles (the last slices may be short or empty).
__device__ __forceinline__ void wave_slice(int64_t b0, int64_t b1, int w, int64_t &j0, int64_t &j1) {
  const int64_t len = b1 - b0;
  const int64_t tiles = (len + TILE - 1) / TILE;
  const int64_t per = (tiles + WAVES - 1) / WAVES * TILE;
  const int64_t s0 = b0 + (int64_t)w * per, s1 = s0 + per;
  j0 = s0 < b1 ? s0 : b1;
  j1 = s1 < b1 ? s1 : b1;
}

// wave index within the block, as a wave-uniform value
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// ---------------------------------------------------------------------------------
// Check sums.
// ---------------------------------------------------------------------------------
// FP64 check sums of the energy launch over sources [j0, j1) that all lie at r <= NEAR_R a.  With
// w = (r/a)^2 + (rc/a)^2 of the source, |c - x|^2 / (a^2 w) = 1 + (c/a).(-2x/(a w)) (rc the check
// sphere's radius): three FMAs from the per-source (-2x/(a w), -2y/(a w), -2z/(a w)), with 1/sqrt(w)
// in the weights (q', q' r/a) / sqrt(w), where the exact differences take six operations.  Every
// term of the sum is at most 1 in magnitude (2 |c||x| <= |c|^2 + |x|^2) and the sum is at least
// ((rc - NEAR_R a)/a)^2 / ((rc/a)^2 + NEAR_R^2) >= 1.2e-5 (rc >= a), so its rounding stays within
// about 5e-11 relative (1e-13 at rc = 1.1 a).  Sources in runs of 8 (their scalar loads batched).
__device__ __forceinline__ void check_range_expanded(const double4 &ck, double ia, const CheckSrc *__restrict__ cs,
                                                     int j0, int j1, double &au, double &av) {
  const double cx = ck.x * ia, cy = ck.y * ia, cz = ck.z * ia;
  double su = 0.0, sv = 0.0;
  int j = j0;
  for (; j + 8 <= j1; j += 8) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const CheckSrc m = cs[j + t];
      const double ri = rinv2(fma(cx, m.x, fma(cy, m.y, fma(cz, m.z, 1.0))));
      su = fma(m.wu, ri, su);
      sv = fma(m.wv, ri, sv);
    }
  }
  for (; j < j1; ++j) {
    const CheckSrc m = cs[j];
    const double ri = rinv2(fma(cx, m.x, fma(cy, m.y, fma(cz, m.z, 1.0))));
    su = fma(m.wu, ri, su);
    sv = fma(m.wv, ri, sv);
  }
  au += 0.5 * ia * su;  // rinv2 holds twice the reciprocal, of the distance over a
  av += 0.5 * ia * sv;
}

template <int MODE>
__device__ __forceinline__ void check_range(const typename PT<MODE>::T4 &ck, const typename PT<MODE>::T4 *__restrict__ src,
                                            const typename PT<MODE>::T *__restrict__ srcw, int j0, int j1,
                                            double &au, double &av) {
  using T = typename PT<MODE>::T;
  using T4 = typename PT<MODE>::T4;
  if constexpr (MODE == HSMA_PAIR_FP32) {
    T su = 0, sv = 0;
    for (int j = j0; j < j1; ++j) {
      const T4 s = src[j];
      const T dx = ck.x - s.x, dy = ck.y - s.y, dz = ck.z - s.z;
      const T ri = rinv(dx * dx + dy * dy + dz * dz);
      su = fma(s.w, ri, su);
      sv = fma(srcw[j], ri, sv);
    }
    au = su;
    av = sv;
  } else {
    au = 0.0;
    av = 0.0;
    int jb = j0;
    for (; jb + TILE <= j1; jb += TILE) {
      T su = 0, sv = 0;
#pragma unroll 8
      for (int t = 0; t < TILE; ++t) {
        const T4 s = src[jb + t];
        const T dx = ck.x - s.x, dy = ck.y - s.y, dz = ck.z - s.z;
        const T ri = rinv(dx * dx + dy * dy + dz * dz);
        su = fma(s.w, ri, su);
        sv = fma(srcw[jb + t], ri, sv);
      }
      au += (double)su;
      av += (double)sv;
    }
    T su = 0, sv = 0;
    for (int j = jb; j < j1; ++j) {
      const T4 s = src[j];
      const T dx = ck.x - s.x, dy = ck.y - s.y, dz = ck.z - s.z;
      const T ri = rinv(dx * dx + dy * dy + dz * dz);
      su = fma(s.w, ri, su);
      sv = fma(srcw[j], ri, sv);
    }
    au += (double)su;
    av += (double)sv;
  }
}

template <int MODE>
__global__ __launch_bounds__(TPB) void k_check(int persistent, int nsys, int M, int chc, const int64_t *__restrict__ base,
                                               const int *__restrict__ sys_c, const PlanDev *__restrict__ plans,
                                               const int32_t *__restrict__ plan_of,
                                               const typename PT<MODE>::T4 *__restrict__ src,
                                               const typename PT<MODE>::T *__restrict__ srcw, int64_t parts_bound,
                                               double *__restrict__ part, const CheckSrc *__restrict__ csrc,
                                               const int64_t *__restrict__ nfar) {
  using T4 = typename PT<MODE>::T4;
  Sched S(const_cast<int64_t *>(base), nsys);
  __shared__ int64_t s_item;
  __shared__ double red[2][WAVES][GRP];
  const int lane = threadIdx.x & 63, w = wave_id();
  if (!sched_ok(S)) return;
  const int64_t total = S.ic[nsys];
  const int64_t Gc = cdiv64(M, GRP);
  int64_t item;
  ItemLoop loop;
  while (loop.next(persistent, total, &S.ctr[CTR_CHECK], &s_item, item)) {
    const int b = sys_c[item];
    const int64_t lo = S.off[b], n = S.off[b + 1] - lo;
    const int64_t loc = item - S.ic[b];
    const int64_t chunks = cdiv64(n, chc);
    const int64_t c = loc / Gc, g = loc % Gc;  // items sharing a source chunk are adjacent
    const PlanDev pd = plans[plan_of ? plan_of[b] : 0];
    const T4 *chk = chk_of<MODE>(pd);
    const int64_t k = g * GRP + lane;
    const T4 ck = chk[k < M ? k : M - 1];
    int64_t j0, j1;
    wave_slice(c * chc, (c + 1) * chc < n ? (c + 1) * chc : n, w, j0, j1);
    double au = 0.0, av = 0.0;
    if constexpr (MODE == HSMA_PAIR_FP64) {
      if (csrc && j0 < j1) {  // energy launch: its far ions (packed first) in the expanded form
        const int64_t je = nfar[b] < j0 ? j0 : (nfar[b] < j1 ? nfar[b] : j1);
        if (j0 < je) check_range_expanded(ck, 1.0 / pd.a, csrc + lo, (int)j0, (int)je, au, av);
        j0 = je;
      }
    }
    if (j0 < j1) {  // (check_range sets its outputs)
      double ru, rv;
      check_range<MODE>(ck, src + lo, srcw + lo, (int)j0, (int)j1, ru, rv);
      au += ru;
      av += rv;
    }
    red[0][w][lane] = au;
    red[1][w][lane] = av;
    __syncthreads();
    if (w == 0) {
      double su = red[0][0][lane], sv = red[1][0][lane];
      for (int ww = 1; ww < WAVES; ++ww) {
        su += red[0][ww][lane];
        sv += red[1][ww][lane];
      }
      const int64_t slot = S.pc[b] + (g * chunks + c) * GRP + lane;
      part[slot] = su;
      part[parts_bound + slot] = sv;
    }
  }
}

// u, v of every system: fixed-order sum of the chunk partials.  uv[(2b)*M + k] = u, [(2b+1)*M + k] = v.
__global__ __launch_bounds__(256) void k_check_finish(int nsys, int M, int chc, const int64_t *__restrict__ base,
                                                      int64_t parts_bound, const double *__restrict__ part,
                                                      double *__restrict__ uv, float *__restrict__ uv32) {
  Sched S(const_cast<int64_t *>(base), nsys);
  if (!sched_ok(S)) return;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)nsys * M) return;
  const int b = (int)(t / M);
  const int k = (int)(t % M);
  const int64_t n = S.off[b + 1] - S.off[b];
  const int64_t chunks = n > 0 ? cdiv64(n, chc) : 0;
  const int64_t g = k / GRP, lane = k % GRP;
  double u = 0.0, v = 0.0;
#pragma unroll 8
  for (int64_t c = 0; c < chunks; ++c) {
    const int64_t slot = S.pc[b] + (g * chunks + c) * GRP + lane;
    u += part[slot];
    v += part[parts_bound + slot];
  }
  uv[(2 * (int64_t)b) * M + k] = u;
  uv[(2 * (int64_t)b + 1) * M + k] = v;
  if (uv32) {
    uv32[(2 * (int64_t)b) * M + k] = (float)u;
    uv32[(2 * (int64_t)b + 1) * M + k] = (float)v;
  }
}

// ---------------------------------------------------------------------------------
// Fit apply, few systems: one wave64 per output row and system.
// ---------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename TM>
__global__ __launch_bounds__(256) void k_fit_moments(int K, int M, const TM *__restrict__ pinv,
                                                     const double *__restrict__ uv, double *__restrict__ ab) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int b = blockIdx.y;
  const int lane = threadIdx.x & 63;
  if (row >= K) return;
  const TM *pr = pinv + (size_t)row * M;
  const double *u = uv + (size_t)(2 * b) * M;
  const double *v = u + M;
  double su = 0.0, sv = 0.0;
#pragma unroll 8
  for (int m = lane; m < M; m += 64) {
    const double wgt = (double)pr[m];
    su = fma(wgt, u[m], su);
    sv = fma(wgt, v[m], sv);
  }
  su = wave_sum(su);
  sv = wave_sum(sv);
  if (lane == 0) {
    ab[(size_t)(2 * b) * K + row] = su;
    ab[(size_t)(2 * b + 1) * K + row] = sv;
  }
}

// The evaluation's surface sources of node s of system b: (Q', D') at s with exact dipoles
// (Pe = P); with the paper's point pairs (Pe = 3P) the monopole (Q', 0) at 3s and the charges
// (-D' R_tau/dy, 0), (+D' R_tau/dy, 0) at its inner and outer point (3s + 1, 3s + 2), whose
// potential D' (R_tau/dy)(1/|x - y+| - 1/|x - y-|) tends to the dipole's D' (x - y).y / |x - y|^3.
template <typename T2>
__device__ __forceinline__ void store_strengths(T2 *__restrict__ qd, int b, int s, int P, int Pe, double q,
                                                double d, double dyc) {
  if (Pe == P) {
    T2 o;
    o.x = q;
    o.y = d;
    qd[(size_t)b * P + s] = o;
  } else {
    T2 o0, o1, o2;
    o0.x = q;
    o0.y = 0;
    o1.x = -d * dyc;
    o1.y = 0;
    o2.x = d * dyc;
    o2.y = 0;
    T2 *e = qd + (size_t)b * Pe + 3 * (size_t)s;
    e[0] = o0;
    e[1] = o1;
    e[2] = o2;
  }
}

template <typename TM, typename T2>
__global__ __launch_bounds__(256) void k_fit_surface(int nsys, const int64_t *__restrict__ base, int P, int Pe, int K,
                                                     const TM *__restrict__ lhat, const PlanDev *__restrict__ plans,
                                                     const int32_t *__restrict__ plan_of, const int *__restrict__ nidx,
                                                     const double *__restrict__ ab, T2 *__restrict__ qd) {
  Sched S(const_cast<int64_t *>(base), nsys);
  if (!sched_ok(S)) return;  // plan_of was checked by the schedule
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int b = blockIdx.y;
  const int lane = threadIdx.x & 63;
  if (s >= P) return;
  const PlanDev &c = plans[plan_of ? plan_of[b] : 0];
  const double *fg = c.fg;
  const TM *lr = lhat + (size_t)s * K;
  const double *al = ab + (size_t)(2 * b) * K;
  const double *be = al + K;
  double sq = 0.0, sd = 0.0;
#pragma unroll 4
  for (int k = lane; k < K; k += 64) {
    const double h = fg[k] * al[k] + fg[K + k] * be[k];
    const double l = (double)lr[k];
    sq = fma(l * (double)degree_weight(nidx[k], c.dipole), h, sq);
    sd = fma(l, h, sd);
  }
  sq = wave_sum(sq);
  sd = wave_sum(sd);
  if (lane == 0) store_strengths(qd, b, s, P, Pe, sq, c.dipole == 2 ? 0.0 : -sd, c.dyc);
}

// ---------------------------------------------------------------------------------
// Fit apply, many systems: C[col][row] = sum_k A[row][k] B[col][k] on MFMA.  Block tile 64 rows
// x 64 cols, four waves of 32 x 32 (2 x 2 tiles of 16 x 16); k staged through LDS 32 at a time,
// and the next 32 values of k read from global memory into registers while the current ones are
// multiplied, so that the loads' latency overlaps the MFMAs (the products are latency-bound
// otherwise: one k step's work is a few hundred cycles).
// ---------------------------------------------------------------------------------
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
constexpr int GK = 32;  // k values per LDS stage

// One thread's share of a stage: 64 rows (cols) x GK values of k of each operand, 8 values each,
// rows read 32 consecutive k by consecutive threads; zero beyond the matrices.
template <typename T>
struct GemmStage {
  T ra[8], rb[8];
  __device__ __forceinline__ void load(const T *__restrict__ A, const T *__restrict__ B, int nrows, int ncols,
                                       int kdim, int row0, int col0, int k0, int t) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = t + 256 * i, r = e >> 5, gk = k0 + (e & 31);
      ra[i] = (row0 + r < nrows && gk < kdim) ? A[(size_t)(row0 + r) * kdim + gk] : (T)0;
      rb[i] = (col0 + r < ncols && gk < kdim) ? B[(size_t)(col0 + r) * kdim + gk] : (T)0;
    }
  }
  __device__ __forceinline__ void store(T (*As)[GK + 1], T (*Bs)[GK + 1], int t) const {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = t + 256 * i;
      As[e >> 5][e & 31] = ra[i];
      Bs[e >> 5][e & 31] = rb[i];
    }
  }
};

// FP32 (v_mfma_f32_16x16x4f32).  The MFMA accumulators are FP32; they are folded into FP64
// registers after every 64 values of k, so the sum over k = 1536-9600 terms loses no more than a
// 64-term FP32 sum.
__global__ __launch_bounds__(256) void k_gemm_nt(int nrows, int ncols, int kdim, const float *__restrict__ A,
                                                 const float *__restrict__ B, float *__restrict__ C) {
  __shared__ float As[64][GK + 1];
  __shared__ float Bs[64][GK + 1];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int row0 = blockIdx.x * 64, col0 = blockIdx.y * 64;
  floatx4 acc[2][2];
  double dacc[2][2][4];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
      for (int r = 0; r < 4; ++r) dacc[i][j][r] = 0.0;
    }
  GemmStage<float> g;
  g.load(A, B, nrows, ncols, kdim, row0, col0, 0, t);
  for (int k0 = 0; k0 < kdim; k0 += GK) {
    __syncthreads();  // every wave is done with the previous stage
    g.store(As, Bs, t);
    __syncthreads();
    if (k0 + GK < kdim) g.load(A, B, nrows, ncols, kdim, row0, col0, k0 + GK, t);
#pragma unroll
    for (int kk = 0; kk < GK; kk += 4) {
      const int kl = kk + (lane >> 4);
      float a[2], bb[2];
      for (int i = 0; i < 2; ++i) a[i] = As[wr * 32 + i * 16 + (lane & 15)][kl];
      for (int j = 0; j < 2; ++j) bb[j] = Bs[wc * 32 + j * 16 + (lane & 15)][kl];
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], bb[j], acc[i][j], 0, 0, 0);
    }
    if ((k0 + GK) % 64 == 0 || k0 + GK >= kdim) {
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          for (int r = 0; r < 4; ++r) dacc[i][j][r] += (double)acc[i][j][r];
          acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
    }
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      const int col = col0 + wc * 32 + j * 16 + (lane & 15);
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + wr * 32 + i * 16 + 4 * (lane >> 4) + r;
        if (row < nrows && col < ncols) C[(size_t)col * nrows + row] = (float)dacc[i][j][r];
      }
    }
}

// The same product in FP64 (v_mfma_f64_16x16x4f64), whose lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] of a 16 x 4 by 4 x 16 step and receives D[l / 16 + 4 v][l % 16], v = 0..3;
// the accumulators are FP64 throughout.
__global__ __launch_bounds__(256) void k_gemm64_nt(int nrows, int ncols, int kdim, const double *__restrict__ A,
                                                   const double *__restrict__ B, double *__restrict__ C) {
  __shared__ double As[64][GK + 1];
  __shared__ double Bs[64][GK + 1];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int row0 = blockIdx.x * 64, col0 = blockIdx.y * 64;
  doublex4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
  GemmStage<double> g;
  g.load(A, B, nrows, ncols, kdim, row0, col0, 0, t);
  for (int k0 = 0; k0 < kdim; k0 += GK) {
    __syncthreads();  // every wave is done with the previous stage
    g.store(As, Bs, t);
    __syncthreads();
    if (k0 + GK < kdim) g.load(A, B, nrows, ncols, kdim, row0, col0, k0 + GK, t);
#pragma unroll
    for (int kk = 0; kk < GK; kk += 4) {
      const int kl = kk + (lane >> 4);
      double a[2], bb[2];
      for (int i = 0; i < 2; ++i) a[i] = As[wr * 32 + i * 16 + (lane & 15)][kl];
      for (int j = 0; j < 2; ++j) bb[j] = Bs[wc * 32 + j * 16 + (lane & 15)][kl];
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], acc[i][j], 0, 0, 0);
    }
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      const int col = col0 + wc * 32 + j * 16 + (lane & 15);
      for (int v = 0; v < 4; ++v) {
        const int row = row0 + wr * 32 + i * 16 + (lane >> 4) + 4 * v;
        if (row < nrows && col < ncols) C[(size_t)col * nrows + row] = acc[i][j][v];
      }
    }
}

// Fit apply on BF16 MFMA with split products.  Every factor x is taken as a sum of BF16
// terms b0 = bf16(x), b1 = bf16(x - b0), b2 = bf16(x - b0 - b1), and the product of two
// factors as the sum of the term products whose orders add to at most NS - 1:
//   NS = 2 (split-BF16x3): a0 c0 + a0 c1 + a1 c0; the two-term split leaves up to 2^-16 |x|,
//           so a product carries up to 3 * 2^-16 relative error;
//   NS = 3 (split-BF16x6): also a0 c2 + a2 c0 + a1 c1, leaving about 2^-24, as FP32.
// C[col][row] = sum_k A[row][k] B[col][k]; A comes pre-split (plane t of nrows rows, row
// stride kp = kdim rounded up to 32, zero padding), B is FP32 with row stride kdim and is
// split while it is staged.  v_mfma_f32_16x16x32_bf16: a lane holds 8 consecutive k of one row
// (A) or column (B); both operands use the same k order, so the contraction does not depend
// on it.  Block tile 64 x 64, four waves of 32 x 32, k staged 32 at a time; the smallest
// products are accumulated first, and the FP32 accumulators are folded into FP64 every 64 k,
// as in k_gemm_nt.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ inline uint32_t bf16_rne_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

template <int NS>
__global__ __launch_bounds__(256) void k_gemm_bf(int nrows, int ncols, int kdim, int kp,
                                                 const uint16_t *__restrict__ A, const float *__restrict__ B,
                                                 float *__restrict__ C) {
  __shared__ __align__(16) uint16_t As[NS][64][40];
  __shared__ __align__(16) uint16_t Bs[NS][64][40];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int row0 = blockIdx.x * 64, col0 = blockIdx.y * 64;
  const int sr = t >> 2, sc = (t & 3) * 8;  // staging: row / column sr, k offset sc
  floatx4 acc[2][2];
  double dacc[2][2][4];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
      for (int r = 0; r < 4; ++r) dacc[i][j][r] = 0.0;
    }
  int step = 0;
  for (int k0 = 0; k0 < kdim; k0 += 32) {
    {
      const int gr = row0 + sr;
#pragma unroll
      for (int p = 0; p < NS; ++p) {
        uint4 h = make_uint4(0, 0, 0, 0);
        if (gr < nrows)  // k0 + sc + 7 < kp: the padded rows cover every staged k
          h = *(const uint4 *)(A + ((size_t)p * nrows + gr) * kp + k0 + sc);
        *(uint4 *)&As[p][sr][sc] = h;
      }
      const int gc = col0 + sr;
      uint32_t bb[NS][8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int gk = k0 + sc + e;
        float v = (gc < ncols && gk < kdim) ? B[(size_t)gc * kdim + gk] : 0.0f;
#pragma unroll
        for (int p = 0; p < NS; ++p) {
          bb[p][e] = bf16_rne_bits(v);
          v -= __uint_as_float(bb[p][e] << 16);
        }
      }
#pragma unroll
      for (int p = 0; p < NS; ++p)
        *(uint4 *)&Bs[p][sr][sc] = make_uint4(bb[p][0] | bb[p][1] << 16, bb[p][2] | bb[p][3] << 16,
                                              bb[p][4] | bb[p][5] << 16, bb[p][6] | bb[p][7] << 16);
    }
    __syncthreads();
    const int kl = 8 * (lane >> 4);
    bf16x8 af[NS][2], bf[NS][2];
#pragma unroll
    for (int p = 0; p < NS; ++p)
      for (int i = 0; i < 2; ++i) {
        af[p][i] = *(const bf16x8 *)&As[p][wr * 32 + i * 16 + (lane & 15)][kl];
        bf[p][i] = *(const bf16x8 *)&Bs[p][wc * 32 + i * 16 + (lane & 15)][kl];
      }
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) {
        floatx4 c = acc[i][j];
        if constexpr (NS == 3) {
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1][i], bf[1][j], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[2][i], bf[0][j], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bf[2][j], c, 0, 0, 0);
        }
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1][i], bf[0][j], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bf[1][j], c, 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bf[0][j], c, 0, 0, 0);
      }
    __syncthreads();
    if (++step == 2 || k0 + 32 >= kdim) {
      step = 0;
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          for (int r = 0; r < 4; ++r) dacc[i][j][r] += (double)acc[i][j][r];
          acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
    }
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      const int col = col0 + wc * 32 + j * 16 + (lane & 15);
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + wr * 32 + i * 16 + 4 * (lane >> 4) + r;
        if (row < nrows && col < ncols) C[(size_t)col * nrows + row] = (float)dacc[i][j][r];
      }
    }
}

// h = f . alpha' + g . beta' from the first GEMM's output ab32 [2 nsys][K]; writes the
// second GEMM's operand h32 [2 nsys][K]: row 2b = n . h, row 2b+1 = h (TF: FP32 or FP64).
template <typename TF>
__global__ __launch_bounds__(256) void k_fit_h(int nsys, const int64_t *__restrict__ base, int K,
                                               const TF *__restrict__ ab32, const PlanDev *__restrict__ plans,
                                               const int32_t *__restrict__ plan_of, const int *__restrict__ nidx,
                                               TF *__restrict__ h32) {
  Sched S(const_cast<int64_t *>(base), nsys);
  if (!sched_ok(S)) return;  // plan_of was checked by the schedule
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)nsys * K) return;
  const int b = (int)(t / K), k = (int)(t % K);
  const PlanDev &c = plans[plan_of ? plan_of[b] : 0];
  const double h = c.fg[k] * (double)ab32[(size_t)(2 * b) * K + k] +
                   c.fg[K + k] * (double)ab32[(size_t)(2 * b + 1) * K + k];
  h32[(size_t)(2 * b) * K + k] = (TF)(h * (double)degree_weight(nidx[k], c.dipole));
  h32[(size_t)(2 * b + 1) * K + k] = (TF)h;
}

// qd[b][s] = (C[2b][s], -C[2b+1][s]) from the second GEMM's output [2 nsys][P].
template <typename T2, typename TF>
__global__ __launch_bounds__(256) void k_fit_qd(int nsys, int P, int Pe, const PlanDev *__restrict__ plans,
                                                const int32_t *__restrict__ plan_of, const TF *__restrict__ Cq,
                                                T2 *__restrict__ qd) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)nsys * P) return;
  const int b = (int)(t / P), s = (int)(t % P);
  const PlanDev &c = plans[plan_of ? plan_of[b] : 0];
  store_strengths(qd, b, s, P, Pe, (double)Cq[(size_t)(2 * b) * P + s],
                  c.dipole == 2 ? 0.0 : -(double)Cq[(size_t)(2 * b + 1) * P + s], c.dyc);
}

// ---------------------------------------------------------------------------------
// Evaluation sums.
// ---------------------------------------------------------------------------------
template <int MODE, bool DIAG>
__device__ __forceinline__ double kelvin_range(const typename PT<MODE>::T4 &t, int i,
                                               const typename PT<MODE>::T4 *__restrict__ img, int j0, int j1) {
  using T = typename PT<MODE>::T;
  using T4 = typename PT<MODE>::T4;
  if constexpr (MODE != HSMA_PAIR_FP32_COMP) {
    T s = 0;
#pragma unroll 8
    for (int j = j0; j < j1; ++j) {
      const T4 v = img[j];
      const T dx = t.x - v.x, dy = t.y - v.y, dz = t.z - v.z;
      T ri = rinv(dx * dx + dy * dy + dz * dz);
      if (DIAG) ri = (j == i) ? (T)0 : ri;
      s = fma(v.w, ri, s);
    }
    return (double)s;
  } else {
    double acc = 0.0;
    int jb = j0;
    for (; jb + TILE <= j1; jb += TILE) {
      float s = 0.0f;
#pragma unroll 8
      for (int u = 0; u < TILE; ++u) {
        const float4 v = img[jb + u];
        const float dx = t.x - v.x, dy = t.y - v.y, dz = t.z - v.z;
        float ri = rinv(dx * dx + dy * dy + dz * dz);
        if (DIAG) ri = (jb + u == i) ? 0.0f : ri;
        s = fmaf(v.w, ri, s);
      }
      acc += (double)s;
    }
    float s = 0.0f;
    for (int j = jb; j < j1; ++j) {
      const float4 v = img[j];
      const float dx = t.x - v.x, dy = t.y - v.y, dz = t.z - v.z;
      float ri = rinv(dx * dx + dy * dy + dz * dz);
      if (DIAG) ri = (j == i) ? 0.0f : ri;
      s = fmaf(v.w, ri, s);
    }
    return acc + (double)s;
  }
}

template <int MODE, bool MONO>
__device__ __forceinline__ double surface_range(const typename PT<MODE>::T4 &t,
                                                const typename PT<MODE>::T4 *__restrict__ nodes,
                                                const typename PT<MODE>::T2 *__restrict__ qd, int s0, int s1) {
  using T = typename PT<MODE>::T;
  using T2 = typename PT<MODE>::T2;
  using T4 = typename PT<MODE>::T4;
  double acc = 0.0;
  for (int sb = s0; sb < s1; sb += TILE) {
    const int se = sb + TILE < s1 ? sb + TILE : s1;
    T s = 0;
#pragma unroll 8
    for (int k = sb; k < se; ++k) {
      const T4 yv = nodes[k];
      const T2 wv = qd[k];
      const T dx = t.x - yv.x, dy = t.y - yv.y, dz = t.z - yv.z;
      const T ri = rinv(dx * dx + dy * dy + dz * dz);
      if constexpr (MONO) {  // single layer: monopoles only
        s = fma(wv.x, ri, s);
      } else {
        const T dot = dx * yv.x + dy * yv.y + dz * yv.z;  // (x - y_s) . y_s = R_tau (x - y_s) . y^_s
        s = fma(ri, fma(wv.y * dot, ri * ri, wv.x), s);
      }
    }
    if constexpr (MODE == HSMA_PAIR_FP32) {
      acc = (double)((T)acc + s);
    } else {
      acc += (double)s;
    }
  }
  return acc;
}

template <int MODE>
__global__ __launch_bounds__(TPB) void k_eval(int persistent, int nsys, int P, int che, const int64_t *__restrict__ base,
                                              const int *__restrict__ sys_e, const PlanDev *__restrict__ plans,
                                              const int32_t *__restrict__ plan_of,
                                              const typename PT<MODE>::T4 *__restrict__ tgt,
                                              const typename PT<MODE>::T4 *__restrict__ img,
                                              const typename PT<MODE>::T4 *__restrict__ nodes,
                                              const typename PT<MODE>::T2 *__restrict__ qd, double *__restrict__ part) {
  using T4 = typename PT<MODE>::T4;
  Sched S(const_cast<int64_t *>(base), nsys);
  __shared__ int64_t s_item;
  __shared__ double red[WAVES][GRP];
  const int lane = threadIdx.x & 63, w = wave_id();
  if (!sched_ok(S)) return;
  const int64_t total = S.ie[nsys];
  int64_t item;
  ItemLoop loop;
  while (loop.next(persistent, total, &S.ctr[CTR_EVAL], &s_item, item)) {
    const int b = sys_e[item];
    const int64_t lo = S.off[b], n = S.off[b + 1] - lo;
    const int64_t loc = item - S.ie[b];
    const int64_t G = cdiv64(n, GRP);
    const int64_t chunks = cdiv64(n + P, che);
    const int64_t c = loc / G, g = loc % G;  // items sharing a source chunk are adjacent
    const int64_t il = g * GRP + lane;       // local target index
    const T4 t = tgt[lo + (il < n ? il : n - 1)];
    const int64_t tot = n + P;
    int64_t j0, j1;
    wave_slice(c * che, (c + 1) * che < tot ? (c + 1) * che : tot, w, j0, j1);
    double acc = 0.0;
    const int64_t k1 = j1 < n ? j1 : n;
    if (j0 < k1) {
      const int64_t t0 = g * GRP;
      const bool diag = (t0 < k1) && (t0 + GRP > j0);
      acc = diag ? kelvin_range<MODE, true>(t, (int)il, img + lo, (int)j0, (int)k1)
                 : kelvin_range<MODE, false>(t, (int)il, img + lo, (int)j0, (int)k1);
    }
    const int64_t s0 = (j0 > n ? j0 : n) - n, s1 = j1 - n;
    if (s0 < s1) {
      const int pl = plan_of ? plan_of[b] : 0;
      const T4 *nd = nodes + (size_t)pl * P;
      const typename PT<MODE>::T2 *qb = qd + (size_t)b * P;
      acc += plans[pl].dipole == 2 ? surface_range<MODE, true>(t, nd, qb, (int)s0, (int)s1)
                                   : surface_range<MODE, false>(t, nd, qb, (int)s0, (int)s1);
    }
    red[w][lane] = acc;
    __syncthreads();
    if (w == 0) {
      double s = red[0][lane];
      for (int ww = 1; ww < WAVES; ++ww) s += red[ww][lane];
      part[S.pe[b] + (g * chunks + c) * GRP + lane] = s;
    }
  }
}

// ---------------------------------------------------------------------------------
// Field sums (Algorithm 1, step 5: potential and field at the ions).  With every image
// held fixed, an image of strength c at s adds c / |x - s| to the potential and
// c (x - s) / |x - s|^3 to E = -grad Phi.  A surface node y_s adds, besides its potential
// Q / r + D' (d . y_s) / r^3 (d = x - y_s), the field
//   d (Q + 3 D' (d . y_s) / r^2) / r^3 - y_s D' / r^3.
// The partial sums are kept per target and source chunk as (Phi, Ex, Ey, Ez).
// ---------------------------------------------------------------------------------
struct F4 {
  double p, x, y, z;
};

// In the FP32 modes the coordinates carry FP32 lo parts (tl for the target, ilo for the
// images): d = (x_hi - s_hi) + (x_lo - s_lo).  The field of an image a distance d away is
// dominated by the nearest images, and for two ions at the interface d can be 1e-4 a, where
// FP32 coordinates alone (2^-24 a) would leave 1e-3 relative error in the term.
template <int MODE, bool DIAG>
__device__ __forceinline__ void kelvin_field_range(const typename PT<MODE>::T4 &t, const float4 &tl, int i,
                                                   const typename PT<MODE>::T4 *__restrict__ img,
                                                   const float4 *__restrict__ ilo, int j0, int j1, F4 &acc) {
  using T = typename PT<MODE>::T;
  using T4 = typename PT<MODE>::T4;
  constexpr bool LO = MODE != HSMA_PAIR_FP64;
  // FP32_COMP: FP32 sums over 32-source tiles folded into FP64; otherwise one running sum
  const int tile = MODE == HSMA_PAIR_FP32_COMP ? TILE : (1 << 30);
  T rp = 0, rx = 0, ry = 0, rz = 0;
  for (int jb = j0; jb < j1; jb += tile) {
    const int je = (j1 - jb) > tile ? jb + tile : j1;
    T sp = 0, sx = 0, sy = 0, sz = 0;
#pragma unroll 8
    for (int j = jb; j < je; ++j) {
      const T4 v = img[j];
      T dx = t.x - v.x, dy = t.y - v.y, dz = t.z - v.z;
      if constexpr (LO) {
        const float4 vl = ilo[j];
        dx += tl.x - vl.x;
        dy += tl.y - vl.y;
        dz += tl.z - vl.z;
      }
      T ri = rinv(dx * dx + dy * dy + dz * dz);
      if (DIAG) ri = (j == i) ? (T)0 : ri;
      const T w = v.w * ri;
      sp += w;
      const T w3 = w * (ri * ri);
      sx = fma(w3, dx, sx);
      sy = fma(w3, dy, sy);
      sz = fma(w3, dz, sz);
    }
    if constexpr (MODE == HSMA_PAIR_FP32_COMP) {
      acc.p += (double)sp;
      acc.x += (double)sx;
      acc.y += (double)sy;
      acc.z += (double)sz;
    } else {
      rp += sp;
      rx += sx;
      ry += sy;
      rz += sz;
    }
  }
  if constexpr (MODE != HSMA_PAIR_FP32_COMP) {
    acc.p += (double)rp;
    acc.x += (double)rx;
    acc.y += (double)ry;
    acc.z += (double)rz;
  }
}

template <int MODE>
__device__ __forceinline__ void surface_field_range(const typename PT<MODE>::T4 &t,
                                                    const typename PT<MODE>::T4 *__restrict__ nodes,
                                                    const typename PT<MODE>::T2 *__restrict__ qd, int s0, int s1,
                                                    F4 &acc) {
  using T = typename PT<MODE>::T;
  using T2 = typename PT<MODE>::T2;
  using T4 = typename PT<MODE>::T4;
  T rp = 0, rx = 0, ry = 0, rz = 0;
  for (int sb = s0; sb < s1; sb += TILE) {
    const int se = sb + TILE < s1 ? sb + TILE : s1;
    T sp = 0, sx = 0, sy = 0, sz = 0;
#pragma unroll 4
    for (int k = sb; k < se; ++k) {
      const T4 yv = nodes[k];
      const T2 wv = qd[k];
      const T dx = t.x - yv.x, dy = t.y - yv.y, dz = t.z - yv.z;
      const T ri = rinv(dx * dx + dy * dy + dz * dz);
      const T ri2 = ri * ri;
      const T dot = dx * yv.x + dy * yv.y + dz * yv.z;  // (x - y_s) . y_s
      const T tq = wv.y * dot * ri2;                      // D' (d . y_s) / r^2
      const T u = wv.x + tq;
      sp = fma(ri, u, sp);
      const T A = ri * ri2;
      const T B = A * fma((T)2, tq, u);
      const T Cy = A * wv.y;
      sx = fma(B, dx, fma(-Cy, yv.x, sx));
      sy = fma(B, dy, fma(-Cy, yv.y, sy));
      sz = fma(B, dz, fma(-Cy, yv.z, sz));
    }
    if constexpr (MODE == HSMA_PAIR_FP32) {
      rp += sp;
      rx += sx;
      ry += sy;
      rz += sz;
    } else {
      acc.p += (double)sp;
      acc.x += (double)sx;
      acc.y += (double)sy;
      acc.z += (double)sz;
    }
  }
  if constexpr (MODE == HSMA_PAIR_FP32) {
    acc.p += (double)rp;
    acc.x += (double)rx;
    acc.y += (double)ry;
    acc.z += (double)rz;
  }
}

// Same items and partial slots as k_eval, with a (Phi, E) quadruple per slot.
template <int MODE>
__global__ __launch_bounds__(TPB) void k_eval_field(int persistent, int nsys, int P, int che,
                                                    const int64_t *__restrict__ base, const int *__restrict__ sys_e,
                                                    const int32_t *__restrict__ plan_of,
                                                    const typename PT<MODE>::T4 *__restrict__ tgt,
                                                    const typename PT<MODE>::T4 *__restrict__ img,
                                                    const typename PT<MODE>::T4 *__restrict__ nodes,
                                                    const typename PT<MODE>::T2 *__restrict__ qd,
                                                    const float4 *__restrict__ tlo, const float4 *__restrict__ ilo,
                                                    double4 *__restrict__ part) {
  using T4 = typename PT<MODE>::T4;
  Sched S(const_cast<int64_t *>(base), nsys);
  __shared__ int64_t s_item;
  __shared__ double4 red[WAVES][GRP];
  const int lane = threadIdx.x & 63, w = wave_id();
  if (!sched_ok(S)) return;
  const int64_t total = S.ie[nsys];
  int64_t item;
  ItemLoop loop;
  while (loop.next(persistent, total, &S.ctr[CTR_EVAL], &s_item, item)) {
    const int b = sys_e[item];
    const int64_t lo = S.off[b], n = S.off[b + 1] - lo;
    const int64_t loc = item - S.ie[b];
    const int64_t G = cdiv64(n, GRP);
    const int64_t chunks = cdiv64(n + P, che);
    const int64_t c = loc / G, g = loc % G;
    const int64_t il = g * GRP + lane;
    const T4 t = tgt[lo + (il < n ? il : n - 1)];
    const float4 tl = tlo ? tlo[lo + (il < n ? il : n - 1)] : make_float4(0.f, 0.f, 0.f, 0.f);
    const int64_t tot = n + P;
    int64_t j0, j1;
    wave_slice(c * che, (c + 1) * che < tot ? (c + 1) * che : tot, w, j0, j1);
    F4 acc = {0.0, 0.0, 0.0, 0.0};
    const int64_t k1 = j1 < n ? j1 : n;
    if (j0 < k1) {
      const int64_t t0 = g * GRP;
      const bool diag = (t0 < k1) && (t0 + GRP > j0);
      const float4 *il4 = ilo ? ilo + lo : nullptr;
      if (diag)
        kelvin_field_range<MODE, true>(t, tl, (int)il, img + lo, il4, (int)j0, (int)k1, acc);
      else
        kelvin_field_range<MODE, false>(t, tl, (int)il, img + lo, il4, (int)j0, (int)k1, acc);
    }
    const int64_t s0 = (j0 > n ? j0 : n) - n, s1 = j1 - n;
    if (s0 < s1) {
      const int pl = plan_of ? plan_of[b] : 0;
      surface_field_range<MODE>(t, nodes + (size_t)pl * P, qd + (size_t)b * P, (int)s0, (int)s1, acc);
    }
    red[w][lane] = make_double4(acc.p, acc.x, acc.y, acc.z);
    __syncthreads();
    if (w == 0) {
      double4 s = red[0][lane];
      for (int ww = 1; ww < WAVES; ++ww) {
        const double4 o = red[ww][lane];
        s.x += o.x;
        s.y += o.y;
        s.z += o.z;
        s.w += o.w;
      }
      part[S.pe[b] + (g * chunks + c) * GRP + lane] = s;
    }
  }
}

// ---------------------------------------------------------------------------------
// Symmetric Kelvin sums.  For ions i, j of one system, |x_i - r_K,j|^2 (r_j/a)^2 =
// r_i^2 r_j^2 / a^2 - 2 x_i.x_j + a^2 is symmetric in i and j, so
//   1 / |x_j - r_K,i| = (r_i / r_j) / |x_i - r_K,j|:
// one reciprocal root gives both q'_j / |x_i - r_K,j| (to ion i) and
// (q'_i r_i) / |x_i - r_K,j| / r_j (to ion j), q' = q_K / (4 pi eps1).
// A system's ions form blocks of TB = 64 R; a wave holds one block as targets (R per lane)
// and sweeps another block J >= I as wave-uniform sources.  Forward sums stay in the lanes;
// the reverse contribution to each source is summed over the wave by DPP steps.  Every ion
// gets one partial slot per partner block (slot K of ion i at K * n + i, K = the other block),
// written exactly once, then one slot per surface-node chunk.  Diagonal blocks and surface
// chunks are one-directional.
// ---------------------------------------------------------------------------------
template <int CTRL, int ROW_MASK, int BANK_MASK, bool BOUND_ZERO>
__device__ __forceinline__ float dpp_read(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, BANK_MASK, BOUND_ZERO));
}

// Sum over the 64 lanes of a wave, complete in lane 63.  Row shifts by 1, 2, 4 and 8 with zero
// fill form the inclusive prefix sum of each row of 16 lanes (its total in the row's lane 15);
// the row-15 broadcast then adds row r-1's total into row r (lane 31 = rows 0+1, lane 63 =
// rows 2+3) and the row-31 broadcast adds lane 31 into rows 2 and 3.  Only lane 63 is used.
__device__ __forceinline__ float wave_total_lane63(float v) {
  v += dpp_read<0x111, 0xf, 0xf, true>(v);  // row_shr:1
  v += dpp_read<0x112, 0xf, 0xf, true>(v);  // row_shr:2
  v += dpp_read<0x114, 0xf, 0xf, true>(v);  // row_shr:4
  v += dpp_read<0x118, 0xf, 0xf, true>(v);  // row_shr:8
  v += dpp_read<0x142, 0xf, 0xf, true>(v);  // row_bcast:15
  v += dpp_read<0x143, 0xf, 0xf, true>(v);  // row_bcast:31
  return v;
}

// The reverse-total buffer moved down one lane (wave_shl:1, lane i reads lane i + 1) with the new
// total t entering lane 63: without zero fill lane 63 has no source lane and keeps the DPP
// move's old operand, t.
__device__ __forceinline__ float shift_in_lane63(float t, float buf) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(t), __float_as_int(buf), 0x130, 0xf, 0xf, false));
}

// One wave-uniform source image v against the lane's R targets of the symmetric kernel: the
// forward terms into sum[k], the lane's part of the source's reverse total returned.
template <int R>
__device__ __forceinline__ float sym_source(const float4 &v, const float (&tx)[R], const float (&ty)[R],
                                            const float (&tz)[R], const float (&tw)[R], float (&sum)[R]) {
  float rev = 0.0f;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const float dx = tx[k] - v.x, dy = ty[k] - v.y, dz = tz[k] - v.z;
    const float ri = rinv(dx * dx + dy * dy + dz * dz);
    sum[k] = fmaf(v.w, ri, sum[k]);
    rev = fmaf(tw[k], ri, rev);
  }
  return rev;
}

// Surface nodes s0..s1-1 onto RS target sets per lane, FP32 tiles of TILE nodes folded into
// FP64.  MONO: the single-layer form, monopoles only (the dipole strengths are zero).
// SPLIT: exact dipoles with every node on the sphere R_tau (r2t = R_tau^2): (x - y).y =
// (|x|^2 - R_tau^2 - d^2)/2 and d^2 r^2 = 1 (r = 1/d from the hardware root, to about 2e-7), so a
// dipole term is w_d ((|x|^2 - R_tau^2)/2 r^3 - r/2): three sums per target, the first scaled at
// each tile's end, both parts of one sign (|x| < R_tau).  The rest: (x - y).y from the differences.
template <int RS, bool MONO, bool SPLIT = false>
__device__ __forceinline__ void sym_surface(const float (&sx)[RS], const float (&sy)[RS], const float (&sz)[RS],
                                            const float4 *__restrict__ nd, const float2 *__restrict__ qb, int s0,
                                            int s1, double (&acc)[RS], float r2t = 0.0f) {
  double hf[RS];
  if constexpr (SPLIT) {
#pragma unroll
    for (int k = 0; k < RS; ++k)
      hf[k] = 0.5 * ((double)sx[k] * sx[k] + (double)sy[k] * sy[k] + (double)sz[k] * sz[k] - (double)r2t);
  }
  for (int sb = s0; sb < s1; sb += TILE) {
    const int se = sb + TILE < s1 ? sb + TILE : s1;
    float sum[RS], s3[RS], s1w[RS];
#pragma unroll
    for (int k = 0; k < RS; ++k) {
      sum[k] = 0.0f;
      s3[k] = 0.0f;
      s1w[k] = 0.0f;
    }
    for (int m = sb; m < se; ++m) {
      const float4 yv = nd[m];
      const float2 wv = qb[m];
#pragma unroll
      for (int k = 0; k < RS; ++k) {
        const float dx = sx[k] - yv.x, dy = sy[k] - yv.y, dz = sz[k] - yv.z;
        const float ri = rinv(dx * dx + dy * dy + dz * dz);
        if constexpr (MONO) {
          sum[k] = fmaf(wv.x, ri, sum[k]);
        } else if constexpr (SPLIT) {
          sum[k] = fmaf(wv.x, ri, sum[k]);
          s3[k] = fmaf(wv.y, ri * ri * ri, s3[k]);
          s1w[k] = fmaf(wv.y, ri, s1w[k]);
        } else {
          const float dot = dx * yv.x + dy * yv.y + dz * yv.z;
          sum[k] = fmaf(ri, fmaf(wv.y * dot, ri * ri, wv.x), sum[k]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < RS; ++k) {
      if constexpr (SPLIT)
        acc[k] += fma(hf[k], (double)s3[k], fma(-0.5, (double)s1w[k], (double)sum[k]));
      else
        acc[k] += (double)sum[k];
    }
  }
}

// One item of the symmetric kernel (a block pair or a surface item), by one wave.
template <int R>
__device__ __forceinline__ void sym_item(int64_t item, const Sched &S, int lane, int P, int sch, int dipole,
                                         const int *__restrict__ sys_e, const int32_t *__restrict__ plan_of,
                                         const float4 *__restrict__ tgt, const float4 *__restrict__ img,
                                         const float *__restrict__ wk, const double *__restrict__ rk,
                                         const float4 *__restrict__ nodes, const float2 *__restrict__ qd,
                                         const PlanDev *__restrict__ plans, double *__restrict__ part) {
  constexpr int TB = 64 * R;
  constexpr int RS = R / SYM_SH;         // target sets per lane of a surface item
  constexpr float FAR_TARGET = 3.0e18f;  // stand-in position of an empty target lane
  const int b = __builtin_amdgcn_readfirstlane(sys_e[item]);
  const bool surface = item >= S.is[b];
  const int64_t lo = S.off[b];
  const int n = (int)(S.off[b + 1] - lo);
  const int64_t B = cdiv64(n, TB);
  double *pb = part + S.pe[b];
  const float4 *im = img + lo;
  if (surface) {
    // surface item: block I, node chunk c, target sets h RS .. h RS + RS - 1 of each lane
    const int64_t t = item - S.is[b];
    const int I = __builtin_amdgcn_readfirstlane((int)(t / (sch * SYM_SH)));
    const int rem = (int)(t % (sch * SYM_SH));
    const int c = __builtin_amdgcn_readfirstlane(rem / SYM_SH), h = __builtin_amdgcn_readfirstlane(rem % SYM_SH);
    const int t0 = I * TB + h * RS * 64;
    float sx[RS], sy[RS], sz[RS];
#pragma unroll
    for (int k = 0; k < RS; ++k) {
      const int i = t0 + k * 64 + lane;
      if (i < n) {
        const float4 tv = tgt[lo + i];
        sx[k] = tv.x;
        sy[k] = tv.y;
        sz[k] = tv.z;
      } else {
        sx[k] = FAR_TARGET;
        sy[k] = 0.0f;
        sz[k] = 0.0f;
      }
    }
    double acc[RS];
#pragma unroll
    for (int k = 0; k < RS; ++k) acc[k] = 0.0;
    const int per = (P + sch - 1) / sch;
    const int s0 = c * per, s1 = s0 + per < P ? s0 + per : P;
    const int pl = plan_of ? plan_of[b] : 0;
    const float4 *nd = nodes + (size_t)pl * P;
    const float2 *qb = qd + (size_t)b * P;
    if (dipole == 2)
      sym_surface<RS, true>(sx, sy, sz, nd, qb, s0, s1, acc);
    else if (dipole == 0)
      sym_surface<RS, false, true>(sx, sy, sz, nd, qb, s0, s1, acc, (float)(plans[pl].Rtau * plans[pl].Rtau));
    else
      sym_surface<RS, false>(sx, sy, sz, nd, qb, s0, s1, acc);
    const int64_t slot = B + c;
#pragma unroll
    for (int k = 0; k < RS; ++k) {
      const int i = t0 + k * 64 + lane;
      if (i < n) pb[(size_t)slot * n + i] = acc[k];
    }
    return;
  }
  int I, J;
  {
    // rows I = 0..B-1 of the triangle J = I..B-1 start at I B - I (I - 1) / 2
    const int64_t loc = item - S.ie[b];
    const double bb = 2.0 * (double)B + 1.0;
    int64_t r = (int64_t)((bb - sqrt(bb * bb - 8.0 * (double)loc)) * 0.5);
    r = r < 0 ? 0 : (r > B - 1 ? B - 1 : r);
    while (r > 0 && r * B - r * (r - 1) / 2 > loc) --r;
    while (r + 1 < B && (r + 1) * B - (r + 1) * r / 2 <= loc) ++r;
    I = (int)r;
    J = (int)(I + (loc - (r * B - r * (r - 1) / 2)));
  }
  I = __builtin_amdgcn_readfirstlane(I);
  J = __builtin_amdgcn_readfirstlane(J);
  const int t0 = I * TB;
  float tx[R], ty[R], tz[R], tw[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int i = t0 + k * 64 + lane;
    if (i < n) {
      const float4 t = tgt[lo + i];
      tx[k] = t.x;
      ty[k] = t.y;
      tz[k] = t.z;
      tw[k] = wk[lo + i];
    } else {
      tx[k] = FAR_TARGET;
      ty[k] = 0.0f;
      tz[k] = 0.0f;
      tw[k] = 0.0f;
    }
  }
  double acc[R];
#pragma unroll
  for (int k = 0; k < R; ++k) acc[k] = 0.0;
  int slot;
  {
    const int j0 = J * TB, j1 = j0 + TB < n ? j0 + TB : n;
    if (I == J) {
      // diagonal block: one-directional, the ion's own image excluded (it is the analytic term)
      for (int jb = j0; jb < j1; jb += TILE) {
        const int je = jb + TILE < j1 ? jb + TILE : j1;
        float sum[R];
#pragma unroll
        for (int k = 0; k < R; ++k) sum[k] = 0.0f;
        for (int j = jb; j < je; ++j) {
          const float4 v = im[j];
#pragma unroll
          for (int k = 0; k < R; ++k) {
            const float dx = tx[k] - v.x, dy = ty[k] - v.y, dz = tz[k] - v.z;
            float ri = rinv(dx * dx + dy * dy + dz * dz);
            ri = (j == t0 + k * 64 + lane) ? 0.0f : ri;
            sum[k] = fmaf(v.w, ri, sum[k]);
          }
        }
#pragma unroll
        for (int k = 0; k < R; ++k) acc[k] += (double)sum[k];
      }
    } else {
      for (int jg = j0; jg < j1; jg += 64) {
        const int ge = jg + 64 < j1 ? jg + 64 : j1;
        // Reverse totals of the group's sources: each source's total arrives in lane 63 and the
        // buffer moves down one lane per source (wave_shl:1, lane i reads lane i + 1), so after
        // the g = ge - jg sources lane 64 - g + t holds source jg + t.
        float rb = 0.0f;
        for (int jb = jg; jb < ge; jb += TILE) {
          const int je = jb + TILE < ge ? jb + TILE : ge;
          float sum[R];
#pragma unroll
          for (int k = 0; k < R; ++k) sum[k] = 0.0f;
          // Blocks of 512: two sources per step, in order (the same sums as one at a time), so
          // that their reductions interleave (C3 potentials 123.3 -> 120.1 ms, and 78 instead of
          // 85 VGPRs); blocks of 256 measured slower that way (C4 22.9 -> 23.5 ms) and take one.
          int j = jb;
          if constexpr (R >= 8)
            for (; j + 2 <= je; j += 2) {
              const float4 v0 = im[j], v1 = im[j + 1];
              float rev0 = sym_source<R>(v0, tx, ty, tz, tw, sum);
              float rev1 = sym_source<R>(v1, tx, ty, tz, tw, sum);
              rev0 = wave_total_lane63(rev0);
              rev1 = wave_total_lane63(rev1);
              rb = shift_in_lane63(rev0, rb);
              rb = shift_in_lane63(rev1, rb);
            }
          for (; j < je; ++j) rb = shift_in_lane63(wave_total_lane63(sym_source<R>(im[j], tx, ty, tz, tw, sum)), rb);
#pragma unroll
          for (int k = 0; k < R; ++k) acc[k] += (double)sum[k];
        }
        const int js = jg + lane - (64 - (ge - jg));
        if (js >= jg) pb[(size_t)I * n + js] = (double)rb * rk[lo + js];  // slot I of ion js
      }
    }
    slot = J;
  }
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int i = t0 + k * 64 + lane;
    if (i < n) pb[(size_t)slot * n + i] = acc[k];
  }
}

// The symmetric kernel: one item per wave (a block's waves take consecutive items), or the
// persistent form, whose waves take items EG at a time from their die's counter in the order of
// die_item until the die's items run out.  Every item writes the same slots either way.
template <int R, bool PERSIST>
__global__ __launch_bounds__(TPB) void k_kelvin_sym(int nsys, int P, int sch, int dipole,
                                                    const int64_t *__restrict__ base,
                                                    const int *__restrict__ sys_e, const int32_t *__restrict__ plan_of,
                                                    const float4 *__restrict__ tgt, const float4 *__restrict__ img,
                                                    const float *__restrict__ wk, const double *__restrict__ rk,
                                                    const float4 *__restrict__ nodes, const float2 *__restrict__ qd,
                                                    const PlanDev *__restrict__ plans, double *__restrict__ part) {
  Sched S(const_cast<int64_t *>(base), nsys);
  const int lane = threadIdx.x & 63, w = wave_id();
  if (!sched_ok(S)) return;
  const int64_t total = S.is[nsys];
  if constexpr (!PERSIST) {
    const int64_t item = uniform64((int64_t)blockIdx.x * WAVES + w);
    if (item < total) sym_item<R>(item, S, lane, P, sch, dipole, sys_e, plan_of, tgt, img, wk, rk, nodes, qd, plans, part);
  } else {
    const int64_t x = blockIdx.x % NXCD;
    for (;;) {
      int64_t t = 0;
      if (lane == 0) t = (int64_t)atomicAdd((unsigned long long *)&S.ctr[CTR_EVAL + x], (unsigned long long)EG);
      t = uniform64(__shfl(t, 0, 64));
      if (die_item(x, t) >= total) return;  // every later claim of this die lies beyond too
      for (int g = 0; g < EG; ++g) {
        const int64_t item = die_item(x, t + g);
        if (item < total) sym_item<R>(item, S, lane, P, sch, dipole, sys_e, plan_of, tgt, img, wk, rk, nodes, qd, plans, part);
      }
    }
  }
}

// The symmetric Kelvin sums in FP64 pairs: the same items, slots and identity as
// k_kelvin_sym, with FP64 positions, strengths and sums throughout.  A pair's reciprocal root
// (an FP32 seed and one FP64 Newton step) is the most expensive part of an FP64 pair, so the
// shared root nearly halves the work.  FP64 values cross lanes as two 32-bit DPP moves.
template <int CTRL, bool BOUND_ZERO>
__device__ __forceinline__ double dpp_move64(double old, double v) {
  const long long ov = __double_as_longlong(old), vv = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)ov, (int)vv, CTRL, 0xf, 0xf, BOUND_ZERO);
  const int hi = __builtin_amdgcn_update_dpp((int)(ov >> 32), (int)(vv >> 32), CTRL, 0xf, 0xf, BOUND_ZERO);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes, complete in lane 63 (the steps of wave_total_lane63).
__device__ __forceinline__ double wave_total_lane63_f64(double v) {
  v += dpp_move64<0x111, true>(0.0, v);  // row_shr:1
  v += dpp_move64<0x112, true>(0.0, v);  // row_shr:2
  v += dpp_move64<0x114, true>(0.0, v);  // row_shr:4
  v += dpp_move64<0x118, true>(0.0, v);  // row_shr:8
  v += dpp_move64<0x142, true>(0.0, v);  // row_bcast:15
  v += dpp_move64<0x143, true>(0.0, v);  // row_bcast:31
  return v;
}

template <int R>
__global__ __launch_bounds__(TPB) void k_kelvin_sym64(int nsys, int P, int sch, int mono,
                                                      const int64_t *__restrict__ base, const int *__restrict__ sys_e,
                                                      const int32_t *__restrict__ plan_of,
                                                      const double4 *__restrict__ tgt, const double4 *__restrict__ img,
                                                      const double *__restrict__ wk, const double *__restrict__ rk,
                                                      const double4 *__restrict__ nodes,
                                                      const double2 *__restrict__ qd, double *__restrict__ part) {
  constexpr int TB = 64 * R;
  constexpr int RS = R / SYM_SH;
  constexpr double FAR_TARGET = 3.0e18;
  Sched S(const_cast<int64_t *>(base), nsys);
  const int lane = threadIdx.x & 63, w = wave_id();
  if (!sched_ok(S)) return;
  const int64_t item = uniform64((int64_t)blockIdx.x * WAVES + w);
  if (item >= S.is[nsys]) return;
  const int b = __builtin_amdgcn_readfirstlane(sys_e[item]);
  const bool surface = item >= S.is[b];
  const int64_t lo = S.off[b];
  const int n = (int)(S.off[b + 1] - lo);
  const int64_t B = cdiv64(n, TB);
  double *pb = part + S.pe[b];
  const double4 *im = img + lo;
  if (surface) {
    const int64_t t = item - S.is[b];
    const int I = __builtin_amdgcn_readfirstlane((int)(t / (sch * SYM_SH)));
    const int rem = (int)(t % (sch * SYM_SH));
    const int c = __builtin_amdgcn_readfirstlane(rem / SYM_SH), h = __builtin_amdgcn_readfirstlane(rem % SYM_SH);
    const int t0 = I * TB + h * RS * 64;
    double sx[RS], sy[RS], sz[RS], acc[RS];
#pragma unroll
    for (int k = 0; k < RS; ++k) {
      const int i = t0 + k * 64 + lane;
      const double4 tv = i < n ? tgt[lo + i] : make_double4(FAR_TARGET, 0.0, 0.0, 0.0);
      sx[k] = tv.x;
      sy[k] = tv.y;
      sz[k] = tv.z;
      acc[k] = 0.0;
    }
    const int per = (P + sch - 1) / sch;
    const int s0 = c * per, s1 = s0 + per < P ? s0 + per : P;
    const int pl = plan_of ? plan_of[b] : 0;
    const double4 *nd = nodes + (size_t)pl * P;
    const double2 *qb = qd + (size_t)b * P;
    for (int m = s0; m < s1; ++m) {
      const double4 yv = nd[m];
      const double2 wv = qb[m];
#pragma unroll
      for (int k = 0; k < RS; ++k) {
        const double dx = sx[k] - yv.x, dy = sy[k] - yv.y, dz = sz[k] - yv.z;
        const double ri = rinv(dx * dx + dy * dy + dz * dz);
        if (mono) {
          acc[k] = fma(wv.x, ri, acc[k]);
        } else {
          const double dot = dx * yv.x + dy * yv.y + dz * yv.z;
          acc[k] = fma(ri, fma(wv.y * dot, ri * ri, wv.x), acc[k]);
        }
      }
    }
    const int64_t slot = B + c;
#pragma unroll
    for (int k = 0; k < RS; ++k) {
      const int i = t0 + k * 64 + lane;
      if (i < n) pb[(size_t)slot * n + i] = acc[k];
    }
    return;
  }
  int I, J;
  {
    const int64_t loc = item - S.ie[b];
    const double bb = 2.0 * (double)B + 1.0;
    int64_t r = (int64_t)((bb - sqrt(bb * bb - 8.0 * (double)loc)) * 0.5);
    r = r < 0 ? 0 : (r > B - 1 ? B - 1 : r);
    while (r > 0 && r * B - r * (r - 1) / 2 > loc) --r;
    while (r + 1 < B && (r + 1) * B - (r + 1) * r / 2 <= loc) ++r;
    I = (int)r;
    J = (int)(I + (loc - (r * B - r * (r - 1) / 2)));
  }
  I = __builtin_amdgcn_readfirstlane(I);
  J = __builtin_amdgcn_readfirstlane(J);
  const int t0 = I * TB;
  double tx[R], ty[R], tz[R], tw[R], acc[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int i = t0 + k * 64 + lane;
    const bool in = i < n;
    const double4 t = in ? tgt[lo + i] : make_double4(FAR_TARGET, 0.0, 0.0, 0.0);
    tx[k] = t.x;
    ty[k] = t.y;
    tz[k] = t.z;
    tw[k] = in ? wk[lo + i] : 0.0;
    acc[k] = 0.0;
  }
  const int j0 = J * TB, j1 = j0 + TB < n ? j0 + TB : n;
  if (I == J) {
    // diagonal block: one-directional, the ion's own image excluded (it is the analytic term)
    for (int j = j0; j < j1; ++j) {
      const double4 v = im[j];
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const double dx = tx[k] - v.x, dy = ty[k] - v.y, dz = tz[k] - v.z;
        double ri = rinv(dx * dx + dy * dy + dz * dz);
        ri = (j == t0 + k * 64 + lane) ? 0.0 : ri;
        acc[k] = fma(v.w, ri, acc[k]);
      }
    }
  } else {
    for (int jg = j0; jg < j1; jg += 64) {
      const int ge = jg + 64 < j1 ? jg + 64 : j1;
      double rb = 0.0;  // reverse totals, moved down one lane per source as in k_kelvin_sym
      for (int j = jg; j < ge; ++j) {
        const double4 v = im[j];
        double rev = 0.0;
#pragma unroll
        for (int k = 0; k < R; ++k) {
          const double dx = tx[k] - v.x, dy = ty[k] - v.y, dz = tz[k] - v.z;
          const double ri = rinv(dx * dx + dy * dy + dz * dz);
          acc[k] = fma(v.w, ri, acc[k]);
          rev = fma(tw[k], ri, rev);
        }
        rev = wave_total_lane63_f64(rev);
        rb = dpp_move64<0x130, false>(rev, rb);  // wave_shl:1; lane 63 keeps the new total
      }
      const int js = jg + lane - (64 - (ge - jg));
      if (js >= jg) pb[(size_t)I * n + js] = rb * rk[lo + js];  // slot I of ion js
    }
  }
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int i = t0 + k * 64 + lane;
    if (i < n) pb[(size_t)J * n + i] = acc[k];
  }
}

// ---------------------------------------------------------------------------------
// Energy sums in FP64 pairs, without potentials.  E = 1/2 sum_i q_i Phi_i is a bilinear form
// in the charges, so a block pair needs no per-ion output: with the image identity above,
// the two ordered terms of an ion pair share one reciprocal root y = 1/|x_i - r_K,j|,
//   q_i q'_j / |x_i - r_K,j| + q_j q'_i / |x_j - r_K,i| = y (q_i q'_j + (q'_i r_i)(q_j / r_j)),
// so a lane keeps two sums per target, S1 = sum_j q'_j y and S2 = sum_j (q_j / r_j) y, and the
// item's energy is sum_i (q_i S1_i + q'_i r_i S2_i), reduced over the wave in a fixed order
// and written to the item's own slot.  Diagonal blocks sum every ordered pair j != i; surface
// items sum q_i times the node potentials.  Every value is FP64; the reciprocal root is the
// hardware FP64 estimate refined by one Newton step.
// ---------------------------------------------------------------------------------
// Block pair (I, J), I <= J, of item number loc within a system's triangle of B blocks:
// rows I = 0..B-1 of the triangle J = I..B-1 start at I B - I (I - 1) / 2.
__device__ __forceinline__ void block_pair(int64_t loc, int64_t B, int &I, int &J) {
  const double bb = 2.0 * (double)B + 1.0;
  int64_t r = (int64_t)((bb - sqrt(bb * bb - 8.0 * (double)loc)) * 0.5);
  r = r < 0 ? 0 : (r > B - 1 ? B - 1 : r);
  while (r > 0 && r * B - r * (r - 1) / 2 > loc) --r;
  while (r + 1 < B && (r + 1) * B - (r + 1) * r / 2 <= loc) ++r;
  I = __builtin_amdgcn_readfirstlane((int)r);
  J = __builtin_amdgcn_readfirstlane((int)(r + (loc - (r * B - r * (r - 1) / 2))));
}

// The energy kernel's expanded pair form: per source (-2x/a, -2y/a, -2z/a, (r/a)^2) and the two
// weights, the plans (for 1/a of the targets), and per system the count of its ions far from the
// interface (packed first).
struct EnergyExt {
  const double4 *emx;
  const double2 *ew;
  const PlanDev *plans;
  const int64_t *nfar;
};

template <int R>
__device__ __forceinline__ void energy_item(int64_t item, int nsys, int P, int sch, int mono, const Sched &S, int lane,
                                            const int *__restrict__ sys_e, const int32_t *__restrict__ plan_of,
                                            const double4 *__restrict__ tgt, const double4 *__restrict__ img,
                                            const double *__restrict__ q, const double *__restrict__ wk,
                                            const double *__restrict__ qr, const double4 *__restrict__ nodes,
                                            const double2 *__restrict__ qd, double *__restrict__ epair,
                                            const EnergyExt ex);

// The launch bound caps the registers at five waves per SIMD (two for blocks of 512 ions): both
// the unbounded kernel and caps of six or seven waves measured slower.
template <int R, bool PERSIST>
__global__ __launch_bounds__(TPB, (R == 8 ? 2 : 5)) void k_energy64(
    int nsys, int P, int sch, int mono, const int64_t *__restrict__ base, const int *__restrict__ sys_e,
    const int32_t *__restrict__ plan_of, const double4 *__restrict__ tgt, const double4 *__restrict__ img,
    const double *__restrict__ q, const double *__restrict__ wk, const double *__restrict__ qr,
    const double4 *__restrict__ nodes, const double2 *__restrict__ qd, double *__restrict__ epair,
    const EnergyExt ex) {
  Sched S(const_cast<int64_t *>(base), nsys);
  const int lane = threadIdx.x & 63, w = wave_id();
  if (!sched_ok(S)) return;
  const int64_t total = S.is[nsys];
  if constexpr (!PERSIST) {  // one item per wave
    const int64_t item = uniform64(xcd_item(w));
    if (item < total)
      energy_item<R>(item, nsys, P, sch, mono, S, lane, sys_e, plan_of, tgt, img, q, wk, qr, nodes, qd, epair, ex);
    return;
  } else {
  // persistent: claims of EG items from this die's counter until the die's items run out
  const int64_t x = blockIdx.x % NXCD;
  for (;;) {
    int64_t t = 0;
    if (lane == 0) t = (int64_t)atomicAdd((unsigned long long *)&S.ctr[CTR_ENERGY + x], (unsigned long long)EG);
    t = uniform64(__shfl(t, 0, 64));
    if (die_item(x, t) >= total) return;  // every later claim of this die lies beyond too
    for (int g = 0; g < EG; ++g) {
      const int64_t item = die_item(x, t + g);
      if (item < total)
        energy_item<R>(item, nsys, P, sch, mono, S, lane, sys_e, plan_of, tgt, img, q, wk, qr, nodes, qd, epair,
                       ex);
    }
  }
  }
}

// One item of the energy kernels (block pair or surface item); writes epair[item].
template <int R>
__device__ __forceinline__ void energy_item(int64_t item, int nsys, int P, int sch, int mono, const Sched &S,
                                            int lane, const int *__restrict__ sys_e,
                                            const int32_t *__restrict__ plan_of, const double4 *__restrict__ tgt,
                                            const double4 *__restrict__ img, const double *__restrict__ q,
                                            const double *__restrict__ wk, const double *__restrict__ qr,
                                            const double4 *__restrict__ nodes, const double2 *__restrict__ qd,
                                            double *__restrict__ epair, const EnergyExt ex) {
  constexpr int TB = 64 * R;
  constexpr int RS = R / SYM_SH;
  constexpr double FAR_TARGET = 3.0e18;  // stand-in position of an empty target lane (zero charge)
  const int b = __builtin_amdgcn_readfirstlane(sys_e[item]);
  const bool surface = item >= S.is[b];
  const int64_t lo = S.off[b];
  const int n = (int)(S.off[b + 1] - lo);
  double e = 0.0;
  if (surface) {
    // half of block I's ions (target sets h RS .. h RS + RS - 1 of each lane) against node chunk c
    const int64_t t = item - S.is[b];
    const int I = __builtin_amdgcn_readfirstlane((int)(t / (sch * SYM_SH)));
    const int rem = (int)(t % (sch * SYM_SH));
    const int c = __builtin_amdgcn_readfirstlane(rem / SYM_SH), h = __builtin_amdgcn_readfirstlane(rem % SYM_SH);
    const int t0 = I * TB + h * RS * 64;
    const int per = (P + sch - 1) / sch;
    const int s0 = c * per, s1 = s0 + per < P ? s0 + per : P;
    const int pl = plan_of ? plan_of[b] : 0;
    const double4 *nd = nodes + (size_t)pl * P;
    const double2 *qb = qd + (size_t)b * P;
    const double Rt = ex.plans[pl].Rtau, R2 = Rt * Rt;
    // Every node on the sphere R_tau (not the point-pair form) with R_tau >= 1.05 a: |x - y|^2 =
    // |x|^2 + R_tau^2 - 2 x.y, three FMAs from the target's -2x and |x|^2 + R_tau^2.  D >=
    // (R_tau - a)^2 >= 0.0025 a^2 there, so it rounds to about 1e-12 relative.  The dipole's
    // (x - y).y = (|x|^2 - R_tau^2 - D)/2, so with r = 2/sqrt(D) (rinv2, D r^2 = 4 up to the Newton
    // step's 1e-14) twice its term is w_d ((|x|^2 - R_tau^2)/8 r^3 - r/2): two sums over the
    // nodes per target, both terms of one sign (|x| < R_tau), the first scaled once at the end.
    // Otherwise the exact differences.  Monopole-only and dipole loops are separate.
    const bool sexp = ex.plans[pl].dipole != 1 && Rt >= SURF_EXPANDED * ex.plans[pl].a;
    double f0[RS], f1[RS], f2[RS], f3[RS], f4[RS], sq[RS], acc[RS], acc3[RS], acc1[RS];
#pragma unroll
    for (int k = 0; k < RS; ++k) {
      const int i = t0 + k * 64 + lane;
      const bool in = i < n;
      // an empty lane: zero charge, at the origin (expanded) or far away
      const double4 tv = in ? tgt[lo + i] : make_double4(sexp ? 0.0 : FAR_TARGET, 0.0, 0.0, 0.0);
      const double xx = fma(tv.x, tv.x, fma(tv.y, tv.y, tv.z * tv.z));
      f0[k] = sexp ? -2.0 * tv.x : tv.x;
      f1[k] = sexp ? -2.0 * tv.y : tv.y;
      f2[k] = sexp ? -2.0 * tv.z : tv.z;
      f3[k] = xx + R2;
      f4[k] = 0.125 * (xx - R2);
      sq[k] = in ? q[lo + i] : 0.0;
      acc[k] = 0.0;
      acc3[k] = 0.0;
      acc1[k] = 0.0;
    }
    if (sexp) {
      // the sums hold twice the terms (rinv2)
      if (mono) {
#pragma unroll 2
        for (int m = s0; m < s1; ++m) {
          const double4 yv = nd[m];
          const double wx = qb[m].x;
#pragma unroll
          for (int k = 0; k < RS; ++k)
            acc[k] = fma(wx, rinv2(fma(f0[k], yv.x, fma(f1[k], yv.y, fma(f2[k], yv.z, f3[k])))), acc[k]);
        }
      } else {
#pragma unroll 2
        for (int m = s0; m < s1; ++m) {
          const double4 yv = nd[m];
          const double2 wv = qb[m];
#pragma unroll
          for (int k = 0; k < RS; ++k) {
            const double ri = rinv2(fma(f0[k], yv.x, fma(f1[k], yv.y, fma(f2[k], yv.z, f3[k]))));
            acc[k] = fma(wv.x, ri, acc[k]);
            acc3[k] = fma(wv.y, ri * ri * ri, acc3[k]);
            acc1[k] = fma(wv.y, ri, acc1[k]);
          }
        }
#pragma unroll
        for (int k = 0; k < RS; ++k) acc[k] = fma(f4[k], acc3[k], fma(-0.5, acc1[k], acc[k]));
      }
#pragma unroll
      for (int k = 0; k < RS; ++k) e = fma(sq[k], acc[k], e);
      e *= 0.5;
    } else {
      if (mono) {
        for (int m = s0; m < s1; ++m) {
          const double4 yv = nd[m];
          const double wx = qb[m].x;
#pragma unroll
          for (int k = 0; k < RS; ++k) {
            const double dx = f0[k] - yv.x, dy = f1[k] - yv.y, dz = f2[k] - yv.z;
            acc[k] = fma(wx, rinv(dx * dx + dy * dy + dz * dz), acc[k]);
          }
        }
      } else {
        for (int m = s0; m < s1; ++m) {
          const double4 yv = nd[m];
          const double2 wv = qb[m];
#pragma unroll
          for (int k = 0; k < RS; ++k) {
            const double dx = f0[k] - yv.x, dy = f1[k] - yv.y, dz = f2[k] - yv.z;
            const double ri = rinv(dx * dx + dy * dy + dz * dz);
            const double dot = dx * yv.x + dy * yv.y + dz * yv.z;
            acc[k] = fma(ri, fma(wv.y * dot, ri * ri, wv.x), acc[k]);
          }
        }
      }
#pragma unroll
      for (int k = 0; k < RS; ++k) e = fma(sq[k], acc[k], e);
    }
  } else {
    const int64_t B = cdiv64(n, TB), sup = super_of(B), loc = item - S.ie[b];
    int I, J;
    if (sup == 1) {
      block_pair(loc, B, I, J);
    } else {
      int SI, SJ;
      block_pair(loc / (sup * sup), cdiv64(B, sup), SI, SJ);
      const int wi = (int)(loc % (sup * sup));
      I = SI * (int)sup + wi / (int)sup;
      J = SJ * (int)sup + wi % (int)sup;
      if (I >= B || J >= B || J < I) {  // a slot of the tile outside the triangle: no pairs
        if (lane == 0) epair[item] = 0.0;
        return;
      }
    }
    const int t0 = I * TB;
    double tx[R], ty[R], tz[R], s1[R], s2[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int i = t0 + k * 64 + lane;
      const double4 t = i < n ? tgt[lo + i] : make_double4(FAR_TARGET, 0.0, 0.0, 0.0);
      tx[k] = t.x;
      ty[k] = t.y;
      tz[k] = t.z;
      s1[k] = 0.0;
      s2[k] = 0.0;
    }
    const double4 *im = img + lo;
    const int j0 = J * TB, j1 = j0 + TB < n ? j0 + TB : n;
    // the sums hold twice the pair terms (rinv2); halved once at the end
    if (R == 8 && I == J) {
      // diagonal block of 512 ions: every ordered pair j != i, one direction (registers)
      for (int j = j0; j < j1; ++j) {
        const double4 v = im[j];
#pragma unroll
        for (int k = 0; k < R; ++k) {
          const double dx = tx[k] - v.x, dy = ty[k] - v.y, dz = tz[k] - v.z;
          double ri = rinv2(dx * dx + dy * dy + dz * dz);
          ri = (j == t0 + k * 64 + lane) ? 0.0 : ri;
          s1[k] = fma(v.w, ri, s1[k]);
        }
      }
    } else if (I == J) {
      // Diagonal block: each unordered pair j > i once, both directions through the symmetric
      // identity as in the off-diagonal blocks (the own image is the analytic term).  Sources in
      // runs of 64: run jb meets the target rows k <= jb, all of whose pairs count for k < jb and
      // those with j > i for k = jb.  A block wholly below n_far takes the expanded form.
      if ((int64_t)j1 <= ex.nfar[b]) {
        const double ia = 1.0 / ex.plans[plan_of ? plan_of[b] : 0].a;
        double uu[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
          tx[k] *= ia;
          ty[k] *= ia;
          tz[k] *= ia;
          uu[k] = fma(tx[k], tx[k], fma(ty[k], ty[k], tz[k] * tz[k]));
        }
        const double4 *em = ex.emx + lo;
        const double2 *ewt = ex.ew + lo;
#pragma unroll
        for (int jb = 0; jb < R; ++jb) {
          const int js = j0 + 64 * jb, je = js + 64 < j1 ? js + 64 : j1;
          for (int j = js; j < je; ++j) {
            const double4 m = em[j];
            const double2 wj = ewt[j];
#pragma unroll
            for (int k = 0; k <= jb; ++k) {
              double ri = rinv2(fma(tx[k], m.x, fma(ty[k], m.y, fma(tz[k], m.z, fma(uu[k], m.w, 1.0)))));
              if (k == jb) ri = j > t0 + k * 64 + lane ? ri : 0.0;
              s1[k] = fma(wj.x, ri, s1[k]);
              s2[k] = fma(wj.y, ri, s2[k]);
            }
          }
        }
      } else {
        const double *cr = qr + lo;
#pragma unroll
        for (int jb = 0; jb < R; ++jb) {
          const int js = j0 + 64 * jb, je = js + 64 < j1 ? js + 64 : j1;
          for (int j = js; j < je; ++j) {
            const double4 v = im[j];
            const double cj = cr[j];
#pragma unroll
            for (int k = 0; k <= jb; ++k) {
              const double dx = tx[k] - v.x, dy = ty[k] - v.y, dz = tz[k] - v.z;
              double ri = rinv2(dx * dx + dy * dy + dz * dz);
              if (k == jb) ri = j > t0 + k * 64 + lane ? ri : 0.0;
              s1[k] = fma(v.w, ri, s1[k]);
              s2[k] = fma(cj, ri, s2[k]);
            }
          }
        }
      }
    } else {
      // Off-diagonal block, in units of a.  When every target of block I lies at r_i <= NEAR_R a
      // (the energy launch packs the ions nearer the interface last, so then do all ions before
      // them), the squared image distance times (r_j/a)^2 is expanded,
      // D = (r_i/a)^2 (r_j/a)^2 + 1 - 2 (x_i/a).(x_j/a) (the identity behind the symmetric form),
      // and 1/|x_i - r_K,j| = (r_j/a^2) D^-1/2 with r_j/a^2 folded into the weights: four
      // operations instead of six.  D >= (1 - r_i r_j/a^2)^2 >= (1 - r_i/a)^2 >= 2.5e-5 there
      // (r_j <= a), so its rounding stays within a few 1e-11 relative.  Only pairs of two ions
      // near the interface take the differences x_i/a - r_K,j/a, with 1/a joining their weights.
      const double ia = 1.0 / ex.plans[plan_of ? plan_of[b] : 0].a;
#pragma unroll
      for (int k = 0; k < R; ++k) {
        tx[k] *= ia;
        ty[k] *= ia;
        tz[k] *= ia;
      }
      if ((int64_t)(t0 + TB) <= ex.nfar[b]) {
        const double4 *em = ex.emx + lo;
        const double2 *ewt = ex.ew + lo;
        double uu[R];
#pragma unroll
        for (int k = 0; k < R; ++k) uu[k] = fma(tx[k], tx[k], fma(ty[k], ty[k], tz[k] * tz[k]));
        for (int j = j0; j < j1; ++j) {
          const double4 m = em[j];
          const double2 wj = ewt[j];
#pragma unroll
          for (int k = 0; k < R; ++k) {
            const double d = fma(tx[k], m.x, fma(ty[k], m.y, fma(tz[k], m.z, fma(uu[k], m.w, 1.0))));
            const double ri = rinv2(d);
            s1[k] = fma(wj.x, ri, s1[k]);
            s2[k] = fma(wj.y, ri, s2[k]);
          }
        }
      } else {
        const double *cr = qr + lo;
        for (int j = j0; j < j1; ++j) {
          const double4 v = im[j];
          const double vx = v.x * ia, vy = v.y * ia, vz = v.z * ia, w1 = v.w * ia, w2 = cr[j] * ia;
#pragma unroll
          for (int k = 0; k < R; ++k) {
            const double dx = tx[k] - vx, dy = ty[k] - vy, dz = tz[k] - vz;
            const double ri = rinv2(dx * dx + dy * dy + dz * dz);
            s1[k] = fma(w1, ri, s1[k]);
            s2[k] = fma(w2, ri, s2[k]);
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int i = t0 + k * 64 + lane;
      if (i < n) e = fma(q[lo + i], s1[k], fma(wk[lo + i], s2[k], e));
    }
    e *= 0.5;
  }
  e = wave_sum(e);
  if (lane == 0) epair[item] = e;
}

// Fixed-order sums of the item energies: chunk f of system b holds EC consecutive items of its
// block pairs, or of its surface items after those; 256 threads sum them lane-strided and by a
// tree.
__global__ __launch_bounds__(256) void k_energy_chunks(int nsys, int P, int sym_tb, int sch,
                                                       const int64_t *__restrict__ base,
                                                       const double *__restrict__ epair, double *__restrict__ echunk) {
  Sched S(const_cast<int64_t *>(base), nsys);
  __shared__ double red[256];
  const int64_t f = blockIdx.x;
  if (!sched_ok(S) || f >= S.ec[nsys]) return;  // uniform across the block
  const int b = system_of(S.ec, nsys, f);
  const int64_t n = S.off[b + 1] - S.off[b];
  int64_t pairs, surf, parts;
  eval_counts(n, P, 0, sym_tb, sch, pairs, surf, parts, true);
  const int64_t k = f - S.ec[b], cp = cdiv64(pairs, EC);
  const int64_t first = k < cp ? S.ie[b] + k * EC : S.is[b] + (k - cp) * EC;
  const int64_t end = k < cp ? S.ie[b] + pairs : S.is[b] + surf;
  const int64_t last = first + EC < end ? first + EC : end;
  double s = 0.0;
  for (int64_t i = first + threadIdx.x; i < last; i += 256) s += epair[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) echunk[f] = red[0];
}

// E_b = (own-image block partials, 1/2 included) + 1/2 (sum of system b's chunk sums), each
// lane-strided and reduced by a shuffle tree.
__global__ __launch_bounds__(64) void k_energy_items(int nsys, const int64_t *__restrict__ base,
                                                     const double *__restrict__ epart,
                                                     const double *__restrict__ echunk, double *__restrict__ E) {
  Sched S(const_cast<int64_t *>(base), nsys);
  if (!sched_ok(S)) return;
  const int b = blockIdx.x;
  double s = 0.0, t = 0.0;
  for (int64_t f = S.fb[b] + threadIdx.x; f < S.fb[b + 1]; f += 64) s += epart[f];
  for (int64_t f = S.ec[b] + threadIdx.x; f < S.ec[b + 1]; f += 64) t += echunk[f];
  s = wave_sum(s);
  t = wave_sum(t);
  if (threadIdx.x == 0) E[b] = s + 0.5 * t;
}

// Block partials of 1/2 sum_i q_i self_i (the own-image energy), for the energy-only path.
__global__ __launch_bounds__(FINB) void k_self_energy(int nsys, const int64_t *__restrict__ base,
                                                      const int *__restrict__ sys_f, const double *__restrict__ self,
                                                      const double *__restrict__ q, double *__restrict__ epart) {
  Sched S(const_cast<int64_t *>(base), nsys);
  __shared__ double red[FINB];
  const int64_t f = blockIdx.x;
  if (!sched_ok(S) || f >= S.fb[nsys]) return;  // uniform across the block
  const int b = sys_f[f];
  const int64_t lo = S.off[b], n = S.off[b + 1] - lo;
  const int64_t il = (f - S.fb[b]) * FINB + threadIdx.x;
  red[threadIdx.x] = il < n ? 0.5 * q[lo + il] * self[lo + il] : 0.0;
  __syncthreads();
  for (int o = FINB / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) epart[f] = red[0];
}

// Phi_i = own-image term + fixed-order sum of the chunk partials; block partial of 1/2 sum q Phi.
__global__ __launch_bounds__(FINB) void k_finish(int nsys, int P, int che, int sym_tb, int sch,
                                                 const int64_t *__restrict__ base,
                                                 const int *__restrict__ sys_f, const double *__restrict__ part,
                                                 const double *__restrict__ self, const double *__restrict__ q,
                                                 double *__restrict__ phi, double *__restrict__ epart) {
  Sched S(const_cast<int64_t *>(base), nsys);
  __shared__ double red[FINB];
  const int64_t f = blockIdx.x;
  if (!sched_ok(S) || f >= S.fb[nsys]) return;  // uniform across the block
  const int b = sys_f[f];
  const int64_t lo = S.off[b], n = S.off[b + 1] - lo;
  const int64_t il = (f - S.fb[b]) * FINB + threadIdx.x;
  double e = 0.0;
  if (il < n) {
    double s = self[lo + il];
    if (sym_tb > 0) {  // one slot per partner block, then the surface chunks: slot K of ion i at K * n + i
      const int slots = (int)(cdiv64(n, sym_tb) + sch);
      const double *pp = part + S.pe[b] + il;
#pragma unroll 8
      for (int k = 0; k < slots; ++k) s += pp[(int64_t)k * n];
    } else {
      const int64_t chunks = cdiv64(n + P, che);
      const int64_t g = il / GRP, lane = il % GRP;
      const double *pp = part + S.pe[b] + g * chunks * GRP + lane;
#pragma unroll 8
      for (int64_t c = 0; c < chunks; ++c) s += pp[c * GRP];
    }
    phi[lo + il] = s;
    e = 0.5 * q[lo + il] * s;
  }
  red[threadIdx.x] = e;
  __syncthreads();
  for (int o = FINB / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) epart[f] = red[0];
}

// Phi_i and E_i = own-image terms + fixed-order sums of the chunk partials (one-directional
// evaluation items); block partial of 1/2 sum q Phi.
__global__ __launch_bounds__(FINB) void k_finish_field(int nsys, int P, int che, const int64_t *__restrict__ base,
                                                       const int *__restrict__ sys_f,
                                                       const double4 *__restrict__ part,
                                                       const double *__restrict__ self,
                                                       const double4 *__restrict__ sfield,
                                                       const double *__restrict__ q, double *__restrict__ phi,
                                                       double *__restrict__ ex, double *__restrict__ ey,
                                                       double *__restrict__ ez, double *__restrict__ epart) {
  Sched S(const_cast<int64_t *>(base), nsys);
  __shared__ double red[FINB];
  const int64_t f = blockIdx.x;
  if (!sched_ok(S) || f >= S.fb[nsys]) return;  // uniform across the block
  const int b = sys_f[f];
  const int64_t lo = S.off[b], n = S.off[b + 1] - lo;
  const int64_t il = (f - S.fb[b]) * FINB + threadIdx.x;
  double e = 0.0;
  if (il < n) {
    const double4 sf = sfield[lo + il];
    double sp = self[lo + il], sx = sf.x, sy = sf.y, sz = sf.z;
    const int64_t chunks = cdiv64(n + P, che);
    const int64_t g = il / GRP, lane = il % GRP;
    const double4 *pp = part + S.pe[b] + g * chunks * GRP + lane;
#pragma unroll 4
    for (int64_t c = 0; c < chunks; ++c) {
      const double4 v = pp[c * GRP];
      sp += v.x;
      sx += v.y;
      sy += v.z;
      sz += v.w;
    }
    phi[lo + il] = sp;
    ex[lo + il] = sx;
    ey[lo + il] = sy;
    ez[lo + il] = sz;
    e = 0.5 * q[lo + il] * sp;
  }
  red[threadIdx.x] = e;
  __syncthreads();
  for (int o = FINB / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) epart[f] = red[0];
}

// E_b = sum of the block partials of system b, lane-strided then a shuffle tree (fixed order).
__global__ __launch_bounds__(64) void k_energy(int nsys, const int64_t *__restrict__ base,
                                               const double *__restrict__ epart, double *__restrict__ E) {
  Sched S(const_cast<int64_t *>(base), nsys);
  if (!sched_ok(S)) return;
  const int b = blockIdx.x;
  double s = 0.0;
  for (int64_t f = S.fb[b] + threadIdx.x; f < S.fb[b + 1]; f += 64) s += epart[f];
  s = wave_sum(s);
  if (threadIdx.x == 0) E[b] = s;
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
inline int round_up(int64_t v, int m) { return (int)((v + m - 1) / m * m); }

template <int MODE>
hsma_status launch(hsma_group_s *grp, const Layout &L, const int64_t *offsets, const int32_t *plan_of, int64_t n1,
                   const double *x, const double *y, const double *z, const double *q, double *phi, double *E,
                   double *ex, double *ey, double *ez, char *ws, hipStream_t st) {
  using T = typename PT<MODE>::T;
  using T2 = typename PT<MODE>::T2;
  using T4 = typename PT<MODE>::T4;
  const Geometry *g = grp->geo;
  const int M = g->M, P = g->P, K = g->K, nsys = L.nsys;
  const int Pe = grp->P_ev;  // surface sources of the evaluation
  int64_t *base = (int64_t *)(ws + L.sched);
  int *sys_c = (int *)(ws + L.item_sys_c);
  int *sys_e = (int *)(ws + L.item_sys_e);
  int *sys_f = (int *)(ws + L.fin_sys);
  T4 *img = (T4 *)(ws + L.img);
  T4 *tgt = (T4 *)(ws + L.tgt);
  T *srcw = (T *)(ws + L.srcw);
  double *self = (double *)(ws + L.self);
  double *chk_part = (double *)(ws + L.chk_part);
  double *uv = (double *)(ws + L.uv);
  float *uv32 = L.mfma ? (float *)(ws + L.uv32) : nullptr;
  double *ab = (double *)(ws + L.ab);
  T2 *qd = (T2 *)(ws + L.qd);
  double *eval_part = (double *)(ws + L.eval_part);
  double *epart = (double *)(ws + L.epart);
  const PlanDev *plans = grp->dev;
  const int persistent = grp->tune.persistent;
  const int64_t pgrid_c = (int64_t)g->ncu * grp->tune.occ_check, pgrid_e = (int64_t)g->ncu * grp->tune.occ_eval;
  // an energy launch on a limited grid (tune.ewaves) runs its check sums persistent on that grid too
  const bool throttle = L.eonly && grp->tune.ewaves > 0;
  const int persistent_c = persistent || throttle;
  const int64_t cap_c = throttle ? (int64_t)grp->tune.ewaves : pgrid_c;
  // persistent grids: resident blocks, at most one per item, a multiple of the die count
  const int64_t grid_c = persistent_c ? round_up(L.items_c < cap_c ? L.items_c : cap_c, NXCD) : L.items_c;
  const int64_t grid_e = persistent ? round_up(L.items_e < pgrid_e ? L.items_e : pgrid_e, NXCD) : L.items_e;

  hipEvent_t pr = prof_begin(grp, ST_PACK, st);
  const int sched_t = nsys >= SCHED_T ? SCHED_T : (int)((nsys + 63) / 64 * 64);
  Bounds bd;
  bd.total_n = n1;
  bd.max_n = L.max_n;
  bd.items_c = L.items_c;
  bd.items_e = L.items_e;
  bd.fin = L.fin;
  bd.parts_c = L.parts_c;
  bd.parts_e = L.parts_e;
  bd.echunks = L.eonly ? L.echunks : INT64_MAX;  // only energy-only launches store the chunk sums
  bd.nplans = grp->nplans;
  // symmetric kernel: surface items last when the block pairs fill at most SYM_TAIL_ROUNDS
  // rounds of the device's resident waves
  const int64_t sym_tail = grp->tune.sym_order == 1 ? -1
                           : grp->tune.sym_order == 2
                               ? INT64_MAX
                               : SYM_TAIL_ROUNDS * g->ncu * WAVES * grp->tune.occ_sym[L.sym_tb == 512];
  k_schedule<<<1, sched_t, 0, st>>>(nsys, offsets, plan_of, bd, M, Pe, L.chc, L.che, L.sym_tb, L.sch, sym_tail,
                                    (L.eonly ? 1 : 0) + 16 * L.prec, base, grp->flag);
  if (L.eonly && L.fin > 0) {  // the energy launch packs the ions near the interface last
    k_near_count<<<(int)L.fin, FINB, 0, st>>>(nsys, base, plans, plan_of, x, y, z, (int *)(ws + L.ncnt));
    k_near_scan<<<nsys, 256, 0, st>>>(nsys, base, (const int *)(ws + L.ncnt), (int64_t *)(ws + L.farst),
                                      (int64_t *)(ws + L.nearst), (int64_t *)(ws + L.nfar));
  }
  if (L.fin > 0)
    k_pack<MODE><<<(int)L.fin, 256, 0, st>>>(nsys, base, sys_c, sys_e, sys_f, plans, plan_of, x, y, z, q, img, tgt,
                                             srcw, self,
                                             (T *)(ws + L.wk), (double *)(ws + L.rk),
                                             L.eonly ? (double *)(ws + L.qr) : nullptr,
                                             L.eonly ? (double4 *)(ws + L.emx) : nullptr,
                                             L.eonly ? (double2 *)(ws + L.ew) : nullptr,
                                             L.eonly ? (CheckSrc *)(ws + L.csrc) : nullptr,
                                             L.eonly ? (const int64_t *)(ws + L.farst) : nullptr,
                                             L.eonly ? (const int64_t *)(ws + L.nearst) : nullptr,
                                             L.eonly ? (double *)(ws + L.qpk) : nullptr,
                                             L.field ? (double4 *)(ws + L.sfield) : nullptr,
                                             L.lo ? (float4 *)(ws + L.tlo) : nullptr,
                                             L.lo ? (float4 *)(ws + L.ilo) : nullptr, grp->flag);
  prof_end(pr, st);

  pr = prof_begin(grp, ST_CHECK, st);
  if (L.items_c > 0)
    k_check<MODE><<<(unsigned)grid_c, TPB, 0, st>>>(persistent_c, nsys, M, L.chc, base, sys_c, plans, plan_of, tgt, srcw,
                                                    L.parts_c, chk_part,
                                                    L.eonly ? (const CheckSrc *)(ws + L.csrc) : nullptr,
                                                    L.eonly ? (const int64_t *)(ws + L.nfar) : nullptr);
  k_check_finish<<<(int)cdiv((int64_t)nsys * M, 256), 256, 0, st>>>(nsys, M, L.chc, base, L.parts_c, chk_part, uv,
                                                                     uv32);
  prof_end(pr, st);

  pr = prof_begin(grp, ST_FIT, st);
  if (L.mfma) {
    float *ab32 = (float *)(ws + L.ab);  // the FP32 path keeps alpha', beta' in FP32
    float *h32 = (float *)(ws + L.h32);
    float *c2 = (float *)(ws + L.gemm2);
    dim3 g1((unsigned)cdiv(K, 64), (unsigned)cdiv(2 * (int64_t)nsys, 64));
    if (L.bf_terms == 2)
      k_gemm_bf<2><<<g1, 256, 0, st>>>(K, 2 * nsys, M, g->Mp, g->pinv_bf, uv32, ab32);
    else if (L.bf_terms == 3)
      k_gemm_bf<3><<<g1, 256, 0, st>>>(K, 2 * nsys, M, g->Mp, g->pinv_bf, uv32, ab32);
    else
      k_gemm_nt<<<g1, 256, 0, st>>>(K, 2 * nsys, M, g->pinv32, uv32, ab32);
    k_fit_h<float><<<(int)cdiv((int64_t)nsys * K, 256), 256, 0, st>>>(nsys, base, K, ab32, plans, plan_of, g->nidx,
                                                                      h32);
    dim3 g2((unsigned)cdiv(P, 64), (unsigned)cdiv(2 * (int64_t)nsys, 64));
    if (L.bf_terms == 2)
      k_gemm_bf<2><<<g2, 256, 0, st>>>(P, 2 * nsys, K, g->Kp, g->lhat_bf, h32, c2);
    else if (L.bf_terms == 3)
      k_gemm_bf<3><<<g2, 256, 0, st>>>(P, 2 * nsys, K, g->Kp, g->lhat_bf, h32, c2);
    else
      k_gemm_nt<<<g2, 256, 0, st>>>(P, 2 * nsys, K, g->lhat32, h32, c2);
    k_fit_qd<T2, float><<<(int)cdiv((int64_t)nsys * P, 256), 256, 0, st>>>(nsys, P, Pe, plans, plan_of, c2, qd);
  } else if (MODE == HSMA_PAIR_FP64 && L.gemm64) {
    double *h64 = (double *)(ws + L.h32);
    double *c2 = (double *)(ws + L.gemm2);
    dim3 g1((unsigned)cdiv(K, 64), (unsigned)cdiv(2 * (int64_t)nsys, 64));
    k_gemm64_nt<<<g1, 256, 0, st>>>(K, 2 * nsys, M, g->pinv64, uv, ab);
    k_fit_h<double><<<(int)cdiv((int64_t)nsys * K, 256), 256, 0, st>>>(nsys, base, K, ab, plans, plan_of, g->nidx,
                                                                       h64);
    dim3 g2((unsigned)cdiv(P, 64), (unsigned)cdiv(2 * (int64_t)nsys, 64));
    k_gemm64_nt<<<g2, 256, 0, st>>>(P, 2 * nsys, K, g->lhat64, h64, c2);
    k_fit_qd<T2, double><<<(int)cdiv((int64_t)nsys * P, 256), 256, 0, st>>>(nsys, P, Pe, plans, plan_of, c2, qd);
  } else if constexpr (MODE == HSMA_PAIR_FP64) {
    k_fit_moments<double><<<dim3((unsigned)cdiv(K, 4), nsys), 256, 0, st>>>(K, M, g->pinv64, uv, ab);
    k_fit_surface<double, T2><<<dim3((unsigned)cdiv(P, 4), nsys), 256, 0, st>>>(nsys, base, P, Pe, K, g->lhat64, plans,
                                                                                plan_of, g->nidx, ab, qd);
  } else {
    k_fit_moments<float><<<dim3((unsigned)cdiv(K, 4), nsys), 256, 0, st>>>(K, M, g->pinv32, uv, ab);
    k_fit_surface<float, T2><<<dim3((unsigned)cdiv(P, 4), nsys), 256, 0, st>>>(nsys, base, P, Pe, K, g->lhat32, plans,
                                                                               plan_of, g->nidx, ab, qd);
  }
  prof_end(pr, st);
  if (L.upto_fit) {
    HSMA_HIP(hipGetLastError());
    return HSMA_OK;
  }

  if constexpr (MODE == HSMA_PAIR_FP64) {
    if (L.eonly) {  // the energy alone: FP64 pair sums without potentials
      double *epair = (double *)(ws + L.eval_part);
      pr = prof_begin(grp, ST_EVAL, st);
      if (L.items_e > 0) {
        // one item per wave, the grid dealt out per die in runs; or a persistent grid of ewaves
        // workgroups (a multiple of the die count) taking items from per-die counters
        const int persist = grp->tune.ewaves > 0;
        const unsigned gs = persist ? (unsigned)(cdiv(grp->tune.ewaves, NXCD) * NXCD)
                                    : (unsigned)(cdiv(cdiv(L.items_e, WAVES), NXCD * XQ) * NXCD * XQ);
        const double *wk = (const double *)(ws + L.wk);
        const double *qr = (const double *)(ws + L.qr);
        const double *qpk = (const double *)(ws + L.qpk);
        auto run = [&](auto kern) {
          kern<<<gs, TPB, 0, st>>>(nsys, Pe, L.sch, grp->dipole == 2, base, sys_e, plan_of, tgt, img, qpk, wk, qr,
                                   grp->nodes64, qd, epair,
                                   EnergyExt{(const double4 *)(ws + L.emx), (const double2 *)(ws + L.ew), plans,
                                             (const int64_t *)(ws + L.nfar)});
        };
        if (L.sym_tb == 128)
          persist ? run(k_energy64<2, true>) : run(k_energy64<2, false>);
        else if (L.sym_tb == 256)
          persist ? run(k_energy64<4, true>) : run(k_energy64<4, false>);
        else
          persist ? run(k_energy64<8, true>) : run(k_energy64<8, false>);
      }
      prof_end(pr, st);
      pr = prof_begin(grp, ST_FINISH, st);
      if (L.fin > 0)
        k_self_energy<<<(int)L.fin, FINB, 0, st>>>(nsys, base, sys_f, self, (const double *)(ws + L.qpk), epart);
      double *echunk = (double *)(ws + L.echunk);
      if (L.echunks > 0)
        k_energy_chunks<<<(unsigned)L.echunks, 256, 0, st>>>(nsys, Pe, L.sym_tb, L.sch, base, epair, echunk);
      if (E) k_energy_items<<<nsys, 64, 0, st>>>(nsys, base, epart, echunk, E);
      prof_end(pr, st);
      HSMA_HIP(hipGetLastError());
      return HSMA_OK;
    }
  }

  pr = prof_begin(grp, ST_EVAL, st);
  bool done = false;
  if constexpr (MODE == HSMA_PAIR_FP32_COMP) {
    if (L.sym_tb > 0 && L.items_e > 0) {
      // one item per wave, or persistent: the kernel's resident blocks, a multiple of the die count
      const unsigned gs = persistent ? (unsigned)round_up((int64_t)g->ncu * grp->tune.occ_sym[L.sym_tb == 512], NXCD)
                                     : (unsigned)cdiv(L.items_e, WAVES);
      const float *wk = (const float *)(ws + L.wk);
      const double *rk = (const double *)(ws + L.rk);
      auto run = [&](auto kern) {
        kern<<<gs, TPB, 0, st>>>(nsys, Pe, L.sch, grp->dipole, base, sys_e, plan_of, tgt, img, wk, rk,
                                 grp->nodes32, qd, plans, eval_part);
      };
      if (L.sym_tb == 256)
        persistent ? run(k_kelvin_sym<4, true>) : run(k_kelvin_sym<4, false>);
      else
        persistent ? run(k_kelvin_sym<8, true>) : run(k_kelvin_sym<8, false>);
      done = true;
    }
  } else if constexpr (MODE == HSMA_PAIR_FP64) {
    if (L.sym_tb > 0 && L.items_e > 0) {
      const unsigned gs = (unsigned)cdiv(L.items_e, WAVES);
      const double *wk = (const double *)(ws + L.wk);
      const double *rk = (const double *)(ws + L.rk);
      if (L.sym_tb == 256)
        k_kelvin_sym64<4><<<gs, TPB, 0, st>>>(nsys, Pe, L.sch, grp->dipole == 2, base, sys_e, plan_of, tgt, img, wk,
                                              rk, grp->nodes64, qd, eval_part);
      else
        k_kelvin_sym64<8><<<gs, TPB, 0, st>>>(nsys, Pe, L.sch, grp->dipole == 2, base, sys_e, plan_of, tgt, img, wk,
                                              rk, grp->nodes64, qd, eval_part);
      done = true;
    }
  }
  if (L.field) {
    if (L.items_e > 0)
      k_eval_field<MODE><<<(unsigned)grid_e, TPB, 0, st>>>(
          persistent, nsys, Pe, L.che, base, sys_e, plan_of, tgt, img, group_nodes<MODE>(grp), qd,
          L.lo ? (const float4 *)(ws + L.tlo) : nullptr, L.lo ? (const float4 *)(ws + L.ilo) : nullptr,
          (double4 *)eval_part);
  } else if (!done && L.items_e > 0) {
    k_eval<MODE><<<(unsigned)grid_e, TPB, 0, st>>>(persistent, nsys, Pe, L.che, base, sys_e, plans, plan_of, tgt, img,
                                                   group_nodes<MODE>(grp), qd, eval_part);
  }
  prof_end(pr, st);

  pr = prof_begin(grp, ST_FINISH, st);
  if (L.fin > 0 && L.field)
    k_finish_field<<<(int)L.fin, FINB, 0, st>>>(nsys, Pe, L.che, base, sys_f, (const double4 *)eval_part, self,
                                                (const double4 *)(ws + L.sfield), q, phi, ex, ey, ez, epart);
  else if (L.fin > 0)
    k_finish<<<(int)L.fin, FINB, 0, st>>>(nsys, Pe, L.che, L.sym_tb, L.sch, base, sys_f, eval_part, self, q, phi,
                                          epart);
  if (E) k_energy<<<nsys, 64, 0, st>>>(nsys, base, epart, E);
  prof_end(pr, st);
  HSMA_HIP(hipGetLastError());
  return HSMA_OK;
}

}  // namespace

// Item sizes are chosen from upper bounds known on the host (system count, total and
// largest system size): the check chunk aims at about 8192 items, the evaluation chunk at
// about 8192 items of the largest possible pair count; both multiples of 4 waves x 32.
Layout layout(const hsma_group_s *grp, int nsys, int64_t total_n, int64_t max_n, bool field, bool no_sym,
              bool eonly) {
  Layout L;
  L.field = field;
  L.eonly = eonly && !field;
  L.prec = L.eonly ? HSMA_PAIR_FP64 : grp->pair_prec;
  const Geometry *g = grp->geo;
  const int64_t M = g->M, Pf = g->P, K = g->K;
  const int64_t P = grp->P_ev;  // surface sources of the evaluation
  const bool fp64 = L.prec == HSMA_PAIR_FP64;
  L.nsys = nsys;
  L.total_n = total_n;
  L.max_n = max_n;
  const int64_t target_items = grp->tune.target_items;
  const int64_t Gc = cdiv(M, GRP);
  int64_t chc = cdiv(Gc * total_n, target_items);
  chc = chc < 512 ? 512 : (chc > 65536 ? 65536 : chc);
  L.chc = round_up(chc, WAVES * TILE);
  const double pairs_bound = (double)total_n * (double)(max_n + P);
  int64_t che = (int64_t)(pairs_bound / (double)(GRP * target_items)) + 1;
  che = che < 1024 ? 1024 : (che > 65536 ? 65536 : che);
  L.che = round_up(che, WAVES * TILE);
  // bounds: sum over systems of ceil(a_b / c) <= sum a_b / c + nsys
  L.items_c = total_n > 0 ? Gc * (total_n / L.chc + nsys) : 0;
  L.parts_c = L.items_c * GRP;
  const int64_t gt = total_n / GRP + nsys;                      // target groups
  const int64_t chunks_max = (max_n + P) / L.che + 1;           // chunks of the largest system
  L.items_e = total_n > 0 ? gt * chunks_max : 0;
  L.parts_e = L.items_e * GRP;
  // Symmetric Kelvin kernel: ion blocks of 256 (4 targets per lane) where they fit, else 512.
  // Each wave works on a whole block pair or surface chunk, so in the automatic mode it is used
  // only when its waves at least cover every SIMD of the device.
  L.sym_tb = 0;
  L.sch = 0;
  const int mode = grp->tune.symmetric;
  if (L.eonly && total_n > 0) {
    // the energy kernel: blocks of 256 ions; of 128 when the launch's block pairs of 256 would
    // fill fewer than ETAIL_ROUNDS rounds of the device's wave slots (more, smaller items fill
    // the end of a small launch); 512 with symmetric mode 3; or as set.  One FP64 value per item.
    const int64_t pairs256 = (total_n / 256 + nsys) * (cdiv(max_n, 256) + 1) / 2;
    const int64_t tb = grp->tune.eblock                                    ? grp->tune.eblock
                       : mode == 3                                         ? 512
                       : pairs256 < ETAIL_ROUNDS * (int64_t)g->ncu * WAVES * 8 ? 128
                                                                           : 256;
    const int64_t bmax = cdiv(max_n, tb);
    const int64_t sch = cdiv(P, (2 * tb) / 3);
    const int64_t sb = total_n / tb + nsys;
    L.sym_tb = (int)tb;
    L.sch = (int)sch;
    // super-tiles: a system of B blocks has at most (B + ST) (B + 2 ST) / 2 pair slots
    L.items_e = (bmax + 2 * ST) * (sb + ST * (int64_t)nsys) / 2 + sb * sch * SYM_SH + 1;
    L.parts_e = total_n * (bmax + sch);  // the schedule's bound check only: no slots are stored
    L.echunks = L.items_e / EC + 2 * (int64_t)nsys + 1;
  } else if ((L.prec == HSMA_PAIR_FP32_COMP || L.prec == HSMA_PAIR_FP64) && mode != 0 && total_n > 0 && !field &&
             !no_sym) {
    for (int r = 4; r <= 8; r *= 2) {
      if ((mode == 2 && r != 4) || (mode == 3 && r != 8)) continue;
      const int64_t tb = 64 * r;
      const int64_t bmax = cdiv(max_n, tb);
      const int64_t sch = cdiv(P, (2 * tb) / 3);     // surface chunks of about 2/3 of a block's cost
      const int64_t parts = total_n * (bmax + sch);  // >= sum_b n_b (B_b + sch)
      const int64_t sb = total_n / tb + nsys;        // >= sum_b B_b
      const int64_t waves = sb * (bmax + 1) / 2 + sb * sch * SYM_SH;
      if (parts * (int64_t)sizeof(double) > SYM_MAX_BYTES || (mode == 1 && waves < 4 * (int64_t)g->ncu)) continue;
      L.sym_tb = (int)tb;
      L.sch = (int)sch;
      L.items_e = waves + 1;  // >= sum_b B_b (B_b + 1) / 2 + B_b sch SYM_SH
      L.parts_e = parts;
      break;
    }
  }
  L.fin = total_n > 0 ? total_n / FINB + nsys : 0;
  const int fit = grp->tune.fit;
  const bool gemm = fit >= 2 || (fit == 0 && nsys >= FIT_MFMA_MIN_SYS);
  L.mfma = !fp64 && gemm;
  L.gemm64 = fp64 && gemm;
  L.bf_terms = fp64 ? 0 : fit == 3 ? 2 : fit == 4 ? 3 : 0;
  const size_t t4 = fp64 ? sizeof(double4) : sizeof(float4);
  const size_t t1 = fp64 ? sizeof(double) : sizeof(float);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  L.sched = take(sizeof(int64_t) * (8 * (size_t)(nsys + 1) + CTR_WORDS));
  L.item_sys_c = take(sizeof(int) * (size_t)L.items_c);
  L.item_sys_e = take(sizeof(int) * (size_t)L.items_e);
  L.fin_sys = take(sizeof(int) * (size_t)L.fin);
  L.img = take(t4 * (size_t)total_n);
  L.tgt = take(t4 * (size_t)total_n);
  L.srcw = take(t1 * (size_t)total_n);
  L.self = take(sizeof(double) * (size_t)total_n);
  L.wk = take(t1 * (size_t)total_n);
  L.rk = take(sizeof(double) * (size_t)total_n);
  L.chk_part = take(sizeof(double) * 2 * (size_t)L.parts_c);
  L.uv = take(sizeof(double) * 2 * (size_t)M * nsys);
  L.uv32 = L.mfma ? take(sizeof(float) * 2 * (size_t)M * nsys) : 0;
  L.ab = take(sizeof(double) * 2 * (size_t)K * nsys);
  L.h32 = L.mfma ? take(sizeof(float) * 2 * (size_t)K * nsys) : L.gemm64 ? take(sizeof(double) * 2 * (size_t)K * nsys) : 0;
  L.gemm2 = L.mfma    ? take(sizeof(float) * 2 * (size_t)Pf * nsys)
            : L.gemm64 ? take(sizeof(double) * 2 * (size_t)Pf * nsys)
                       : 0;
  L.qd = take(sizeof(double2) * (size_t)P * nsys);
  L.eval_part = take(L.eonly ? sizeof(double) * (size_t)L.items_e
                             : (field ? sizeof(double4) : sizeof(double)) * (size_t)L.parts_e);
  L.qr = L.eonly ? take(sizeof(double) * (size_t)total_n) : 0;
  L.emx = L.eonly ? take(sizeof(double4) * (size_t)total_n) : 0;
  L.csrc = L.eonly ? take(sizeof(CheckSrc) * (size_t)total_n) : 0;
  L.ew = L.eonly ? take(sizeof(double2) * (size_t)total_n) : 0;
  L.ncnt = L.eonly ? take(sizeof(int) * (size_t)L.fin) : 0;
  L.farst = L.eonly ? take(sizeof(int64_t) * (size_t)L.fin) : 0;
  L.nearst = L.eonly ? take(sizeof(int64_t) * (size_t)L.fin) : 0;
  L.nfar = L.eonly ? take(sizeof(int64_t) * (size_t)nsys) : 0;
  L.qpk = L.eonly ? take(sizeof(double) * (size_t)total_n) : 0;
  L.echunk = L.eonly ? take(sizeof(double) * (size_t)(L.echunks + 1)) : 0;
  L.sfield = field ? take(sizeof(double4) * (size_t)total_n) : 0;
  L.lo = field && !fp64;
  L.tlo = L.lo ? take(sizeof(float4) * (size_t)total_n) : 0;
  L.ilo = L.lo ? take(sizeof(float4) * (size_t)total_n) : 0;
  L.phi = take(sizeof(double) * (size_t)total_n);
  L.epart = take(sizeof(double) * (size_t)(L.fin + 1));
  L.E = take(sizeof(double) * (size_t)nsys);
  L.total = o;
  return L;
}

size_t call_workspace_bytes(const hsma_group_s *grp, int nsys, int64_t total_n, int64_t max_n, bool field) {
  const size_t a = layout(grp, nsys, total_n, max_n, field).total;
  const size_t b = layout(grp, nsys, total_n, max_n, false, false, true).total;
  return a > b ? a : b;
}

namespace {
hsma_status launch_prec(hsma_group_s *grp, const Layout &L, const int64_t *offsets, const int32_t *plan_of,
                        int64_t total_n, const double *x, const double *y, const double *z, const double *q,
                        double *phi, double *E, double *ex, double *ey, double *ez, char *w, hipStream_t st) {
  switch (L.prec) {
    case HSMA_PAIR_FP32:
      return launch<HSMA_PAIR_FP32>(grp, L, offsets, plan_of, total_n, x, y, z, q, phi, E, ex, ey, ez, w, st);
    case HSMA_PAIR_FP32_COMP:
      return launch<HSMA_PAIR_FP32_COMP>(grp, L, offsets, plan_of, total_n, x, y, z, q, phi, E, ex, ey, ez, w, st);
    case HSMA_PAIR_FP64:
      return launch<HSMA_PAIR_FP64>(grp, L, offsets, plan_of, total_n, x, y, z, q, phi, E, ex, ey, ez, w, st);
    default:
      return HSMA_EINVAL;
  }
}
}  // namespace

// Energies always come from FP64 pair sums: a call that asks for E runs the energy-only launch,
// and then, if it also asks for potentials (or fields), the potential launch in the group's pair
// precision on the same workspace.  An energy is therefore the same bit for bit whether or not
// the call also asks for potentials.
hsma_status run_batched(hsma_group_s *grp, int nsys, const int64_t *offsets, const int32_t *plan_of, int64_t total_n,
                        int64_t max_n, const double *x, const double *y, const double *z, const double *q,
                        double *phi, double *E, void *ws, size_t ws_bytes, hipStream_t st, double *ex, double *ey,
                        double *ez) {
  if (!grp || nsys < 1 || total_n < 0 || max_n < 0 || max_n > total_n || !ws) return HSMA_EINVAL;
  const bool field = ex || ey || ez;
  if (field && (!ex || !ey || !ez)) return HSMA_EINVAL;
  if (total_n + grp->P_ev > ((int64_t)1 << 31) - 1) return HSMA_EINVAL;  // 32-bit source indices
  if (total_n > 0 && (!x || !y || !z || !q)) return HSMA_EINVAL;
  if (((uintptr_t)ws & 255) != 0) return HSMA_EINVAL;
  if (nsys > 1 && !offsets) return HSMA_EINVAL;
  int dev = -1;
  HSMA_HIP(hipGetDevice(&dev));
  if (dev != grp->device) return HSMA_ESTATE;
  const bool one_pass = !E;
  const bool want_pot = phi || field;
  const Layout L = layout(grp, nsys, total_n, max_n, field);
  const Layout Le = layout(grp, nsys, total_n, max_n, false, false, true);
  // workspace sized for other sizes or launch parameters
  if (ws_bytes < (one_pass ? L.total : (want_pot ? (L.total > Le.total ? L.total : Le.total) : Le.total)))
    return HSMA_EINVAL;
  char *w = (char *)ws;
  if (one_pass) {
    if (!phi) phi = (double *)(w + L.phi);
    return launch_prec(grp, L, offsets, plan_of, total_n, x, y, z, q, phi, E, ex, ey, ez, w, st);
  }
  hsma_status rc =
      launch_prec(grp, Le, offsets, plan_of, total_n, x, y, z, q, nullptr, E, nullptr, nullptr, nullptr, w, st);
  if (rc != HSMA_OK || !want_pot) return rc;
  if (!phi) phi = (double *)(w + L.phi);
  return launch_prec(grp, L, offsets, plan_of, total_n, x, y, z, q, phi, nullptr, ex, ey, ez, w, st);
}

hsma_status run_front(hsma_group_s *grp, const Layout &L, int64_t n, const double *x, const double *y,
                      const double *z, const double *q, char *ws, hipStream_t st) {
  if (!L.upto_fit || L.nsys != 1) return HSMA_EINVAL;
  switch (grp->pair_prec) {
    case HSMA_PAIR_FP32:
      return launch<HSMA_PAIR_FP32>(grp, L, nullptr, nullptr, n, x, y, z, q, nullptr, nullptr, nullptr, nullptr,
                                    nullptr, ws, st);
    case HSMA_PAIR_FP32_COMP:
      return launch<HSMA_PAIR_FP32_COMP>(grp, L, nullptr, nullptr, n, x, y, z, q, nullptr, nullptr, nullptr,
                                         nullptr, nullptr, ws, st);
    default:
      return HSMA_EINVAL;
  }
}

template <int MODE>
hsma_status occupancy_of(int *oc, int *oe) {
  int a = 0, b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_check<MODE>, TPB, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_eval<MODE>, TPB, 0) != hipSuccess)
    return HSMA_EDEVICE;
  *oc = a > 0 ? a : 1;
  *oe = b > 0 ? b : 1;
  return HSMA_OK;
}

hsma_status sym_occupancy(int *o256, int *o512) {
  int a = 0, b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_kelvin_sym<4, true>, TPB, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_kelvin_sym<8, true>, TPB, 0) != hipSuccess)
    return HSMA_EDEVICE;
  *o256 = a > 0 ? a : 1;
  *o512 = b > 0 ? b : 1;
  return HSMA_OK;
}

hsma_status pair_occupancy(int pair_prec, int *occ_check, int *occ_eval) {
  switch (pair_prec) {
    case HSMA_PAIR_FP32:
      return occupancy_of<HSMA_PAIR_FP32>(occ_check, occ_eval);
    case HSMA_PAIR_FP32_COMP:
      return occupancy_of<HSMA_PAIR_FP32_COMP>(occ_check, occ_eval);
    case HSMA_PAIR_FP64:
      return occupancy_of<HSMA_PAIR_FP64>(occ_check, occ_eval);
    default:
      return HSMA_EINVAL;
  }
}

// ---------------------------------------------------------------------------------
// Stage timing.
// ---------------------------------------------------------------------------------
hipEvent_t prof_begin(hsma_group_s *grp, int stage, hipStream_t st) {
  if (!grp->prof_on) return nullptr;
  Profile *p = (Profile *)grp->prof;
  std::lock_guard<std::mutex> lk(p->mu);
  if (p->n == p->cap) {
    const int nc = p->cap ? 2 * p->cap : 256;
    ProfRec *r = (ProfRec *)realloc(p->recs, sizeof(ProfRec) * nc);
    if (!r) return nullptr;
    p->recs = r;
    p->cap = nc;
  }
  ProfRec *r = &p->recs[p->n];
  if (hipEventCreate(&r->a) != hipSuccess) return nullptr;
  if (hipEventCreate(&r->b) != hipSuccess) {
    (void)hipEventDestroy(r->a);
    return nullptr;
  }
  r->stage = stage;
  p->n++;
  (void)hipEventRecord(r->a, st);
  return r->b;
}

void prof_end(hipEvent_t end, hipStream_t st) {
  if (end) (void)hipEventRecord(end, st);
}

void prof_free(hsma_group_s *grp) {
  Profile *p = (Profile *)grp->prof;
  if (!p) return;
  for (int i = 0; i < p->n; ++i) {
    (void)hipEventDestroy(p->recs[i].a);
    (void)hipEventDestroy(p->recs[i].b);
  }
  free(p->recs);
  delete p;
  grp->prof = nullptr;
}

}  // namespace hsma

using namespace hsma;

// ---------------------------------------------------------------------------------
// Scratch of the allocation-free entry point: a device array of HSMA_NOALLOC_BYTES in the code
// object, so every device the library runs on holds one until the process ends.  In host code
// its name is only a stand-in: the device address comes from hipGetSymbolAddress, taken once per
// device with that device current (at plan creation, else at the entry point's first call there),
// and only that address is passed to kernels.
// ---------------------------------------------------------------------------------
namespace {
__device__ __align__(256) char scratch[HSMA_NOALLOC_BYTES];
constexpr int NOALLOC_DEVICES = 64;
std::mutex noalloc_mu;
void *noalloc_ptr[NOALLOC_DEVICES];
}  // namespace

namespace hsma {
// The scratch address on device dev (the current device), looked up on first use.
void *noalloc_scratch(int dev) {
  if (dev < 0 || dev >= NOALLOC_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(noalloc_mu);
  if (!noalloc_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    noalloc_ptr[dev] = ptr;
  }
  return noalloc_ptr[dev];
}
}  // namespace hsma

extern "C" hsma_status hsma_energy_noalloc(hsma_plan_t pl, int64_t N, const double *x, const double *y,
                                           const double *z, const double *q, double *phi, double *E,
                                           hipStream_t st) {
  if (!pl || N < 0) return HSMA_EINVAL;
  int dev = -1;
  HSMA_HIP(hipGetDevice(&dev));
  if (dev != pl->device) return HSMA_ESTATE;
  if (call_workspace_bytes(pl->self, 1, N, N, false) > (size_t)HSMA_NOALLOC_BYTES) return HSMA_EINVAL;
  void *ws = noalloc_scratch(dev);
  if (!ws) return HSMA_EDEVICE;
  return run_batched(pl->self, 1, nullptr, nullptr, N, N, x, y, z, q, phi, E, ws, (size_t)HSMA_NOALLOC_BYTES, st);
}

// ---------------------------------------------------------------------------------
// C ABI.
// ---------------------------------------------------------------------------------
extern "C" size_t hsma_workspace_bytes(hsma_plan_t pl, int64_t N) {
  if (!pl || N < 0) return 0;
  return call_workspace_bytes(pl->self, 1, N, N, false);
}

extern "C" hsma_status hsma_potential(hsma_plan_t pl, int64_t N, const double *x, const double *y, const double *z,
                                      const double *q, double *phi, void *ws, size_t ws_bytes, hipStream_t st) {
  if (!pl || (N > 0 && !phi)) return HSMA_EINVAL;
  return run_batched(pl->self, 1, nullptr, nullptr, N, N, x, y, z, q, phi, nullptr, ws, ws_bytes, st);
}

extern "C" hsma_status hsma_energy(hsma_plan_t pl, int64_t N, const double *x, const double *y, const double *z,
                                   const double *q, double *phi, double *E, void *ws, size_t ws_bytes,
                                   hipStream_t st) {
  if (!pl || !E) return HSMA_EINVAL;
  return run_batched(pl->self, 1, nullptr, nullptr, N, N, x, y, z, q, phi, E, ws, ws_bytes, st);
}

extern "C" size_t hsma_field_workspace_bytes(hsma_plan_t pl, int64_t N) {
  if (!pl || N < 0) return 0;
  return call_workspace_bytes(pl->self, 1, N, N, true);
}

extern "C" hsma_status hsma_field(hsma_plan_t pl, int64_t N, const double *x, const double *y, const double *z,
                                  const double *q, double *phi, double *ex, double *ey, double *ez, double *E,
                                  void *ws, size_t ws_bytes, hipStream_t st) {
  if (!pl || (N > 0 && (!ex || !ey || !ez))) return HSMA_EINVAL;
  return run_batched(pl->self, 1, nullptr, nullptr, N, N, x, y, z, q, phi, E, ws, ws_bytes, st, ex, ey, ez);
}

extern "C" size_t hsma_field_batched_workspace_bytes(hsma_group_t grp, int nsys, int64_t total_n, int64_t max_n) {
  if (!grp || nsys < 1 || total_n < 0 || max_n < 0) return 0;
  return call_workspace_bytes(grp, nsys, total_n, max_n, true);
}

extern "C" hsma_status hsma_field_batched(hsma_group_t grp, int nsys, const int64_t *offsets, const int32_t *plan_of,
                                          int64_t total_n, int64_t max_n, const double *x, const double *y,
                                          const double *z, const double *q, double *phi, double *ex, double *ey,
                                          double *ez, double *E, void *ws, size_t ws_bytes, hipStream_t st) {
  if (!grp || !offsets || !ex || !ey || !ez) return HSMA_EINVAL;
  return run_batched(grp, nsys, offsets, plan_of, total_n, max_n, x, y, z, q, phi, E, ws, ws_bytes, st, ex, ey, ez);
}

extern "C" size_t hsma_batched_workspace_bytes(hsma_group_t grp, int nsys, int64_t total_n, int64_t max_n) {
  if (!grp || nsys < 1 || total_n < 0 || max_n < 0) return 0;
  return call_workspace_bytes(grp, nsys, total_n, max_n, false);
}

extern "C" hsma_status hsma_energy_batched(hsma_group_t grp, int nsys, const int64_t *offsets, const int32_t *plan_of,
                                           int64_t total_n, int64_t max_n, const double *x, const double *y,
                                           const double *z, const double *q, double *phi, double *E, void *ws,
                                           size_t ws_bytes, hipStream_t st) {
  if (!grp || !offsets) return HSMA_EINVAL;
  return run_batched(grp, nsys, offsets, plan_of, total_n, max_n, x, y, z, q, phi, E, ws, ws_bytes, st);
}

extern "C" hsma_status hsma_group_tune(hsma_group_t grp, int persistent, int target_items) {
  if (!grp || (persistent != 0 && persistent != 1) || target_items < 64 || target_items > (1 << 22))
    return HSMA_EINVAL;
  grp->tune.persistent = persistent;
  grp->tune.target_items = target_items;
  return HSMA_OK;
}

extern "C" int hsma_group_eval_kernel(hsma_group_t grp, int nsys, int64_t total_n, int64_t max_n) {
  if (!grp || nsys < 1 || total_n < 0 || max_n < 0 || max_n > total_n) return -1;
  return layout(grp, nsys, total_n, max_n).sym_tb;
}

extern "C" hsma_status hsma_group_set_symmetric(hsma_group_t grp, int on) {
  if (!grp || on < 0 || on > 3) return HSMA_EINVAL;
  grp->tune.symmetric = on;
  return HSMA_OK;
}

extern "C" hsma_status hsma_group_set_sym_order(hsma_group_t grp, int mode) {
  if (!grp || mode < 0 || mode > 2) return HSMA_EINVAL;
  grp->tune.sym_order = mode;
  return HSMA_OK;
}

extern "C" hsma_status hsma_group_set_fit(hsma_group_t grp, int mode) {
  if (!grp || mode < 0 || mode > 4) return HSMA_EINVAL;
  grp->tune.fit = mode;
  return HSMA_OK;
}

extern "C" int hsma_group_fit_route(hsma_group_t grp, int nsys) {
  if (!grp || nsys < 1) return -1;
  const Layout L = layout(grp, nsys, 0, 0);
  return L.bf_terms == 3 ? 4 : L.bf_terms == 2 ? 3 : (L.mfma || L.gemm64) ? 2 : 1;
}

extern "C" hsma_status hsma_debug_intermediates(hsma_plan_t pl, int64_t N, const void *ws, hipStream_t st, double *u,
                                                double *v, double *Q, double *D) {
  if (!pl || !ws || N < 0) return HSMA_EINVAL;
  const char *w = (const char *)ws;
  const int M = pl->geo->M, P = pl->geo->P;
  HSMA_HIP(hipStreamSynchronize(st));
  // the schedule of the last launch on ws records which layout it used (both start with it)
  int64_t kind = 0;
  HSMA_HIP(hipMemcpy(&kind, w + layout(pl->self, 1, N, N).sched + sizeof(int64_t) * (8 * 2 + 3), sizeof(int64_t),
                     hipMemcpyDeviceToHost));
  const bool eonly = (kind & 15) == 1;
  const int prec = (int)(kind >> 4);
  if (prec < HSMA_PAIR_FP32 || prec > HSMA_PAIR_FP64) return HSMA_ESTATE;  // no launch recorded
  const Layout L = layout(pl->self, 1, N, N, false, false, eonly);
  if (u) HSMA_HIP(hipMemcpy(u, w + L.uv, sizeof(double) * M, hipMemcpyDeviceToHost));
  if (v) HSMA_HIP(hipMemcpy(v, w + L.uv + sizeof(double) * M, sizeof(double) * M, hipMemcpyDeviceToHost));
  if (Q || D) {
    // (Q', D') per node, or from the point-pair layout: Q' at 3s, D' = (outer charge) dy / R_tau
    const int Pe = pl->self->P_ev, stride = Pe / P;
    const double dyc = pl->host.dyc;
    double2 *h = new double2[Pe];
    hipError_t e;
    if (prec == HSMA_PAIR_FP64) {
      e = hipMemcpy(h, w + L.qd, sizeof(double2) * Pe, hipMemcpyDeviceToHost);
    } else {
      float2 *f = new float2[Pe];
      e = hipMemcpy(f, w + L.qd, sizeof(float2) * Pe, hipMemcpyDeviceToHost);
      for (int s = 0; s < Pe; ++s) h[s] = make_double2(f[s].x, f[s].y);
      delete[] f;
    }
    if (e == hipSuccess)
      for (int s = 0; s < P; ++s) {
        if (Q) Q[s] = h[stride * s].x;
        if (D) D[s] = stride == 1 ? h[s].y : h[3 * s + 2].x / dyc;
      }
    delete[] h;
    if (e != hipSuccess) return HSMA_EDEVICE;
  }
  return HSMA_OK;
}

extern "C" hsma_status hsma_profile_enable(hsma_group_t grp, int on) {
  if (!grp) return HSMA_EINVAL;
  if (!grp->prof) grp->prof = new Profile();
  grp->prof_on = on ? 1 : 0;
  return HSMA_OK;
}

extern "C" hsma_status hsma_profile_read(hsma_group_t grp, double *ms, int64_t *count) {
  if (!grp || !ms || !count) return HSMA_EINVAL;
  for (int s = 0; s < ST_COUNT; ++s) {
    ms[s] = 0.0;
    count[s] = 0;
  }
  Profile *p = (Profile *)grp->prof;
  if (!p) return HSMA_OK;
  std::lock_guard<std::mutex> lk(p->mu);
  hsma_status rc = HSMA_OK;
  for (int i = 0; i < p->n; ++i) {
    ProfRec &r = p->recs[i];
    float t = 0.0f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) rc = HSMA_EDEVICE;
    ms[r.stage] += t;
    count[r.stage] += 1;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  p->n = 0;
  return rc;
}

// flag bit 1: an ion outside the cavity or a non-finite input; bit 2: device offsets or plan
// indices inconsistent with the host sizes (the call did no work).
static hsma_status flag_check(hsma_group_s *grp, hipStream_t st) {
  HSMA_HIP(hipStreamSynchronize(st));
  int f = 0;
  HSMA_HIP(hipMemcpy(&f, grp->flag, sizeof(int), hipMemcpyDeviceToHost));
  if (f) {
    HSMA_HIP(hipMemset(grp->flag, 0, sizeof(int)));
    return (f & 2) ? HSMA_EINVAL : HSMA_EDOMAIN;
  }
  return HSMA_OK;
}

extern "C" hsma_status hsma_stream_check(hsma_plan_t pl, hipStream_t st) {
  if (!pl) return HSMA_EINVAL;
  return flag_check(pl->self, st);
}

extern "C" hsma_status hsma_group_stream_check(hsma_group_t grp, hipStream_t st) {
  if (!grp) return HSMA_EINVAL;
  return flag_check(grp, st);
}

extern "C" const char *hsma_status_string(hsma_status s) {
  switch (s) {
    case HSMA_OK: return "ok";
    case HSMA_EINVAL: return "invalid argument";
    case HSMA_EDOMAIN: return "ion outside the cavity or non-finite input";
    case HSMA_ENOMEM: return "out of memory";
    case HSMA_EBUSY: return "busy";
    case HSMA_EDEVICE: return "HIP runtime error";
    case HSMA_ESTATE: return "wrong state or device";
  }
  return "unknown status";
}

extern "C" int hsma_version(void) { return 200; }
