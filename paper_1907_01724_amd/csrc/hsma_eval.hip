// Hot path of the HSMA reaction potential (Algorithm 1, steps 2-5) for gfx950.
//
//   K1 k_pack        Kelvin images (Sec. 2.4: r_K = (a/r)^2 x, q_K), exact FP64 self term,
//                    packed SoA sources/targets in the pair precision, domain check.
//   K2 k_check       check fields u_k = sum_i q_i G0(c_k, x_i), v_k = sum_i q_i (r_i/a) G0(c_k, x_i)
//                    (Algorithm 1, step 2), partial sums per source chunk.
//   K3 k_fit_*       alpha' = pinv u, beta' = pinv v, then the surface strengths
//                    Q' = Lhat (n . h), D' = -Lhat h with h = f . alpha' + g . beta'
//                    (steps 3-4; Green's second identity on the Fibonacci nodes).
//   K4 k_eval        Phi_i = sum_{j != i} q_K,j / |x_i - r_K,j| + sum_s [Q'_s + D'_s (d.y_s)/|d|^2]/|d|
//                    (eq. "phirffinall", step 5), partial sums per source chunk.
//   K5 k_finish_*    fixed-order FP64 reductions: Phi_i = self_i + sum of partials; E = 1/2 sum q_i Phi_i.
//
// Pair sums are VALU-bound: a target per lane, sources read at wave-uniform addresses
// (scalar loads, no LDS traffic), one v_rsq per pair.  Blocks are mapped so that the
// blocks sharing a source chunk land on the same XCD (same L2).
#include <math.h>

#include "hsma_internal.h"

namespace hsma {
namespace {

constexpr int TPB = 256;   // threads (targets) per block in the pair kernels
constexpr int TILE = 32;   // sources per FP32 partial sum before folding into FP64
constexpr int NXCD = 8;

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

// 1/sqrt(r2) in FP64: FP32 hardware estimate (relative error ~1e-7) refined by one
// Newton step y <- y + y (1 - r2 y^2) / 2, giving ~2e-14.
__device__ __forceinline__ double rinv(double r2) {
  const double y = (double)__builtin_amdgcn_rsqf((float)r2);
  const double t = r2 * y;
  const double e = fma(-t, y, 1.0);
  return fma(y * 0.5, e, y);
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

// Block id -> logical id so that consecutive logical ids share an XCD (hardware deals
// block ids round-robin over the XCDs).  The grid is padded to a multiple of NXCD.
__device__ __forceinline__ int xcd_logical(int bid, int grid) {
  const int per = grid / NXCD;
  return (bid % NXCD) * per + bid / NXCD;
}

// ---------------------------------------------------------------------------------
// K1: Kelvin images and packing.
// ---------------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(256) void k_pack(int64_t N, const double *__restrict__ x, const double *__restrict__ y,
                                              const double *__restrict__ z, const double *__restrict__ q, Consts c,
                                              typename PT<MODE>::T4 *__restrict__ img,
                                              typename PT<MODE>::T4 *__restrict__ tgt,
                                              typename PT<MODE>::T *__restrict__ srcw, double *__restrict__ self,
                                              int *__restrict__ flag) {
  using T4 = typename PT<MODE>::T4;
  using T = typename PT<MODE>::T;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double xi = x[i], yi = y[i], zi = z[i], qi = q[i];
  const double r2 = xi * xi + yi * yi + zi * zi;
  const double r = sqrt(r2);
  const bool ok = isfinite(xi) && isfinite(yi) && isfinite(zi) && isfinite(qi) && r < c.a;
  if (!ok) {
    atomicOr(flag, 1);
    img[i] = make4<T4>(0.0, 0.0, 2.0 * c.far, 0.0);
    tgt[i] = make4<T4>(0.0, 0.0, 0.0, 0.0);
    srcw[i] = (T)0;
    self[i] = 0.0;
    return;
  }
  const double qp = qi * c.c0;  // q / (4 pi eps1)
  double kx, ky, kz, qk;
  if (r >= c.rmin) {
    const double f = c.a2 / r2;  // r_K = (a/r)^2 x
    kx = f * xi;
    ky = f * yi;
    kz = f * zi;
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
  }
  // own image: q_K / (4 pi eps1 |x - r_K|) with |x - r_K| = (a^2 - r^2) / r, written so
  // that it stays regular at r = 0 and keeps FP64 accuracy as r -> a
  self[i] = qp / c.a * (c.gamma * c.a2 + 0.5 * c.dbar * (c.Rtau * r - c.a2)) / ((c.a - r) * (c.a + r));
  img[i] = make4<T4>(kx, ky, kz, qk);
  tgt[i] = make4<T4>(xi, yi, zi, qp);
  srcw[i] = (T)(qp * r / c.a);
}

// ---------------------------------------------------------------------------------
// K2: check fields.  grid = padded (chunks x target blocks); one check point per lane.
// ---------------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(TPB) void k_check(int M, const typename PT<MODE>::T4 *__restrict__ chk, int64_t N,
                                               const typename PT<MODE>::T4 *__restrict__ src,
                                               const typename PT<MODE>::T *__restrict__ srcw, int chunk, int ntb,
                                               int nblocks, double *__restrict__ part) {
  using T = typename PT<MODE>::T;
  using T4 = typename PT<MODE>::T4;
  const int lg = xcd_logical(blockIdx.x, gridDim.x);
  if (lg >= nblocks) return;
  const int cidx = lg / ntb, tb = lg % ntb;
  const int k = tb * TPB + threadIdx.x;
  const T4 ck = chk[k < M ? k : M - 1];
  const int64_t j0 = (int64_t)cidx * chunk;
  const int64_t j1 = j0 + chunk < N ? j0 + chunk : N;
  double au = 0.0, av = 0.0;
  if constexpr (MODE == HSMA_PAIR_FP32) {
    T su = 0, sv = 0;
    for (int64_t j = j0; j < j1; ++j) {
      const T4 s = src[j];
      const T dx = ck.x - s.x, dy = ck.y - s.y, dz = ck.z - s.z;
      const T ri = rinv(dx * dx + dy * dy + dz * dz);
      su = fma(s.w, ri, su);
      sv = fma(srcw[j], ri, sv);
    }
    au = su;
    av = sv;
  } else {
    int64_t jb = j0;
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
    for (int64_t j = jb; j < j1; ++j) {
      const T4 s = src[j];
      const T dx = ck.x - s.x, dy = ck.y - s.y, dz = ck.z - s.z;
      const T ri = rinv(dx * dx + dy * dy + dz * dz);
      su = fma(s.w, ri, su);
      sv = fma(srcw[j], ri, sv);
    }
    au += (double)su;
    av += (double)sv;
  }
  if (k < M) {
    const int nch = nblocks / ntb;
    part[(size_t)cidx * M + k] = au;
    part[(size_t)(nch + cidx) * M + k] = av;
  }
}

// u_k, v_k = sum over chunks in order.
__global__ void k_check_reduce(int M, int nch, const double *__restrict__ part, double *__restrict__ uv) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  double u = 0.0, v = 0.0;
  for (int c = 0; c < nch; ++c) {
    u += part[(size_t)c * M + k];
    v += part[(size_t)(nch + c) * M + k];
  }
  uv[k] = u;
  uv[M + k] = v;
}

// ---------------------------------------------------------------------------------
// K3: fixed fit apply (single system): two GEMVs, one wave64 per output row.
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
  const int lane = threadIdx.x & 63;
  if (row >= K) return;
  const TM *pr = pinv + (size_t)row * M;
  double su = 0.0, sv = 0.0;
  for (int m = lane; m < M; m += 64) {
    const double w = (double)pr[m];
    su = fma(w, uv[m], su);
    sv = fma(w, uv[M + m], sv);
  }
  su = wave_sum(su);
  sv = wave_sum(sv);
  if (lane == 0) {
    ab[row] = su;
    ab[K + row] = sv;
  }
}

template <typename TM, typename T2>
__global__ __launch_bounds__(256) void k_fit_surface(int P, int K, const TM *__restrict__ lhat,
                                                     const double *__restrict__ fg, const int *__restrict__ nidx,
                                                     const double *__restrict__ ab, T2 *__restrict__ qd) {
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (s >= P) return;
  const TM *lr = lhat + (size_t)s * K;
  double sq = 0.0, sd = 0.0;
  for (int k = lane; k < K; k += 64) {
    const double h = fg[k] * ab[k] + fg[K + k] * ab[K + k];
    const double l = (double)lr[k];
    sq = fma(l * (double)nidx[k], h, sq);
    sd = fma(l, h, sd);
  }
  sq = wave_sum(sq);
  sd = wave_sum(sd);
  if (lane == 0) {
    T2 o;
    o.x = sq;
    o.y = -sd;
    qd[s] = o;
  }
}

// ---------------------------------------------------------------------------------
// K4: evaluation pair sums.
// ---------------------------------------------------------------------------------
template <int MODE, bool DIAG>
__device__ __forceinline__ double kelvin_range(const typename PT<MODE>::T4 &t, int64_t i,
                                               const typename PT<MODE>::T4 *__restrict__ img, int64_t j0,
                                               int64_t j1) {
  using T = typename PT<MODE>::T;
  using T4 = typename PT<MODE>::T4;
  if constexpr (MODE != HSMA_PAIR_FP32_COMP) {
    T s = 0;
#pragma unroll 8
    for (int64_t j = j0; j < j1; ++j) {
      const T4 v = img[j];
      const T dx = t.x - v.x, dy = t.y - v.y, dz = t.z - v.z;
      T ri = rinv(dx * dx + dy * dy + dz * dz);
      if (DIAG) ri = (j == i) ? (T)0 : ri;
      s = fma(v.w, ri, s);
    }
    return (double)s;
  } else {
    double acc = 0.0;
    int64_t jb = j0;
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
    for (int64_t j = jb; j < j1; ++j) {
      const float4 v = img[j];
      const float dx = t.x - v.x, dy = t.y - v.y, dz = t.z - v.z;
      float ri = rinv(dx * dx + dy * dy + dz * dz);
      if (DIAG) ri = (j == i) ? 0.0f : ri;
      s = fmaf(v.w, ri, s);
    }
    return acc + (double)s;
  }
}

template <int MODE>
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
    for (int k = sb; k < se; ++k) {
      const T4 y = nodes[k];
      const T2 w = qd[k];
      const T dx = t.x - y.x, dy = t.y - y.y, dz = t.z - y.z;
      const T ri = rinv(dx * dx + dy * dy + dz * dz);
      const T dot = dx * y.x + dy * y.y + dz * y.z;  // (x - y_s) . y_s = R_tau (x - y_s) . y^_s
      s = fma(ri, fma(w.y * dot, ri * ri, w.x), s);
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
__global__ __launch_bounds__(TPB) void k_eval(int64_t N, int P, const typename PT<MODE>::T4 *__restrict__ tgt,
                                              const typename PT<MODE>::T4 *__restrict__ img,
                                              const typename PT<MODE>::T4 *__restrict__ nodes,
                                              const typename PT<MODE>::T2 *__restrict__ qd, int64_t chunk, int ntb,
                                              int nblocks, double *__restrict__ part) {
  using T4 = typename PT<MODE>::T4;
  const int lg = xcd_logical(blockIdx.x, gridDim.x);
  if (lg >= nblocks) return;
  const int cidx = lg / ntb, tb = lg % ntb;
  const int64_t i = (int64_t)tb * TPB + threadIdx.x;
  const T4 t = tgt[i < N ? i : N - 1];
  const int64_t total = N + P;
  const int64_t j0 = (int64_t)cidx * chunk;
  const int64_t j1 = j0 + chunk < total ? j0 + chunk : total;
  double acc = 0.0;
  const int64_t k1 = j1 < N ? j1 : N;
  if (j0 < k1) {
    const int64_t t0 = (int64_t)tb * TPB;
    const bool diag = (t0 < k1) && (t0 + TPB > j0);
    acc = diag ? kelvin_range<MODE, true>(t, i, img, j0, k1) : kelvin_range<MODE, false>(t, i, img, j0, k1);
  }
  const int64_t s0 = (j0 > N ? j0 : N) - N, s1 = j1 - N;
  if (s0 < s1) acc += surface_range<MODE>(t, nodes, qd, (int)s0, (int)s1);
  if (i < N) part[(size_t)cidx * N + i] = acc;
}

// Phi_i = self_i + sum of chunk partials (fixed order); block partial of 1/2 sum q Phi.
__global__ __launch_bounds__(256) void k_finish_phi(int64_t N, int nch, const double *__restrict__ part,
                                                    const double *__restrict__ self, const double *__restrict__ q,
                                                    double *__restrict__ phi, double *__restrict__ epart) {
  __shared__ double red[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double e = 0.0;
  if (i < N) {
    double s = self[i];
    for (int c = 0; c < nch; ++c) s += part[(size_t)c * N + i];
    phi[i] = s;
    e = 0.5 * q[i] * s;
  }
  red[threadIdx.x] = e;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) epart[blockIdx.x] = red[0];
}

// E = sum of block partials, strided per thread then a tree: fixed order.
__global__ __launch_bounds__(256) void k_finish_energy(int nb, const double *__restrict__ epart,
                                                       double *__restrict__ E) {
  __shared__ double red[256];
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) s += epart[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *E = red[0];
}

// Clear n doubles with a kernel (memset nodes misbehave when replayed inside graphs).
__global__ void k_zero(int64_t n, double *__restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
inline int pad8(int n) { return (n + NXCD - 1) / NXCD * NXCD; }

template <int MODE>
hsma_status launch_all(const hsma_plan_s *pl, int64_t N, const double *x, const double *y, const double *z,
                       const double *q, double *phi, double *E, char *ws, const Workspace &L, hipStream_t st) {
  using T = typename PT<MODE>::T;
  using T2 = typename PT<MODE>::T2;
  using T4 = typename PT<MODE>::T4;
  const Geometry *g = pl->geo;
  const int M = g->M, P = g->P, K = g->K;
  T4 *img = (T4 *)(ws + L.img);
  T4 *tgt = (T4 *)(ws + L.tgt);
  T *srcw = (T *)(ws + L.srcw);
  double *self = (double *)(ws + L.self);
  double *chk_part = (double *)(ws + L.chk_part);
  double *uv = (double *)(ws + L.uv);
  double *ab = (double *)(ws + L.ab);
  T2 *qd = (T2 *)(ws + L.qd);
  double *eval_part = (double *)(ws + L.eval_part);
  double *epart = (double *)(ws + L.e_part);
  const T4 *chk = nullptr;
  const T4 *nodes = nullptr;
  if constexpr (MODE == HSMA_PAIR_FP64) {
    chk = (const T4 *)pl->chk64;
    nodes = (const T4 *)pl->nodes64;
  } else {
    chk = (const T4 *)pl->chk32;
    nodes = (const T4 *)pl->nodes32;
  }
  hsma_plan_s *pm = const_cast<hsma_plan_s *>(pl);
  hipEvent_t pr = nullptr;
  if (N > 0) {
    pr = prof_begin(pm, ST_PACK, st);
    k_pack<MODE><<<cdiv(N, 256), 256, 0, st>>>(N, x, y, z, q, pl->c, img, tgt, srcw, self, pl->flag);
    prof_end(pr, st);
    const int ntb_c = cdiv(M, TPB);
    const int nb_c = L.chk_chunks * ntb_c;
    pr = prof_begin(pm, ST_CHECK, st);
    k_check<MODE><<<pad8(nb_c), TPB, 0, st>>>(M, chk, N, tgt, srcw, L.chk_chunk, ntb_c, nb_c, chk_part);
    k_check_reduce<<<cdiv(M, 256), 256, 0, st>>>(M, L.chk_chunks, chk_part, uv);
    prof_end(pr, st);
  } else {
    k_zero<<<cdiv(2 * M, 256), 256, 0, st>>>(2 * (int64_t)M, uv);
  }
  pr = prof_begin(pm, ST_FIT, st);
  if constexpr (MODE == HSMA_PAIR_FP64) {
    k_fit_moments<double><<<cdiv(K, 4), 256, 0, st>>>(K, M, g->pinv64, uv, ab);
    k_fit_surface<double, T2><<<cdiv(P, 4), 256, 0, st>>>(P, K, g->lhat64, pl->fg, g->nidx, ab, qd);
  } else {
    k_fit_moments<float><<<cdiv(K, 4), 256, 0, st>>>(K, M, g->pinv32, uv, ab);
    k_fit_surface<float, T2><<<cdiv(P, 4), 256, 0, st>>>(P, K, g->lhat32, pl->fg, g->nidx, ab, qd);
  }
  prof_end(pr, st);
  if (N > 0) {
    const int ntb_e = cdiv(N, TPB);
    const int nb_e = L.eval_chunks * ntb_e;
    pr = prof_begin(pm, ST_EVAL, st);
    k_eval<MODE><<<pad8(nb_e), TPB, 0, st>>>(N, P, tgt, img, nodes, qd, L.eval_chunk, ntb_e, nb_e, eval_part);
    prof_end(pr, st);
    pr = prof_begin(pm, ST_FINISH, st);
    k_finish_phi<<<L.e_blocks, 256, 0, st>>>(N, L.eval_chunks, eval_part, self, q, phi, epart);
    if (E) k_finish_energy<<<1, 256, 0, st>>>(L.e_blocks, epart, E);
    prof_end(pr, st);
  } else if (E) {
    k_zero<<<1, 256, 0, st>>>(1, E);
  }
  HSMA_HIP(hipGetLastError());
  return HSMA_OK;
}

}  // namespace

Workspace workspace_layout(const hsma_plan_s *pl, int64_t N) {
  Workspace L;
  const Geometry *g = pl->geo;
  const int M = g->M, P = g->P, K = g->K;
  const size_t t4 = pl->opts.pair_prec == HSMA_PAIR_FP64 ? sizeof(double4) : sizeof(float4);
  const size_t t1 = pl->opts.pair_prec == HSMA_PAIR_FP64 ? sizeof(double) : sizeof(float);
  // check sums: about 2048 blocks, chunks of at least 64 sources, multiples of TILE
  const int ntb_c = cdiv(M, TPB);
  int nch = N > 0 ? cdiv(2048, ntb_c) : 0;
  if (N > 0) {
    const int maxch = cdiv(N, 64);
    if (nch > maxch) nch = maxch;
    if (nch < 1) nch = 1;
    int64_t chunk = (N + nch - 1) / nch;
    chunk = (chunk + TILE - 1) / TILE * TILE;
    L.chk_chunk = (int)chunk;
    L.chk_chunks = cdiv(N, chunk);
  } else {
    L.chk_chunk = 0;
    L.chk_chunks = 0;
  }
  // evaluation sums: about 4096 blocks, chunks of at least 256 sources
  const int64_t S = N + P;
  const int ntb_e = N > 0 ? cdiv(N, TPB) : 0;
  if (N > 0) {
    int ech = cdiv(4096, ntb_e);
    const int maxch = cdiv(S, 256);
    if (ech > maxch) ech = maxch;
    if (ech < 1) ech = 1;
    int64_t chunk = (S + ech - 1) / ech;
    chunk = (chunk + TILE - 1) / TILE * TILE;
    L.eval_chunk = (int)chunk;
    L.eval_chunks = cdiv(S, chunk);
  } else {
    L.eval_chunk = 0;
    L.eval_chunks = 0;
  }
  L.e_blocks = N > 0 ? cdiv(N, 256) : 0;
  size_t o = 0;
  const size_t n = (size_t)(N > 0 ? N : 0);
  L.img = o;
  o = align256(o + t4 * n);
  L.tgt = o;
  o = align256(o + t4 * n);
  L.srcw = o;
  o = align256(o + t1 * n);
  L.self = o;
  o = align256(o + sizeof(double) * n);
  L.chk_part = o;
  o = align256(o + sizeof(double) * 2 * (size_t)L.chk_chunks * M);
  L.uv = o;
  o = align256(o + sizeof(double) * 2 * M);
  L.ab = o;
  o = align256(o + sizeof(double) * 2 * K);
  L.qd = o;
  o = align256(o + sizeof(double2) * P);
  L.eval_part = o;
  o = align256(o + sizeof(double) * (size_t)L.eval_chunks * n);
  L.phi = o;
  o = align256(o + sizeof(double) * n);
  L.e_part = o;
  o = align256(o + sizeof(double) * (L.e_blocks + 1));
  L.total = o;
  return L;
}

}  // namespace hsma

namespace hsma {

hipEvent_t prof_begin(hsma_plan_s *pl, int stage, hipStream_t st) {
  if (!pl->prof_on) return nullptr;
  Profile *p = (Profile *)pl->prof;
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

void prof_free(hsma_plan_s *pl) {
  Profile *p = (Profile *)pl->prof;
  if (!p) return;
  for (int i = 0; i < p->n; ++i) {
    (void)hipEventDestroy(p->recs[i].a);
    (void)hipEventDestroy(p->recs[i].b);
  }
  free(p->recs);
  delete p;
  pl->prof = nullptr;
}

}  // namespace hsma

using namespace hsma;

extern "C" hsma_status hsma_profile_enable(hsma_plan_t pl, int on) {
  if (!pl) return HSMA_EINVAL;
  if (!pl->prof) pl->prof = new Profile();
  pl->prof_on = on ? 1 : 0;
  return HSMA_OK;
}

extern "C" hsma_status hsma_profile_read(hsma_plan_t pl, double *ms, int64_t *count) {
  if (!pl || !ms || !count) return HSMA_EINVAL;
  for (int s = 0; s < ST_COUNT; ++s) {
    ms[s] = 0.0;
    count[s] = 0;
  }
  Profile *p = (Profile *)pl->prof;
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

static hsma_status check_device(const hsma_plan_s *pl) {
  int dev = -1;
  HSMA_HIP(hipGetDevice(&dev));
  return dev == pl->device ? HSMA_OK : HSMA_ESTATE;
}

static hsma_status run(hsma_plan_t pl, int64_t N, const double *x, const double *y, const double *z,
                       const double *q, double *phi, double *E, void *ws, hipStream_t st) {
  if (!pl || N < 0 || N > ((int64_t)1 << 31) - 1 || !ws) return HSMA_EINVAL;
  if (N > 0 && (!x || !y || !z || !q)) return HSMA_EINVAL;
  if (((uintptr_t)ws & 255) != 0) return HSMA_EINVAL;
  hsma_status rc = check_device(pl);
  if (rc != HSMA_OK) return rc;
  const Workspace L = workspace_layout(pl, N);
  char *w = (char *)ws;
  if (!phi) phi = (double *)(w + L.phi);
  switch (pl->opts.pair_prec) {
    case HSMA_PAIR_FP32:
      return launch_all<HSMA_PAIR_FP32>(pl, N, x, y, z, q, phi, E, w, L, st);
    case HSMA_PAIR_FP32_COMP:
      return launch_all<HSMA_PAIR_FP32_COMP>(pl, N, x, y, z, q, phi, E, w, L, st);
    case HSMA_PAIR_FP64:
      return launch_all<HSMA_PAIR_FP64>(pl, N, x, y, z, q, phi, E, w, L, st);
    default:
      return HSMA_EINVAL;
  }
}

extern "C" size_t hsma_workspace_bytes(hsma_plan_t pl, int64_t N) {
  if (!pl || N < 0) return 0;
  return workspace_layout(pl, N).total;
}

extern "C" hsma_status hsma_potential(hsma_plan_t pl, int64_t N, const double *x, const double *y, const double *z,
                                      const double *q, double *phi, void *ws, hipStream_t st) {
  if (N > 0 && !phi) return HSMA_EINVAL;
  return run(pl, N, x, y, z, q, phi, nullptr, ws, st);
}

extern "C" hsma_status hsma_energy(hsma_plan_t pl, int64_t N, const double *x, const double *y, const double *z,
                                   const double *q, double *phi, double *E, void *ws, hipStream_t st) {
  if (!E) return HSMA_EINVAL;
  return run(pl, N, x, y, z, q, phi, E, ws, st);
}

extern "C" hsma_status hsma_debug_intermediates(hsma_plan_t pl, int64_t N, const void *ws, hipStream_t st, double *u,
                                                double *v, double *Q, double *D) {
  if (!pl || !ws || N < 0) return HSMA_EINVAL;
  const Workspace L = workspace_layout(pl, N);
  const char *w = (const char *)ws;
  const int M = pl->geo->M, P = pl->geo->P;
  HSMA_HIP(hipStreamSynchronize(st));
  if (u) HSMA_HIP(hipMemcpy(u, w + L.uv, sizeof(double) * M, hipMemcpyDeviceToHost));
  if (v) HSMA_HIP(hipMemcpy(v, w + L.uv + sizeof(double) * M, sizeof(double) * M, hipMemcpyDeviceToHost));
  if (Q || D) {
    if (pl->opts.pair_prec == HSMA_PAIR_FP64) {
      double2 *h = new double2[P];
      hipError_t e = hipMemcpy(h, w + L.qd, sizeof(double2) * P, hipMemcpyDeviceToHost);
      if (e == hipSuccess)
        for (int s = 0; s < P; ++s) {
          if (Q) Q[s] = h[s].x;
          if (D) D[s] = h[s].y;
        }
      delete[] h;
      if (e != hipSuccess) return HSMA_EDEVICE;
    } else {
      float2 *h = new float2[P];
      hipError_t e = hipMemcpy(h, w + L.qd, sizeof(float2) * P, hipMemcpyDeviceToHost);
      if (e == hipSuccess)
        for (int s = 0; s < P; ++s) {
          if (Q) Q[s] = h[s].x;
          if (D) D[s] = h[s].y;
        }
      delete[] h;
      if (e != hipSuccess) return HSMA_EDEVICE;
    }
  }
  return HSMA_OK;
}

extern "C" hsma_status hsma_stream_check(hsma_plan_t pl, hipStream_t st) {
  if (!pl) return HSMA_EINVAL;
  HSMA_HIP(hipStreamSynchronize(st));
  int f = 0;
  HSMA_HIP(hipMemcpy(&f, pl->flag, sizeof(int), hipMemcpyDeviceToHost));
  if (f) {
    HSMA_HIP(hipMemset(pl->flag, 0, sizeof(int)));
    return HSMA_EDOMAIN;
  }
  return HSMA_OK;
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

extern "C" int hsma_version(void) { return 100; }
