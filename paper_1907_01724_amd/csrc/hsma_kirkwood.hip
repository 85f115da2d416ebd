// The Kirkwood series of Sec. 2.2 on the GPU: the paper's comparison method for the
// reaction potential, truncated after a given order.  For a source q_j at x_j and a target x
// (both inside the cavity), the spherical-harmonic expansion of eq. "phirf" with the
// coefficients of eq. "Anm", summed over m by the addition theorem, is
//   Phi(x) = sum_j q_j / (4 pi eps1 a) sum_{n <= order} M_n t^n P_n(c),
//   t = |x| |x_j| / a^2,  c = x^.x_j^,
// with the Kirkwood factor M_n of eq. "Anuapp1".  Every source acts on every target, the
// ion's own term (j = i) included, as in the image form of the library.  FP64 throughout.
//
// The Legendre terms are built by the three-term recurrence in the scaled form
//   u_0 = 1, u_1 = t c, u_{n+1} = A_n (t c) u_n - B_n t^2 u_{n-1},
//   A_n = (2n+1)/(n+1), B_n = n/(n+1), u_n = t^n P_n(c),
// whose coefficients (M_n, A_n, B_n) are a table read with wave-uniform loads.
#include "hsma_internal.h"

namespace hsma {
namespace {

constexpr int KW_TGT = 64;    // targets per wave (one per lane)
constexpr int KW_FIN = 256;   // ions per finish block

// coef[n] = (M_n, A_n, B_n, 0), n = 0..order
__global__ void k_kw_coeffs(int order, double eps, double mu, double4 *coef) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n > order) return;
  coef[n] = make_double4(kirkwood_factor(n, eps, mu), (2.0 * n + 1.0) / (n + 1.0), (double)n / (n + 1.0), 0.0);
}

// dir[i] = (x^, |x| / a); qw[i] = q / (4 pi eps1 a).  An ion at the centre has t = 0 with every
// partner, so only the n = 0 term survives and its direction is immaterial.
__global__ void k_kw_pack(int64_t N, const double *__restrict__ x, const double *__restrict__ y,
                          const double *__restrict__ z, const double *__restrict__ q, double a, double c0a,
                          double4 *__restrict__ dir, double *__restrict__ qw, int *__restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double xi = x[i], yi = y[i], zi = z[i], qi = q[i];
  const double r = sqrt(xi * xi + yi * yi + zi * zi);
  const bool ok = isfinite(xi) && isfinite(yi) && isfinite(zi) && isfinite(qi) && r < a;
  if (!ok) {
    atomicOr(flag, 1);
    dir[i] = make_double4(0.0, 0.0, 1.0, 0.0);
    qw[i] = 0.0;
    return;
  }
  const double inv = r > 0.0 ? 1.0 / r : 0.0;
  dir[i] = make_double4(xi * inv, yi * inv, r > 0.0 ? zi * inv : 1.0, r / a);
  qw[i] = qi * c0a;
}

// Partial sums: wave = 64 targets, grid.y = source chunk; partial[c * N + i].
__global__ __launch_bounds__(KW_TGT) void k_kw_pairs(int64_t N, int chunk, int order,
                                                     const double4 *__restrict__ coef,
                                                     const double4 *__restrict__ dir,
                                                     const double *__restrict__ qw, double *__restrict__ partial) {
  const int64_t i = (int64_t)blockIdx.x * KW_TGT + threadIdx.x;
  const int64_t c = blockIdx.y;
  const int64_t j0 = c * chunk, j1 = j0 + chunk < N ? j0 + chunk : N;
  const double4 ti = dir[i < N ? i : N - 1];
  double s = 0.0;
  for (int64_t j = j0; j < j1; ++j) {
    const double4 sj = dir[j];
    const double t = ti.w * sj.w;
    const double cs = ti.x * sj.x + ti.y * sj.y + ti.z * sj.z;
    const double tc = t * cs, t2 = t * t;
    double um = 1.0, u = tc;  // u_0, u_1
    double sum = coef[0].x;
    if (order >= 1) sum = fma(coef[1].x, u, sum);
    for (int n = 1; n < order; ++n) {
      const double4 k = coef[n];  // A_n, B_n in .y, .z
      const double un = fma(k.y * tc, u, -(k.z * t2) * um);
      um = u;
      u = un;
      sum = fma(coef[n + 1].x, u, sum);
    }
    s = fma(qw[j], sum, s);
  }
  if (i < N) partial[c * N + i] = s;
}

// phi_i = sum of the chunk partials in chunk order; block partial of (1/2) sum q phi.
__global__ __launch_bounds__(KW_FIN) void k_kw_finish(int64_t N, int nchunks, const double *__restrict__ partial,
                                                      const double *__restrict__ q, double *__restrict__ phi,
                                                      double *__restrict__ epart) {
  __shared__ double red[KW_FIN];
  const int64_t i = (int64_t)blockIdx.x * KW_FIN + threadIdx.x;
  double e = 0.0;
  if (i < N) {
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += partial[(int64_t)c * N + i];
    phi[i] = s;
    e = 0.5 * q[i] * s;
  }
  red[threadIdx.x] = e;
  __syncthreads();
  for (int o = KW_FIN / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) epart[blockIdx.x] = red[0];
}

// E = sum of the block partials, one block, strided then a fixed tree.
__global__ __launch_bounds__(KW_FIN) void k_kw_energy(int nb, const double *__restrict__ epart, double *__restrict__ E) {
  __shared__ double red[KW_FIN];
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += KW_FIN) s += epart[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = KW_FIN / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *E = red[0];
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Source chunks so that the launch has about 4096 waves; at least 64 sources per chunk.
inline int kw_chunks(int64_t N) {
  if (N <= 0) return 0;
  const int64_t waves = cdiv(N, KW_TGT);
  int64_t nc = cdiv(4096, waves);
  const int64_t most = cdiv(N, 64);
  if (nc > most) nc = most;
  return (int)(nc < 1 ? 1 : nc);
}

struct KwLayout {
  size_t coef, dir, qw, partial, phi, epart, total;
  int nchunks, chunk;
};

KwLayout kw_layout(int order, int64_t N) {
  KwLayout L;
  L.nchunks = kw_chunks(N);
  L.chunk = N > 0 ? (int)cdiv(N, L.nchunks) : 0;
  size_t o = 0;
  auto take = [&](size_t b) {
    const size_t at = o;
    o = align256(o + b);
    return at;
  };
  L.coef = take(sizeof(double4) * (size_t)(order + 1));
  L.dir = take(sizeof(double4) * (size_t)N);
  L.qw = take(sizeof(double) * (size_t)N);
  L.partial = take(sizeof(double) * (size_t)N * L.nchunks);
  L.phi = take(sizeof(double) * (size_t)N);
  L.epart = take(sizeof(double) * (size_t)cdiv(N, KW_FIN));
  L.total = o;
  return L;
}

}  // namespace
}  // namespace hsma

using namespace hsma;

extern "C" size_t hsma_kirkwood_workspace_bytes(int order, int64_t N) {
  if (order < 0 || order > HSMA_KIRKWOOD_MAX_ORDER || N < 0) return 0;
  return kw_layout(order, N).total;
}

extern "C" hsma_status hsma_kirkwood(hsma_plan_t pl, int order, int64_t N, const double *x, const double *y,
                                     const double *z, const double *q, double *phi, double *E, void *ws,
                                     size_t ws_bytes, hipStream_t st) {
  if (!pl || order < 0 || order > HSMA_KIRKWOOD_MAX_ORDER || N < 0 || !ws) return HSMA_EINVAL;
  if (N > 0 && (!x || !y || !z || !q)) return HSMA_EINVAL;
  if (((uintptr_t)ws & 255) != 0) return HSMA_EINVAL;
  int dev = -1;
  HSMA_HIP(hipGetDevice(&dev));
  if (dev != pl->device) return HSMA_ESTATE;
  const KwLayout L = kw_layout(order, N);
  if (ws_bytes < L.total) return HSMA_EINVAL;
  char *w = (char *)ws;
  if (N == 0) {
    if (E) k_kw_energy<<<1, KW_FIN, 0, st>>>(0, nullptr, E);  // no ions: E = 0 (a kernel, so graphs can hold it)
    HSMA_HIP(hipGetLastError());
    return HSMA_OK;
  }
  if (!phi) phi = (double *)(w + L.phi);
  double4 *coef = (double4 *)(w + L.coef);
  double4 *dir = (double4 *)(w + L.dir);
  double *qw = (double *)(w + L.qw);
  double *partial = (double *)(w + L.partial);
  double *epart = (double *)(w + L.epart);
  const double a = pl->a;
  k_kw_coeffs<<<(unsigned)cdiv(order + 1, 64), 64, 0, st>>>(order, pl->eps1 / pl->eps2, pl->kappa * a, coef);
  k_kw_pack<<<(unsigned)cdiv(N, 256), 256, 0, st>>>(N, x, y, z, q, a, 1.0 / (4.0 * HSMA_PI * pl->eps1 * a), dir, qw,
                                                    pl->self->flag);
  dim3 grid((unsigned)cdiv(N, KW_TGT), (unsigned)L.nchunks);
  k_kw_pairs<<<grid, KW_TGT, 0, st>>>(N, L.chunk, order, coef, dir, qw, partial);
  const int nb = (int)cdiv(N, KW_FIN);
  k_kw_finish<<<nb, KW_FIN, 0, st>>>(N, L.nchunks, partial, q, phi, epart);
  if (E) k_kw_energy<<<1, KW_FIN, 0, st>>>(nb, epart, E);
  HSMA_HIP(hipGetLastError());
  return HSMA_OK;
}
