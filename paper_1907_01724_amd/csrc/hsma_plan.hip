// Plan construction for the HSMA reaction potential: all arithmetic in FP64 kernels.
//
//  * Kirkwood factors M_n (Sec. 2.2, eq. "Anuapp1") from the finite sum for the
//    modified spherical Bessel function k_n printed in Sec. 2.2, with the decomposition
//    constants gamma, sigma, dbar of eq. "Anuapp" (Sec. 2.3).
//  * Node sets: the Fibonacci rule of Sec. 2.4 on the auxiliary sphere, and a
//    golden-angle lattice of check points on the sphere of radius rc (the least-squares
//    stand-in for the quadrature grid of Algorithm 1, step 1).
//  * The fixed fit (Algorithm 1, step 3, done as least squares): Yc (M x K real SH at
//    the check points), its Gram matrix, a blocked Cholesky factorisation, and the
//    pseudo-inverse (Yc^T Yc)^{-1} Yc^T.
//  * The surface operator mapping the fitted harmonic coefficients to the monopole and
//    dipole strengths of Green's second identity (eq. "GreenSecond") on the nodes.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <tuple>

#include "hsma_internal.h"

namespace hsma {
namespace {

// ---------------------------------------------------------------------------------
// Kirkwood factors.
// ---------------------------------------------------------------------------------

// One thread: M_n, gamma, sigma, dbar and the plan diagonals
//   f_nm = R_tau (rc/a)^{n+1} (M_n - gamma + dbar/2),  g_nm = R_tau (rc/a)^{n+1} (-dbar R_tau / (2a)),
// so that R_tau Ahat_nm = f_nm alpha'_nm + g_nm beta'_nm for the fitted alpha' = pinv u,
// beta' = pinv v (the ion-dependent correction factor of Sec. 2.4 is c_n + e r_i / a).
// out: [gamma, sigma, dbar, M_0..M_p], fg: [f (K), g (K)].
__global__ void k_plan_constants(int p, double eps, double mu, double tau, double rc_over_a, double a,
                                 double *out, double *fg) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const double gamma = (eps - 1.0) / (eps + 1.0);
  const double sigma = (1.0 + mu) / (1.0 + eps);
  const double dbar = gamma * (1.0 - sigma) - mu / (1.0 + eps);
  out[0] = gamma;
  out[1] = sigma;
  out[2] = dbar;
  const double Rtau = (1.0 + tau) * a;
  const double e = -dbar * (1.0 + tau) * 0.5;
  const int K = (p + 1) * (p + 1);
  double scale = rc_over_a;  // (rc/a)^{n+1}
  for (int n = 0; n <= p; ++n) {
    const double Mn = kirkwood_factor(n, eps, mu);
    out[3 + n] = Mn;
    const double cn = Mn - gamma + 0.5 * dbar;
    for (int m = -n; m <= n; ++m) {
      fg[n * n + n + m] = Rtau * scale * cn;
      fg[K + n * n + n + m] = Rtau * scale * e;
    }
    scale *= rc_over_a;
  }
}

// ---------------------------------------------------------------------------------
// Node sets.
// ---------------------------------------------------------------------------------

// Fibonacci rule (Sec. 2.4) on the unit sphere: node 2j and 2j+1 share
// z_j = -1 + 2j/F2, polar angle arccos(z_j + sin(pi z_j)/pi) and weight
// (2 pi / F2)(1 + cos(pi z_j)); their azimuths are pi j F1 / F2 and that plus pi
// (j F1 is reduced modulo 2 F2 first, which leaves the angle unchanged).
__global__ void k_fibonacci(int F1, int F2, double *nodes, double *w) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int P = 2 * (F2 + 1);
  if (s >= P) return;
  const int j = s >> 1, h = s & 1;
  const double zj = -1.0 + 2.0 * j / (double)F2;
  double c = zj + sin(HSMA_PI * zj) / HSMA_PI;
  c = fmin(1.0, fmax(-1.0, c));
  const double st = sqrt(fmax(0.0, 1.0 - c * c));
  const long long red = ((long long)j * (long long)F1) % (2LL * F2);
  const double ph = HSMA_PI * (double)red / (double)F2 + (h ? HSMA_PI : 0.0);
  nodes[3 * s + 0] = st * cos(ph);
  nodes[3 * s + 1] = st * sin(ph);
  nodes[3 * s + 2] = c;
  w[s] = 2.0 * HSMA_PI / (double)F2 * (1.0 + cos(HSMA_PI * zj));
}

// Golden-angle lattice on the unit sphere: z_k = 1 - (2k+1)/M, azimuth
// pi (1 + sqrt 5)(k + 1/2) mod 2 pi.
__global__ void k_check_lattice(int M, double *pts) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  const double zk = 1.0 - (2.0 * k + 1.0) / (double)M;
  const double sk = sqrt(fmax(0.0, 1.0 - zk * zk));
  const double ph = fmod(HSMA_PI * (1.0 + sqrt(5.0)) * (k + 0.5), 2.0 * HSMA_PI);
  pts[3 * k + 0] = sk * cos(ph);
  pts[3 * k + 1] = sk * sin(ph);
  pts[3 * k + 2] = zk;
}

// Algorithm 1, step 1: 2p Gauss-Legendre nodes in cos(theta) times 2p + 1 equispaced
// azimuths 2 pi j / (2p + 1) on the unit sphere, point k = i (2p + 1) + j.  Node i is the
// i-th root of P_2p in decreasing order, found by Newton's method from
// cos(pi (i + 3/4) / (2p + 1/2)) with P_2p and P_2p' from the three-term recurrence and
// (1 - x^2) P_n' = n (P_{n-1} - x P_n).  One thread per point.
__global__ void k_check_gl(int p, double *pts) {
  const int n = 2 * p, nph = 2 * p + 1;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n * nph) return;
  const int i = k / nph, j = k % nph;
  double z = cos(HSMA_PI * (i + 0.75) / (n + 0.5));
  for (int it = 0; it < 100; ++it) {
    double p0 = 1.0, p1 = z;
    for (int l = 2; l <= n; ++l) {
      const double p2 = ((2.0 * l - 1.0) * z * p1 - (l - 1.0) * p0) / l;
      p0 = p1;
      p1 = p2;
    }
    const double dp = n * (p0 - z * p1) / (1.0 - z * z);
    const double dz = p1 / dp;
    z -= dz;
    if (fabs(dz) < 1e-16) break;
  }
  const double st = sqrt(fmax(0.0, 1.0 - z * z));
  const double ph = 2.0 * HSMA_PI * j / nph;
  pts[3 * k + 0] = st * cos(ph);
  pts[3 * k + 1] = st * sin(ph);
  pts[3 * k + 2] = z;
}

// ---------------------------------------------------------------------------------
// Real orthonormal spherical harmonics of a unit vector (x, y, z), degree <= p.
// Y_nm = N_nm P_n^m(z) times cos(m phi) (m > 0, with sqrt 2) or sin(|m| phi) (m < 0).
// Written through the polynomials q_n^m = N_nm P_n^m / sin^m(theta) and the real and
// imaginary parts of (x + i y)^m = sin^m(theta) e^{i m phi}, so no angle is formed.
// Calls emit(index, value) for index n*n + n + m.
// ---------------------------------------------------------------------------------
template <typename Emit>
__device__ void real_sh_unit(int p, double x, double y, double z, Emit emit) {
  double cm = 1.0, sm = 0.0;           // Re, Im of (x + i y)^m
  double qmm = 0.28209479177387814;    // q_0^0 = 1 / sqrt(4 pi)
  for (int m = 0; m <= p; ++m) {
    if (m > 0) {
      qmm *= sqrt((2.0 * m + 1.0) / (2.0 * m));
      const double c2 = cm * x - sm * y;
      sm = cm * y + sm * x;
      cm = c2;
    }
    const double rc = (m == 0) ? 1.0 : 1.4142135623730951 * cm;
    const double rs = 1.4142135623730951 * sm;
    double q2 = 0.0, q1 = qmm;  // q_{n-2}, q_{n-1}
    for (int n = m; n <= p; ++n) {
      double qn;
      if (n == m) {
        qn = qmm;
      } else if (n == m + 1) {
        qn = sqrt(2.0 * m + 3.0) * z * qmm;
      } else {
        const double an = sqrt((4.0 * n * n - 1.0) / ((double)n * n - (double)m * m));
        const double bn = sqrt(((n - 1.0) * (n - 1.0) - (double)m * m) / (4.0 * (n - 1.0) * (n - 1.0) - 1.0));
        qn = an * (z * q1 - bn * q2);
      }
      if (n > m) {
        q2 = q1;
        q1 = qn;
      }
      emit(n * n + n + m, qn * rc);
      if (m > 0) emit(n * n + n - m, qn * rs);
    }
  }
}

// YT[nm * M + k] = Y_nm(check point k): the transpose of Yc, one thread per point.
__global__ void k_check_basis(int p, int M, const double *pts, double *YT) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  real_sh_unit(p, pts[3 * k], pts[3 * k + 1], pts[3 * k + 2],
               [&](int idx, double v) { YT[(size_t)idx * M + k] = v; });
}

// lhat[s * K + nm] = what_s (1 + tau)^n Y_nm(node s) / (4 pi), one thread per node.
__global__ void k_surface_basis(int p, int P, double tau, const double *nodes, const double *what,
                                double *lhat64, float *lhat32) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= P) return;
  const int K = (p + 1) * (p + 1);
  const double ws = what[s] / (4.0 * HSMA_PI);
  real_sh_unit(p, nodes[3 * s], nodes[3 * s + 1], nodes[3 * s + 2], [&](int idx, double v) {
    int n = 0;
    while ((n + 1) * (n + 1) <= idx) ++n;
    const double val = ws * pow(1.0 + tau, (double)n) * v;
    lhat64[(size_t)s * K + idx] = val;
    lhat32[(size_t)s * K + idx] = (float)val;
  });
}

// BF16 with round-to-nearest-even (finite inputs).
__device__ inline uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Split the FP64 matrix src (rows x cols) into three BF16 terms, plane t at
// dst[(t * rows + r) * cp + c]: b0 = bf16(x), b1 = bf16(x - b0), b2 = bf16(x - b0 - b1); the
// padding columns c >= cols are zero.
__global__ void k_split_bf16(int rows, int cols, int cp, const double *src, uint16_t *dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)rows * cp) return;
  const int r = (int)(t / cp), c = (int)(t % cp);
  double x = c < cols ? src[(size_t)r * cols + c] : 0.0;
  for (int k = 0; k < 3; ++k) {
    const uint16_t b = bf16_rne((float)x);
    dst[(size_t)k * rows * cp + t] = b;
    x -= (double)__uint_as_float((uint32_t)b << 16);
  }
}

__global__ void k_degree_index(int K, int *nidx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  int n = 0;
  while ((n + 1) * (n + 1) <= i) ++n;
  nidx[i] = n;
}

// ---------------------------------------------------------------------------------
// Normal equations: G = YT YT^T (K x K, lower triangle), 16 x 16 tiles through LDS.
// ---------------------------------------------------------------------------------
constexpr int GT = 16;

__global__ void k_gram(int K, int M, const double *YT, double *G) {
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bj > bi) return;  // lower triangle of tiles only
  __shared__ double As[GT][GT + 1], Bs[GT][GT + 1];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int i = bi * GT + ty, j = bj * GT + tx;
  double acc = 0.0;
  for (int k0 = 0; k0 < M; k0 += GT) {
    const int ri = bi * GT + ty, rj = bj * GT + ty, kk = k0 + tx;
    As[ty][tx] = (ri < K && kk < M) ? YT[(size_t)ri * M + kk] : 0.0;
    Bs[ty][tx] = (rj < K && kk < M) ? YT[(size_t)rj * M + kk] : 0.0;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < GT; ++t) acc += As[ty][t] * Bs[tx][t];
    __syncthreads();
  }
  if (i < K && j < K && j <= i) G[(size_t)i * K + j] = acc;
}

// ---------------------------------------------------------------------------------
// Blocked right-looking Cholesky G = L L^T (lower, in place, row-major K x K).
// ---------------------------------------------------------------------------------
constexpr int NB = 32;

// Factor the jb x jb diagonal block at (j0, j0) in LDS; flags a non-positive pivot.
__global__ void k_potrf_diag(int K, int j0, int jb, double *G, int *bad) {
  __shared__ double A[NB][NB + 1];
  const int t = threadIdx.x;  // 256 threads
  for (int e = t; e < jb * jb; e += blockDim.x) {
    const int r = e / jb, c = e % jb;
    A[r][c] = (c <= r) ? G[(size_t)(j0 + r) * K + (j0 + c)] : 0.0;
  }
  __syncthreads();
  for (int c = 0; c < jb; ++c) {
    if (t == 0) {
      const double d = A[c][c];
      if (!(d > 0.0)) *bad = 1;
      A[c][c] = sqrt(fmax(d, 1e-300));
    }
    __syncthreads();
    const double d = A[c][c];
    for (int r = c + 1 + t; r < jb; r += blockDim.x) A[r][c] /= d;
    __syncthreads();
    for (int e = t; e < jb * jb; e += blockDim.x) {
      const int r = e / jb, cc = e % jb;
      if (cc > c && r >= cc) A[r][cc] -= A[r][c] * A[cc][c];
    }
    __syncthreads();
  }
  for (int e = t; e < jb * jb; e += blockDim.x) {
    const int r = e / jb, c = e % jb;
    if (c <= r) G[(size_t)(j0 + r) * K + (j0 + c)] = A[r][c];
  }
}

// Rows below the diagonal block: solve X L_d^T = G[i, j0:j0+jb] for each row i.
__global__ void k_trsm_panel(int K, int j0, int jb, double *G) {
  __shared__ double L[NB][NB + 1];
  for (int e = threadIdx.x; e < jb * jb; e += blockDim.x) {
    const int r = e / jb, c = e % jb;
    L[r][c] = (c <= r) ? G[(size_t)(j0 + r) * K + (j0 + c)] : 0.0;
  }
  __syncthreads();
  const int i = j0 + jb + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  double x[NB];
  double *row = G + (size_t)i * K + j0;
  for (int c = 0; c < jb; ++c) {
    double s = row[c];
    for (int t = 0; t < c; ++t) s -= x[t] * L[c][t];
    x[c] = s / L[c][c];
  }
  for (int c = 0; c < jb; ++c) row[c] = x[c];
}

// Trailing update G[i][k] -= sum_t G[i][j0+t] G[k][j0+t] for k <= i, both >= j0 + jb.
__global__ void k_syrk_update(int K, int j0, int jb, double *G) {
  const int base = j0 + jb;
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bj > bi) return;
  __shared__ double Ai[GT][NB + 1], Ak[GT][NB + 1];
  const int tx = threadIdx.x, ty = threadIdx.y;
  for (int e = ty * GT + tx; e < GT * jb; e += GT * GT) {
    const int r = e / jb, c = e % jb;
    const int gi = base + bi * GT + r, gk = base + bj * GT + r;
    Ai[r][c] = gi < K ? G[(size_t)gi * K + j0 + c] : 0.0;
    Ak[r][c] = gk < K ? G[(size_t)gk * K + j0 + c] : 0.0;
  }
  __syncthreads();
  const int i = base + bi * GT + ty, k = base + bj * GT + tx;
  if (i >= K || k >= K || k > i) return;
  double s = 0.0;
  for (int t = 0; t < jb; ++t) s += Ai[ty][t] * Ak[tx][t];
  G[(size_t)i * K + k] -= s;
}

// ---------------------------------------------------------------------------------
// X = G^{-1} B = L^{-T} (L^{-1} B) for the K x M right-hand side B held in X (row-major, one
// column per check point), in blocks of SB rows.  The diagonal blocks of L are inverted once;
// then block row I of the forward substitution is  X_I <- Linv_I (X_I - L_{I,<I} X_{<I})  and of
// the backward one  X_I <- Linv_I^T (X_I - (L_{>I,I})^T X_{>I}):  one launch per block row and
// direction, one workgroup per tile of CT columns (the columns are independent right-hand sides).
// ---------------------------------------------------------------------------------
constexpr int SB = 64, CT = 32, KC = 32, SOLVE_T = 256;

// Linv_I: the inverse of L's diagonal block I (order jb = min(SB, K - I SB)), zero-padded to
// SB x SB; thread t forms its column t by forward substitution of the unit vector e_t.
__global__ __launch_bounds__(SB) void k_trtri_diag(int K, const double *L, double *Linv) {
  __shared__ double A[SB][SB + 1], Y[SB][SB + 1];
  const int I = blockIdx.x, j0 = I * SB, jb = min(SB, K - j0), t = threadIdx.x;
  for (int r = 0; r < SB; ++r) A[r][t] = (r < jb && t <= r) ? L[(size_t)(j0 + r) * K + j0 + t] : 0.0;
  __syncthreads();
  for (int r = 0; r < SB; ++r) {  // only column t of Y is touched by thread t
    double s = 0.0;
    if (r < jb && t < jb && r >= t) {
      s = r == t ? 1.0 : 0.0;
      for (int u = t; u < r; ++u) s -= A[r][u] * Y[u][t];
      s /= A[r][r];
    }
    Y[r][t] = s;
  }
  double *out = Linv + (size_t)I * SB * SB;
  for (int r = 0; r < SB; ++r) out[(size_t)r * SB + t] = Y[r][t];
}

// One block row I of the forward (BACK = false) or backward (BACK = true) substitution for the
// columns [blockIdx.x CT, + CT).  Thread (tr, tc) holds rows tr + 8u (u < SB / 8) of column tc.
// The backward pass also writes the FP32 copy X32.
template <bool BACK>
__global__ __launch_bounds__(SOLVE_T) void k_solve_block(int K, int M, int I, const double *L, const double *Linv,
                                                         double *X, float *X32) {
  constexpr int RU = SB / (SOLVE_T / CT);  // rows per thread
  __shared__ double As[SB][KC + 1], Bs[KC][CT + 1], Ys[SB][CT + 1];
  const int j0 = I * SB, jb = min(SB, K - j0), c0 = blockIdx.x * CT;
  const int tc = threadIdx.x % CT, tr = threadIdx.x / CT;
  const int kbeg = BACK ? j0 + jb : 0, kend = BACK ? K : j0;
  double acc[RU];
#pragma unroll
  for (int u = 0; u < RU; ++u) acc[u] = 0.0;
  for (int k0 = kbeg; k0 < kend; k0 += KC) {
    for (int e = threadIdx.x; e < SB * KC; e += SOLVE_T) {
      if (!BACK) {  // As[r][k] = L[j0 + r][k0 + k]
        const int r = e / KC, k = e % KC;
        As[r][k] = (r < jb && k0 + k < kend) ? L[(size_t)(j0 + r) * K + k0 + k] : 0.0;
      } else {  // As[r][k] = L[k0 + k][j0 + r], read along the row of L
        const int k = e / SB, r = e % SB;
        As[r][k] = (r < jb && k0 + k < kend) ? L[(size_t)(k0 + k) * K + j0 + r] : 0.0;
      }
    }
    for (int e = threadIdx.x; e < KC * CT; e += SOLVE_T) {
      const int k = e / CT, c = e % CT;
      Bs[k][c] = (k0 + k < kend && c0 + c < M) ? X[(size_t)(k0 + k) * M + c0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < KC; ++k) {
      const double bv = Bs[k][tc];
#pragma unroll
      for (int u = 0; u < RU; ++u) acc[u] = fma(As[tr + 8 * u][k], bv, acc[u]);
    }
    __syncthreads();
  }
  const bool col = c0 + tc < M;
#pragma unroll
  for (int u = 0; u < RU; ++u) {
    const int r = tr + 8 * u;
    Ys[r][tc] = (r < jb && col) ? X[(size_t)(j0 + r) * M + c0 + tc] - acc[u] : 0.0;
  }
  __syncthreads();
  const double *Li = Linv + (size_t)I * SB * SB;
#pragma unroll
  for (int u = 0; u < RU; ++u) {
    const int r = tr + 8 * u;
    double v = 0.0;
    for (int w = 0; w < SB; ++w) v = fma(BACK ? Li[(size_t)w * SB + r] : Li[(size_t)r * SB + w], Ys[w][tc], v);
    if (r < jb && col) {
      X[(size_t)(j0 + r) * M + c0 + tc] = v;
      if (BACK) X32[(size_t)(j0 + r) * M + c0 + tc] = (float)v;
    }
  }
}

// Per-plan node coordinates: check points at radius rc, surface nodes at R_tau.
// Point-pair dipoles (eq. "approxG"): node s at 3s (radius R), its inner charge at radius
// R - dy/2 (3s + 1) and its outer charge at R + dy/2 (3s + 2), along the unit normal.
__global__ void k_pair_points(int P, const double *unit, double R, double dy, float4 *p32, double4 *p64) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * P) return;
  const int s = i / 3, t = i % 3;
  const double r = t == 0 ? R : (t == 1 ? R - 0.5 * dy : R + 0.5 * dy);
  const double x = r * unit[3 * s], y = r * unit[3 * s + 1], z = r * unit[3 * s + 2];
  p32[i] = make_float4((float)x, (float)y, (float)z, 0.f);
  p64[i] = make_double4(x, y, z, 0.0);
}

__global__ void k_scale_points(int n, const double *unit, double r, float4 *p32, double4 *p64) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = r * unit[3 * i], y = r * unit[3 * i + 1], z = r * unit[3 * i + 2];
  p32[i] = make_float4((float)x, (float)y, (float)z, 0.0f);
  p64[i] = make_double4(x, y, z, 0.0);
}

// ---------------------------------------------------------------------------------
// Geometry cache.
// ---------------------------------------------------------------------------------
std::mutex g_mu;
std::map<std::tuple<int, int, int, int, double, double, int, int>, Geometry *> g_cache;

inline int blocks(int64_t n, int b) { return (int)((n + b - 1) / b); }

void geometry_free(Geometry *g) {
  (void)hipFree(g->unit_check);
  (void)hipFree(g->unit_nodes);
  (void)hipFree(g->what);
  (void)hipFree(g->pinv64);
  (void)hipFree(g->pinv32);
  (void)hipFree(g->lhat64);
  (void)hipFree(g->lhat32);
  (void)hipFree(g->pinv_bf);
  (void)hipFree(g->lhat_bf);
  (void)hipFree(g->nidx);
  delete g;
}

hsma_status geometry_build(Geometry *g) {
  const int p = g->p, K = g->K, P = g->P, M = g->M;
  hipStream_t st;
  HSMA_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  double *YT = nullptr, *G = nullptr, *Linv = nullptr;
  int *bad = nullptr;
  hsma_status rc = HSMA_OK;
#define HSMA_TRY(call)                   \
  do {                                   \
    if ((call) != hipSuccess) {          \
      rc = HSMA_EDEVICE;                 \
      goto out;                          \
    }                                    \
  } while (0)
  HSMA_TRY(hipMalloc(&g->unit_check, sizeof(double) * 3 * M));
  HSMA_TRY(hipMalloc(&g->unit_nodes, sizeof(double) * 3 * P));
  HSMA_TRY(hipMalloc(&g->what, sizeof(double) * P));
  HSMA_TRY(hipMalloc(&g->pinv64, sizeof(double) * (size_t)K * M));
  HSMA_TRY(hipMalloc(&g->pinv32, sizeof(float) * (size_t)K * M));
  HSMA_TRY(hipMalloc(&g->lhat64, sizeof(double) * (size_t)P * K));
  HSMA_TRY(hipMalloc(&g->lhat32, sizeof(float) * (size_t)P * K));
  g->Mp = (M + 31) / 32 * 32;
  g->Kp = (K + 31) / 32 * 32;
  HSMA_TRY(hipMalloc(&g->pinv_bf, sizeof(uint16_t) * 3 * (size_t)K * g->Mp));
  HSMA_TRY(hipMalloc(&g->lhat_bf, sizeof(uint16_t) * 3 * (size_t)P * g->Kp));
  HSMA_TRY(hipMalloc(&g->nidx, sizeof(int) * K));
  HSMA_TRY(hipMalloc(&G, sizeof(double) * (size_t)K * K));
  HSMA_TRY(hipMalloc(&bad, sizeof(int)));
  HSMA_TRY(hipMemsetAsync(bad, 0, sizeof(int), st));
  HSMA_TRY(hipMemsetAsync(G, 0, sizeof(double) * (size_t)K * K, st));

  if (g->check_set == 1)
    k_check_gl<<<blocks(M, 256), 256, 0, st>>>(p, g->unit_check);
  else
    k_check_lattice<<<blocks(M, 256), 256, 0, st>>>(M, g->unit_check);
  k_fibonacci<<<blocks(P, 256), 256, 0, st>>>(g->F1, g->F2, g->unit_nodes, g->what);
  k_degree_index<<<blocks(K, 256), 256, 0, st>>>(K, g->nidx);
  k_surface_basis<<<blocks(P, 64), 64, 0, st>>>(p, P, g->tau, g->unit_nodes, g->what, g->lhat64, g->lhat32);
  // YT is built in the pinv64 buffer and solved in place
  YT = g->pinv64;
  k_check_basis<<<blocks(M, 64), 64, 0, st>>>(p, M, g->unit_check, YT);
  {
    dim3 tb(GT, GT), gr(blocks(K, GT), blocks(K, GT));
    k_gram<<<gr, tb, 0, st>>>(K, M, YT, G);
  }
  for (int j0 = 0; j0 < K; j0 += NB) {
    const int jb = (K - j0) < NB ? (K - j0) : NB;
    k_potrf_diag<<<1, 256, 0, st>>>(K, j0, jb, G, bad);
    const int rest = K - j0 - jb;
    if (rest > 0) {
      k_trsm_panel<<<blocks(rest, 64), 64, 0, st>>>(K, j0, jb, G);
      dim3 tb(GT, GT), gr(blocks(rest, GT), blocks(rest, GT));
      k_syrk_update<<<gr, tb, 0, st>>>(K, j0, jb, G);
    }
  }
  {
    const int nsb = blocks(K, SB), ncol = blocks(M, CT);
    HSMA_TRY(hipMalloc(&Linv, sizeof(double) * (size_t)nsb * SB * SB));
    k_trtri_diag<<<nsb, SB, 0, st>>>(K, G, Linv);
    for (int I = 0; I < nsb; ++I)
      k_solve_block<false><<<ncol, SOLVE_T, 0, st>>>(K, M, I, G, Linv, g->pinv64, g->pinv32);
    for (int I = nsb - 1; I >= 0; --I)
      k_solve_block<true><<<ncol, SOLVE_T, 0, st>>>(K, M, I, G, Linv, g->pinv64, g->pinv32);
  }
  k_split_bf16<<<blocks((int64_t)K * g->Mp, 256), 256, 0, st>>>(K, M, g->Mp, g->pinv64, g->pinv_bf);
  k_split_bf16<<<blocks((int64_t)P * g->Kp, 256), 256, 0, st>>>(P, K, g->Kp, g->lhat64, g->lhat_bf);
  HSMA_TRY(hipGetLastError());
  HSMA_TRY(hipStreamSynchronize(st));
  {
    int hbad = 0;
    HSMA_TRY(hipMemcpy(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost));
    if (hbad) rc = HSMA_EINVAL;  // the check set does not determine the coefficients
  }
out:
#undef HSMA_TRY
  (void)hipFree(G);
  (void)hipFree(Linv);
  (void)hipFree(bad);
  (void)hipStreamDestroy(st);
  return rc;
}

}  // namespace

hsma_status geometry_acquire(int p, int P, int M, int F1, double tau, double rc_over_a, int check_set,
                             Geometry **out) {
  int dev = 0;
  HSMA_HIP(hipGetDevice(&dev));
  auto key = std::make_tuple(p, P, M, F1, tau, rc_over_a, dev, check_set);
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_cache.find(key);
  if (it != g_cache.end()) {
    it->second->refs++;
    *out = it->second;
    return HSMA_OK;
  }
  Geometry *g = new Geometry();
  memset(g, 0, sizeof(*g));
  g->p = p;
  g->K = (p + 1) * (p + 1);
  g->P = P;
  g->M = M;
  g->F1 = F1;
  g->F2 = P / 2 - 1;
  g->tau = tau;
  g->rc_over_a = rc_over_a;
  g->check_set = check_set;
  g->device = dev;
  g->ncu = 0;
  if (hipDeviceGetAttribute(&g->ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || g->ncu <= 0)
    g->ncu = 256;
  hsma_status rc = geometry_build(g);
  if (rc != HSMA_OK) {
    geometry_free(g);
    return rc;
  }
  g->refs = 1;
  g_cache[key] = g;
  *out = g;
  return HSMA_OK;
}

void geometry_release(Geometry *g) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (--g->refs > 0) return;
  for (auto it = g_cache.begin(); it != g_cache.end(); ++it) {
    if (it->second == g) {
      g_cache.erase(it);
      break;
    }
  }
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(g->device);
  geometry_free(g);
  (void)hipSetDevice(cur);
}

}  // namespace hsma

using namespace hsma;

static int gcd_int(int a, int b) {
  while (b) {
    const int t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// F1 for F2 (the Fibonacci rule wants consecutive Fibonacci numbers, i.e. F2/F1 near the
// golden ratio and coprime): the integer nearest F2/phi, moved to the nearest coprime value.
static int default_f1(int F2) {
  const double g = (1.0 + sqrt(5.0)) / 2.0;
  const int base = (int)lround(F2 / g);
  for (int d = 0; d < F2; ++d) {
    const int c1 = base - d, c2 = base + d;
    if (c1 > 0 && c1 < F2 && gcd_int(c1, F2) == 1) return c1;
    if (c2 > 0 && c2 < F2 && gcd_int(c2, F2) == 1) return c2;
  }
  return 1;
}

extern "C" hsma_plan_opts hsma_plan_opts_default(void) {
  hsma_plan_opts o;
  o.p = -1;
  o.tau = 0.1;
  o.rc_over_a = 0.0;
  o.F1 = 0;
  o.pair_prec = HSMA_PAIR_FP32_COMP;
  o.check_set = 0;
  o.dipole = 0;
  o.dy_over_Rtau = 0.0;
  return o;
}

extern "C" hsma_status hsma_plan(double a, double eps1, double eps2, double kappa, int P, int M, hsma_plan_t *out) {
  return hsma_plan_ex(a, eps1, eps2, kappa, P, M, nullptr, out);
}

extern "C" hsma_status hsma_plan_ex(double a, double eps1, double eps2, double kappa, int P, int M,
                                    const hsma_plan_opts *opts_in, hsma_plan_t *out) {
  if (!out) return HSMA_EINVAL;
  *out = nullptr;
  hsma_plan_opts o = opts_in ? *opts_in : hsma_plan_opts_default();
  if (!(isfinite(a) && isfinite(eps1) && isfinite(eps2) && isfinite(kappa))) return HSMA_EINVAL;
  if (!(a > 0.0 && a < 1e6 && eps1 > 0.0 && eps2 > 0.0 && kappa >= 0.0)) return HSMA_EINVAL;
  if (P < 8 || (P & 1)) return HSMA_EINVAL;
  if (!(isfinite(o.tau) && o.tau > 0.0 && o.tau < 10.0)) return HSMA_EINVAL;
  if (o.rc_over_a <= 0.0) o.rc_over_a = 1.0 + o.tau;
  if (!(isfinite(o.rc_over_a) && o.rc_over_a >= 1.0 && o.rc_over_a < 10.0)) return HSMA_EINVAL;
  if (o.check_set != 0 && o.check_set != 1) return HSMA_EINVAL;
  if (o.dipole < 0 || o.dipole > 2) return HSMA_EINVAL;
  if (o.dy_over_Rtau <= 0.0) o.dy_over_Rtau = 1e-5;
  if (!(isfinite(o.dy_over_Rtau) && o.dy_over_Rtau < 0.1)) return HSMA_EINVAL;
  if (o.p < 0) {
    int s = (int)floor(sqrt((double)P));
    while ((long)(s + 1) * (s + 1) <= P) ++s;
    while ((long)s * s > P) --s;
    o.p = s / 2;
  }
  if (o.p > 120) return HSMA_EINVAL;
  const int K = (o.p + 1) * (o.p + 1);
  if ((long)2 * M < 3L * K) return HSMA_EINVAL;  // M >= 1.5 K
  if (o.check_set == 1 && (o.p < 1 || M != 2 * o.p * (2 * o.p + 1))) return HSMA_EINVAL;
  const int F2 = P / 2 - 1;
  if (o.F1 == 0) o.F1 = default_f1(F2);
  if (o.F1 <= 0 || o.F1 >= F2) return HSMA_EINVAL;
  if (o.pair_prec < HSMA_PAIR_FP32 || o.pair_prec > HSMA_PAIR_FP64) return HSMA_EINVAL;

  Geometry *g = nullptr;
  hsma_status rc = geometry_acquire(o.p, P, M, o.F1, o.tau, o.rc_over_a, o.check_set, &g);
  if (rc != HSMA_OK) return rc;

  hsma_plan_s *pl = new hsma_plan_s();
  memset(pl, 0, sizeof(*pl));
  pl->a = a;
  pl->eps1 = eps1;
  pl->eps2 = eps2;
  pl->kappa = kappa;
  pl->opts = o;
  pl->geo = g;
  pl->device = g->device;
  double *consts = nullptr;
  double hc[3];
  hipStream_t st = nullptr;
  hsma_plan_t self_list[1];
#define HSMA_TRY(call)          \
  do {                          \
    if ((call) != hipSuccess) { \
      rc = HSMA_EDEVICE;        \
      goto fail;                \
    }                           \
  } while (0)
  HSMA_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  HSMA_TRY(hipMalloc(&pl->fg, sizeof(double) * 2 * K));
  HSMA_TRY(hipMalloc(&consts, sizeof(double) * (3 + o.p + 1)));
  HSMA_TRY(hipMalloc(&pl->chk32, sizeof(float4) * M));
  HSMA_TRY(hipMalloc(&pl->chk64, sizeof(double4) * M));
  HSMA_TRY(hipMalloc(&pl->nodes32, sizeof(float4) * P * (o.dipole == 1 ? 3 : 1)));
  HSMA_TRY(hipMalloc(&pl->nodes64, sizeof(double4) * P * (o.dipole == 1 ? 3 : 1)));
  k_plan_constants<<<1, 1, 0, st>>>(o.p, eps1 / eps2, kappa * a, o.tau, o.rc_over_a, a, consts, pl->fg);
  k_scale_points<<<blocks(M, 256), 256, 0, st>>>(M, g->unit_check, o.rc_over_a * a, pl->chk32, pl->chk64);
  if (o.dipole == 1)
    k_pair_points<<<blocks(3 * P, 256), 256, 0, st>>>(P, g->unit_nodes, (1.0 + o.tau) * a,
                                                      o.dy_over_Rtau * (1.0 + o.tau) * a, pl->nodes32, pl->nodes64);
  else
    k_scale_points<<<blocks(P, 256), 256, 0, st>>>(P, g->unit_nodes, (1.0 + o.tau) * a, pl->nodes32,
                                                   pl->nodes64);
  HSMA_TRY(hipGetLastError());
  HSMA_TRY(hipMemcpyAsync(hc, consts, sizeof(hc), hipMemcpyDeviceToHost, st));
  HSMA_TRY(hipStreamSynchronize(st));
  pl->host.a = a;
  pl->host.a2 = a * a;
  pl->host.c0 = 1.0 / (4.0 * HSMA_PI * eps1);
  pl->host.gamma = hc[0];
  pl->host.sigma = hc[1];
  pl->host.dbar = hc[2];
  pl->host.Rtau = (1.0 + o.tau) * a;
  pl->host.rc = o.rc_over_a * a;
  pl->host.rmin = 1e-12 * a;
  pl->host.far = 1e12 * a;
  pl->host.fg = pl->fg;
  pl->host.chk32 = pl->chk32;
  pl->host.chk64 = pl->chk64;
  pl->host.nodes32 = pl->nodes32;
  pl->host.nodes64 = pl->nodes64;
  pl->host.dipole = o.dipole;
  pl->host.dyc = 1.0 / o.dy_over_Rtau;
  (void)hipFree(consts);
  consts = nullptr;
  (void)hipStreamDestroy(st);
  st = nullptr;
  self_list[0] = pl;
  rc = group_build(1, self_list, 1, &pl->self);
  if (rc != HSMA_OK) goto fail;
  (void)noalloc_scratch(pl->device);  // set-up of hsma_energy_noalloc on this device (retried there)
  *out = pl;
  return HSMA_OK;
fail:
#undef HSMA_TRY
  (void)hipFree(consts);
  if (st) (void)hipStreamDestroy(st);
  hsma_plan_destroy(pl);
  return rc;
}

extern "C" hsma_status hsma_plan_destroy(hsma_plan_t pl) {
  if (!pl) return HSMA_EINVAL;
  if (pl->self) group_free(pl->self);
  (void)hipFree(pl->fg);
  (void)hipFree(pl->chk32);
  (void)hipFree(pl->chk64);
  (void)hipFree(pl->nodes32);
  (void)hipFree(pl->nodes64);
  if (pl->geo) geometry_release(pl->geo);
  delete pl;
  return HSMA_OK;
}

extern "C" hsma_status hsma_plan_get_info(hsma_plan_t pl, hsma_plan_info *info) {
  if (!pl || !info) return HSMA_EINVAL;
  info->a = pl->a;
  info->eps1 = pl->eps1;
  info->eps2 = pl->eps2;
  info->kappa = pl->kappa;
  info->tau = pl->opts.tau;
  info->R_tau = pl->host.Rtau;
  info->rc = pl->host.rc;
  info->gamma = pl->host.gamma;
  info->sigma = pl->host.sigma;
  info->dbar = pl->host.dbar;
  info->p = pl->geo->p;
  info->K = pl->geo->K;
  info->P = pl->geo->P;
  info->M = pl->geo->M;
  info->F1 = pl->geo->F1;
  info->F2 = pl->geo->F2;
  info->pair_prec = pl->opts.pair_prec;
  info->device = pl->device;
  info->check_set = pl->geo->check_set;
  info->dipole = pl->opts.dipole;
  info->dy_over_Rtau = pl->opts.dy_over_Rtau;
  return HSMA_OK;
}

// ---------------------------------------------------------------------------------
// Groups: plans that share one discretisation, evaluated together.
// ---------------------------------------------------------------------------------
namespace hsma {

hsma_status group_build(int nplans, const hsma_plan_t *plans, int owned_by_plan, hsma_group_s **out) {
  if (nplans < 1 || !plans || !out) return HSMA_EINVAL;
  for (int i = 0; i < nplans; ++i)
    if (!plans[i]) return HSMA_EINVAL;
  Geometry *g = plans[0]->geo;
  const int prec = plans[0]->opts.pair_prec;
  const int dipole = plans[0]->opts.dipole;
  for (int i = 1; i < nplans; ++i)
    if (plans[i]->geo != g || plans[i]->opts.pair_prec != prec || plans[i]->opts.dipole != dipole)
      return HSMA_ESTATE;
  int dev = -1;
  HSMA_HIP(hipGetDevice(&dev));
  if (dev != g->device) return HSMA_ESTATE;
  hsma_group_s *grp = new hsma_group_s();
  memset(grp, 0, sizeof(*grp));
  grp->nplans = nplans;
  grp->geo = g;
  grp->pair_prec = prec;
  grp->device = g->device;
  grp->owned_by_plan = owned_by_plan;
  grp->P_ev = g->P * (dipole == 1 ? 3 : 1);
  grp->dipole = dipole;
  grp->tune.persistent = 0;
  grp->tune.target_items = 65536;
  grp->tune.symmetric = 1;
  grp->tune.fit = 0;
  grp->tune.sym_order = 0;
  grp->tune.eblock = 0;
  grp->tune.ewaves = 0;
  if (pair_occupancy(prec, &grp->tune.occ_check, &grp->tune.occ_eval) != HSMA_OK ||
      sym_occupancy(&grp->tune.occ_sym[0], &grp->tune.occ_sym[1]) != HSMA_OK) {
    delete grp;
    return HSMA_EDEVICE;
  }
  PlanDev *h = new PlanDev[nplans];
  for (int i = 0; i < nplans; ++i) h[i] = plans[i]->host;
  hsma_status rc = HSMA_OK;
  const size_t P = (size_t)grp->P_ev;
  if (hipMalloc(&grp->dev, sizeof(PlanDev) * nplans) != hipSuccess ||
      hipMalloc(&grp->flag, sizeof(int)) != hipSuccess ||
      hipMalloc(&grp->nodes32, sizeof(float4) * P * nplans) != hipSuccess ||
      hipMalloc(&grp->nodes64, sizeof(double4) * P * nplans) != hipSuccess ||
      hipMemcpy(grp->dev, h, sizeof(PlanDev) * nplans, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(grp->flag, 0, sizeof(int)) != hipSuccess)
    rc = HSMA_EDEVICE;
  // one array of every plan's nodes, so that the evaluation kernel reads them through a kernel
  // argument (scalar loads) rather than through pointers stored in device memory
  for (int i = 0; i < nplans && rc == HSMA_OK; ++i)
    if (hipMemcpy(grp->nodes32 + P * i, plans[i]->nodes32, sizeof(float4) * P, hipMemcpyDeviceToDevice) != hipSuccess ||
        hipMemcpy(grp->nodes64 + P * i, plans[i]->nodes64, sizeof(double4) * P, hipMemcpyDeviceToDevice) != hipSuccess)
      rc = HSMA_EDEVICE;
  delete[] h;
  if (rc != HSMA_OK) {
    group_free(grp);
    return rc;
  }
  *out = grp;
  return HSMA_OK;
}

void group_free(hsma_group_s *grp) {
  if (!grp) return;
  prof_free(grp);
  (void)hipFree(grp->dev);
  (void)hipFree(grp->flag);
  (void)hipFree(grp->nodes32);
  (void)hipFree(grp->nodes64);
  delete grp;
}

}  // namespace hsma

extern "C" hsma_status hsma_group_create(int nplans, const hsma_plan_t *plans, hsma_group_t *out) {
  if (!out) return HSMA_EINVAL;
  *out = nullptr;
  return group_build(nplans, plans, 0, out);
}

extern "C" hsma_status hsma_group_destroy(hsma_group_t grp) {
  if (!grp || grp->owned_by_plan) return HSMA_EINVAL;
  group_free(grp);
  return HSMA_OK;
}

extern "C" hsma_group_t hsma_plan_group(hsma_plan_t pl) { return pl ? pl->self : nullptr; }
