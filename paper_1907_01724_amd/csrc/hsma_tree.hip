// Treecode far field for the Kelvin-image and surface sums (the role of the paper's FMM in Sec. 3 and
// Sec. 4.2, as a Barnes-Hut treecode): one system, FP32 pair modes.
//
// Every Kelvin image lies outside the cavity and every target inside it.  The images are
// sorted by the Morton code of their position in the cube [-L, L]^3, L = 8a, at depth D; the
// few images outside the cube (ions within a/8 of the centre, whose images are more than 8a
// away) sort last and form the far set, summed directly.  Each level l = 0..D of the octree is
// the run-length encoding of the codes shifted by 3 (D - l) bits.  Per cell, Cartesian
// multipole moments about the cell centre
//   M_k = sum_j q_K,j (y_j - c)^k,  |k| <= p,
// and the potential at x of an accepted cell is sum_k a_k(x - c) M_k with the Taylor
// coefficients a_k(R) = (1/k!) d^k/dy^k 1/|x - y| at y = c, from the recurrence
//   |R|^2 a_k = ((2n - 1)/n) sum_i R_i a_{k - e_i} - ((n - 1)/n) sum_i a_{k - 2e_i},  n = |k|,
// a_0 = 1/|R| (the recurrence for the Taylor coefficients of 1/|x - y| used by Cartesian
// treecodes, e.g. Lindsay and Krasny; it follows from 1/|x - y| satisfying Laplace's equation).
// A cell is accepted for a group of 64 targets when (r_cell + r_group) < theta |c_cell - c_group|;
// leaves that are not accepted are summed directly, the ion's own image excluded (it is the
// analytic FP64 term of the packing kernel).  If an ion's own image lies in an accepted cell,
// its exact FP32 term is subtracted again.  theta = 0 accepts nothing: the traversal then sums
// every image directly.  The targets are grouped by their own positions, not by their images:
// sorted by Morton code in [-a, a]^3 and cut into runs of up to 64 within the cells of a coarse
// level, so that groups are compact and nearly full everywhere in the cavity.  (Grouped by their
// images' cells, the ions near the centre, whose images are spread thinly far out, formed groups
// of one or two targets, each with a whole traversal.)
//
// The check sums, the fit and the surface strengths are those of the direct path
// (run_front).  The surface nodes are sorted the same way into patches of up to 64, with
// moments that include their radial dipoles, and each group takes them by the same rule after
// the traversal.  The moments of cells and patches are folded onto the multi-indices with
// k_z <= 1 by the harmonic identity of the Taylor coefficients (see fold_rec), so that an
// accepted cell costs (p + 1)^2 terms.
#include <cmath>
#include <type_traits>

#include "hsma_internal.h"

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

namespace hsma {
namespace {

constexpr int TR_WAVES = 1;             // waves per block, one target group each
constexpr int TR_STACK = 96;            // traversal stack entries per wave (>= 7 (D + 1) + 8)
constexpr int TR_MAX_DEPTH = 10;        // codes of 3 D bits plus the far flag fit in 31 bits
constexpr unsigned TR_FAR = 1u << 30;   // code of an image outside the cube
constexpr double TR_CUBE = 8.0;         // cube half-width in units of a
constexpr int TR_TBITS = 10;            // bits per axis of the targets' codes in [-a, a]^3
constexpr int TR_LEAF = 64;             // cells of at most this many images are leaves at any level
constexpr int TR_CELL_BLOCKS = 8192;    // blocks of the moment kernels (one wave each, grid-stride)

// Graded multi-index order: degree n, then kx descending, then ky descending.
constexpr int ncoef(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }
__host__ __device__ constexpr int kidx(int kx, int ky, int kz) {
  const int n = kx + ky + kz;
  return n * (n + 1) * (n + 2) / 6 + (n - kx) * (n - kx + 1) / 2 + (n - kx - ky);
}
struct K3 {
  int x, y, z;
};
__host__ __device__ constexpr K3 kof(int k) {  // the k-th multi-index of the graded order
  int i = 0;
  for (int n = 0; n <= 16; ++n)
    for (int x = n; x >= 0; --x)
      for (int y = n - x; y >= 0; --y) {
        if (i == k) return K3{x, y, n - x - y};
        ++i;
      }
  return K3{0, 0, 0};
}

// The Taylor coefficients of 1/|x - y| are harmonic in y: for k = m + 2 e_z,
//   k! a_k = -(m + 2 e_x)! a_{m + 2 e_x} - (m + 2 e_y)! a_{m + 2 e_y},
// so a sum over all |k| <= p of a_k M_k equals one over the k with k_z <= 1 only (2n + 1 per
// degree n, (p + 1)^2 in all) against folded moments, and the recurrence above, restricted to
// k_z <= 1, only ever refers to such k.  Reduced order: degree n from index n^2, first k_z = 0
// (k_x = n .. 0), then k_z = 1 (k_x = n - 1 .. 0).
constexpr int nred(int p) { return (p + 1) * (p + 1); }
__host__ __device__ constexpr int ridx(int kx, int ky, int kz) {
  const int n = kx + ky + kz;
  return n * n + (kz == 0 ? n - kx : n + 1 + (n - 1 - kx));
}
__host__ __device__ constexpr K3 rof(int k) {  // the k-th multi-index of the reduced order
  int n = 0;
  while ((n + 1) * (n + 1) <= k) ++n;
  const int j = k - n * n;
  return j <= n ? K3{n - j, j, 0} : K3{n - 1 - (j - n - 1), j - n - 1, 1};
}

// a_k(R) for |k| <= P, k_z <= 1, into a[nred(P)], one coefficient per instantiation, each
// added into v = sum_k a_k m_k as soon as it is formed (so that a coefficient is dead two
// degrees later, which keeps the registers of high orders down).
template <int P, int K, bool DOT = true>
__device__ __forceinline__ void taylor_rec(float rx, float ry, float rz, float ir2, float (&a)[nred(P)],
                                           const float *__restrict__ m, float &v) {
  if constexpr (K < nred(P)) {
    constexpr K3 t = rof(K);
    constexpr int n = t.x + t.y + t.z;
    constexpr float c1 = (float)(2 * n - 1) / (float)n, c2 = (float)(n - 1) / (float)n;
    float s1 = 0.0f, s2 = 0.0f;
    if constexpr (t.x >= 1) s1 = fmaf(rx, a[ridx(t.x - 1, t.y, t.z)], s1);
    if constexpr (t.y >= 1) s1 = fmaf(ry, a[ridx(t.x, t.y - 1, t.z)], s1);
    if constexpr (t.z >= 1) s1 = fmaf(rz, a[ridx(t.x, t.y, t.z - 1)], s1);
    if constexpr (t.x >= 2) s2 += a[ridx(t.x - 2, t.y, t.z)];
    if constexpr (t.y >= 2) s2 += a[ridx(t.x, t.y - 2, t.z)];
    a[K] = (c1 * s1 - c2 * s2) * ir2;
    if constexpr (DOT) v = fmaf(a[K], m[K], v);
    taylor_rec<P, K + 1, DOT>(rx, ry, rz, ir2, a, m, v);
  }
}

// sum over |k| <= P, k_z <= 1 of a_k(R) m_k, in the order of k
template <int P>
__device__ __forceinline__ float taylor_dot(float rx, float ry, float rz, const float *__restrict__ m) {
  float a[nred(P)];
  const float ir = __builtin_amdgcn_rsqf(rx * rx + ry * ry + rz * rz);
  a[0] = ir;
  float v = fmaf(ir, m[0], 0.0f);
  taylor_rec<P, 1>(rx, ry, rz, ir * ir, a, m, v);
  return v;
}

// the reduced coefficients a_k(R) alone
template <int P>
__device__ __forceinline__ void taylor_coef(float rx, float ry, float rz, float (&a)[nred(P)]) {
  const float ir = __builtin_amdgcn_rsqf(rx * rx + ry * ry + rz * rz);
  a[0] = ir;
  float unused = 0.0f;
  taylor_rec<P, 1, false>(rx, ry, rz, ir * ir, a, nullptr, unused);
}

// The coefficients with k_z >= 2 of a harmonic expansion from those with k_z <= 1, by the
// identity above, in increasing index order (both terms of a k have a lower index).
template <int P, int K>
__device__ __forceinline__ void unfold_rec(float (&f)[ncoef(P)]) {
  if constexpr (K < ncoef(P)) {
    constexpr K3 t = kof(K);
    if constexpr (t.z >= 2) {
      constexpr float d = (float)(t.z * (t.z - 1));
      constexpr float cx = (float)((t.x + 2) * (t.x + 1)) / d, cy = (float)((t.y + 2) * (t.y + 1)) / d;
      f[K] = -fmaf(cx, f[kidx(t.x + 2, t.y, t.z - 2)], cy * f[kidx(t.x, t.y + 2, t.z - 2)]);
    }
    unfold_rec<P, K + 1>(f);
  }
}

// sum_k L_k x^k over |k| <= P, the monomials built along the graded order
template <int P, int K>
__device__ __forceinline__ void local_rec(float x, float y, float z, float (&xk)[ncoef(P)],
                                          const float *__restrict__ L, float &v) {
  if constexpr (K < ncoef(P)) {
    constexpr K3 t = kof(K);
    if constexpr (t.x >= 1)
      xk[K] = xk[kidx(t.x - 1, t.y, t.z)] * x;
    else if constexpr (t.y >= 1)
      xk[K] = xk[kidx(t.x, t.y - 1, t.z)] * y;
    else
      xk[K] = xk[kidx(t.x, t.y, t.z - 1)] * z;
    v = fmaf(L[K], xk[K], v);
    local_rec<P, K + 1>(x, y, z, xk, L, v);
  }
}

// Folds the moments with k_z >= 2 into those of two lower k_z (the identity above), from the
// highest index down: both targets of a k have the same degree and a lower index.
template <int P, int K>
__device__ __forceinline__ void fold_rec(float (&f)[ncoef(P)]) {
  if constexpr (K >= 0) {
    constexpr K3 t = kof(K);
    if constexpr (t.z >= 2) {
      constexpr float d = (float)(t.z * (t.z - 1));
      constexpr float cx = (float)((t.x + 2) * (t.x + 1)) / d, cy = (float)((t.y + 2) * (t.y + 1)) / d;
      f[kidx(t.x + 2, t.y, t.z - 2)] = fmaf(-cx, f[K], f[kidx(t.x + 2, t.y, t.z - 2)]);
      f[kidx(t.x, t.y + 2, t.z - 2)] = fmaf(-cy, f[K], f[kidx(t.x, t.y + 2, t.z - 2)]);
    }
    fold_rec<P, K - 1>(f);
  }
}

template <int P, int K>
__device__ __forceinline__ void scatter_red(const float (&r)[nred(P)], float (&f)[ncoef(P)]) {
  if constexpr (K < nred(P)) {
    constexpr K3 t = rof(K);
    f[kidx(t.x, t.y, t.z)] = r[K];
    scatter_red<P, K + 1>(r, f);
  }
}

template <int P, int K>
__device__ __forceinline__ void reduce_rec(const float (&f)[ncoef(P)], float *__restrict__ out) {
  if constexpr (K < nred(P)) {
    constexpr K3 t = rof(K);
    out[K] = f[kidx(t.x, t.y, t.z)];
    reduce_rec<P, K + 1>(f, out);
  }
}

__device__ __forceinline__ unsigned spread3(unsigned v) {  // 10 bits -> every third bit
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}
__device__ __forceinline__ unsigned compact3(unsigned v) {
  v &= 0x09249249u;
  v = (v | (v >> 2)) & 0x030c30c3u;
  v = (v | (v >> 4)) & 0x0300f00fu;
  v = (v | (v >> 8)) & 0x030000ffu;
  v = (v | (v >> 16)) & 0x3ffu;
  return v;
}

// codes[i], ids[i] = i for every ion's image.
__global__ void k_tree_keys(int n, int D, float L, const float4 *__restrict__ img, unsigned *__restrict__ codes,
                            int *__restrict__ ids) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 v = img[i];
  unsigned code = TR_FAR;
  if (fabsf(v.x) < L && fabsf(v.y) < L && fabsf(v.z) < L) {
    const float sc = (float)(1 << D) / (2.0f * L);
    const int m = (1 << D) - 1;
    const int ix = min(m, max(0, (int)((v.x + L) * sc)));
    const int iy = min(m, max(0, (int)((v.y + L) * sc)));
    const int iz = min(m, max(0, (int)((v.z + L) * sc)));
    code = spread3((unsigned)ix) | (spread3((unsigned)iy) << 1) | (spread3((unsigned)iz) << 2);
  }
  codes[i] = code;
  ids[i] = i;
}

// Sorted images; inv[i] = sorted position of ion i's image.
__global__ void k_tree_gather(int n, const int *__restrict__ perm, const float4 *__restrict__ img,
                              float4 *__restrict__ simg, int *__restrict__ inv) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int i = perm[s];
  simg[s] = img[i];
  inv[i] = s;
}

// Codes of the targets (the ions) in the cube [-a, a]^3 at TR_TBITS bits per axis.
__global__ void k_tree_tkeys(int n, float a, const float4 *__restrict__ tgt, unsigned *__restrict__ codes,
                             int *__restrict__ ids) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 v = tgt[i];
  const float sc = (float)(1 << TR_TBITS) / (2.0f * a);
  const int m = (1 << TR_TBITS) - 1;
  const int ix = min(m, max(0, (int)((v.x + a) * sc)));
  const int iy = min(m, max(0, (int)((v.y + a) * sc)));
  const int iz = min(m, max(0, (int)((v.z + a) * sc)));
  codes[i] = spread3((unsigned)ix) | (spread3((unsigned)iy) << 1) | (spread3((unsigned)iz) << 2);
  ids[i] = i;
}

// Targets in their own sorted order, with the sorted position of each one's image.
__global__ void k_tree_tgather(int n, const int *__restrict__ tperm, const float4 *__restrict__ tgt,
                               const int *__restrict__ inv, float4 *__restrict__ stgt, int *__restrict__ town) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int i = tperm[s];
  stgt[s] = tgt[i];
  town[s] = inv[i];
}

// Run-length flags of the level-l keys: from the sorted codes (leaf level, src_key = codes,
// shift 0) or from the level-(l+1) cell keys (shift 3).  m = number of valid source entries
// (*m_dev, on the device); entries from m up to cap get flag 0.
__global__ void k_tree_flags(int cap, const int *__restrict__ m_dev, int m_host, const unsigned *__restrict__ src_key,
                             int shift, int *__restrict__ flags) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cap) return;
  const int m = m_dev ? *m_dev : m_host;
  int f = 0;
  if (j < m) f = (j == 0 || (src_key[j] >> shift) != (src_key[j - 1] >> shift)) ? 1 : 0;
  flags[j] = f;
}

// Cells of a level from the flags and their exclusive scan: key, first source entry (child),
// and first image (start).  The last thread also stores the count and the end sentinel.
__global__ void k_tree_cells(int cap, const int *__restrict__ m_dev, int m_host, int n_img,
                             const unsigned *__restrict__ src_key, int shift, const int *__restrict__ src_start,
                             const int *__restrict__ flags, const int *__restrict__ scan, unsigned *__restrict__ key,
                             int *__restrict__ child, int *__restrict__ start, int *__restrict__ count_out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = m_dev ? *m_dev : m_host;
  if (j < m && flags[j]) {
    const int c = scan[j];
    key[c] = src_key[j] >> shift;
    child[c] = j;
    start[c] = src_start ? src_start[j] : j;
  }
  if (j == 0) {
    const int nc = m > 0 ? scan[m - 1] + flags[m - 1] : 0;
    *count_out = nc;
    start[nc] = n_img;  // end sentinel of the last cell's images
    child[nc] = m;      // ... and of its children
  }
}

// Centre of the level-l octree cell of key k.
__device__ __forceinline__ float3 cell_centre(unsigned k, int level, float L) {
  const float h = 2.0f * L / (float)(1 << level);
  return make_float3(-L + ((float)compact3(k) + 0.5f) * h, -L + ((float)compact3(k >> 1) + 0.5f) * h,
                     -L + ((float)compact3(k >> 2) + 0.5f) * h);
}

// Moments, centre and radius of the leaf cells: one wave per cell (a grid-stride loop over the
// cells), the lanes over the coefficients k.  The images are taken 64 at a time: each lane
// stages the powers of one image's offset from the centre in LDS, then every lane adds
// q d_x^kx d_y^ky d_z^kz for its own k over the chunk, in image order.  The centre is the
// geometric centre of the octree cell; the far cell (outside the cube) gets radius +inf.
template <int P>
__global__ __launch_bounds__(64) void k_tree_moments(const int *__restrict__ ncell, int level, float L,
                                                    const unsigned *__restrict__ key, const int *__restrict__ start,
                                                    const float4 *__restrict__ simg, float4 *__restrict__ cen,
                                                    float *__restrict__ mom) {
  constexpr int NC = ncoef(P), NRND = (NC + 63) / 64;
  __shared__ float pw[64][3][P + 1];
  __shared__ float sq[64];
  const int lane = threadIdx.x;
  K3 kk[NRND];
  for (int r = 0; r < NRND; ++r) kk[r] = kof(lane + 64 * r < NC ? lane + 64 * r : 0);
  const int nc = *ncell;
  for (int c = blockIdx.x; c < nc; c += gridDim.x) {
    const unsigned k = key[c];
    if ((k >> (3 * level)) != 0) {  // cube cells of level l have keys below 8^l; the far cell has no moments
      if (lane == 0) cen[c] = make_float4(0.f, 0.f, 0.f, INFINITY);
      continue;
    }
    const float3 ce = cell_centre(k, level, L);
    const int s0 = start[c], s1 = start[c + 1];
    float acc[NRND];
    for (int r = 0; r < NRND; ++r) acc[r] = 0.0f;
    float rmax = 0.0f;
    for (int sb = s0; sb < s1; sb += 64) {
      const int cnt = s1 - sb < 64 ? s1 - sb : 64;
      __syncthreads();  // the previous chunk's powers are no longer read
      if (lane < cnt) {
        const float4 v = simg[sb + lane];
        const float d[3] = {v.x - ce.x, v.y - ce.y, v.z - ce.z};
        rmax = fmaxf(rmax, sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]));
        for (int a = 0; a < 3; ++a) {
          float p = 1.0f;
          for (int e = 0; e <= P; ++e) {
            pw[lane][a][e] = p;
            p *= d[a];
          }
        }
        sq[lane] = v.w;
      }
      __syncthreads();
      for (int r = 0; r < NRND; ++r) {
        if (lane + 64 * r >= NC) break;
        const K3 t = kk[r];
        float m = acc[r];
        for (int i = 0; i < cnt; ++i) m = fmaf(sq[i], pw[i][0][t.x] * pw[i][1][t.y] * pw[i][2][t.z], m);
        acc[r] = m;
      }
    }
    for (int o = 32; o > 0; o >>= 1) rmax = fmaxf(rmax, __shfl_xor(rmax, o));
    for (int r = 0; r < NRND; ++r)
      if (lane + 64 * r < NC) mom[(size_t)c * NC + lane + 64 * r] = acc[r];
    if (lane == 0) cen[c] = make_float4(ce.x, ce.y, ce.z, rmax);
  }
}

// Moments of the cells of level l < D from their children (level l + 1), about the parent's
// centre: M_k(parent) = sum over children and j <= k of C(k, j) (c_child - c_parent)^(k - j)
// M_j(child), with C the product of the three binomial coefficients.  The shift factorises into
// three one-dimensional shifts, taken as three passes over (child, k) in LDS (z, then y, then x,
// the last one also summing over the children in order), so that no lane sums more than p + 1
// terms per item.  One wave per parent (a grid-stride loop; a cell of the cube has at most 8
// children, stored consecutively).  The radius bound is max over children of
// |c_child - c_parent| + r_child.  Every group centre lies in the cavity, |g| <= a, so a cell with
// r_c >= theta (|c| + a) fails the acceptance test for every group: its moments are never read
// and are written as zeros instead (the upper levels, whose cells span much of the cube, and
// every cell at theta = 0).
template <int P>
__global__ __launch_bounds__(64) void k_tree_m2m(const int *__restrict__ ncell, int level, float L, float theta,
                                                float a, const unsigned *__restrict__ key,
                                                const int *__restrict__ child, const float4 *__restrict__ ccen,
                                                const float *__restrict__ cmom, float4 *__restrict__ cen,
                                                float *__restrict__ mom) {
  constexpr int NC = ncoef(P);
  __shared__ float sa[8 * NC], sb[8 * NC];
  __shared__ float pw[8][3][P + 1];
  __shared__ float bin[P + 1][P + 1];
  __shared__ float rad8[8];
  __shared__ int kt[NC];  // k_x | k_y << 8 | k_z << 16 of each index
  const int lane = threadIdx.x;
  for (int e = lane; e < (P + 1) * (P + 1); e += 64) {  // C(i, j), exact in FP32 for i <= 8
    const int i = e / (P + 1), j = e % (P + 1);
    float b = 1.0f;
    for (int u = 1; u <= j; ++u) b = b * (float)(i - j + u) / (float)u;
    bin[i][j] = j <= i ? b : 0.0f;
  }
  for (int k = lane; k < NC; k += 64) {
    const K3 t = kof(k);
    kt[k] = t.x | (t.y << 8) | (t.z << 16);
  }
  const int nc = *ncell;
  for (int c = blockIdx.x; c < nc; c += gridDim.x) {
    const unsigned k = key[c];
    if ((k >> (3 * level)) != 0) {  // the far cell: never accepted
      if (lane == 0) cen[c] = make_float4(0.f, 0.f, 0.f, INFINITY);
      continue;
    }
    const float3 ce = cell_centre(k, level, L);
    const int k0 = child[c];
    const int nch = min(child[c + 1] - k0, 8);
    __syncthreads();  // the previous parent's tables are no longer read
    if (lane < nch) {
      const float4 cc = ccen[k0 + lane];
      const float d[3] = {cc.x - ce.x, cc.y - ce.y, cc.z - ce.z};
      rad8[lane] = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) + cc.w;
      for (int ax = 0; ax < 3; ++ax) {
        float pv = 1.0f;
        for (int e = 0; e <= P; ++e) {
          pw[lane][ax][e] = pv;
          pv *= d[ax];
        }
      }
    }
    __syncthreads();
    float rad = 0.0f;
    for (int ch = 0; ch < nch; ++ch) rad = fmaxf(rad, rad8[ch]);
    if (lane == 0) cen[c] = make_float4(ce.x, ce.y, ce.z, rad);
    // never accepted (a margin of 1e-4 over the rounding of the traversal's test)
    if (rad >= 1.0001f * theta * (sqrtf(ce.x * ce.x + ce.y * ce.y + ce.z * ce.z) + a)) {
      for (int e = lane; e < NC; e += 64) mom[(size_t)c * NC + e] = 0.0f;
      continue;
    }
    for (int e = lane; e < nch * NC; e += 64) sa[e] = cmom[(size_t)k0 * NC + e];
    __syncthreads();
    // z: sb(x, y, z) = sum_{j <= z} C(z, j) d_z^(z - j) sa(x, y, j)
    for (int e = lane; e < nch * NC; e += 64) {
      const int ch = e / NC, t = kt[e - ch * NC];
      const int x = t & 255, y = (t >> 8) & 255, z = t >> 16;
      const float *src = sa + ch * NC;
      float v = 0.0f;
      for (int j = 0; j <= z; ++j) v = fmaf(bin[z][j] * pw[ch][2][z - j], src[kidx(x, y, j)], v);
      sb[e] = v;
    }
    __syncthreads();
    // y: sa(x, y, z) = sum_{j <= y} C(y, j) d_y^(y - j) sb(x, j, z)
    for (int e = lane; e < nch * NC; e += 64) {
      const int ch = e / NC, t = kt[e - ch * NC];
      const int x = t & 255, y = (t >> 8) & 255, z = t >> 16;
      const float *src = sb + ch * NC;
      float v = 0.0f;
      for (int j = 0; j <= y; ++j) v = fmaf(bin[y][j] * pw[ch][1][y - j], src[kidx(x, j, z)], v);
      sa[e] = v;
    }
    __syncthreads();
    // x, summed over the children in order: M(x, y, z) = sum_ch sum_{j <= x} C(x, j) d_x^(x - j) sa(j, y, z)
    for (int e = lane; e < NC; e += 64) {
      const int t = kt[e];
      const int x = t & 255, y = (t >> 8) & 255, z = t >> 16;
      float v = 0.0f;
      for (int ch = 0; ch < nch; ++ch) {
        const float *src = sa + ch * NC;
        for (int j = 0; j <= x; ++j) v = fmaf(bin[x][j] * pw[ch][0][x - j], src[kidx(j, y, z)], v);
      }
      mom[(size_t)c * NC + e] = v;
    }
  }
}

// Surface nodes and their strengths (Q, D) in their sorted order.
__global__ void k_tree_ngather(int pn, const int *__restrict__ perm, const float4 *__restrict__ nodes,
                               const float2 *__restrict__ qd, float4 *__restrict__ snodes, float2 *__restrict__ sqd) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= pn) return;
  const int i = perm[s];
  snodes[s] = nodes[i];
  sqd[s] = qd[i];
}

// Moments of the patches of surface nodes (runs of up to 64 sorted nodes within cells): one
// wave per patch, a grid-stride loop.  A node y of strengths (Q, D) is a charge Q and the
// radial dipole p = D y (its potential at x is Q / |x - y| + D (x - y).y / |x - y|^3, the form
// of the direct sum), so with d = y - c
//   M_k += Q d^k + sum_i p_i k_i d^(k - e_i),
// the dipole's moments being p . grad_y of the charge's.  The centre is the centre of the
// patch's bounding box; pstart gets each patch's first node and the end sentinel.
template <int P>
__global__ __launch_bounds__(64) void k_tree_patch(const int *__restrict__ npatch, const int2 *__restrict__ pr,
                                                  const float4 *__restrict__ snodes, const float2 *__restrict__ sqd,
                                                  int mono, float4 *__restrict__ pcen, int *__restrict__ pstart,
                                                  float *__restrict__ pm) {
  constexpr int NC = ncoef(P), NRND = (NC + 63) / 64;
  __shared__ float pw[64][3][P + 1];
  __shared__ float4 sw[64];  // Q, p
  const int lane = threadIdx.x;
  K3 kk[NRND];
  for (int r = 0; r < NRND; ++r) kk[r] = kof(lane + 64 * r < NC ? lane + 64 * r : 0);
  const int np = *npatch;
  for (int g = blockIdx.x; g < np; g += gridDim.x) {
    const int2 rg = pr[g];
    const bool in = lane < rg.y;
    const float4 y = snodes[rg.x + (in ? lane : 0)];
    const float2 w = sqd[rg.x + (in ? lane : 0)];
    float lo[3] = {y.x, y.y, y.z}, hi[3] = {y.x, y.y, y.z};
    for (int o = 32; o > 0; o >>= 1)
      for (int a = 0; a < 3; ++a) {
        lo[a] = fminf(lo[a], __shfl_xor(lo[a], o));
        hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], o));
      }
    const float c[3] = {0.5f * (lo[0] + hi[0]), 0.5f * (lo[1] + hi[1]), 0.5f * (lo[2] + hi[2])};
    const float d[3] = {y.x - c[0], y.y - c[1], y.z - c[2]};
    float rad = in ? sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) : 0.0f;
    for (int o = 32; o > 0; o >>= 1) rad = fmaxf(rad, __shfl_xor(rad, o));
    __syncthreads();  // the previous patch's tables are no longer read
    if (in) {
      for (int a = 0; a < 3; ++a) {
        float pv = 1.0f;
        for (int e = 0; e <= P; ++e) {
          pw[lane][a][e] = pv;
          pv *= d[a];
        }
      }
      const float D = mono ? 0.0f : w.y;
      sw[lane] = make_float4(w.x, D * y.x, D * y.y, D * y.z);
    }
    __syncthreads();
    for (int r = 0; r < NRND; ++r) {
      if (lane + 64 * r >= NC) break;
      const K3 t = kk[r];
      float m = 0.0f;
      for (int i = 0; i < rg.y; ++i) {
        const float px = pw[i][0][t.x], py = pw[i][1][t.y], pz = pw[i][2][t.z];
        const float4 q = sw[i];
        float v = q.x * px * py * pz;
        if (t.x > 0) v = fmaf(q.y * (float)t.x, pw[i][0][t.x - 1] * py * pz, v);
        if (t.y > 0) v = fmaf(q.z * (float)t.y, px * pw[i][1][t.y - 1] * pz, v);
        if (t.z > 0) v = fmaf(q.w * (float)t.z, px * py * pw[i][2][t.z - 1], v);
        m += v;
      }
      pm[(size_t)g * NC + lane + 64 * r] = m;
    }
    if (lane == 0) {
      pcen[g] = make_float4(c[0], c[1], c[2], rad);
      pstart[g] = rg.x;
      if (g == np - 1) pstart[np] = rg.x + rg.y;
    }
  }
}

// Target groups: the sorted targets of each cell of the targets' grouping level in runs of up
// to 64, so that no group straddles a jump of the space-filling order.  ng[c] = groups of cell c.
__global__ void k_tree_gcount(int cap, const int *__restrict__ ncell, const int *__restrict__ start,
                              int *__restrict__ ng) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cap) return;
  ng[c] = c < *ncell ? (start[c + 1] - start[c] + 63) / 64 : 0;
}

__global__ void k_tree_gfill(int cap, const int *__restrict__ ncell, const int *__restrict__ start,
                             const int *__restrict__ ng, const int *__restrict__ gofs, int2 *__restrict__ gr,
                             int *__restrict__ ngroups) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int nc = *ncell;
  if (c == 0) *ngroups = nc > 0 ? gofs[nc - 1] + ng[nc - 1] : 0;
  if (c >= cap || c >= nc) return;
  const int s0 = start[c], cnt = start[c + 1] - s0;
  for (int k = 0; k < ng[c]; ++k) gr[gofs[c] + k] = make_int2(s0 + 64 * k, min(64, cnt - 64 * k));
}

// Bounding sphere of each target group, and a sort key that orders the groups by decreasing
// distance of their centre from the cavity's: groups near the interface, close to the dense
// shell of images just outside it, open the most cells, and are launched first so that the
// light ones fill the end of the launch.  Slots beyond the group count get the largest key.
__global__ __launch_bounds__(64) void k_tree_groups(const int *__restrict__ ngroups, const int2 *__restrict__ gr,
                                                    const float4 *__restrict__ stgt, float4 *__restrict__ grp,
                                                    unsigned *__restrict__ gkey, int *__restrict__ gid) {
  const int g = blockIdx.x, lane = threadIdx.x;
  if (g >= *ngroups) {
    if (lane == 0) {
      gkey[g] = 0xffffffffu;
      gid[g] = g;
    }
    return;
  }
  const int2 rg = gr[g];
  const bool in = lane < rg.y;
  const float4 t = stgt[rg.x + (in ? lane : 0)];
  float lo[3] = {t.x, t.y, t.z}, hi[3] = {t.x, t.y, t.z};
  for (int o = 32; o > 0; o >>= 1)
    for (int d = 0; d < 3; ++d) {
      lo[d] = fminf(lo[d], __shfl_xor(lo[d], o));
      hi[d] = fmaxf(hi[d], __shfl_xor(hi[d], o));
    }
  const float cx = 0.5f * (lo[0] + hi[0]), cy = 0.5f * (lo[1] + hi[1]), cz = 0.5f * (lo[2] + hi[2]);
  float r = in ? sqrtf((t.x - cx) * (t.x - cx) + (t.y - cy) * (t.y - cy) + (t.z - cz) * (t.z - cz)) : 0.0f;
  for (int o = 32; o > 0; o >>= 1) r = fmaxf(r, __shfl_xor(r, o));
  if (lane == 0) {
    grp[g] = make_float4(cx, cy, cz, r);
    // non-negative floats order as their bit patterns; the complement reverses the order
    gkey[g] = ~__float_as_uint(sqrtf(cx * cx + cy * cy + cz * cz)) & 0x7fffffffu;
    gid[g] = g;
  }
}

// One cell of any level, as the traversal reads it: one 32-byte scalar load per visit.  Cells
// are numbered globally, level by level (level l from off[l]); a leaf has k0 == k1.
struct __align__(32) CellRec {
  float cx, cy, cz, r;  // geometric centre and radius bound (+inf for the far cell)
  int s0, s1;           // sorted images [s0, s1)
  int k0, k1;           // children [k0, k1), global numbers
};

// Records of the cells of level l (children of level l + 1 numbered from off_next), and their
// moments folded to the reduced set (zero for the far cell, which is never accepted).
template <int P>
__global__ void k_tree_pack(int cap, const int *__restrict__ ncell, int leaf, int off_l, int off_next,
                            const float4 *__restrict__ cen, const int *__restrict__ start,
                            const int *__restrict__ child, const float *__restrict__ mom, CellRec *__restrict__ rec,
                            float *__restrict__ red) {
  constexpr int NC = ncoef(P), NR = nred(P);
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cap || c >= *ncell) return;
  const float4 cc = cen[c];
  float *out = red + (size_t)(off_l + c) * NR;
  if (cc.w == INFINITY) {
    for (int k = 0; k < NR; ++k) out[k] = 0.0f;
  } else {
    float f[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) f[k] = mom[(size_t)c * NC + k];
    fold_rec<P, NC - 1>(f);
    reduce_rec<P, 0>(f, out);
  }
  CellRec r;
  r.cx = cc.x;
  r.cy = cc.y;
  r.cz = cc.z;
  r.r = cc.w;
  r.s0 = start[c];
  r.s1 = start[c + 1];
  const bool lf = leaf || r.s1 - r.s0 <= TR_LEAF;
  r.k0 = lf ? 0 : off_next + child[c];
  r.k1 = lf ? 0 : off_next + child[c + 1];
  rec[off_l + c] = r;
}

template <int U, bool MASK>
__device__ __forceinline__ void direct_terms(float tx, float ty, float tz, int own, const float4 *__restrict__ simg,
                                             int j, float &sum) {
  float4 v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) v[u] = simg[j + u];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const float dx = tx - v[u].x, dy = ty - v[u].y, dz = tz - v[u].z;
    float ri = __builtin_amdgcn_rsqf(dx * dx + dy * dy + dz * dz);
    if constexpr (MASK) ri = (j + u == own) ? 0.0f : ri;
    sum = fmaf(v[u].w, ri, sum);
  }
}

template <bool MASK>
__device__ __forceinline__ void direct_blocks(float tx, float ty, float tz, int own, const float4 *__restrict__ simg,
                                              int s0, int s1, double &acc) {
  for (int sb = s0; sb < s1; sb += 32) {
    const int se = sb + 32 < s1 ? sb + 32 : s1;
    float sum = 0.0f;
    int j = sb;
    for (; j + 4 <= se; j += 4) direct_terms<4, MASK>(tx, ty, tz, own, simg, j, sum);
    for (; j < se; ++j) direct_terms<1, MASK>(tx, ty, tz, own, simg, j, sum);
    acc += (double)sum;
  }
}

// sum over the images [s0, s1) but the ion's own, in FP32 blocks of 32 terms added into FP64;
// the loads are issued four at a time.  The own image is masked only where some lane's own
// image lies in the range (the same sums either way).
__device__ __forceinline__ void direct_range(float tx, float ty, float tz, int own, const float4 *__restrict__ simg,
                                             int s0, int s1, double &acc) {
  if (__ballot(own >= s0 && own < s1) != 0)
    direct_blocks<true>(tx, ty, tz, own, simg, s0, s1, acc);
  else
    direct_blocks<false>(tx, ty, tz, own, simg, s0, s1, acc);
}

// Local expansion about the centre of the far set (the images outside the cube, beyond 8a,
// of ions within a/8 of the centre), for theta > 0: every target lies within a of the centre,
// so 1/|y - x| = sum_k a_k(y) x^k converges like (1/8)^(p+1), far below the treecode's own
// truncation.  L_k = sum_far q_K a_k(y_K) over the reduced k (one lane per image, then a fixed
// butterfly over the lanes), the others from the harmonic identity.  One wave.
template <int P>
__global__ __launch_bounds__(64) void k_tree_local(int n, const unsigned *__restrict__ key0,
                                                  const int *__restrict__ start0, const int *__restrict__ ncell,
                                                  const float4 *__restrict__ simg, float *__restrict__ Lout) {
  constexpr int NR = nred(P), NC = ncoef(P);
  const int lane = threadIdx.x;
  int far_start = n;
  for (int c = 0; c < ncell[0]; ++c)
    if (key0[c] != 0u) far_start = start0[c];
  float acc[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) acc[k] = 0.0f;
  for (int j = far_start + lane; j < n; j += 64) {
    const float4 v = simg[j];
    float a[NR];
    taylor_coef<P>(v.x, v.y, v.z, a);
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[k] = fmaf(v.w, a[k], acc[k]);
  }
#pragma unroll
  for (int k = 0; k < NR; ++k)
    for (int o = 32; o > 0; o >>= 1) acc[k] += __shfl_xor(acc[k], o);
  if (lane == 0) {
    float f[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) f[k] = 0.0f;
    scatter_red<P, 0>(acc, f);
    unfold_rec<P, 0>(f);
#pragma unroll
    for (int k = 0; k < NC; ++k) Lout[k] = f[k];
  }
}

template <int U>
__device__ __forceinline__ void surface_terms(float tx, float ty, float tz, int mono, const float4 *__restrict__ nodes,
                                              const float2 *__restrict__ qd, int m, float &sum) {
  float4 yv[U];
  float2 wv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    yv[u] = nodes[m + u];
    wv[u] = qd[m + u];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const float dx = tx - yv[u].x, dy = ty - yv[u].y, dz = tz - yv[u].z;
    const float ri = __builtin_amdgcn_rsqf(dx * dx + dy * dy + dz * dz);
    if (mono) {
      sum = fmaf(wv[u].x, ri, sum);
    } else {
      const float dot = dx * yv[u].x + dy * yv[u].y + dz * yv[u].z;
      sum = fmaf(ri, fmaf(wv[u].y * dot, ri * ri, wv[u].x), sum);
    }
  }
}

// One wave per group of up to 64 sorted targets: traversal, far set, surface nodes; writes phi
// in the ions' original order (own-image term included).  Every decision of the traversal is
// taken from cell and group data alone, so it is uniform over the wave and runs on the scalar
// unit; the acceptance test is compared in squares, (r_c + r_g)^2 < theta^2 d^2.
template <int P>
__global__ __launch_bounds__(64 * TR_WAVES) void k_tree_eval(int n, float theta2, const CellRec *__restrict__ rec,
                                                            const float *__restrict__ red,
                                                            const unsigned *__restrict__ key0,
                                                            const int *__restrict__ start0,
                                                            const int *__restrict__ ncell,
                                                            const float4 *__restrict__ simg,
                                                            const float4 *__restrict__ stgt,
                                                            const int *__restrict__ town,
                                                            const int *__restrict__ perm,
                                                            const int *__restrict__ ngroups,
                                                            const int *__restrict__ gorder,
                                                            const int2 *__restrict__ gr,
                                                            const float4 *__restrict__ grp,
                                                            const double *__restrict__ self, int mono,
                                                            const float *__restrict__ Lfar,
                                                            const CellRec *__restrict__ prec,
                                                            const float *__restrict__ pred,
                                                            const int *__restrict__ npatch,
                                                            const float4 *__restrict__ snodes,
                                                            const float2 *__restrict__ sqd, double *__restrict__ phi) {
  constexpr int NR = nred(P);
  __shared__ int stack[TR_WAVES][TR_STACK];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int slot = blockIdx.x * TR_WAVES + w;
  if (slot >= *ngroups) return;
  const int g = gorder[slot];  // the valid groups sort first
  const int2 gg = gr[g];
  const bool in = lane < gg.y;
  const int s = gg.x + (in ? lane : 0);
  const float4 t = stgt[s];
  const int own = in ? town[s] : -1;  // sorted position of the target's own image
  const float4 G = grp[g];
  double acc = 0.0;
  int sp = 0;
  // level 0 (cells 0 and 1): the cube, key 0, pushed as the root, and the cell of the images
  // outside the cube, the far set, summed directly below
  int far_start = n;
  const int n0 = ncell[0];
  for (int c = 0; c < n0; ++c) {
    if (key0[c] == 0u)
      stack[w][sp++] = c;
    else
      far_start = start0[c];
  }
  while (sp > 0) {
    const int c = __builtin_amdgcn_readfirstlane(stack[w][--sp]);
    const CellRec rc = rec[c];
    const float dx = rc.cx - G.x, dy = rc.cy - G.y, dz = rc.cz - G.z;
    const float rs = rc.r + G.w;
    const int accept = __builtin_amdgcn_readfirstlane((int)(rs * rs < theta2 * (dx * dx + dy * dy + dz * dz)));
    if (accept) {
      float v = taylor_dot<P>(t.x - rc.cx, t.y - rc.cy, t.z - rc.cz, red + (size_t)c * NR);
      if (own >= rc.s0 && own < rc.s1) {  // the ion's own image is in the cell: take its term out again
        const float4 o = simg[own];
        const float ox = t.x - o.x, oy = t.y - o.y, oz = t.z - o.z;
        v -= o.w * __builtin_amdgcn_rsqf(ox * ox + oy * oy + oz * oz);
      }
      acc += (double)v;
    } else if (rc.k0 == rc.k1) {  // a leaf
      direct_range(t.x, t.y, t.z, own, simg, rc.s0, rc.s1, acc);
    } else {
      for (int k = rc.k1 - 1; k >= rc.k0 && sp < TR_STACK; --k) stack[w][sp++] = k;
    }
  }
  if (far_start < n) {
    if (theta2 > 0.0f) {  // the local expansion of the far set; an own image there is taken out
      float xk[ncoef(P)];  // monomials t^k
      xk[0] = 1.0f;
      float v = Lfar[0];
      local_rec<P, 1>(t.x, t.y, t.z, xk, Lfar, v);
      if (own >= far_start) {
        const float4 o = simg[own];
        const float ox = t.x - o.x, oy = t.y - o.y, oz = t.z - o.z;
        v -= o.w * __builtin_amdgcn_rsqf(ox * ox + oy * oy + oz * oz);
      }
      acc += (double)v;
    } else {
      direct_range(t.x, t.y, t.z, own, simg, far_start, n, acc);
    }
  }
  // surface nodes: each patch from its multipoles when the same test accepts it, else directly
  const int np = *npatch;
  for (int pc = 0; pc < np; ++pc) {
    const CellRec rc = prec[pc];
    const float dx = rc.cx - G.x, dy = rc.cy - G.y, dz = rc.cz - G.z;
    const float rs = rc.r + G.w;
    const int accept = __builtin_amdgcn_readfirstlane((int)(rs * rs < theta2 * (dx * dx + dy * dy + dz * dz)));
    if (accept) {
      acc += (double)taylor_dot<P>(t.x - rc.cx, t.y - rc.cy, t.z - rc.cz, pred + (size_t)pc * NR);
    } else {
      float sum = 0.0f;
      int m = rc.s0;
      for (; m + 4 <= rc.s1; m += 4) surface_terms<4>(t.x, t.y, t.z, mono, snodes, sqd, m, sum);
      for (; m < rc.s1; ++m) surface_terms<1>(t.x, t.y, t.z, mono, snodes, sqd, m, sum);
      acc += (double)sum;
    }
  }
  if (in) {
    const int i = perm[s];
    phi[i] = self[i] + acc;
  }
}

// Block partials of (1/2) sum q phi in the original ion order, then one block adds them.
__global__ __launch_bounds__(256) void k_tree_epart(int n, const double *__restrict__ q,
                                                    const double *__restrict__ phi, double *__restrict__ ep) {
  __shared__ double red[256];
  const int i = blockIdx.x * 256 + threadIdx.x;
  red[threadIdx.x] = i < n ? 0.5 * q[i] * phi[i] : 0.0;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) ep[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_tree_esum(int nb, const double *__restrict__ ep, double *__restrict__ E) {
  __shared__ double red[256];
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) s += ep[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *E = red[0];
}

inline int64_t cdivl(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Calls f with the multipole order as a compile-time constant (decltype(o)::value): 2, 4, 6, 8 or 10.
template <typename F>
void with_order(int P, F &&f) {
  switch (P) {
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    default: f(std::integral_constant<int, 10>{}); break;
  }
}

// Level of the targets' cells in [-a, a]^3 that no group crosses: about 8 groups of 64 per cell
// of a uniformly filled cavity (the ball fills pi/6 of the cube), so that groups are nearly full.
int target_level(int64_t n) {
  const int l = (int)std::lround(std::log2((double)(n > 1 ? n : 1) / 200.0) / 3.0);
  return l < 0 ? 0 : (l > TR_TBITS ? TR_TBITS : l);
}
inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// Level of the nodes' cells in the cube of half-width 1.125 R_tau: the sphere crosses about
// pi 4^l cells of level l, so that about 32 nodes fall in each.
int patch_level(int pn) {
  const int l = (int)std::lround(std::log2((double)(pn > 1 ? pn : 1) / 100.0) / 2.0);
  return l < 0 ? 0 : (l > TR_TBITS ? TR_TBITS : l);
}

int auto_depth(int64_t n) {
  // the fastest depth measured on uniformly filled cavities: 7 at N = 10^6, 6 at 2 10^5
  const double d = 7.0 + (std::log2((double)(n > 1 ? n : 1)) - std::log2(1e6)) / 3.0;
  int D = (int)std::lround(d);
  return D < 2 ? 2 : (D > TR_MAX_DEPTH - 1 ? TR_MAX_DEPTH - 1 : D);
}

struct TreeLayout {
  int D, P, nc, ngroups, lt, pn, lp, npcap;
  int64_t cap[TR_MAX_DEPTH + 1], tcap, ncap;
  size_t codes_a, codes_b, ids_a, ids_b, codes_t, ids_t, town, simg, stgt, inv, flags, scan, grp, gr, gng, gofs,
      tkey, tstart, tchild, gkey_a, gkey_b, gid_a, gid_b, ncell, ep, temp, temp_bytes;
  size_t key[TR_MAX_DEPTH + 1], start[TR_MAX_DEPTH + 1], child[TR_MAX_DEPTH + 1], cen[TR_MAX_DEPTH + 1];
  int64_t off[TR_MAX_DEPTH + 2];  // global number of each level's first cell; off[D + 1] = all cells
  size_t rec, mom, red;           // records, moments and folded moments of every cell, by global number
  size_t lfar;                    // local expansion of the far set, ncoef(P) floats
  // surface nodes: sort, cells of level lp, patches and their records and moments
  size_t ncodes_a, ncodes_b, nids_a, nids_b, nflags, nscan, snodes, sqd, nkey, nstart, nchild, nng, ngofs, pr, pcen,
      pstart, pm, prec, pred;
  size_t total;
};

hsma_status tree_layout(int64_t n, int D, int P, int pn, size_t base, TreeLayout &T) {
  T.D = D;
  T.P = P;
  T.nc = ncoef(P);
  size_t o = al256(base);
  auto take = [&](size_t b) {
    const size_t at = o;
    o = al256(o + (b > 0 ? b : 1));
    return at;
  };
  const size_t N = (size_t)(n > 0 ? n : 1);
  T.codes_a = take(4 * N);
  T.codes_b = take(4 * N);
  T.ids_a = take(4 * N);
  T.ids_b = take(4 * N);
  T.codes_t = take(4 * N);
  T.ids_t = take(4 * N);
  T.town = take(4 * N);
  T.simg = take(16 * N);
  T.stgt = take(16 * N);
  T.inv = take(4 * N);
  T.flags = take(4 * N);
  T.scan = take(4 * N);

  // cells per level; at TR_MAX_DEPTH + 1 the number of target groups, at + 2 of target cells,
  // at + 3 of node cells, at + 4 of node patches
  T.ncell = take(4 * (TR_MAX_DEPTH + 5));
  T.ep = take(8 * (size_t)cdivl(n, 256));
  for (int l = 0; l <= D; ++l) {
    int64_t c = (int64_t)1 << (3 * l);
    c = (c + 1 < (int64_t)N ? c + 1 : (int64_t)N);  // level l holds at most 8^l cube cells and the far cell
    T.cap[l] = c;
  }
  // target cells: at most 8^lt, and at most one per target
  T.lt = target_level(n);
  T.tcap = std::min<int64_t>((int64_t)1 << (3 * T.lt), (int64_t)N);
  T.tkey = take(4 * (size_t)T.tcap);
  T.tstart = take(4 * ((size_t)T.tcap + 1));
  T.tchild = take(4 * ((size_t)T.tcap + 1));
  // target groups: at most one partial group per target cell
  T.ngroups = (int)(cdivl(n, 64) + T.tcap);
  T.grp = take(16 * (size_t)T.ngroups);
  T.gr = take(8 * (size_t)T.ngroups);
  T.gng = take(4 * (size_t)T.tcap);
  T.gofs = take(4 * (size_t)T.tcap);
  T.gkey_a = take(4 * (size_t)T.ngroups);  // launch order of the groups, sorted by key
  T.gkey_b = take(4 * (size_t)T.ngroups);
  T.gid_a = take(4 * (size_t)T.ngroups);
  T.gid_b = take(4 * (size_t)T.ngroups);
  T.off[0] = 0;
  for (int l = 0; l <= D; ++l) {
    const int64_t c = T.cap[l];
    T.key[l] = take(4 * (size_t)c);
    T.start[l] = take(4 * ((size_t)c + 1));
    T.child[l] = take(4 * ((size_t)c + 1));
    T.cen[l] = take(16 * (size_t)c);
    T.off[l + 1] = T.off[l] + c;
  }
  T.rec = take(sizeof(CellRec) * (size_t)T.off[D + 1]);
  T.pn = pn;
  const size_t PN = (size_t)(pn > 0 ? pn : 1);
  T.lp = patch_level(pn);
  T.ncap = std::min<int64_t>((int64_t)1 << (3 * T.lp), (int64_t)PN);
  T.npcap = (int)(cdivl((int64_t)PN, 64) + T.ncap);
  T.ncodes_a = take(4 * PN);
  T.ncodes_b = take(4 * PN);
  T.nids_a = take(4 * PN);
  T.nids_b = take(4 * PN);
  T.nflags = take(4 * PN);
  T.nscan = take(4 * PN);
  T.snodes = take(16 * PN);
  T.sqd = take(8 * PN);
  T.nkey = take(4 * (size_t)T.ncap);
  T.nstart = take(4 * ((size_t)T.ncap + 1));
  T.nchild = take(4 * ((size_t)T.ncap + 1));
  T.nng = take(4 * (size_t)T.ncap);
  T.ngofs = take(4 * (size_t)T.ncap);
  T.pr = take(8 * (size_t)T.npcap);
  T.pcen = take(16 * (size_t)T.npcap);
  T.pstart = take(4 * ((size_t)T.npcap + 1));
  T.pm = take(4 * (size_t)T.npcap * T.nc);
  T.prec = take(sizeof(CellRec) * (size_t)T.npcap);
  T.pred = take(4 * (size_t)T.npcap * nred(P));
  T.mom = take(4 * (size_t)T.off[D + 1] * T.nc);
  T.red = take(4 * (size_t)T.off[D + 1] * nred(P));
  T.lfar = take(4 * (size_t)T.nc);
  size_t sort_b = 0, scan_b = 0;
  // the images' sort, the targets', and the groups' launch order (up to 2 N groups)
  const unsigned ns = (unsigned)std::max<int64_t>(std::max<int64_t>((int64_t)N, T.ngroups), (int64_t)PN);
  for (int bits : {31, 3 * TR_TBITS, 32}) {
    size_t b = 0;
    if (rocprim::radix_sort_pairs(nullptr, b, (const unsigned *)nullptr, (unsigned *)nullptr, (const int *)nullptr,
                                  (int *)nullptr, ns, 0, bits) != hipSuccess)
      return HSMA_EDEVICE;
    sort_b = b > sort_b ? b : sort_b;
  }
  if (rocprim::exclusive_scan(nullptr, scan_b, (const int *)nullptr, (int *)nullptr, 0, std::max(N, PN),
                              rocprim::plus<int>()) !=
      hipSuccess)
    return HSMA_EDEVICE;
  T.temp_bytes = sort_b > scan_b ? sort_b : scan_b;
  T.temp = take(T.temp_bytes);
  T.total = o;
  return HSMA_OK;
}

}  // namespace
}  // namespace hsma

using namespace hsma;

static hsma_status tree_args(hsma_plan_t pl, int64_t N, const hsma_tree_opts *opts, int &D, int &P, float &theta) {
  if (!pl || N < 0 || !opts) return HSMA_EINVAL;
  if (pl->opts.pair_prec != HSMA_PAIR_FP32 && pl->opts.pair_prec != HSMA_PAIR_FP32_COMP) return HSMA_EINVAL;
  if (!(opts->theta >= 0.0 && opts->theta < 1.0)) return HSMA_EINVAL;
  if (opts->order != 2 && opts->order != 4 && opts->order != 6 && opts->order != 8 &&
      opts->order != 10)
    return HSMA_EINVAL;
  if (opts->depth != 0 && (opts->depth < 2 || opts->depth > TR_MAX_DEPTH - 1)) return HSMA_EINVAL;
  if (N > ((int64_t)1 << 27) - 1) return HSMA_EINVAL;  // global cell numbers, at most (D + 1) N, in an int
  D = opts->depth ? opts->depth : auto_depth(N);
  P = opts->order;
  theta = (float)opts->theta;
  return HSMA_OK;
}

extern "C" size_t hsma_tree_workspace_bytes(hsma_plan_t pl, int64_t N, const hsma_tree_opts *opts) {
  int D, P;
  float th;
  if (tree_args(pl, N, opts, D, P, th) != HSMA_OK) return 0;
  Layout L = layout(pl->self, 1, N, N, false, true);
  TreeLayout T;
  if (tree_layout(N, D, P, pl->self->P_ev, L.total, T) != HSMA_OK) return 0;
  return T.total;
}

extern "C" hsma_status hsma_energy_tree(hsma_plan_t pl, int64_t N, const double *x, const double *y, const double *z,
                                        const double *q, double *phi, double *E, const hsma_tree_opts *opts, void *ws,
                                        size_t ws_bytes, hipStream_t st) {
  int D, P;
  float theta;
  hsma_status rc = tree_args(pl, N, opts, D, P, theta);
  if (rc != HSMA_OK) return rc;
  if (!ws || ((uintptr_t)ws & 255) != 0 || (N > 0 && (!x || !y || !z || !q || !phi))) return HSMA_EINVAL;
  int dev = -1;
  HSMA_HIP(hipGetDevice(&dev));
  if (dev != pl->device) return HSMA_ESTATE;
  Layout L = layout(pl->self, 1, N, N, false, true);
  L.upto_fit = true;
  TreeLayout T;
  rc = tree_layout(N, D, P, pl->self->P_ev, L.total, T);
  if (rc != HSMA_OK) return rc;
  if (ws_bytes < T.total) return HSMA_EINVAL;
  char *w = (char *)ws;
  if (N == 0) {
    if (E) k_tree_esum<<<1, 256, 0, st>>>(0, nullptr, E);
    HSMA_HIP(hipGetLastError());
    return HSMA_OK;
  }
  rc = run_front(pl->self, L, N, x, y, z, q, w, st);
  if (rc != HSMA_OK) return rc;
  const int n = (int)N;
  const float4 *img = (const float4 *)(w + L.img);
  const float4 *tgt = (const float4 *)(w + L.tgt);
  const double *self = (const double *)(w + L.self);
  const float2 *qd = (const float2 *)(w + L.qd);
  unsigned *codes_a = (unsigned *)(w + T.codes_a), *codes_b = (unsigned *)(w + T.codes_b);
  int *ids_a = (int *)(w + T.ids_a), *ids_b = (int *)(w + T.ids_b);
  float4 *simg = (float4 *)(w + T.simg), *stgt = (float4 *)(w + T.stgt);
  int *inv = (int *)(w + T.inv), *flags = (int *)(w + T.flags), *scan = (int *)(w + T.scan);
  int *ncell = (int *)(w + T.ncell);
  const float Lc = (float)(TR_CUBE * pl->a);
  const int nb = (int)cdivl(n, 256);
  k_tree_keys<<<nb, 256, 0, st>>>(n, D, Lc, img, codes_a, ids_a);
  size_t tb = T.temp_bytes;
  HSMA_HIP(rocprim::radix_sort_pairs(w + T.temp, tb, codes_a, codes_b, ids_a, ids_b, (unsigned)n, 0, 31, st));
  k_tree_gather<<<nb, 256, 0, st>>>(n, ids_b, img, simg, inv);
  // levels from the leaves up
  for (int l = D; l >= 0; --l) {
    const int64_t cap_src = l == D ? N : T.cap[l + 1];
    const unsigned *src_key = l == D ? codes_b : (const unsigned *)(w + T.key[l + 1]);
    const int *src_start = l == D ? nullptr : (const int *)(w + T.start[l + 1]);
    const int *m_dev = l == D ? nullptr : ncell + (l + 1);
    const int shift = l == D ? 0 : 3;
    const int gsrc = (int)cdivl(cap_src, 256);
    k_tree_flags<<<gsrc, 256, 0, st>>>((int)cap_src, m_dev, n, src_key, shift, flags);
    size_t sb = T.temp_bytes;
    HSMA_HIP(rocprim::exclusive_scan(w + T.temp, sb, flags, scan, 0, (size_t)cap_src, rocprim::plus<int>(), st));
    k_tree_cells<<<gsrc, 256, 0, st>>>((int)cap_src, m_dev, n, n, src_key, shift, src_start, flags, scan,
                                       (unsigned *)(w + T.key[l]), (int *)(w + T.child[l]), (int *)(w + T.start[l]),
                                       ncell + l);
  }
  float *mom = (float *)(w + T.mom), *red = (float *)(w + T.red);
  CellRec *rec = (CellRec *)(w + T.rec);
  for (int l = D; l >= 0; --l) {
    const int gm = (int)std::min<int64_t>(T.cap[l], TR_CELL_BLOCKS);  // grid-stride over the cells
    const unsigned *kl = (const unsigned *)(w + T.key[l]);
    float4 *cl = (float4 *)(w + T.cen[l]);
    float *ml = mom + (size_t)T.off[l] * T.nc;
    if (l == D) {  // leaves: moments from their images
      with_order(P, [&](auto o) {
        k_tree_moments<decltype(o)::value><<<gm, 64, 0, st>>>(ncell + l, l, Lc, kl, (const int *)(w + T.start[l]),
                                                              simg, cl, ml);
      });
    } else {  // upper levels: translated from the children
      const int *chl = (const int *)(w + T.child[l]);
      const float4 *cc = (const float4 *)(w + T.cen[l + 1]);
      const float *cm = mom + (size_t)T.off[l + 1] * T.nc;
      with_order(P, [&](auto o) {
        k_tree_m2m<decltype(o)::value><<<gm, 64, 0, st>>>(ncell + l, l, Lc, theta, (float)pl->a, kl, chl, cc, cm,
                                                          cl, ml);
      });
    }
    const int gpk = (int)cdivl(T.cap[l], 256);
    const int *sl = (const int *)(w + T.start[l]), *chp = (const int *)(w + T.child[l]);
    with_order(P, [&](auto o) {
      k_tree_pack<decltype(o)::value><<<gpk, 256, 0, st>>>((int)T.cap[l], ncell + l, l == D, (int)T.off[l], (int)T.off[l + 1],
                                                cl, sl, chp, ml, rec, red);
    });
  }
  {
    // targets: sorted by their own codes (codes_a and ids_a are free again), cells of level lt,
    // then groups of up to 64 within each cell
    unsigned *codes_t = (unsigned *)(w + T.codes_t);
    int *ids_t = (int *)(w + T.ids_t);
    k_tree_tkeys<<<nb, 256, 0, st>>>(n, (float)pl->a, tgt, codes_a, ids_a);
    size_t tb2 = T.temp_bytes;
    HSMA_HIP(rocprim::radix_sort_pairs(w + T.temp, tb2, codes_a, codes_t, ids_a, ids_t, (unsigned)n, 0,
                                       3 * TR_TBITS, st));
    k_tree_tgather<<<nb, 256, 0, st>>>(n, ids_t, tgt, inv, stgt, (int *)(w + T.town));
    const int tshift = 3 * (TR_TBITS - T.lt);
    int *tcount = ncell + TR_MAX_DEPTH + 2;
    k_tree_flags<<<nb, 256, 0, st>>>(n, nullptr, n, codes_t, tshift, flags);
    size_t sb = T.temp_bytes;
    HSMA_HIP(rocprim::exclusive_scan(w + T.temp, sb, flags, scan, 0, (size_t)n, rocprim::plus<int>(), st));
    k_tree_cells<<<nb, 256, 0, st>>>(n, nullptr, n, n, codes_t, tshift, nullptr, flags, scan, (unsigned *)(w + T.tkey),
                                     (int *)(w + T.tchild), (int *)(w + T.tstart), tcount);
    const int gc = (int)cdivl(T.tcap, 256);
    int *gng = (int *)(w + T.gng), *gofs = (int *)(w + T.gofs);
    const int *tstart = (const int *)(w + T.tstart);
    k_tree_gcount<<<gc, 256, 0, st>>>((int)T.tcap, tcount, tstart, gng);
    sb = T.temp_bytes;
    HSMA_HIP(rocprim::exclusive_scan(w + T.temp, sb, gng, gofs, 0, (size_t)T.tcap, rocprim::plus<int>(), st));
    k_tree_gfill<<<gc, 256, 0, st>>>((int)T.tcap, tcount, tstart, gng, gofs, (int2 *)(w + T.gr),
                                     ncell + TR_MAX_DEPTH + 1);
    unsigned *gka = (unsigned *)(w + T.gkey_a), *gkb = (unsigned *)(w + T.gkey_b);
    int *gia = (int *)(w + T.gid_a), *gib = (int *)(w + T.gid_b);
    k_tree_groups<<<T.ngroups, 64, 0, st>>>(ncell + TR_MAX_DEPTH + 1, (const int2 *)(w + T.gr), stgt,
                                            (float4 *)(w + T.grp), gka, gia);
    size_t tb3 = T.temp_bytes;
    HSMA_HIP(rocprim::radix_sort_pairs(w + T.temp, tb3, gka, gkb, gia, gib, (unsigned)T.ngroups, 0, 32, st));
  }
  {
    // surface nodes: sorted by their codes in the cube of half-width 1.125 R_tau (the nodes of
    // point pairs lie within R_tau (1 + dy/2R_tau)), cells of level lp, patches of up to 64
    // nodes within each cell, their moments and records
    const int pn = T.pn;
    const int nbp = (int)cdivl(pn, 256);
    unsigned *nca = (unsigned *)(w + T.ncodes_a), *ncb = (unsigned *)(w + T.ncodes_b);
    int *nia = (int *)(w + T.nids_a), *nib = (int *)(w + T.nids_b);
    int *nfl = (int *)(w + T.nflags), *nsc = (int *)(w + T.nscan);
    float4 *snodes = (float4 *)(w + T.snodes);
    float2 *sqd = (float2 *)(w + T.sqd);
    const float Rn = (float)(1.125 * (1.0 + pl->opts.tau) * pl->a);
    k_tree_tkeys<<<nbp, 256, 0, st>>>(pn, Rn, pl->self->nodes32, nca, nia);
    size_t tb4 = T.temp_bytes;
    HSMA_HIP(rocprim::radix_sort_pairs(w + T.temp, tb4, nca, ncb, nia, nib, (unsigned)pn, 0, 3 * TR_TBITS, st));
    k_tree_ngather<<<nbp, 256, 0, st>>>(pn, nib, pl->self->nodes32, qd, snodes, sqd);
    const int nshift = 3 * (TR_TBITS - T.lp);
    int *nccount = ncell + TR_MAX_DEPTH + 3, *npatch = ncell + TR_MAX_DEPTH + 4;
    k_tree_flags<<<nbp, 256, 0, st>>>(pn, nullptr, pn, ncb, nshift, nfl);
    size_t sb = T.temp_bytes;
    HSMA_HIP(rocprim::exclusive_scan(w + T.temp, sb, nfl, nsc, 0, (size_t)pn, rocprim::plus<int>(), st));
    k_tree_cells<<<nbp, 256, 0, st>>>(pn, nullptr, pn, pn, ncb, nshift, nullptr, nfl, nsc, (unsigned *)(w + T.nkey),
                                      (int *)(w + T.nchild), (int *)(w + T.nstart), nccount);
    const int gcn = (int)cdivl(T.ncap, 256);
    int *nng = (int *)(w + T.nng), *ngofs = (int *)(w + T.ngofs);
    const int *nstart = (const int *)(w + T.nstart);
    k_tree_gcount<<<gcn, 256, 0, st>>>((int)T.ncap, nccount, nstart, nng);
    sb = T.temp_bytes;
    HSMA_HIP(rocprim::exclusive_scan(w + T.temp, sb, nng, ngofs, 0, (size_t)T.ncap, rocprim::plus<int>(), st));
    k_tree_gfill<<<gcn, 256, 0, st>>>((int)T.ncap, nccount, nstart, nng, ngofs, (int2 *)(w + T.pr), npatch);
    float4 *pcen = (float4 *)(w + T.pcen);
    int *pstart = (int *)(w + T.pstart);
    float *pm = (float *)(w + T.pm);
    with_order(P, [&](auto o) {
      k_tree_patch<decltype(o)::value><<<std::min(T.npcap, 1024), 64, 0, st>>>(
          npatch, (const int2 *)(w + T.pr), snodes, sqd, pl->self->dipole == 2, pcen, pstart, pm);
      k_tree_pack<decltype(o)::value><<<(int)cdivl(T.npcap, 256), 256, 0, st>>>(
          T.npcap, npatch, 1, 0, 0, pcen, pstart, pstart, pm, (CellRec *)(w + T.prec), (float *)(w + T.pred));
    });
  }
  const hsma_group_s *grp = pl->self;
  const int ge = (int)cdivl(T.ngroups, TR_WAVES);
  const float4 *gp = (const float4 *)(w + T.grp);
  const float th2 = theta * theta;
  const unsigned *key0 = (const unsigned *)(w + T.key[0]);
  const int *start0 = (const int *)(w + T.start[0]);
  const int *ngp = ncell + TR_MAX_DEPTH + 1;
  const int *town = (const int *)(w + T.town), *ids_t = (const int *)(w + T.ids_t);
  const int *gord = (const int *)(w + T.gid_b);
  const int2 *grr = (const int2 *)(w + T.gr);
  with_order(P, [&](auto o) {
    k_tree_local<decltype(o)::value><<<1, 64, 0, st>>>(n, key0, start0, ncell, simg, (float *)(w + T.lfar));
    k_tree_eval<decltype(o)::value><<<ge, 64 * TR_WAVES, 0, st>>>(
        n, th2, rec, red, key0, start0, ncell, simg, stgt, town, ids_t, ngp, gord, grr, gp, self, grp->dipole == 2,
        (const float *)(w + T.lfar), (const CellRec *)(w + T.prec), (const float *)(w + T.pred), ncell + TR_MAX_DEPTH + 4,
        (const float4 *)(w + T.snodes), (const float2 *)(w + T.sqd), phi);
  });
  if (E) {
    double *ep = (double *)(w + T.ep);
    k_tree_epart<<<nb, 256, 0, st>>>(n, q, phi, ep);
    k_tree_esum<<<1, 256, 0, st>>>(nb, ep, E);
  }
  HSMA_HIP(hipGetLastError());
  return HSMA_OK;
}
