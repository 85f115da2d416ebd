// Resident ion configurations and single-ion-move energy changes (FP64 throughout).
//
// The HSMA energy E = 1/2 sum_i q_i Phi_RF(x_i) (Sec. 4.1, eq. "phirffinall") is a bilinear
// form in the charges:
//   E = 1/2 sum_ij q_i q_j g(x_i, x_j) + 1/2 w . s,
// with g(x, x') = kappa_K(|x'|) c0 / |x - r_K(x')| the modified Kelvin image of a unit charge
// at x' seen at x (g(x, x) is the ion's own image), w = sum_i q_i S(x_i) the surface kernel
// rows (S(x) = (1/|x - y_s|, (x - y_s).y_s / |x - y_s|^3) over the P nodes) and s = T c the
// surface strengths, c = sum_i q_i C(x_i) the check fields and T the fixed fit operator
// (Algorithm 1, steps 2-4).  Moving ion k from x to x' therefore changes E by
//   dE = 1/2 [q_k sum_{j != k} q_j (g(x', x_j) - g(x, x_j) + g(x_j, x') - g(x_j, x)) + q_k^2 (g(x', x') - g(x, x))]
//      + 1/2 [dw . s + (w + dw) . ds],   dw = q_k (S(x') - S(x)),  ds = T q_k (C(x') - C(x)),
// which costs O(N + M + P) pairs and two small GEMVs instead of a full evaluation.
//
// Optionally (HSMA_SYSTEM_COULOMB) the state's energy also holds the direct Coulomb energy of
// the ions inside the cavity, E_C = 1/2 sum_{i != j} q_i q_j c0 / |x_i - x_j| (eq. "phicoul"),
// so that a move's change is the total one: dE_C = q_k sum_{j != k} q_j c0 (1/|x' - x_j| -
// 1/|x - x_j|), summed in the same pass over j as the image terms.
#include <math.h>
#include <string.h>

#include "hsma_internal.h"

namespace hsma {
namespace {

constexpr int DB = 256;

__device__ __forceinline__ double rinv64(double r2) { return 1.0 / sqrt(r2); }

// Image strength per unit charge times c0, and the image position, of an ion at (x, y, z):
// q_K / q = (1/a)[gamma r_K + dbar (R_tau - r_K)/2] with r_K = a^2 / r (Sec. 2.4).  For r below
// rmin the image is at infinity; its potential tends to (gamma - dbar/2) c0 / a everywhere.
struct Img {
  double X, Y, Z, s;  // position and c0 * strength per unit charge
  bool inf;           // at infinity: potential = s everywhere
};

__device__ __forceinline__ Img image_of(const PlanDev &c, double x, double y, double z) {
  Img m;
  const double r2 = x * x + y * y + z * z, r = sqrt(r2);
  if (r < c.rmin) {
    m.inf = true;
    m.X = m.Y = m.Z = 0.0;
    m.s = c.c0 * (c.gamma - 0.5 * c.dbar) / c.a;
    return m;
  }
  m.inf = false;
  const double f = c.a2 / r2;
  m.X = f * x;
  m.Y = f * y;
  m.Z = f * z;
  const double rK = c.a2 / r;
  m.s = c.c0 / c.a * (c.gamma * rK + c.dbar * (c.Rtau - rK) * 0.5);
  return m;
}

__device__ __forceinline__ double img_pot(const Img &m, double x, double y, double z) {
  if (m.inf) return m.s;
  const double dx = x - m.X, dy = y - m.Y, dz = z - m.Z;
  return m.s * rinv64(dx * dx + dy * dy + dz * dz);
}

// g(x, x) of a unit charge: its own image, regular at r = 0 (as in the packing kernel).
__device__ __forceinline__ double self_g(const PlanDev &c, double x, double y, double z) {
  const double r = sqrt(x * x + y * y + z * z);
  return c.c0 / c.a * (c.gamma * c.a2 + 0.5 * c.dbar * (c.Rtau * r - c.a2)) / ((c.a - r) * (c.a + r));
}

// Row S(x) of node s for a unit charge at x: the monopole 1/|x - y_s| and the dipole kernel,
// (x - y_s).y_s / |x - y_s|^3 for exact dipoles or (R_tau/dy)(1/|x - y+| - 1/|x - y-|) for the
// paper's point pairs (nodes at 3s, 3s + 1, 3s + 2).
__device__ __forceinline__ void surface_row(const PlanDev &c, int s, double x, double y, double z, double &m,
                                            double &t) {
  if (c.dipole != 1) {
    const double4 yv = c.nodes64[s];
    const double dx = x - yv.x, dy = y - yv.y, dz = z - yv.z;
    const double ir = rinv64(dx * dx + dy * dy + dz * dz);
    m = ir;
    t = (dx * yv.x + dy * yv.y + dz * yv.z) * ir * ir * ir;
  } else {
    const double4 y0 = c.nodes64[3 * s], ym = c.nodes64[3 * s + 1], yp = c.nodes64[3 * s + 2];
    const double ax = x - y0.x, ay = y - y0.y, az = z - y0.z;
    const double bx = x - ym.x, by = y - ym.y, bz = z - ym.z;
    const double px = x - yp.x, py = y - yp.y, pz = z - yp.z;
    m = rinv64(ax * ax + ay * ay + az * az);
    t = c.dyc * (rinv64(px * px + py * py + pz * pz) - rinv64(bx * bx + by * by + bz * bz));
  }
}

__device__ __forceinline__ double block_sum(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = DB / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// prio: the request server's move batches raise their waves' issue priority, so that a move
// sharing a SIMD with a long full-energy launch issues first (results are unchanged).
__device__ __forceinline__ void move_priority(int prio) {
  if (prio) __builtin_amdgcn_s_setprio(3);
}

// Stage 1: Kelvin row/column sums (blocks [0, nA)), check-field changes (next nB blocks),
// surface-row changes (last nD blocks).  grid.y = request.
__global__ __launch_bounds__(DB) void k_de_pairs(const SysDev *__restrict__ systems, const DeReq *__restrict__ reqs,
                                                 DeReq one, int nA, int nB, int prio) {
  __shared__ double red[DB];
  move_priority(prio);
  const DeReq r = reqs ? reqs[blockIdx.y] : one;
  const SysDev &S = systems[r.sys];
  const PlanDev &c = S.pl;
  const double x0 = S.x[r.k], y0 = S.y[r.k], z0 = S.z[r.k], qk = S.q[r.k];
  const double x1 = r.x, y1 = r.y, z1 = r.z;
  const int blk = blockIdx.x;
  if (blk < nA) {
    if ((int64_t)blk * DB >= S.n) return;  // nA covers the largest system of the batch
    const Img ik0 = image_of(c, x0, y0, z0), ik1 = image_of(c, x1, y1, z1);
    const int64_t j = (int64_t)blk * DB + threadIdx.x;
    double v = 0.0;
    if (j < S.n && j != r.k) {
      const double xj = S.x[j], yj = S.y[j], zj = S.z[j];
      const Img ij = image_of(c, xj, yj, zj);
      // row: ion k at its new and old place in the field of j's image; column: j in the field
      // of k's new and old image
      double t = (img_pot(ij, x1, y1, z1) - img_pot(ij, x0, y0, z0)) +
                 (img_pot(ik1, xj, yj, zj) - img_pot(ik0, xj, yj, zj));
      if (S.coulomb) {  // 2 c0 (1/r' - 1/r): the final 1/2 q_k makes it q_k q_j c0 (1/r' - 1/r)
        const double ax = x1 - xj, ay = y1 - yj, az = z1 - zj, bx = x0 - xj, by = y0 - yj, bz = z0 - zj;
        t += 2.0 * c.c0 * (rinv64(ax * ax + ay * ay + az * az) - rinv64(bx * bx + by * by + bz * bz));
      }
      v = S.q[j] * t;
    }
    const double b = block_sum(v, red);
    if (threadIdx.x == 0) S.partA[blk] = b;
    return;
  }
  if (blk < nA + nB) {
    const int m = (blk - nA) * DB + threadIdx.x;  // nB covers the largest M of the batch
    if (m < S.M) {
      const double4 ck = c.chk64[m];
      const double dx1 = ck.x - x1, dy1 = ck.y - y1, dz1 = ck.z - z1;
      const double dx0 = ck.x - x0, dy0 = ck.y - y0, dz0 = ck.z - z0;
      const double g1 = c.c0 * rinv64(dx1 * dx1 + dy1 * dy1 + dz1 * dz1);
      const double g0 = c.c0 * rinv64(dx0 * dx0 + dy0 * dy0 + dz0 * dz0);
      const double r1 = sqrt(x1 * x1 + y1 * y1 + z1 * z1) / c.a, r0 = sqrt(x0 * x0 + y0 * y0 + z0 * z0) / c.a;
      S.dc[m] = qk * (g1 - g0);
      S.dc[S.M + m] = qk * (r1 * g1 - r0 * g0);
    }
    return;
  }
  const int s = (blk - nA - nB) * DB + threadIdx.x;
  if (s < S.P) {
    double m1, m0, t1, t0;
    surface_row(c, s, x1, y1, z1, m1, t1);
    surface_row(c, s, x0, y0, z0, m0, t0);
    S.dw[s] = qk * (m1 - m0);
    S.dw[S.P + s] = qk * (t1 - t0);
  }
}

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Stage 2: alpha'' = pinv du, beta'' = pinv dv; one wave per coefficient row.
__global__ __launch_bounds__(256) void k_de_fit1(const SysDev *__restrict__ systems, const DeReq *__restrict__ reqs,
                                                 DeReq one, int prio) {
  move_priority(prio);
  const DeReq r = reqs ? reqs[blockIdx.y] : one;
  const SysDev &S = systems[r.sys];
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= S.K) return;
  const double *pr = S.pinv64 + (size_t)row * S.M;
  double a = 0.0, b = 0.0;
  for (int m = lane; m < S.M; m += 64) {
    a = fma(pr[m], S.dc[m], a);
    b = fma(pr[m], S.dc[S.M + m], b);
  }
  a = wave_sum64(a);
  b = wave_sum64(b);
  if (lane == 0) {
    S.ab[row] = a;
    S.ab[S.K + row] = b;
  }
}

// Stage 3: ds = (Lhat (n . h), -Lhat h), h = f . alpha'' + g . beta''; per node also the
// energy terms dw . s + (w + dw) . ds.
__global__ __launch_bounds__(256) void k_de_fit2(const SysDev *__restrict__ systems, const DeReq *__restrict__ reqs,
                                                 DeReq one, int prio) {
  move_priority(prio);
  const DeReq r = reqs ? reqs[blockIdx.y] : one;
  const SysDev &S = systems[r.sys];
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (s >= S.P) return;
  const double *lr = S.lhat64 + (size_t)s * S.K;
  const double *fg = S.pl.fg;
  double sq = 0.0, sd = 0.0;
  for (int k = lane; k < S.K; k += 64) {
    const double h = fg[k] * S.ab[k] + fg[S.K + k] * S.ab[S.K + k];
    sq = fma(lr[k] * (double)degree_weight(S.nidx[k], S.pl.dipole), h, sq);
    sd = fma(lr[k], h, sd);
  }
  sq = wave_sum64(sq);
  sd = wave_sum64(sd);
  if (lane == 0) {
    const double dq = sq, dd = S.pl.dipole == 2 ? 0.0 : -sd;
    S.ds[s] = dq;
    S.ds[S.P + s] = dd;
    const double dwq = S.dw[s], dwd = S.dw[S.P + s];
    S.partE[s] = dwq * S.s[s] + dwd * S.s[S.P + s] + (S.w[s] + dwq) * dq + (S.w[S.P + s] + dwd) * dd;
  }
}

// Stage 4 (one block per request): dE in a fixed order; with commit, apply the move.
__global__ __launch_bounds__(DB) void k_de_final(const SysDev *__restrict__ systems, const DeReq *__restrict__ reqs,
                                                 DeReq one, int prio) {
  __shared__ double red[DB];
  move_priority(prio);
  const DeReq r = reqs ? reqs[blockIdx.x] : one;
  const SysDev &S = systems[r.sys];
  const PlanDev &c = S.pl;
  const double x0 = S.x[r.k], y0 = S.y[r.k], z0 = S.z[r.k], qk = S.q[r.k];
  const int nA = (int)((S.n + DB - 1) / DB);  // this system's own blocks: the order does not depend on the batch
  double a = 0.0;
  for (int i = threadIdx.x; i < nA; i += DB) a += S.partA[i];
  double e = 0.0;
  for (int i = threadIdx.x; i < S.P; i += DB) e += S.partE[i];
  const double sa = block_sum(a, red);
  const double se = block_sum(e, red);
  const double dself = self_g(c, r.x, r.y, r.z) - self_g(c, x0, y0, z0);
  const double dE = 0.5 * (qk * sa + qk * qk * dself) + 0.5 * se;
  if (threadIdx.x == 0 && r.dE) *r.dE = dE;
  if (r.commit) {
    __syncthreads();  // every thread has read the old position
    for (int i = threadIdx.x; i < 2 * S.P; i += DB) {
      S.s[i] += S.ds[i];
      S.w[i] += S.dw[i];
    }
    if (threadIdx.x == 0) {
      S.x[r.k] = r.x;
      S.y[r.k] = r.y;
      S.z[r.k] = r.z;
      *S.E += dE;
    }
  }
}

// w = sum_i q_i S(x_i) over the nodes: one block per node, fixed order.
__global__ __launch_bounds__(DB) void k_sys_w(SysDev *__restrict__ sd) {
  __shared__ double red[DB];
  const SysDev &S = *sd;
  const int s = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < S.n; i += DB) {
    double m, t;
    surface_row(S.pl, s, S.x[i], S.y[i], S.z[i], m, t);
    a += S.q[i] * m;
    b += S.q[i] * t;
  }
  a = block_sum(a, red);
  b = block_sum(b, red);
  if (threadIdx.x == 0) {
    S.w[s] = a;
    S.w[S.P + s] = b;
  }
}

// s from the full evaluation's strengths (double2 per surface source) into the Q', D' layout;
// with point pairs node i's sources are at 3i (Q') and 3i + 2 (D' R_tau / dy).
__global__ void k_sys_s(int P, int dipole, double dyc, const double2 *__restrict__ qd, double *__restrict__ s) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  s[i] = dipole == 1 ? qd[3 * i].x : qd[i].x;
  s[P + i] = dipole == 1 ? qd[3 * i + 2].x / dyc : qd[i].y;
}

// Direct Coulomb energy in FP64: partials of sum_{j != i} q_j / |x_i - x_j| per target and
// source chunk (one target per thread, wave-uniform sources), then per block
// 1/2 c0 sum_i q_i (chunk sum in chunk order), then one block adds the block partials in
// order to E.
constexpr int CB = 256;

__global__ __launch_bounds__(CB) void k_coul_pairs(int64_t N, int64_t chunk, const double *__restrict__ x,
                                                   const double *__restrict__ y, const double *__restrict__ z,
                                                   const double *__restrict__ q, double *__restrict__ part) {
  const int64_t i = (int64_t)blockIdx.x * CB + threadIdx.x;
  const int64_t c = blockIdx.y;
  const int64_t ii = i < N ? i : N - 1;
  const double xi = x[ii], yi = y[ii], zi = z[ii];
  const int64_t j0 = c * chunk, j1 = j0 + chunk < N ? j0 + chunk : N;
  double s = 0.0;
  for (int64_t j = j0; j < j1; ++j) {
    const double dx = xi - x[j], dy = yi - y[j], dz = zi - z[j];
    const double r2 = dx * dx + dy * dy + dz * dz;
    s += (j == ii) ? 0.0 : q[j] * rinv64(r2);
  }
  if (i < N) part[c * N + i] = s;
}

__global__ __launch_bounds__(CB) void k_coul_finish(int64_t N, int nchunks, const double *__restrict__ part,
                                                    const double *__restrict__ q, double c0,
                                                    double *__restrict__ epart) {
  __shared__ double red[CB];
  const int64_t i = (int64_t)blockIdx.x * CB + threadIdx.x;
  double e = 0.0;
  if (i < N) {
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += part[(int64_t)c * N + i];
    e = 0.5 * c0 * q[i] * s;
  }
  red[threadIdx.x] = e;
  __syncthreads();
  for (int o = CB / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) epart[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(CB) void k_coul_add(int nb, const double *__restrict__ epart, double *__restrict__ E) {
  __shared__ double red[CB];
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += CB) s += epart[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = CB / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *E += red[0];
}

inline int coul_chunks(int64_t N) {
  const int64_t tb = (N + CB - 1) / CB;
  int64_t nc = (2048 + tb - 1) / tb;
  nc = nc < 1 ? 1 : (nc > 64 ? 64 : nc);
  const int64_t most = (N + 255) / 256;  // at least 256 sources per chunk
  return (int)(nc > most ? (most < 1 ? 1 : most) : nc);
}

inline size_t align256s(size_t v) { return (v + 255) & ~(size_t)255; }

// Bytes of the Coulomb scratch, placed at the end of a full-evaluation workspace.
size_t coul_bytes(int64_t N) {
  return align256s(sizeof(double) * (size_t)N * coul_chunks(N)) + align256s(sizeof(double) * (size_t)((N + CB - 1) / CB));
}

// E += E_C of the system's current positions, with scratch at ws.
hsma_status add_coulomb(const SysDev &h, int64_t N, double *E, char *ws, hipStream_t st) {
  const int nc = coul_chunks(N);
  const int64_t chunk = (N + nc - 1) / nc;
  double *part = (double *)ws;
  double *epart = (double *)(ws + align256s(sizeof(double) * (size_t)N * nc));
  const int nb = (int)((N + CB - 1) / CB);
  k_coul_pairs<<<dim3((unsigned)nb, (unsigned)nc), CB, 0, st>>>(N, chunk, h.x, h.y, h.z, h.q, part);
  k_coul_finish<<<nb, CB, 0, st>>>(N, nc, part, h.q, h.pl.c0, epart);
  k_coul_add<<<1, CB, 0, st>>>(nb, epart, E);
  HSMA_HIP(hipGetLastError());
  return HSMA_OK;
}

}  // namespace

hsma_status launch_delta(const SysDev *systems, const DeReq *reqs, DeReq one, int nreq, int64_t max_n, int max_M,
                         int max_P, int max_K, hipStream_t st, int prio) {
  const int nA = (int)((max_n + DB - 1) / DB), nB = (max_M + DB - 1) / DB, nD = (max_P + DB - 1) / DB;
  k_de_pairs<<<dim3(nA + nB + nD, nreq), DB, 0, st>>>(systems, reqs, one, nA, nB, prio);
  k_de_fit1<<<dim3((max_K + 3) / 4, nreq), 256, 0, st>>>(systems, reqs, one, prio);
  k_de_fit2<<<dim3((max_P + 3) / 4, nreq), 256, 0, st>>>(systems, reqs, one, prio);
  k_de_final<<<nreq, DB, 0, st>>>(systems, reqs, one, prio);
  HSMA_HIP(hipGetLastError());
  return HSMA_OK;
}

hsma_status system_full_energy_at(hsma_system_s *sys, const double *x, const double *y, const double *z,
                                  const double *q, double *E, void *ws, size_t ws_bytes, hipStream_t st) {
  if (ws_bytes < system_workspace_bytes(sys)) return HSMA_EINVAL;
  const size_t lt = layout(sys->g64, 1, sys->n, sys->n, false, false, true).total;
  hsma_status rc = run_batched(sys->g64, 1, nullptr, nullptr, sys->n, sys->n, x, y, z, q, nullptr, E, ws, lt, st);
  if (rc != HSMA_OK || !sys->h.coulomb) return rc;
  SysDev at = sys->h;
  at.x = const_cast<double *>(x);
  at.y = const_cast<double *>(y);
  at.z = const_cast<double *>(z);
  at.q = const_cast<double *>(q);
  return add_coulomb(at, sys->n, E, (char *)ws + lt, st);
}

hsma_status system_full_energy(hsma_system_s *sys, double *E, void *ws, size_t ws_bytes, hipStream_t st) {
  return system_full_energy_at(sys, sys->h.x, sys->h.y, sys->h.z, sys->h.q, E, ws, ws_bytes, st);
}

size_t system_workspace_bytes(const hsma_system_s *sys) {
  return layout(sys->g64, 1, sys->n, sys->n, false, false, true).total + (sys->h.coulomb ? coul_bytes(sys->n) : 0);
}

}  // namespace hsma

using namespace hsma;

static void system_free(hsma_system_s *sys) {
  if (!sys) return;
  SysDev &h = sys->h;
  double *bufs[] = {h.x, h.y, h.z, h.q, h.s, h.w, h.E, h.dc, h.ab, h.ds, h.dw, h.partA, h.partE};
  for (double *b : bufs) (void)hipFree(b);
  (void)hipFree(sys->d);
  (void)hipFree(sys->ws);
  if (sys->g64) group_free(sys->g64);
  delete sys;
}

extern "C" hsma_status hsma_system_create_ex(hsma_plan_t pl, int64_t N, const double *x, const double *y,
                                             const double *z, const double *q, int flags, hipStream_t st,
                                             hsma_system_t *out) {
  if (!pl || !out || N < 1 || N > ((int64_t)1 << 31) - 1 || !x || !y || !z || !q) return HSMA_EINVAL;
  if (flags & ~HSMA_SYSTEM_COULOMB) return HSMA_EINVAL;
  *out = nullptr;
  int dev = -1;
  HSMA_HIP(hipGetDevice(&dev));
  if (dev != pl->device) return HSMA_ESTATE;
  hsma_system_s *sys = new hsma_system_s();
  memset(sys, 0, sizeof(*sys));
  sys->plan = pl;
  sys->n = N;
  sys->device = dev;
  const Geometry *g = pl->geo;
  const int K = g->K, M = g->M, P = g->P;
  SysDev &h = sys->h;
  h.pl = pl->host;
  h.pinv64 = g->pinv64;
  h.lhat64 = g->lhat64;
  h.nidx = g->nidx;
  h.K = K;
  h.M = M;
  h.P = P;
  h.n = N;
  h.coulomb = (flags & HSMA_SYSTEM_COULOMB) ? 1 : 0;
  hsma_status rc = group_build(1, &pl, 1, &sys->g64);
  if (rc != HSMA_OK) {
    system_free(sys);
    return rc;
  }
  sys->g64->pair_prec = HSMA_PAIR_FP64;  // full evaluations of the state in FP64
  // Full energies of a resident system in blocks of 256 ions whatever its size: the request
  // server needs that size beside its move batches (blocks of 128 raised the moves' p99 several
  // times), and the same size here keeps a served energy the same bit for bit as this API's.
  sys->g64->tune.eblock = 256;
  const size_t nb = sizeof(double) * (size_t)N;
  const int nA = (int)((N + DB - 1) / DB);
  sys->footprint = 4 * nb + sizeof(double) * (6 * (size_t)P + 2 * (size_t)M + 2 * (size_t)K + 1 + (size_t)nA + P) +
                   sizeof(SysDev);
  double *phi = nullptr;
  Layout L = layout(sys->g64, 1, N, N);
  const size_t wsb = call_workspace_bytes(sys->g64, 1, N, N, false);  // energy and potential launches
  sys->ws_bytes = wsb + (h.coulomb ? coul_bytes(N) : 0);
#define HSMA_TRY(call)          \
  do {                          \
    if ((call) != hipSuccess) { \
      rc = HSMA_EDEVICE;        \
      goto fail;                \
    }                           \
  } while (0)
  HSMA_TRY(hipMalloc(&h.x, nb));
  HSMA_TRY(hipMalloc(&h.y, nb));
  HSMA_TRY(hipMalloc(&h.z, nb));
  HSMA_TRY(hipMalloc(&h.q, nb));
  HSMA_TRY(hipMalloc(&h.s, sizeof(double) * 2 * P));
  HSMA_TRY(hipMalloc(&h.w, sizeof(double) * 2 * P));
  HSMA_TRY(hipMalloc(&h.E, sizeof(double)));
  HSMA_TRY(hipMalloc(&h.dc, sizeof(double) * 2 * M));
  HSMA_TRY(hipMalloc(&h.ab, sizeof(double) * 2 * K));
  HSMA_TRY(hipMalloc(&h.ds, sizeof(double) * 2 * P));
  HSMA_TRY(hipMalloc(&h.dw, sizeof(double) * 2 * P));
  HSMA_TRY(hipMalloc(&h.partA, sizeof(double) * nA));
  HSMA_TRY(hipMalloc(&h.partE, sizeof(double) * P));
  HSMA_TRY(hipMalloc(&sys->d, sizeof(SysDev)));
  HSMA_TRY(hipMalloc(&sys->ws, sys->ws_bytes));
  HSMA_TRY(hipMemcpyAsync(h.x, x, nb, hipMemcpyDeviceToDevice, st));
  HSMA_TRY(hipMemcpyAsync(h.y, y, nb, hipMemcpyDeviceToDevice, st));
  HSMA_TRY(hipMemcpyAsync(h.z, z, nb, hipMemcpyDeviceToDevice, st));
  HSMA_TRY(hipMemcpyAsync(h.q, q, nb, hipMemcpyDeviceToDevice, st));
  HSMA_TRY(hipMemcpyAsync(sys->d, &h, sizeof(SysDev), hipMemcpyHostToDevice, st));
  phi = (double *)((char *)sys->ws + L.phi);
  rc = run_batched(sys->g64, 1, nullptr, nullptr, N, N, h.x, h.y, h.z, h.q, phi, h.E, sys->ws, wsb, st);
  if (rc != HSMA_OK) goto fail;
  if (h.coulomb) {
    rc = add_coulomb(h, N, h.E, (char *)sys->ws + wsb, st);
    if (rc != HSMA_OK) goto fail;
  }
  k_sys_s<<<(P + 255) / 256, 256, 0, st>>>(P, h.pl.dipole, h.pl.dyc, (const double2 *)((char *)sys->ws + L.qd), h.s);
  k_sys_w<<<P, DB, 0, st>>>(sys->d);
  HSMA_TRY(hipGetLastError());
  HSMA_TRY(hipStreamSynchronize(st));
  {
    int f = 0;
    HSMA_TRY(hipMemcpy(&f, sys->g64->flag, sizeof(int), hipMemcpyDeviceToHost));
    if (f) {
      rc = (f & 2) ? HSMA_EINVAL : HSMA_EDOMAIN;
      goto fail;
    }
  }
  (void)hipFree(sys->ws);  // the resident state is small; full evaluations bring their own workspace
  sys->ws = nullptr;
  sys->ws_bytes = 0;
  *out = sys;
  return HSMA_OK;
fail:
#undef HSMA_TRY
  (void)hipStreamSynchronize(st);
  system_free(sys);
  return rc;
}

extern "C" hsma_status hsma_system_create(hsma_plan_t pl, int64_t N, const double *x, const double *y, const double *z,
                                          const double *q, hipStream_t st, hsma_system_t *out) {
  return hsma_system_create_ex(pl, N, x, y, z, q, 0, st, out);
}

extern "C" size_t hsma_system_workspace_bytes(hsma_system_t sys) { return sys ? system_workspace_bytes(sys) : 0; }

extern "C" hsma_status hsma_system_full_energy(hsma_system_t sys, double *E, void *ws, size_t ws_bytes,
                                               hipStream_t st) {
  if (!sys || !E || !ws) return HSMA_EINVAL;
  return system_full_energy(sys, E, ws, ws_bytes, st);
}

static hsma_status delta(hsma_system_t sys, int64_t k, double xk, double yk, double zk, double *dE, int commit,
                         hipStream_t st) {
  if (!sys || k < 0 || k >= sys->n) return HSMA_EINVAL;
  if (!(isfinite(xk) && isfinite(yk) && isfinite(zk))) return HSMA_EINVAL;
  if (!(sqrt(xk * xk + yk * yk + zk * zk) < sys->h.pl.a)) return HSMA_EINVAL;
  int dev = -1;
  HSMA_HIP(hipGetDevice(&dev));
  if (dev != sys->device) return HSMA_ESTATE;
  DeReq r;
  r.sys = 0;
  r.commit = commit;
  r.k = k;
  r.x = xk;
  r.y = yk;
  r.z = zk;
  r.dE = dE;
  return launch_delta(sys->d, nullptr, r, 1, sys->n, sys->h.M, sys->h.P, sys->h.K, st, 0);
}

extern "C" hsma_status hsma_delta_energy(hsma_system_t sys, int64_t k, double xk, double yk, double zk, double *dE,
                                         hipStream_t st) {
  if (!dE) return HSMA_EINVAL;
  return delta(sys, k, xk, yk, zk, dE, 0, st);
}

extern "C" hsma_status hsma_system_commit(hsma_system_t sys, int64_t k, double xk, double yk, double zk,
                                          hipStream_t st) {
  return delta(sys, k, xk, yk, zk, nullptr, 1, st);
}

extern "C" hsma_status hsma_system_energy(hsma_system_t sys, double *E, hipStream_t st) {
  if (!sys || !E) return HSMA_EINVAL;
  HSMA_HIP(hipMemcpyAsync(E, sys->h.E, sizeof(double), hipMemcpyDeviceToDevice, st));
  return HSMA_OK;
}

extern "C" hsma_status hsma_system_positions(hsma_system_t sys, double *x, double *y, double *z, hipStream_t st) {
  if (!sys || !x || !y || !z) return HSMA_EINVAL;
  const size_t nb = sizeof(double) * (size_t)sys->n;
  HSMA_HIP(hipMemcpyAsync(x, sys->h.x, nb, hipMemcpyDeviceToDevice, st));
  HSMA_HIP(hipMemcpyAsync(y, sys->h.y, nb, hipMemcpyDeviceToDevice, st));
  HSMA_HIP(hipMemcpyAsync(z, sys->h.z, nb, hipMemcpyDeviceToDevice, st));
  return HSMA_OK;
}

extern "C" hsma_status hsma_system_destroy(hsma_system_t sys) {
  if (!sys) return HSMA_EINVAL;
  (void)hipDeviceSynchronize();
  system_free(sys);
  return HSMA_OK;
}
