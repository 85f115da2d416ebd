/*
 * HSMA reaction-potential ORACLE -- test infrastructure only.
 *
 * A plain, slow, double-precision CPU implementation of what the GPU library
 * computes, written from the paper (J. Fu and Z. Gan, "Harmonic surface mapping
 * algorithm for electrostatic potentials in an atomistic/continuum hybrid model
 * for electrolyte solutions", arXiv:1907.01724).  Only the test suite, the
 * package smoke check and the CPU-baseline leg of the benchmark may load it; the
 * library path never does.  It shares no code with the GPU library.
 *
 * Two oracles live here:
 *   O1  the HSMA itself (Sec. 2.3-2.4 and Algorithm 1) with direct O(N^2) sums and
 *       the same discretisation as the GPU library -- the parity target;
 *   O2  the Kirkwood series (Sec. 2.2, eqs. "phirf" and "Anm"), summed until the
 *       tail is below a tolerance, with its Kelvin part in closed form -- the
 *       truth the O1 physics is checked against.
 *
 * Units: the potential of a charge q in medium eps1 is q/(4 pi eps1 r) (eq. "phicoul").
 * Readings of the paper that it is silent or ambiguous about:
 *   - the harmonic coefficients are obtained by a least-squares fit of check-point
 *     potentials (Algorithm 1, steps 1-3 use a discrete SH transform on the
 *     interface instead); check points sit on a golden-angle lattice of radius rc;
 *   - the correction coefficient of Sec. 2.4 depends on the ion through its Kelvin
 *     radius, so two check fields are fitted: u for q_i and v for q_i r_i / a;
 *   - the normal derivative of G in Green's second identity (eq. "GreenSecond") is
 *     used exactly (a surface dipole) by default; the paper's central difference
 *     with step dy (eq. "approxG") is selectable;
 *   - a single-layer variant (dipole = 2) keeps only the monopole integral of
 *     eq. "threeintegrals": the density on the auxiliary sphere whose single-layer
 *     potential is the same interior harmonic, sigma_nm = (2n+1)/R_tau (R_tau/a)^n
 *     Ahat_nm for Phi_corr = sum Ahat_nm (r/a)^n Y_nm (the classical single-layer
 *     expansion of a harmonic function inside a sphere), and no dipoles;
 *   - the Fibonacci rule (Sec. 2.4) is used as printed, with F2 = P/2 - 1 and any
 *     F1 coprime to F2 when F2 is not a Fibonacci number.
 *
 * parity unpinned: none of the exported functions; each is pinned by the tests.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846264338327950288

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* Sec. 2.2: the factor M_n(mu) of the Kirkwood coefficients (eq. "Anuapp1").  */
/* ------------------------------------------------------------------------- */

/* lambda_n = mu k_{n-1}(mu) / k_n(mu) for n = 0..nmax, where k_n is the modified
 * spherical Bessel function of the second kind defined in Sec. 2.2 and k_{-1} = k_0.
 * From the three-term relation k_{n+1} = k_{n-1} + (2n+1)/mu k_n it follows that
 * lambda_{n+1} = mu^2 / (lambda_n + 2n + 1), with lambda_0 = mu.  The forward
 * direction is stable because k_n grows with n.                                 */
void orc_lambda(int nmax, double mu, double *lam) {
  lam[0] = mu;
  for (int n = 0; n < nmax; n++) lam[n + 1] = mu * mu / (lam[n] + 2.0 * n + 1.0);
}

/* S_n = k_n / (mu k_n') and M_n of eq. "Anuapp1", n = 0..nmax.
 * With k_n' = -k_{n-1} - (n+1)/mu k_n one gets S_n = -1/(n + 1 + lambda_n).   */
void orc_kirkwood_factor(int nmax, double eps, double mu, double *S, double *M) {
  double *lam = (double *)malloc(sizeof(double) * (size_t)(nmax + 1));
  orc_lambda(nmax, mu, lam);
  for (int n = 0; n <= nmax; n++) {
    double s = -1.0 / (n + 1.0 + lam[n]);
    if (S) S[n] = s;
    M[n] = (eps * (n + 1.0) * s + 1.0) / (eps * n * s - 1.0);
  }
  free(lam);
}

/* gamma, sigma, delta-bar of eq. "Anuapp" (Sec. 2.3). */
void orc_image_constants(double eps, double mu, double *out3) {
  double gamma = (eps - 1.0) / (eps + 1.0);
  double sigma = (1.0 + mu) / (1.0 + eps);
  double dbar = gamma * (1.0 - sigma) - mu / (1.0 + eps);
  out3[0] = gamma;
  out3[1] = sigma;
  out3[2] = dbar;
}

/* ------------------------------------------------------------------------- */
/* Real orthonormal spherical harmonics, degree <= p.                          */
/* ------------------------------------------------------------------------- */

/* Y[n*n + n + m] for -n <= m <= n at the direction of (vx, vy, vz):
 *   m = 0: Pbar_n0(cos t);  m > 0: sqrt2 Pbar_nm cos(m f);  m < 0: sqrt2 Pbar_n|m| sin(|m| f),
 * with Pbar_nm = sqrt((2n+1)/(4 pi) (n-m)!/(n+m)!) P_n^m (no Condon-Shortley phase),
 * from the standard normalised three-term recurrences in n.  Any orthonormal real
 * basis of each degree gives the same fitted field, which is all the method uses. */
void orc_real_sh(int p, double vx, double vy, double vz, double *Y) {
  double r = sqrt(vx * vx + vy * vy + vz * vz);
  double ct = 1.0, st = 0.0, f = 0.0;
  if (r > 0.0) {
    ct = vz / r;
    st = sqrt(vx * vx + vy * vy) / r;
    f = atan2(vy, vx);
  }
  int L = p + 1;
  double *P = (double *)malloc(sizeof(double) * (size_t)L * L); /* P[n*L + m] */
  P[0] = sqrt(1.0 / (4.0 * ORC_PI));
  for (int m = 1; m <= p; m++) P[m * L + m] = sqrt((2.0 * m + 1.0) / (2.0 * m)) * st * P[(m - 1) * L + (m - 1)];
  for (int m = 0; m < p; m++) P[(m + 1) * L + m] = sqrt(2.0 * m + 3.0) * ct * P[m * L + m];
  for (int m = 0; m <= p; m++) {
    for (int n = m + 2; n <= p; n++) {
      double an = sqrt((4.0 * n * n - 1.0) / ((double)n * n - (double)m * m));
      double bn = sqrt(((n - 1.0) * (n - 1.0) - (double)m * m) / (4.0 * (n - 1.0) * (n - 1.0) - 1.0));
      P[n * L + m] = an * (ct * P[(n - 1) * L + m] - bn * P[(n - 2) * L + m]);
    }
  }
  for (int n = 0; n <= p; n++) {
    Y[n * n + n] = P[n * L];
    for (int m = 1; m <= n; m++) {
      Y[n * n + n + m] = sqrt(2.0) * P[n * L + m] * cos(m * f);
      Y[n * n + n - m] = sqrt(2.0) * P[n * L + m] * sin(m * f);
    }
  }
  free(P);
}

/* ------------------------------------------------------------------------- */
/* Node sets.                                                                   */
/* ------------------------------------------------------------------------- */

/* Fibonacci (Hannay-Nye) rule of Sec. 2.4 on the sphere of radius R: for j = 0..F2,
 * z_j = -1 + 2j/F2, polar angle arccos(z_j + sin(pi z_j)/pi), azimuths pi j F1/F2 and
 * pi + pi j F1/F2, both with weight (2 pi R^2 / F2)(1 + cos(pi z_j)).
 * Node 2j takes the first azimuth, node 2j+1 the second; 2(F2+1) nodes in all.  */
void orc_fibonacci_nodes(int F1, int F2, double R, double *xyz, double *w) {
  for (int j = 0; j <= F2; j++) {
    double zj = -1.0 + 2.0 * j / (double)F2;
    double c = zj + sin(ORC_PI * zj) / ORC_PI;
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    double th = acos(c);
    double wt = 2.0 * ORC_PI * R * R / (double)F2 * (1.0 + cos(ORC_PI * zj));
    for (int h = 0; h < 2; h++) {
      double ph = ORC_PI * j * (double)F1 / (double)F2 + (h ? ORC_PI : 0.0);
      int s = 2 * j + h;
      xyz[3 * s + 0] = R * sin(th) * cos(ph);
      xyz[3 * s + 1] = R * sin(th) * sin(ph);
      xyz[3 * s + 2] = R * cos(th);
      w[s] = wt;
    }
  }
}

/* Check points: a golden-angle lattice of M points on the sphere of radius rc,
 * z_k = 1 - (2k+1)/M, azimuth pi (1 + sqrt5)(k + 1/2) taken mod 2 pi.           */
void orc_check_lattice(int M, double rc, double *xyz) {
  for (int k = 0; k < M; k++) {
    double zk = 1.0 - (2.0 * k + 1.0) / (double)M;
    double sk = sqrt(fmax(0.0, 1.0 - zk * zk));
    double ph = fmod(ORC_PI * (1.0 + sqrt(5.0)) * (k + 0.5), 2.0 * ORC_PI);
    xyz[3 * k + 0] = rc * sk * cos(ph);
    xyz[3 * k + 1] = rc * sk * sin(ph);
    xyz[3 * k + 2] = rc * zk;
  }
}

/* Gauss-Legendre rule of n nodes on [-1, 1]: the roots of P_n, found by Newton's method
 * from cos(pi (i + 3/4) / (n + 1/2)), with weights 2 / ((1 - x^2) P_n'(x)^2).  P_n and its
 * derivative come from the three-term recurrence and (1 - x^2) P_n' = n (P_{n-1} - x P_n).
 * Nodes are returned in decreasing order.                                       */
void orc_gl_nodes(int n, double *x, double *w) {
  for (int i = 0; i < n; i++) {
    double z = cos(ORC_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; it++) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; k++) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) p0 = 1.0;
      dp = n * (p0 - z * p1) / (1.0 - z * z);
      double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    /* derivative at the converged root */
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; k++) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    if (n == 1) p0 = 1.0;
    dp = n * (p0 - z * p1) / (1.0 - z * z);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

/* Algorithm 1, step 1: 2p Gauss-Legendre nodes in cos(theta) times equispaced azimuths on the
 * sphere of radius rc.  The paper takes 2p azimuths; at phi_j = pi j / p the harmonic
 * sin(p phi) vanishes, so degree p could not be fitted.  Here 2p + 1 azimuths
 * phi_j = 2 pi j / (2p + 1) are taken (M = 2p (2p + 1)), which resolve every order |m| <= p.
 * Point k = i (2p + 1) + j.  wq (optional, M): the quadrature weights w_i 2 pi / (2p + 1) of
 * the grid on the unit sphere, exact for products of harmonics of degree <= p.            */
void orc_check_gl(int p, double rc, double *xyz, double *wq) {
  int n = 2 * p, nph = 2 * p + 1;
  double *x = (double *)malloc(sizeof(double) * (size_t)n);
  double *w = (double *)malloc(sizeof(double) * (size_t)n);
  orc_gl_nodes(n, x, w);
  for (int i = 0; i < n; i++) {
    double st = sqrt(fmax(0.0, 1.0 - x[i] * x[i]));
    for (int j = 0; j < nph; j++) {
      int k = i * nph + j;
      double ph = 2.0 * ORC_PI * j / nph;
      xyz[3 * k + 0] = rc * st * cos(ph);
      xyz[3 * k + 1] = rc * st * sin(ph);
      xyz[3 * k + 2] = rc * x[i];
      if (wq) wq[k] = w[i] * 2.0 * ORC_PI / nph;
    }
  }
  free(x);
  free(w);
}

/* ------------------------------------------------------------------------- */
/* Dense least squares by Householder QR.                                       */
/* ------------------------------------------------------------------------- */

/* X (n x nrhs, row-major) minimising ||A X - B||_F for A (m x n, row-major, m >= n,
 * full column rank) and B (m x nrhs, row-major).  Returns 0, or -1 when m < n or a
 * column is numerically zero.                                                   */
int orc_lstsq(int m, int n, const double *A, int nrhs, const double *B, double *X) {
  if (m < n) return -1;
  double *W = (double *)malloc(sizeof(double) * (size_t)m * n);    /* column-major */
  double *C = (double *)malloc(sizeof(double) * (size_t)m * nrhs); /* column-major */
  for (int i = 0; i < m; i++) {
    for (int j = 0; j < n; j++) W[(size_t)j * m + i] = A[(size_t)i * n + j];
    for (int j = 0; j < nrhs; j++) C[(size_t)j * m + i] = B[(size_t)i * nrhs + j];
  }
  int status = 0;
  for (int k = 0; k < n; k++) {
    double *v = W + (size_t)k * m; /* column k, rows k..m-1 become the reflector */
    double nrm = 0.0;
    for (int i = k; i < m; i++) nrm += v[i] * v[i];
    nrm = sqrt(nrm);
    if (nrm == 0.0) { status = -1; break; }
    double alpha = v[k] > 0.0 ? -nrm : nrm; /* R_kk */
    v[k] -= alpha;                          /* v = x - alpha e1 */
    double vv = 0.0;
    for (int i = k; i < m; i++) vv += v[i] * v[i];
    /* apply H = I - 2 v v^T / (v^T v) to the remaining columns of W and to C */
#pragma omp parallel for schedule(static)
    for (int j = k + 1; j < n + nrhs; j++) {
      double *col = j < n ? W + (size_t)j * m : C + (size_t)(j - n) * m;
      double d = 0.0;
      for (int i = k; i < m; i++) d += v[i] * col[i];
      double f = 2.0 * d / vv;
      for (int i = k; i < m; i++) col[i] -= f * v[i];
    }
    /* keep R_kk in the diagonal slot; the reflector is no longer needed */
    v[k] = alpha;
  }
  if (status == 0) {
    for (int r = 0; r < nrhs; r++) {
      const double *c = C + (size_t)r * m;
      for (int i = n - 1; i >= 0; i--) {
        double s = c[i];
        for (int j = i + 1; j < n; j++) s -= W[(size_t)j * m + i] * X[(size_t)j * nrhs + r];
        X[(size_t)i * nrhs + r] = s / W[(size_t)i * m + i];
      }
    }
  }
  free(W);
  free(C);
  return status;
}

/* ------------------------------------------------------------------------- */
/* O1: the HSMA, step by step.                                                 */
/* ------------------------------------------------------------------------- */

typedef struct {
  double a, eps1, eps2, kappa; /* cavity radius, inner/outer dielectric, inverse Debye length */
  double tau;                  /* auxiliary sphere radius R_tau = (1 + tau) a */
  double rc_over_a;            /* check-point radius / a */
  int p;                       /* SH truncation order */
  int P;                       /* surface nodes = 2 (F2 + 1) */
  int M;                       /* check points */
  int F1;                      /* Fibonacci F1 (F2 = P/2 - 1) */
  int dipole;                  /* 0 exact normal dipole, 1 central-difference point pair,
                                  2 no dipole layer (single layer of monopoles only) */
  double dy_over_Rtau;         /* central-difference step / R_tau (dipole = 1) */
  int check_set;               /* 0 golden-angle lattice of M points, 1 the Gauss-Legendre grid (M = 2p (2p+1)) */
} orc_params;

/* Optional intermediate outputs; any pointer may be NULL. */
typedef struct {
  double *u, *v;         /* M: check fields */
  double *alpha, *beta;  /* K = (p+1)^2: fitted moments */
  double *Ahat;          /* K: correction coefficients, Phi_corr = sum Ahat (r/a)^n Y */
  double *Q, *D;         /* P: surface monopole strength and dipole strength */
  double *nodes, *w;     /* 3P, P */
  double *checks;        /* 3M */
  double *kelvin;        /* nt: the Kelvin-image part of the potential at each target */
} orc_diag;

static int orc_params_ok(const orc_params *pp) {
  if (!(pp->a > 0.0 && pp->eps1 > 0.0 && pp->eps2 > 0.0 && pp->kappa >= 0.0)) return 0;
  if (!(pp->tau > 0.0 && pp->rc_over_a >= 1.0)) return 0;
  if (pp->p < 0 || pp->P < 4 || (pp->P & 1) || pp->M < (pp->p + 1) * (pp->p + 1)) return 0;
  if (pp->check_set != 0 && (pp->check_set != 1 || pp->M != 2 * pp->p * (2 * pp->p + 1))) return 0;
  if (pp->dipole < 0 || pp->dipole > 2) return 0;
  return 1;
}

/* Step 1 of Algorithm 1: the check points of the chosen set on the sphere of radius rc. */
static void orc_check_points(const orc_params *pp, double *chk) {
  if (pp->check_set == 1)
    orc_check_gl(pp->p, pp->rc_over_a * pp->a, chk, NULL);
  else
    orc_check_lattice(pp->M, pp->rc_over_a * pp->a, chk);
}

/* Step S2 of Algorithm 1, realised at check points: the potential of the sources
 * (eq. "phicoul") and of the sources weighted by r_i / a at each check point.    */
void orc_check_fields(const orc_params *pp, long N, const double *x, const double *y, const double *z,
                      const double *q, const double *chk, double *u, double *v) {
  const double c0 = 1.0 / (4.0 * ORC_PI * pp->eps1);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < pp->M; k++) {
    double su = 0.0, sv = 0.0;
    for (long i = 0; i < N; i++) {
      double dx = chk[3 * k] - x[i], dy = chk[3 * k + 1] - y[i], dz = chk[3 * k + 2] - z[i];
      double g = c0 / sqrt(dx * dx + dy * dy + dz * dz);
      double ri = sqrt(x[i] * x[i] + y[i] * y[i] + z[i] * z[i]);
      su += q[i] * g;
      sv += q[i] * (ri / pp->a) * g;
    }
    u[k] = su;
    v[k] = sv;
  }
}

/* Step S3: least-squares fit of the exterior expansion of eq. "phicoul_final",
 *   u(c) = sum_nm alpha_nm (a/rc)^{n+1} Y_nm(c^) / ((2n+1) eps1 a),
 * alpha_nm = sum_i q_i (r_i/a)^n Y_nm(x_i^) when the sources are band-limited;
 * beta is fitted the same way from v.                                           */
int orc_fit_moments(const orc_params *pp, const double *chk, const double *u, const double *v,
                    double *alpha, double *beta) {
  int p = pp->p, K = (p + 1) * (p + 1), M = pp->M;
  double rc = pp->rc_over_a * pp->a;
  double *B = (double *)malloc(sizeof(double) * (size_t)M * K);
  double *rhs = (double *)malloc(sizeof(double) * (size_t)M * 2);
  double *X = (double *)malloc(sizeof(double) * (size_t)K * 2);
  double *Y = (double *)malloc(sizeof(double) * (size_t)K);
  for (int k = 0; k < M; k++) {
    orc_real_sh(p, chk[3 * k], chk[3 * k + 1], chk[3 * k + 2], Y);
    for (int n = 0; n <= p; n++) {
      double f = pow(pp->a / rc, n + 1) / ((2.0 * n + 1.0) * pp->eps1 * pp->a);
      for (int m = -n; m <= n; m++) B[(size_t)k * K + n * n + n + m] = f * Y[n * n + n + m];
    }
    rhs[2 * k] = u[k];
    rhs[2 * k + 1] = v[k];
  }
  int st = orc_lstsq(M, K, B, 2, rhs, X);
  for (int i = 0; i < K; i++) {
    alpha[i] = X[2 * i];
    beta[i] = X[2 * i + 1];
  }
  free(B);
  free(rhs);
  free(X);
  free(Y);
  return st;
}

/* Correction coefficients of eq. "phim" with the ion-dependent factor of Sec. 2.4,
 *   Mhat'_{n,i} = M_n - gamma - dbar (R_tau - r_K,i) / (2 r_K,i),   r_K,i = a^2 / r_i,
 * written as c_n + e r_i/a with c_n = M_n - gamma + dbar/2, e = -dbar R_tau / (2a).
 * Output: Ahat_nm with Phi_corr(x) = sum Ahat_nm (|x|/a)^n Y_nm(x^).             */
void orc_correction_coeffs(const orc_params *pp, const double *alpha, const double *beta, double *Ahat) {
  int p = pp->p;
  double eps = pp->eps1 / pp->eps2, mu = pp->kappa * pp->a, Rt = (1.0 + pp->tau) * pp->a;
  double g3[3];
  orc_image_constants(eps, mu, g3);
  double *Mn = (double *)malloc(sizeof(double) * (size_t)(p + 1));
  orc_kirkwood_factor(p, eps, mu, NULL, Mn);
  double e = -g3[2] * Rt / (2.0 * pp->a);
  for (int n = 0; n <= p; n++) {
    double cn = Mn[n] - g3[0] + 0.5 * g3[2];
    double den = (2.0 * n + 1.0) * pp->eps1 * pp->a;
    for (int m = -n; m <= n; m++) {
      int i = n * n + n + m;
      Ahat[i] = (cn * alpha[i] + e * beta[i]) / den;
    }
  }
  free(Mn);
}

/* Surface strengths from Green's second identity (eq. "GreenSecond") discretised by
 * the Fibonacci rule: at node y_s with weight w_s,
 *   Q_s = w_s dPhi_corr/dr (y_s),  D_s = -w_s Phi_corr(y_s),
 * so that Phi_corr(x) ~ sum_s [Q_s / |x - y_s| + D_s (x - y_s).y^_s / |x - y_s|^3] / (4 pi).
 * Single layer (dipole = 2): 1/|x - y| = sum_n 4 pi r^n / ((2n+1) R^(n+1)) sum_m Y_nm(x^) Y_nm(y^)
 * for r < R gives, for a density sigma = sum sigma_nm Y_nm on the sphere of radius R,
 *   (1/4 pi) int sigma(y) / |x - y| dS = sum R / (2n+1) (r/R)^n sigma_nm Y_nm(x^),
 * so Phi_corr is reproduced by sigma_nm = (2n+1)/R (R/a)^n Ahat_nm: Q_s = w_s sigma(y_s), D_s = 0. */
void orc_surface_strengths(const orc_params *pp, const double *Ahat, const double *nodes, const double *w,
                           double *Q, double *D) {
  int p = pp->p, K = (p + 1) * (p + 1);
  double Rt = (1.0 + pp->tau) * pp->a;
#pragma omp parallel
  {
    double *Y = (double *)malloc(sizeof(double) * (size_t)K);
#pragma omp for schedule(static)
    for (int s = 0; s < pp->P; s++) {
      orc_real_sh(p, nodes[3 * s], nodes[3 * s + 1], nodes[3 * s + 2], Y);
      double phi = 0.0, dphi = 0.0;
      for (int n = 0; n <= p; n++) {
        double rn = pow(Rt / pp->a, n);
        for (int m = -n; m <= n; m++) {
          double t = Ahat[n * n + n + m] * rn * Y[n * n + n + m];
          phi += t;
          dphi += t * (pp->dipole == 2 ? 2.0 * n + 1.0 : (double)n) / Rt;
        }
      }
      Q[s] = w[s] * dphi;
      D[s] = pp->dipole == 2 ? 0.0 : -w[s] * phi;
    }
    free(Y);
  }
}

/* Potential of the surface images at targets: exact dipole (dipole = 0), or the
 * paper's three point images (eq. "threeintegrals"): Q_s at y_s, -D_s/dy at
 * y_s^- = (R_tau - dy/2) y^_s and +D_s/dy at y_s^+ = (R_tau + dy/2) y^_s.        */
void orc_surface_potential(const orc_params *pp, const double *nodes, const double *Q, const double *D,
                           long nt, const double *tx, const double *ty, const double *tz, double *phi) {
  double Rt = (1.0 + pp->tau) * pp->a;
  double dy = pp->dy_over_Rtau * Rt;
#pragma omp parallel for schedule(static)
  for (long t = 0; t < nt; t++) {
    double s = 0.0;
    for (int k = 0; k < pp->P; k++) {
      double ux = nodes[3 * k] / Rt, uy = nodes[3 * k + 1] / Rt, uz = nodes[3 * k + 2] / Rt;
      double dx = tx[t] - nodes[3 * k], dyy = ty[t] - nodes[3 * k + 1], dz = tz[t] - nodes[3 * k + 2];
      double r = sqrt(dx * dx + dyy * dyy + dz * dz);
      s += Q[k] / (4.0 * ORC_PI * r);
      if (pp->dipole == 0) {
        s += D[k] * (dx * ux + dyy * uy + dz * uz) / (4.0 * ORC_PI * r * r * r);
      } else if (pp->dipole == 1) {
        double rm = Rt - 0.5 * dy, rp = Rt + 0.5 * dy;
        double mx = tx[t] - rm * ux, my = ty[t] - rm * uy, mz = tz[t] - rm * uz;
        double px = tx[t] - rp * ux, py = ty[t] - rp * uy, pz = tz[t] - rp * uz;
        s += (-D[k] / dy) / (4.0 * ORC_PI * sqrt(mx * mx + my * my + mz * mz));
        s += (D[k] / dy) / (4.0 * ORC_PI * sqrt(px * px + py * py + pz * pz));
      }
    }
    phi[t] = s;
  }
}

/* The modified Kelvin images of Sec. 2.4: at r_K,i = (a / r_i)^2 x_i a charge
 *   q_K,i = (q_i / a) [gamma r_K,i + dbar (R_tau - r_K,i) / 2],
 * potential q_K,i / (4 pi eps1 |x - r_K,i|).  An ion at the centre has its image at
 * infinity; the limit is the constant q_i (gamma - dbar/2) / (4 pi eps1 a).       */
void orc_kelvin_potential(const orc_params *pp, long N, const double *x, const double *y, const double *z,
                          const double *q, long nt, const double *tx, const double *ty, const double *tz,
                          double *phi) {
  double eps = pp->eps1 / pp->eps2, mu = pp->kappa * pp->a, Rt = (1.0 + pp->tau) * pp->a;
  double g3[3];
  orc_image_constants(eps, mu, g3);
  double a = pp->a, c0 = 1.0 / (4.0 * ORC_PI * pp->eps1);
#pragma omp parallel for schedule(static)
  for (long t = 0; t < nt; t++) {
    double s = 0.0;
    for (long i = 0; i < N; i++) {
      double ri = sqrt(x[i] * x[i] + y[i] * y[i] + z[i] * z[i]);
      if (ri == 0.0) {
        s += q[i] * (g3[0] - 0.5 * g3[2]) / a * c0;
        continue;
      }
      double f = (a / ri) * (a / ri);
      double kx = f * x[i], ky = f * y[i], kz = f * z[i];
      double rK = a * a / ri;
      double qK = q[i] / a * (g3[0] * rK + g3[2] * (Rt - rK) / 2.0);
      double dx = tx[t] - kx, dy = ty[t] - ky, dz = tz[t] - kz;
      s += c0 * qK / sqrt(dx * dx + dy * dy + dz * dz);
    }
    phi[t] = s;
  }
}

/* O1: the HSMA reaction potential (eq. "phirffinall") at nt targets for N sources,
 * following Algorithm 1: Kelvin images, check fields, fit, surface images, sum.
 * Returns 0, -1 for bad parameters, -2 for a source outside the cavity, -3 when
 * the fit fails.                                                                */
int orc_hsma_eval(const orc_params *pp, long N, const double *x, const double *y, const double *z,
                  const double *q, long nt, const double *tx, const double *ty, const double *tz,
                  double *phi, orc_diag *dg) {
  if (!orc_params_ok(pp)) return -1;
  for (long i = 0; i < N; i++)
    if (!(sqrt(x[i] * x[i] + y[i] * y[i] + z[i] * z[i]) < pp->a)) return -2;
  int p = pp->p, K = (p + 1) * (p + 1), M = pp->M, P = pp->P, F2 = P / 2 - 1;
  double Rt = (1.0 + pp->tau) * pp->a;
  double *chk = (double *)malloc(sizeof(double) * 3 * (size_t)M);
  double *u = (double *)malloc(sizeof(double) * (size_t)M);
  double *v = (double *)malloc(sizeof(double) * (size_t)M);
  double *al = (double *)malloc(sizeof(double) * (size_t)K);
  double *be = (double *)malloc(sizeof(double) * (size_t)K);
  double *Ah = (double *)malloc(sizeof(double) * (size_t)K);
  double *nodes = (double *)malloc(sizeof(double) * 3 * (size_t)P);
  double *w = (double *)malloc(sizeof(double) * (size_t)P);
  double *Q = (double *)malloc(sizeof(double) * (size_t)P);
  double *D = (double *)malloc(sizeof(double) * (size_t)P);
  double *pk = (double *)malloc(sizeof(double) * (size_t)(nt > 0 ? nt : 1));
  double *ps = (double *)malloc(sizeof(double) * (size_t)(nt > 0 ? nt : 1));
  int st = 0;

  orc_check_points(pp, chk);                                               /* step 1 */
  orc_check_fields(pp, N, x, y, z, q, chk, u, v);                          /* step 2 */
  if (orc_fit_moments(pp, chk, u, v, al, be) != 0) { st = -3; goto done; } /* step 3 */
  orc_correction_coeffs(pp, al, be, Ah);
  orc_fibonacci_nodes(pp->F1, F2, Rt, nodes, w);                           /* step 4 */
  orc_surface_strengths(pp, Ah, nodes, w, Q, D);
  orc_kelvin_potential(pp, N, x, y, z, q, nt, tx, ty, tz, pk);             /* step 5 */
  orc_surface_potential(pp, nodes, Q, D, nt, tx, ty, tz, ps);
  for (long t = 0; t < nt; t++) phi[t] = pk[t] + ps[t];

  if (dg) {
    if (dg->u) memcpy(dg->u, u, sizeof(double) * (size_t)M);
    if (dg->v) memcpy(dg->v, v, sizeof(double) * (size_t)M);
    if (dg->alpha) memcpy(dg->alpha, al, sizeof(double) * (size_t)K);
    if (dg->beta) memcpy(dg->beta, be, sizeof(double) * (size_t)K);
    if (dg->Ahat) memcpy(dg->Ahat, Ah, sizeof(double) * (size_t)K);
    if (dg->Q) memcpy(dg->Q, Q, sizeof(double) * (size_t)P);
    if (dg->D) memcpy(dg->D, D, sizeof(double) * (size_t)P);
    if (dg->nodes) memcpy(dg->nodes, nodes, sizeof(double) * 3 * (size_t)P);
    if (dg->w) memcpy(dg->w, w, sizeof(double) * (size_t)P);
    if (dg->checks) memcpy(dg->checks, chk, sizeof(double) * 3 * (size_t)M);
    if (dg->kelvin) memcpy(dg->kelvin, pk, sizeof(double) * (size_t)nt);
  }
done:
  free(chk); free(u); free(v); free(al); free(be); free(Ah);
  free(nodes); free(w); free(Q); free(D); free(pk); free(ps);
  return st;
}

/* ------------------------------------------------------------------------- */
/* Field at the targets (Algorithm 1, step 5 evaluates the field with the potential). */
/* ------------------------------------------------------------------------- */

/* E = -grad Phi at the target with every source held fixed: for an image charge c at
 * position s, the field c (x - s) / |x - s|^3 in units of the potential's prefactor.
 * Kelvin images (Sec. 2.4): c = q_K,i / (4 pi eps1) at r_K,i; an ion at the centre
 * has its image at infinity and adds a constant potential, hence no field.        */
void orc_kelvin_field(const orc_params *pp, long N, const double *x, const double *y, const double *z,
                      const double *q, long nt, const double *tx, const double *ty, const double *tz,
                      double *ex, double *ey, double *ez) {
  double eps = pp->eps1 / pp->eps2, mu = pp->kappa * pp->a, Rt = (1.0 + pp->tau) * pp->a;
  double g3[3];
  orc_image_constants(eps, mu, g3);
  double a = pp->a, c0 = 1.0 / (4.0 * ORC_PI * pp->eps1);
#pragma omp parallel for schedule(static)
  for (long t = 0; t < nt; t++) {
    double fx = 0.0, fy = 0.0, fz = 0.0;
    for (long i = 0; i < N; i++) {
      double ri = sqrt(x[i] * x[i] + y[i] * y[i] + z[i] * z[i]);
      if (ri == 0.0) continue;
      double f = (a / ri) * (a / ri);
      double rK = a * a / ri;
      double qK = q[i] / a * (g3[0] * rK + g3[2] * (Rt - rK) / 2.0);
      double dx = tx[t] - f * x[i], dy = ty[t] - f * y[i], dz = tz[t] - f * z[i];
      double r = sqrt(dx * dx + dy * dy + dz * dz);
      double c = c0 * qK / (r * r * r);
      fx += c * dx;
      fy += c * dy;
      fz += c * dz;
    }
    ex[t] = fx;
    ey[t] = fy;
    ez[t] = fz;
  }
}

/* Field of the surface images (eq. "GreenSecond" discretised by the Fibonacci rule).
 * Monopole Q at y: Q d / (4 pi |d|^3), d = x - y.  Exact dipole (dipole = 0), potential
 * D (d . u) / (4 pi |d|^3) with u the outward unit normal: its negative gradient is
 * D [3 (d . u) d / |d|^5 - u / |d|^3] / (4 pi).  Paper form (dipole = 1): the two point
 * charges -D/dy at (R_tau - dy/2) u and +D/dy at (R_tau + dy/2) u (eq. "threeintegrals"). */
void orc_surface_field(const orc_params *pp, const double *nodes, const double *Q, const double *D, long nt,
                       const double *tx, const double *ty, const double *tz, double *ex, double *ey, double *ez) {
  double Rt = (1.0 + pp->tau) * pp->a;
  double dy = pp->dy_over_Rtau * Rt;
  double k4 = 1.0 / (4.0 * ORC_PI);
#pragma omp parallel for schedule(static)
  for (long t = 0; t < nt; t++) {
    double fx = 0.0, fy = 0.0, fz = 0.0;
    for (int k = 0; k < pp->P; k++) {
      double ux = nodes[3 * k] / Rt, uy = nodes[3 * k + 1] / Rt, uz = nodes[3 * k + 2] / Rt;
      double dx = tx[t] - nodes[3 * k], dyy = ty[t] - nodes[3 * k + 1], dz = tz[t] - nodes[3 * k + 2];
      double r = sqrt(dx * dx + dyy * dyy + dz * dz);
      double r3 = r * r * r;
      double c = k4 * Q[k] / r3;
      fx += c * dx;
      fy += c * dyy;
      fz += c * dz;
      if (pp->dipole == 0) {
        double du = dx * ux + dyy * uy + dz * uz;
        double cd = k4 * D[k] * 3.0 * du / (r3 * r * r), cu = k4 * D[k] / r3;
        fx += cd * dx - cu * ux;
        fy += cd * dyy - cu * uy;
        fz += cd * dz - cu * uz;
      } else if (pp->dipole == 1) {
        double rm = Rt - 0.5 * dy, rp = Rt + 0.5 * dy;
        double mx = tx[t] - rm * ux, my = ty[t] - rm * uy, mz = tz[t] - rm * uz;
        double px = tx[t] - rp * ux, py = ty[t] - rp * uy, pz = tz[t] - rp * uz;
        double rmm = sqrt(mx * mx + my * my + mz * mz), rpp = sqrt(px * px + py * py + pz * pz);
        double cm = k4 * (-D[k] / dy) / (rmm * rmm * rmm), cp = k4 * (D[k] / dy) / (rpp * rpp * rpp);
        fx += cm * mx + cp * px;
        fy += cm * my + cp * py;
        fz += cm * mz + cp * pz;
      }
    }
    ex[t] = fx;
    ey[t] = fy;
    ez[t] = fz;
  }
}

/* O1 with the field: Algorithm 1 as in orc_hsma_eval (steps 1-4 give the images and
 * the surface strengths), then step 5 evaluates both the potential and the field
 * E = -grad Phi_RF at the targets, every image held fixed.  Return codes as
 * orc_hsma_eval.                                                                */
int orc_hsma_field(const orc_params *pp, long N, const double *x, const double *y, const double *z,
                   const double *q, long nt, const double *tx, const double *ty, const double *tz,
                   double *phi, double *ex, double *ey, double *ez) {
  if (!orc_params_ok(pp)) return -1;
  for (long i = 0; i < N; i++)
    if (!(sqrt(x[i] * x[i] + y[i] * y[i] + z[i] * z[i]) < pp->a)) return -2;
  int p = pp->p, K = (p + 1) * (p + 1), M = pp->M, P = pp->P, F2 = P / 2 - 1;
  double Rt = (1.0 + pp->tau) * pp->a;
  size_t n1 = (size_t)(nt > 0 ? nt : 1);
  double *chk = (double *)malloc(sizeof(double) * 3 * (size_t)M);
  double *u = (double *)malloc(sizeof(double) * (size_t)M);
  double *v = (double *)malloc(sizeof(double) * (size_t)M);
  double *al = (double *)malloc(sizeof(double) * (size_t)K);
  double *be = (double *)malloc(sizeof(double) * (size_t)K);
  double *Ah = (double *)malloc(sizeof(double) * (size_t)K);
  double *nodes = (double *)malloc(sizeof(double) * 3 * (size_t)P);
  double *w = (double *)malloc(sizeof(double) * (size_t)P);
  double *Q = (double *)malloc(sizeof(double) * (size_t)P);
  double *D = (double *)malloc(sizeof(double) * (size_t)P);
  double *pk = (double *)malloc(sizeof(double) * n1);
  double *ps = (double *)malloc(sizeof(double) * n1);
  double *fk = (double *)malloc(sizeof(double) * 3 * n1);
  double *fs = (double *)malloc(sizeof(double) * 3 * n1);
  int st = 0;

  orc_check_points(pp, chk);                                               /* step 1 */
  orc_check_fields(pp, N, x, y, z, q, chk, u, v);                          /* step 2 */
  if (orc_fit_moments(pp, chk, u, v, al, be) != 0) { st = -3; goto done; } /* step 3 */
  orc_correction_coeffs(pp, al, be, Ah);
  orc_fibonacci_nodes(pp->F1, F2, Rt, nodes, w);                           /* step 4 */
  orc_surface_strengths(pp, Ah, nodes, w, Q, D);
  orc_kelvin_potential(pp, N, x, y, z, q, nt, tx, ty, tz, pk);             /* step 5 */
  orc_surface_potential(pp, nodes, Q, D, nt, tx, ty, tz, ps);
  orc_kelvin_field(pp, N, x, y, z, q, nt, tx, ty, tz, fk, fk + n1, fk + 2 * n1);
  orc_surface_field(pp, nodes, Q, D, nt, tx, ty, tz, fs, fs + n1, fs + 2 * n1);
  for (long t = 0; t < nt; t++) {
    phi[t] = pk[t] + ps[t];
    ex[t] = fk[t] + fs[t];
    ey[t] = fk[n1 + t] + fs[n1 + t];
    ez[t] = fk[2 * n1 + t] + fs[2 * n1 + t];
  }
done:
  free(chk); free(u); free(v); free(al); free(be); free(Ah);
  free(nodes); free(w); free(Q); free(D); free(pk); free(ps); free(fk); free(fs);
  return st;
}

/* Direct Coulomb energy of the ions in medium eps1 (eq. "phicoul"):
 * E_C = (1/2) sum_{i != j} q_i q_j / (4 pi eps1 |x_i - x_j|), the definition summed in FP64. */
double orc_coulomb_energy(double eps1, long N, const double *x, const double *y, const double *z,
                          const double *q) {
  double e = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : e)
  for (long i = 0; i < N; i++) {
    double s = 0.0;
    for (long j = 0; j < N; j++) {
      if (j == i) continue;
      double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
      s += q[j] / sqrt(dx * dx + dy * dy + dz * dz);
    }
    e += q[i] * s;
  }
  return 0.5 * e / (4.0 * ORC_PI * eps1);
}

/* ------------------------------------------------------------------------- */
/* O2: the Kirkwood series (Sec. 2.2).                                          */
/* ------------------------------------------------------------------------- */

/* Reaction potential at nt targets from eq. "phirf" with the coefficients of eq.
 * "Anm".  Summing over m by the addition theorem gives, for a source q at x' and a
 * target x, q/(4 pi eps1 a) sum_n M_n t^n P_n(c) with t = |x||x'|/a^2 and
 * c = cos(angle between x and x').
 *   order > 0: the series truncated after n = order (the paper's comparison method);
 *   order <= 0: summed to convergence, with the gamma part of M_n summed in closed
 *     form, gamma / sqrt(1 - 2tc + t^2) (the Kelvin image of eq. "Phihybrid"), and
 *     the rest, sum (M_n - gamma) t^n P_n(c), continued until the bound
 *     max|M_n - gamma| t^n / (1 - t) of the remaining tail is below tol * |first term|
 *     or n reaches nmax; the largest remaining bound is returned in *tail.
 * Every source contributes to every target, including the ion's own image.       */
int orc_kirkwood_eval(double a, double eps1, double eps2, double kappa, long N, const double *x, const double *y,
                      const double *z, const double *q, long nt, const double *tx, const double *ty,
                      const double *tz, int order, int nmax, double tol, double *phi, double *tail) {
  if (!(a > 0.0 && eps1 > 0.0 && eps2 > 0.0 && kappa >= 0.0)) return -1;
  double eps = eps1 / eps2, mu = kappa * a;
  int nm = order > 0 ? order : nmax;
  double *Mn = (double *)malloc(sizeof(double) * (size_t)(nm + 1));
  orc_kirkwood_factor(nm, eps, mu, NULL, Mn);
  double g3[3];
  orc_image_constants(eps, mu, g3);
  double gamma = g3[0];
  double cmax = 0.0;
  for (int n = 0; n <= nm; n++) cmax = fmax(cmax, fabs(Mn[n] - gamma));
  double worst = 0.0;
#pragma omp parallel for schedule(dynamic, 1) reduction(max : worst)
  for (long t = 0; t < nt; t++) {
    double rt = sqrt(tx[t] * tx[t] + ty[t] * ty[t] + tz[t] * tz[t]);
    double s = 0.0;
    for (long j = 0; j < N; j++) {
      double rj = sqrt(x[j] * x[j] + y[j] * y[j] + z[j] * z[j]);
      double tt = rt * rj / (a * a);
      double c = (rt > 0.0 && rj > 0.0) ? (tx[t] * x[j] + ty[t] * y[j] + tz[t] * z[j]) / (rt * rj) : 1.0;
      if (c > 1.0) c = 1.0;
      if (c < -1.0) c = -1.0;
      double sum = 0.0;
      if (order > 0) {
        double P0 = 1.0, P1 = c, tn = 1.0;
        sum = Mn[0];
        for (int n = 1; n <= order; n++) {
          tn *= tt;
          if (n > 1) {
            double P2 = ((2.0 * n - 1.0) * c * P1 - (n - 1.0) * P0) / n;
            P0 = P1;
            P1 = P2;
          }
          sum += Mn[n] * tn * P1;
        }
      } else {
        sum = gamma / sqrt(1.0 - 2.0 * tt * c + tt * tt);
        double P0 = 1.0, P1 = c, tn = 1.0;
        sum += Mn[0] - gamma;
        double lim = tol * fabs(sum) + 1e-300;
        int n = 1;
        for (; n <= nmax; n++) {
          tn *= tt;
          if (tt == 0.0) break;
          if (n > 1) {
            double P2 = ((2.0 * n - 1.0) * c * P1 - (n - 1.0) * P0) / n;
            P0 = P1;
            P1 = P2;
          }
          sum += (Mn[n] - gamma) * tn * P1;
          if (cmax * tn * tt / (1.0 - tt) < lim) break;
        }
        if (n > nmax && tt > 0.0) {
          double b = cmax * tn / (1.0 - tt) / (fabs(sum) + 1e-300);
          if (b > worst) worst = b;
        }
      }
      s += q[j] * sum;
    }
    phi[t] = s / (4.0 * ORC_PI * eps1 * a);
  }
  if (tail) *tail = worst;
  free(Mn);
  return 0;
}
