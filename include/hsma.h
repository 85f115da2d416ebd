/*
 * hsma.h -- C ABI of the MI355X (gfx950) implementation of the harmonic surface
 * mapping algorithm (HSMA) for the reaction potential of N ions in a dielectric
 * sphere embedded in a linearised Poisson-Boltzmann continuum.
 *
 * Method: J. Fu and Z. Gan, arXiv:1907.01724.  The interface problem is Sec. 2.1
 * (eqs. "phiinsideeq", "phioutsideeq", "boundarycondition"); the quantity computed
 * is the reaction potential Phi_RF of eq. "phiin" at the ions, in the
 * image-plus-surface form of eq. "phirffinall" (Sec. 2.4, Algorithm 1):
 *
 *   Phi_RF(x_i) = sum_{j} q_K,j / (4 pi eps1 |x_i - r_K,j|)           (modified Kelvin images)
 *               + sum_{s<P} [Q_s + D_s (x_i - y_s).y^_s / |x_i - y_s|^2] / (4 pi |x_i - y_s|)
 *
 * with r_K,j = (a/r_j)^2 x_j and q_K,j = (q_j/a)[gamma r_K,j + dbar (R_tau - r_K,j)/2]
 * (Sec. 2.4), surface nodes y_s of the Fibonacci rule on the auxiliary sphere of
 * radius R_tau = (1 + tau) a, and monopole/dipole strengths Q_s, D_s obtained from a
 * fixed least-squares fit of the ions' potential at M check points (Algorithm 1,
 * steps 1-3) mapped through Green's second identity (eq. "GreenSecond").
 * The ion's own image (j = i) is included: it is the ion's self polarisation.
 *
 * Units: a charge q in medium eps1 has potential q / (4 pi eps1 r) (eq. "phicoul").
 * Multiply by the caller's Coulomb constant if another unit system is wanted.
 *
 * Conventions shared by every entry point:
 *  - Every double is IEEE binary64.  Arrays marked [device] are device pointers on
 *    the plan's device; [host] marks host pointers.  Coordinates and charges are
 *    structure-of-arrays: x[i], y[i], z[i], q[i], i < N, with the sphere centred at
 *    the origin.
 *  - Ownership: the caller owns every input/output array and the workspace and must
 *    keep them alive until the stream has executed the call.  Plans and systems own
 *    their internal device buffers and free them in the matching destroy call.
 *  - Streams: compute entry points only enqueue work on the given stream (0 = the
 *    null stream); they never synchronise, allocate or free, so they may be captured
 *    into a HIP graph.  hsma_plan*, hsma_system_create/destroy and hsma_stream_check
 *    synchronise and may allocate.
 *  - Validation: scalar arguments are checked on the host before anything is
 *    enqueued (HSMA_EINVAL).  An ion with |x_i| >= a or a non-finite input value is
 *    detected on the device: it raises the plan's domain flag, which
 *    hsma_stream_check reports as HSMA_EDOMAIN; the outputs of that call are
 *    undefined.
 *  - Determinism: every reduction runs in a fixed order, so a result is bitwise
 *    reproducible for the same inputs, plan and device.
 *  - Thread safety: a plan is immutable after creation and may be used from several
 *    threads and streams at once (they share its domain flag); a system must not be
 *    used concurrently.
 */
#ifndef HSMA_H
#define HSMA_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HSMA_OK = 0,
  HSMA_EINVAL = 1,  /* invalid scalar argument or null pointer */
  HSMA_EDOMAIN = 2, /* an ion outside the cavity or a non-finite input (device flag) */
  HSMA_ENOMEM = 3,  /* device or host allocation failed */
  HSMA_EBUSY = 4,   /* reserved for admission control */
  HSMA_EDEVICE = 5, /* a HIP runtime call failed */
  HSMA_ESTATE = 6   /* object in the wrong state (e.g. plan built for another device) */
} hsma_status;

/* Arithmetic of the pair sums of the potentials (the two Coulomb sums of Algorithm 1, steps 2
 * and 5).  Energies do not depend on it: every entry point that returns E sums them from FP64
 * pairs (see hsma_energy). */
typedef enum {
  HSMA_PAIR_FP32 = 0,      /* FP32 pairs, FP32 running sum per target (precision sweep only) */
  HSMA_PAIR_FP32_COMP = 1, /* FP32 pairs, FP32 sums over 32-source tiles folded into FP64 (default) */
  HSMA_PAIR_FP64 = 2       /* FP64 coordinates and pairs, FP32-seeded FP64 Newton reciprocal root */
} hsma_pair_precision;

typedef struct hsma_plan_s *hsma_plan_t;
typedef struct hsma_group_s *hsma_group_t;
typedef struct hsma_system_s *hsma_system_t;

/* Discretisation options.  Fields left at the values of hsma_plan_opts_default()
 * give: p = floor(sqrt(P)/2), tau = 0.1, rc_over_a = 1 + tau, F1 = the integer
 * nearest F2/golden-ratio that is coprime to F2, FP32 compensated pair sums. */
typedef struct {
  int p;            /* spherical-harmonic truncation order (eq. "phim"); < 0: default */
  double tau;       /* auxiliary sphere R_tau = (1 + tau) a, tau > 0 (Sec. 2.4) */
  double rc_over_a; /* radius of the check points / a, >= 1; <= 0: 1 + tau */
  int F1;           /* Fibonacci-rule F1 (Sec. 2.4), 0 < F1 < F2; 0: default */
  int pair_prec;    /* hsma_pair_precision */
  int check_set;    /* check points: 0 golden-angle lattice of M points (default); 1 the
                       Gauss-Legendre grid of Algorithm 1 step 1: 2p nodes in cos(theta) times
                       2p + 1 equispaced azimuths (the paper's 2p azimuths are zeros of
                       sin(p phi) and cannot fit degree p), so M must be 2p (2p + 1).  Set
                       rc_over_a = 1 for the paper's placement on the interface. */
  int dipole;       /* surface dipoles (eq. "GreenSecond"): 0 exact normal dipoles (default);
                       1 the paper's pair of point charges -+D/dy at R_tau -+ dy/2 along the
                       normal (eq. "approxG"); the pair cancels about log10(R_tau/dy) digits, so
                       it is meant for FP64 pairs or a large dy; 2 no dipole layer: a single
                       layer of monopoles alone (the first integral of eq. "threeintegrals"),
                       with the density that has the same harmonic potential inside the
                       sphere, Q'_s = w_s sum (2n+1)/R_tau (R_tau/a)^n Ahat_nm Y_nm(y_s), D' = 0.
                       Plans of one group must share this choice. */
  double dy_over_Rtau; /* dy / R_tau for dipole = 1, in (0, 0.1); <= 0: 1e-5 */
} hsma_plan_opts;

/* Read-only description of a plan (for callers and tests). */
typedef struct {
  double a, eps1, eps2, kappa;
  double tau, R_tau, rc;           /* auxiliary radius and check-point radius */
  double gamma, sigma, dbar;       /* constants of eq. "Anuapp" */
  int p, K, P, M, F1, F2;          /* K = (p+1)^2 fitted coefficients; P = 2 (F2 + 1) */
  int pair_prec;
  int device;
  int check_set;
  int dipole;
  double dy_over_Rtau;
} hsma_plan_info;

hsma_plan_opts hsma_plan_opts_default(void);

/* Build a plan for one cavity: a > 0 (radius), eps1, eps2 > 0 (dielectric constants
 * inside/outside), kappa >= 0 (inverse Debye length outside), P surface nodes (even,
 * >= 8; P = 2 (F2 + 1) nodes of the Fibonacci rule of Sec. 2.4) and M check points
 * (M >= ceil(1.5 (p+1)^2)).  Runs the FP64 plan kernels on the current device
 * (Kirkwood factors M_n of eq. "Anuapp1", node sets, real SH bases, the normal
 * equations' Cholesky factor and the fixed fit/surface operators) and synchronises.
 * Plans with equal (p, P, M, F1, tau, rc/a) share their dimensionless operators.
 * Errors: HSMA_EINVAL (bad scalar), HSMA_ENOMEM, HSMA_EDEVICE. */
hsma_status hsma_plan(double a, double eps1, double eps2, double kappa, int P, int M, hsma_plan_t *out);
hsma_status hsma_plan_ex(double a, double eps1, double eps2, double kappa, int P, int M,
                         const hsma_plan_opts *opts /* [host], NULL = defaults */, hsma_plan_t *out);
hsma_status hsma_plan_destroy(hsma_plan_t plan);
hsma_status hsma_plan_get_info(hsma_plan_t plan, hsma_plan_info *info /* [host] */);

/* Bytes of device workspace hsma_potential / hsma_energy need for N ions, covering both
 * launches of hsma_energy (256-byte aligned pointer required). */
size_t hsma_workspace_bytes(hsma_plan_t plan, int64_t N);

/* Reaction potential Phi_RF at every ion (eq. "phirffinall"), N >= 0.
 * x, y, z, q: [device] N doubles each; phi: [device] N doubles (output);
 * ws: [device] workspace of ws_bytes >= hsma_workspace_bytes(plan, N) bytes (a smaller one,
 * e.g. one sized before a change of hsma_group_tune, is refused with HSMA_EINVAL).
 * Errors: HSMA_EINVAL, HSMA_ESTATE (current device is not the plan's), HSMA_EDEVICE. */
hsma_status hsma_potential(hsma_plan_t plan, int64_t N, const double *x, const double *y, const double *z,
                           const double *q, double *phi, void *ws, size_t ws_bytes, hipStream_t stream);

/* Reaction energy E = (1/2) sum_i q_i Phi_RF(x_i) (the self energy of Sec. 4.1
 * generalised to N ions), from FP64 pair sums whatever the plan's pair precision, reduced in
 * a fixed order: relative error 1e-16 to 1e-12 against an FP64 evaluation (target 1e-9).  E is
 * a bilinear form in the charges, so it is summed without forming the potentials: per ion pair
 * one reciprocal root serves both ordered image terms (the symmetric image distance of Sec. 2.4),
 * and every ion block pair and surface-node chunk adds one FP64 value; check sums and fit are
 * FP64 as well.  Ion pairs of which one ion lies within 0.995 a of the centre, check sums over
 * such ions, and surface pairs when the nodes lie on one sphere R_tau >= 1.05 a, take their
 * squared distance in expanded form (|x|^2 + |y|^2 - 2 x.y scaled, for the check sums divided
 * by |x|^2 + |y|^2; a pair's form rounds to at most about 5e-11 relative, for the pairs nearest
 * the interface); the rest take exact differences.  E: [device] one double.  phi: [device] N doubles, or NULL for the energy alone;
 * when given, a second launch on the same workspace writes the potentials in the plan's pair
 * precision (E is the same bit for bit either way). */
hsma_status hsma_energy(hsma_plan_t plan, int64_t N, const double *x, const double *y, const double *z,
                        const double *q, double *phi, double *E, void *ws, size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): hsma_energy without a caller workspace.  The
 * workspace is a device array of HSMA_NOALLOC_BYTES in the library's code object, one per
 * device, held until the process ends; the call allocates and frees nothing.  Arguments,
 * results and errors as hsma_energy; N whose hsma_workspace_bytes(plan, N) exceeds
 * HSMA_NOALLOC_BYTES is refused with HSMA_EINVAL before anything is enqueued (64 MiB: up to
 * N = 42797 with P = 1600 surface nodes and M = 2400 check points).  Every call on a device shares that
 * device's array, so calls that overlap on one device (several streams or threads) race and
 * must be ordered by the caller.  The array needs no clearing: each call writes what it
 * reads. */
#define HSMA_NOALLOC_BYTES (64u << 20)
hsma_status hsma_energy_noalloc(hsma_plan_t plan, int64_t N, const double *x, const double *y, const double *z,
                                const double *q, double *phi, double *E, hipStream_t stream);

/* Potential and field at every ion (Algorithm 1, step 5, which evaluates both at the ions):
 * E_i = -grad Phi_RF(x) at x = x_i with every image, the ion's own
 * included, and every surface charge held fixed; the force on ion i is q_i E_i up to the
 * method's error (the fixed-image field of eq. "phirffinall").  Same units as the
 * potential (divide by the length unit).  The evaluation runs the one-directional pair
 * kernel with four sums (Phi, Ex, Ey, Ez) per target; the own image's field is added in
 * FP64 as -x_i Phi_own,i / (a^2 - r_i^2).
 *   ex, ey, ez: [device] N doubles each (output; required when N > 0);
 *   phi: [device] N doubles or NULL; E: [device] one double or NULL (when given, computed by
 *   the FP64 energy launch of hsma_energy before the field launch);
 *   ws: [device] ws_bytes >= hsma_field_workspace_bytes(plan, N).
 * Errors as hsma_potential. */
size_t hsma_field_workspace_bytes(hsma_plan_t plan, int64_t N);
hsma_status hsma_field(hsma_plan_t plan, int64_t N, const double *x, const double *y, const double *z,
                       const double *q, double *phi, double *ex, double *ey, double *ez, double *E, void *ws,
                       size_t ws_bytes, hipStream_t stream);

/* The Kirkwood series of Sec. 2.2 (eqs. "phirf", "Anm", "Anuapp1"), the paper's comparison
 * method, for the plan's cavity (a, eps1, eps2, kappa; its discretisation is not used):
 *   Phi_i = sum_j q_j / (4 pi eps1 a) sum_{n=0}^{order} M_n t^n P_n(c),
 *   t = |x_i| |x_j| / a^2, c = cos(angle between x_i and x_j),
 * truncated after n = order (0 <= order <= HSMA_KIRKWOOD_MAX_ORDER), every source on every
 * ion including its own term, in FP64, summed in a fixed order.  The series converges like
 * t^order, i.e. slowly for ions near the interface (Sec. 4.1); it is O(N^2 order).
 *   x, y, z, q: [device] N doubles; phi: [device] N doubles or NULL; E: [device] one double
 *   (E = (1/2) sum q_i Phi_i) or NULL; ws: [device] ws_bytes >=
 *   hsma_kirkwood_workspace_bytes(order, N), 256-byte aligned.
 * Ions outside the cavity raise the plan's domain flag (hsma_stream_check).  Errors as
 * hsma_potential. */
#define HSMA_KIRKWOOD_MAX_ORDER 100000
size_t hsma_kirkwood_workspace_bytes(int order, int64_t N);
hsma_status hsma_kirkwood(hsma_plan_t plan, int order, int64_t N, const double *x, const double *y, const double *z,
                          const double *q, double *phi, double *E, void *ws, size_t ws_bytes, hipStream_t stream);

/* Intermediate results of the last launch that used ws (the potential launch of hsma_potential,
 * or of hsma_energy with phi, in the plan's pair precision; the FP64 energy launch of hsma_energy
 * without phi),
 * copied to host arrays (for tests and diagnostics; synchronises the stream).
 * Any output pointer may be NULL.  u, v: M check fields; Q, D: P surface strengths
 * (Q_s and D_s of the header comment, divided by 4 pi and 4 pi R_tau). */
hsma_status hsma_debug_intermediates(hsma_plan_t plan, int64_t N, const void *ws, hipStream_t stream,
                                     double *u, double *v, double *Q, double *D);

/* Groups: nplans plans built with the same discretisation (p, P, M, F1, tau, rc/a) and
 * pair precision, evaluated together.  Each plan keeps its own cavity (a, eps1, eps2,
 * kappa); a group stores the plans' constants on the device.  The plans must outlive
 * the group.  Errors: HSMA_EINVAL, HSMA_ESTATE (plans of different discretisations,
 * precisions or devices), HSMA_EDEVICE.  hsma_plan_group returns the one-plan group a
 * plan owns (freed with the plan; not to be passed to hsma_group_destroy). */
hsma_status hsma_group_create(int nplans, const hsma_plan_t *plans /* [host] */, hsma_group_t *out);
hsma_status hsma_group_destroy(hsma_group_t group);
hsma_group_t hsma_plan_group(hsma_plan_t plan);

/* Batched reaction potentials and energies of nsys independent ion configurations in
 * one set of launches (the persistent pair kernels take (system, 64 ions, source chunk)
 * items from a device work counter; the fit is applied to all systems at once, as FP32
 * MFMA GEMMs when nsys >= 192 in the FP32 pair modes).
 *   offsets: [device] nsys + 1 int64, offsets[0] = 0, non-decreasing; system b owns ions
 *            [offsets[b], offsets[b+1]) of x, y, z, q, phi;
 *   plan_of: [device] nsys int32 plan indices into the group, or NULL (all use plan 0);
 *   total_n = offsets[nsys] and max_n >= every system's size: [host] scalars that size
 *            the work and the workspace (hsma_batched_workspace_bytes);
 *   phi: [device] total_n doubles or NULL; E: [device] nsys energies or NULL;
 *   ws: [device] ws_bytes >= hsma_batched_workspace_bytes(group, nsys, total_n, max_n).
 * Energies come from the FP64 energy launch and potentials from the pair-precision launch, as in
 * hsma_energy; a system's energy does not depend on the batch it is in beyond the rounding of
 * its check sums, whose chunk lengths follow the call's sizes.
 * A system of 0 ions has energy 0.  The device checks offsets and plan_of against
 * total_n, max_n and the group size before any work: on a mismatch the call does nothing
 * and hsma_group_stream_check reports HSMA_EINVAL.  Errors: HSMA_EINVAL, HSMA_ESTATE,
 * HSMA_EDEVICE. */
size_t hsma_batched_workspace_bytes(hsma_group_t group, int nsys, int64_t total_n, int64_t max_n);
hsma_status hsma_energy_batched(hsma_group_t group, int nsys, const int64_t *offsets, const int32_t *plan_of,
                                int64_t total_n, int64_t max_n, const double *x, const double *y, const double *z,
                                const double *q, double *phi, double *E, void *ws, size_t ws_bytes,
                                hipStream_t stream);

/* Batched potentials, fields and energies: hsma_energy_batched's arguments and checks, plus
 * ex, ey, ez ([device] total_n doubles each, required) as in hsma_field; ws_bytes >=
 * hsma_field_batched_workspace_bytes(group, nsys, total_n, max_n). */
size_t hsma_field_batched_workspace_bytes(hsma_group_t group, int nsys, int64_t total_n, int64_t max_n);
hsma_status hsma_field_batched(hsma_group_t group, int nsys, const int64_t *offsets, const int32_t *plan_of,
                               int64_t total_n, int64_t max_n, const double *x, const double *y, const double *z,
                               const double *q, double *phi, double *ex, double *ey, double *ez, double *E,
                               void *ws, size_t ws_bytes, hipStream_t stream);

/* Launch shape of the group's pair kernels (check and evaluation sums).  persistent = 1:
 * one grid of resident blocks (the occupancy limit on every compute unit) whose blocks
 * take (system, 64 targets, source chunk) items from a device counter; 0 (default): one
 * item per block, the hardware workgroup dispatcher balancing the load.  target_items
 * (default 65536, 64..2^22): the number of items each pair kernel aims for, which sets the
 * source-chunk length.  Results depend on the launch shape only through the summation
 * order (rounding).  Errors: HSMA_EINVAL. */
hsma_status hsma_group_tune(hsma_group_t group, int persistent, int target_items);

/* Kelvin sums by the symmetric kernel.  The image distance of an ion pair satisfies
 * |x_j - r_K,i| = (r_j / r_i) |x_i - r_K,j| (Sec. 2.4 images), so one reciprocal root serves
 * both ions of a pair.  The kernel works on blocks of 256 or 512 ions and applies to the
 * compensated FP32 and the FP64 pair precisions (not to the plain FP32 sweep mode, nor to the
 * field) when its partial sums (8 bytes per ion and block) fit in 16 GiB.  mode 0: never; 1 (default): blocks of 256, else 512, when it applies and the launch
 * is large enough (see hsma_group_eval_kernel); 2 / 3: blocks of 256 / 512 whenever they
 * apply.  Results differ only in rounding.  Errors: HSMA_EINVAL. */
hsma_status hsma_group_set_symmetric(hsma_group_t group, int mode);

/* Which evaluation kernel hsma_energy_batched would run for these sizes: the ion-block size
 * (256 or 512) of the symmetric Kelvin kernel, 0 for the one-directional kernel, -1 for invalid
 * arguments.  In mode 1 the symmetric kernel is chosen when its waves (one per block pair or
 * surface chunk) at least cover every SIMD of the device. */
int hsma_group_eval_kernel(hsma_group_t group, int nsys, int64_t total_n, int64_t max_n);

/* Order of the symmetric kernel's work items (one wave each: a block pair of one system, or
 * half of one ion block against one chunk of surface nodes).  mode 1: each system's surface
 * items right after its own block pairs, so its ion blocks are read again while still in L2;
 * 2: every system's block pairs first, then every surface item, so that the shorter surface
 * items fill the end of the launch; 0 (default): 2 when the launch's block pairs number at
 * most four waves per resident-wave slot of the device (compute units x resident waves of the
 * kernel), else 1.  Every item computes the same sums in either order: results are
 * bit-identical.  Errors: HSMA_EINVAL. */
hsma_status hsma_group_set_sym_order(hsma_group_t group, int mode);

/* Fit apply (Algorithm 1, steps 3-4: alpha' = Y^+ u, beta' = Y^+ v, then the surface
 * strengths Q', D' through the fixed operator of eq. "GreenSecond") in the FP32 pair modes.
 * mode 0 (default): FP32 GEMVs below 192 systems per call, FP32 MFMA GEMMs from 192 systems
 * (the GEMMs have few row tiles, K / 64, and stay near 0.25-0.4 ms at any smaller batch);
 * 1: always the GEMVs; 2: always the FP32 MFMA GEMMs; 3: always BF16 MFMA GEMMs with
 * split-BF16x3 products (each factor split into two BF16 terms, three term products: about
 * 2^-16 relative per product); 4: the same with split-BF16x6 products (three BF16 terms, six
 * term products: about 2^-24, as FP32).  The fit amplifies the rounding of the check fields
 * and of the operators strongly (balanced charges cancel in u, v), so mode 3 can miss the 1e-6
 * potential target where the surface term is a large share of the potential; modes 1, 2 and
 * 4 hold it.  In FP64 pairs (the FP64 mode and every energy launch) the fit is applied with
 * FP64 GEMVs below 192 systems and FP64 MFMA GEMMs (v_mfma_f64_16x16x4f64) from 192 on; mode 1
 * forces the GEMVs there, modes 2-4 the FP64 GEMMs.
 * Errors: HSMA_EINVAL (mode outside 0..4). */
hsma_status hsma_group_set_fit(hsma_group_t group, int mode);

/* Which fit route hsma_energy_batched would take for nsys systems in the group's pair precision:
 * 1 GEMV, 2 MFMA GEMMs (FP32, or FP64 in the FP64 mode), 3 split-BF16x3 MFMA, 4 split-BF16x6
 * MFMA; -1 for invalid arguments. */
int hsma_group_fit_route(hsma_group_t group, int nsys);

/* Energy launch shape (the FP64 energy-only launch of hsma_energy / hsma_energy_batched):
 * block = 128, 256 or 512 ions per block of the symmetric pair kernel; 0 (default): 512 when
 * hsma_group_set_symmetric chose mode 3, else 128 for launches whose block pairs of 256 would
 * fill fewer than four rounds of the device's wave slots, else 256; workgroups = 0 (default): one item per
 * wave over the whole device; > 0: a persistent grid of that many workgroups (rounded up to a
 * multiple of the die count) taking items from per-die counters, the check sums persistent on
 * the same grid.  Energies depend on block only through the summation order (rounding) and
 * not at all on workgroups.  Errors: HSMA_EINVAL. */
hsma_status hsma_group_set_energy_launch(hsma_group_t group, int block, int workgroups);

/* The group's launch settings, as set by hsma_group_tune, hsma_group_set_symmetric,
 * hsma_group_set_sym_order, hsma_group_set_fit and hsma_group_set_energy_launch. */
typedef struct {
  int persistent, target_items, symmetric, sym_order, fit; /* check and potential launches */
  int energy_block, energy_workgroups;                      /* energy launches */
} hsma_launch_settings;
hsma_status hsma_group_get_settings(hsma_group_t group, hsma_launch_settings *out /* [host] */);
/* Sets all of them at once, each validated as by its own setter.  Errors: HSMA_EINVAL. */
hsma_status hsma_group_apply_settings(hsma_group_t group, const hsma_launch_settings *s /* [host] */);

/* Timing-based choice of the group's launch settings for one call shape: the call
 * hsma_energy_batched(group, nsys, offsets, plan_of, total_n, max_n, x, y, z, q, phi, E, ws,
 * ws_bytes, stream) is run with candidate settings and timed with HIP events on the stream, one
 * setting at a time from the group's current ones (coordinate descent over: for potentials the
 * Kelvin kernel (symmetric mode), its item order and the fit route of the FP32 modes (never
 * split-BF16x3, which can miss the potential target); for energies the energy block and grid;
 * for both the persistent form and the chunk length (target_items)), a change kept when it
 * is at least 2% faster.  Candidates whose workspace exceeds ws_bytes are skipped.  The best
 * settings are left on the group and kept in a process-wide cache under (device architecture,
 * compute units, pair precision, surface form, M, P, K, which outputs, and the bit lengths of
 * nsys, total_n and max_n); a later call with the same key applies the cached settings without
 * running anything, unless flags has HSMA_TUNE_FORCE.  Tuned settings change results only in
 * rounding (summation order), as each setter states.  The call overwrites phi, E and ws,
 * synchronises the stream, creates HIP events and must not be captured into a graph.
 * Errors: those of hsma_energy_batched for the group's current settings; HSMA_EDEVICE. */
#define HSMA_TUNE_FORCE 1
#define HSMA_TUNE_MAX_TRIALS 32
typedef struct {
  hsma_launch_settings s;
  double ms; /* mean time of one call; < 0: refused (its workspace exceeds ws_bytes) */
} hsma_tune_trial;
typedef struct {
  hsma_launch_settings chosen;
  double ms_start, ms_tuned; /* the call with the settings found on entry, and with the chosen
                                ones (0 when taken from the cache) */
  int timed;                 /* settings timed, the entry settings included (0 from the cache) */
  int cached;                /* 1: applied from the cache without timing */
  hsma_tune_trial trials[HSMA_TUNE_MAX_TRIALS]; /* the first min(timed, 32) trials, in order */
} hsma_tune_result;
hsma_status hsma_group_autotune(hsma_group_t group, int nsys, const int64_t *offsets, const int32_t *plan_of,
                                int64_t total_n, int64_t max_n, const double *x, const double *y, const double *z,
                                const double *q, double *phi, double *E, void *ws, size_t ws_bytes,
                                hipStream_t stream, int flags, hsma_tune_result *out /* [host] */);
/* A workspace size that admits every candidate setting of hsma_group_autotune for these sizes
 * (the largest over all combinations, 256-byte multiple); 0 for invalid arguments. */
size_t hsma_group_autotune_workspace_bytes(hsma_group_t group, int nsys, int64_t total_n, int64_t max_n);

/* Stage timing: when enabled, every compute call on the group records HIP events on its
 * stream around its kernel groups (0 schedule/Kelvin images/packing, 1 check sums, 2 fit
 * apply, 3 evaluation pair sums, 4 final reductions).  hsma_profile_read waits for the
 * recorded events, returns the summed milliseconds and event-pair counts per stage
 * (arrays of 5, [host]) and clears the records.  For measurement only: while enabled the
 * compute calls create events and must not be captured into a graph. */
hsma_status hsma_profile_enable(hsma_group_t group, int on);
hsma_status hsma_profile_read(hsma_group_t group, double *ms /* [host] 5 */, int64_t *count /* [host] 5 */);

/* Treecode far field for the Kelvin-image and surface sums of one system (the role of the FMM
 * the paper uses for N up to 10^6, Sec. 3 and Sec. 4.2), as a Barnes-Hut treecode in the FP32
 * pair modes.  The check sums and the fit are those of hsma_energy; the sums over the other
 * ions' Kelvin images and over the surface nodes are approximated.  The images are sorted into
 * an octree over the cube of half-width 8a (depth levels below the root; images farther out, of
 * ions within a/8 of the centre, are summed directly at theta = 0 and as one local expansion about
 * the centre otherwise), the surface nodes into patches of up to 64.  The targets are grouped
 * by their own positions, in groups of up to 64.  A cell or patch of radius r_c at distance d
 * from a group of radius r_g is evaluated from its Cartesian multipole moments of the given
 * order when r_c + r_g < theta d, else opened; leaves and patches that are not accepted are
 * summed directly.
 *   theta: in [0, 1); 0 accepts no cell (every image and node is then summed directly, the
 *          check of the traversal); order: 2, 4, 6, 8 or 10; depth: 2..9, or 0 for a depth
 *          from N (7 at N = 10^6).
 * The error is the treecode's. On 10^6 ions uniform in a cavity with balanced charges, the
 * relative L2 errors of 2048 sampled potentials against an FP64 evaluation are 9.1e-4 (order 4,
 * theta 0.5), 1.2e-6 (order 8, theta 0.4), 6.3e-7 (order 8, theta 0.35) and 7.5e-7 (order 10,
 * theta 0.45); the direct sum in compensated FP32 pairs is at 3.0e-7.  Against that direct sum
 * these run 14, 4.5, 3.4 and 3.8 times faster; at 2 10^5 ions 2.1 times at order 4, theta 0.5;
 * below about 10^5 ions the direct path is faster at any setting.
 *   phi: [device] N doubles (required); E: [device] one double or NULL (1/2 sum q_i phi_i of the
 *   treecode's potentials, so of the treecode's accuracy);
 *   ws: [device] ws_bytes >= hsma_tree_workspace_bytes(plan, N, opts) (0 for invalid arguments).
 * Like the other compute calls it allocates nothing and does not synchronise; unlike them it
 * is not meant for graph capture, since its radix sorts and scans (rocPRIM, with their
 * temporary storage in ws) may enqueue memory fills.
 * Errors: HSMA_EINVAL (also for the FP64 pair mode), HSMA_ESTATE, HSMA_EDEVICE. */
typedef struct {
  double theta;
  int order;
  int depth;
} hsma_tree_opts;
size_t hsma_tree_workspace_bytes(hsma_plan_t plan, int64_t N, const hsma_tree_opts *opts);
hsma_status hsma_energy_tree(hsma_plan_t plan, int64_t N, const double *x, const double *y, const double *z,
                             const double *q, double *phi, double *E, const hsma_tree_opts *opts, void *ws,
                             size_t ws_bytes, hipStream_t stream);

/* Resident system (a Monte Carlo state): copies x, y, z, q ([device], N >= 1 ions) and keeps
 * on the device what a single-ion move needs: the positions, the surface strengths s and
 * surface rows w = sum_i q_i S(x_i) of the HSMA energy, and the energy itself, all from a
 * full evaluation in FP64 pairs.  Synchronises; the plan must outlive the system.
 *
 * hsma_delta_energy: the change of the energy E = (1/2) sum_i q_i Phi_RF(x_i) when ion k
 * moves to (xk, yk, zk) ([host] scalars, |x| < a), written to dE ([device] one double),
 * without changing the state.  The energy is a bilinear form in the charges (the Kelvin
 * images of Sec. 2.4 and the fitted surface images of eq. "phicorrfinall"), so the change
 * is evaluated exactly from the row and column of ion k: O(N) image pairs, O(M + P)
 * check/surface pairs and two GEMVs of the fixed fit operator, in FP64, in four launches.
 * hsma_system_commit: apply that move (positions, s, w and the stored energy).
 * hsma_system_energy: the stored energy (initial value plus committed changes) to E
 * ([device]).  hsma_system_positions: copy the current positions ([device] N each).
 * Errors: HSMA_EINVAL (k out of range, non-finite or |x| >= a), HSMA_EDOMAIN (an initial
 * ion outside the cavity), HSMA_ESTATE (wrong device), HSMA_ENOMEM, HSMA_EDEVICE.
 * A system is not thread safe: its calls must be ordered (one stream). */
hsma_status hsma_system_create(hsma_plan_t plan, int64_t N, const double *x, const double *y, const double *z,
                               const double *q, hipStream_t stream, hsma_system_t *out);
/* As hsma_system_create, with flags: HSMA_SYSTEM_COULOMB makes the system's energy the total
 * E_RF + E_C, where E_C = (1/2) sum_{i != j} q_i q_j / (4 pi eps1 |x_i - x_j|) is the direct
 * Coulomb energy of the ions in the cavity (eq. "phicoul"); hsma_delta_energy, commits,
 * hsma_system_energy and hsma_system_full_energy then all refer to the total.  E_C is summed
 * directly in FP64 (O(N^2) at creation and in full evaluations, O(N) per move).  Other flag
 * bits: HSMA_EINVAL. */
#define HSMA_SYSTEM_COULOMB 1
hsma_status hsma_system_create_ex(hsma_plan_t plan, int64_t N, const double *x, const double *y, const double *z,
                                  const double *q, int flags, hipStream_t stream, hsma_system_t *out);
hsma_status hsma_delta_energy(hsma_system_t sys, int64_t k, double xk, double yk, double zk, double *dE,
                              hipStream_t stream);
hsma_status hsma_system_commit(hsma_system_t sys, int64_t k, double xk, double yk, double zk, hipStream_t stream);
hsma_status hsma_system_energy(hsma_system_t sys, double *E, hipStream_t stream);
hsma_status hsma_system_positions(hsma_system_t sys, double *x, double *y, double *z, hipStream_t stream);
hsma_status hsma_system_destroy(hsma_system_t sys);
/* A fresh FP64 full evaluation of the system's current energy (E [device]), with a
 * caller workspace of ws_bytes >= hsma_system_workspace_bytes(sys); the state is unchanged. */
size_t hsma_system_workspace_bytes(hsma_system_t sys);
hsma_status hsma_system_full_energy(hsma_system_t sys, double *E, void *ws, size_t ws_bytes, hipStream_t stream);

/* Request server over resident systems.
 *
 * Systems are admitted against a device-memory budget (hsma_server_add_system returns
 * HSMA_EBUSY when the system's resident bytes, plus any growth of the shared full-energy
 * workspaces to its size, would exceed it; 0 = half the free memory at creation).  Requests
 * -- a single-ion move (energy change, optionally committed) or a fresh FP64 full energy --
 * are queued by hsma_server_submit (thread safe) and served by a scheduler thread with
 * continuous batching: whenever one of delta_slots batch slots is free, it launches every
 * waiting move whose system is idle, in arrival order, up to max_batch; full energies use
 * energy_slots streams of their own (defaults: 1 and 2).  Every slot's stream is created with
 * a hardware queue of its own (a CU mask enabling every CU), so that a move batch never waits
 * in a queue behind a full energy or behind other work of the process; such streams
 * synchronise with the legacy default stream (stream 0): device work enqueued there while the
 * server runs waits for the server's work in flight, and the reverse, so the caller's own
 * device work belongs on other streams.  Each system sees its requests in arrival order:
 * a full energy first copies the system's positions and charges, and the system takes its
 * next requests as soon as that copy is done, so a full energy can complete after later
 * requests of its system while its value is still that of the state at its place in the
 * order.  New batches start while earlier ones run, and a request's result does not depend on
 * the batch it lands in.  The scheduler sleeps while idle and is woken by submits.  Results,
 * with submit/start/done times in seconds since the server's creation, are collected with
 * hsma_server_poll.  Requests that name an unknown system, an ion out of range or a position
 * outside the cavity complete at once with status HSMA_EINVAL.  hsma_server_run_load submits
 * reqs[i] at arrival[i] seconds (open-loop load) and returns when all are done, with times
 * relative to its start.  hsma_server_remove_system waits until no request of the system is
 * queued or running. */
typedef struct hsma_server_s *hsma_server_t;
enum { HSMA_REQ_DELTA = 0, HSMA_REQ_ENERGY = 1 };
typedef struct {
  int type;      /* HSMA_REQ_DELTA or HSMA_REQ_ENERGY */
  int sys;       /* system id from hsma_server_add_system */
  int commit;    /* HSMA_REQ_DELTA: apply the move after evaluating it */
  int64_t k;     /* HSMA_REQ_DELTA: ion index */
  double x, y, z;/* HSMA_REQ_DELTA: new position */
  uint64_t tag;  /* caller's identifier, returned with the result */
} hsma_request;
typedef struct {
  uint64_t tag;
  int type, sys;
  int status;    /* hsma_status */
  double value;  /* energy change or energy */
  double t_submit, t_start, t_done;
} hsma_result;
typedef struct {
  size_t memory_budget; /* bytes; 0 = half of the free device memory */
  int max_systems, max_batch, delta_slots, energy_slots;
  int energy_workgroups; /* full energies run their pair kernels persistent on this many workgroups,
                            leaving the rest of the device's wave slots to the move batches, so that a
                            move does not wait for a long energy to drain; 0 (default): the compute
                            units' count (one workgroup per compute unit and energy slot); < 0: no
                            limit (one item per wave on the whole device: more full energies per
                            second, longer move tails).  Results do not depend on it. */
  int move_priority;     /* 1 (default): the move kernels raise their waves' issue priority
                            (s_setprio) above the full energies' on a shared SIMD; 0: equal.
                            Results do not depend on it. */
} hsma_server_opts;
typedef struct {
  size_t memory_used, memory_budget;
  int64_t pending;
  uint64_t completed, batches, batched_requests;
  int systems;
  double now;
} hsma_server_info;
hsma_server_opts hsma_server_opts_default(void);
hsma_status hsma_server_create(const hsma_server_opts *opts /* [host], NULL = defaults */, hsma_server_t *out);
hsma_status hsma_server_destroy(hsma_server_t server);
hsma_status hsma_server_add_system(hsma_server_t server, hsma_plan_t plan, int64_t N, const double *x,
                                   const double *y, const double *z, const double *q /* [device] */, int *id);
hsma_status hsma_server_remove_system(hsma_server_t server, int id);
hsma_status hsma_server_submit(hsma_server_t server, const hsma_request *reqs /* [host] */, int n);
int hsma_server_poll(hsma_server_t server, hsma_result *out /* [host] */, int max);
hsma_status hsma_server_stats(hsma_server_t server, hsma_server_info *info /* [host] */);
hsma_status hsma_server_run_load(hsma_server_t server, const hsma_request *reqs, const double *arrival, int n,
                                 hsma_result *out /* all [host] */);

/* Synchronise the stream and report a device-side error raised since the last check
 * (then clear it): HSMA_EDOMAIN for an ion outside the cavity or a non-finite input,
 * HSMA_EINVAL for device offsets or plan indices inconsistent with the host sizes; for the
 * plan's single-system calls, or for a group's batched calls. */
hsma_status hsma_stream_check(hsma_plan_t plan, hipStream_t stream);
hsma_status hsma_group_stream_check(hsma_group_t group, hipStream_t stream);

const char *hsma_status_string(hsma_status s);
int hsma_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HSMA_H */
