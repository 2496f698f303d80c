/*
 * qmc.h -- randomly shifted rank-1 lattice quasi-Monte Carlo estimator on
 * AMD Instinct MI355X (gfx950), FP64 throughout.
 *
 * The method (arXiv:1811.11722, Sec. 2):
 *   I_d[f] = integral of f over [0,1]^d, f real or complex            eq. (1)
 *   Q_k    = (1/n) sum_{j=1..n} fhat({(j-1) g / n + Delta_k}),
 *   Qbar   = (1/m) sum_{k=1..m} Q_k                                   eq. (2)
 *   sigma^2 = sum_k (Q_k - Qbar)^2 / (m (m - 1))                       eq. (3)
 *   fhat(x) = f(z(x)) prod_i z_i'(x_i) with the Korobov transform      eq. (4)
 *             or the baker's transform                                eq. (5)
 * The sector integrand family follows eq. (6) with two polynomials
 * (U and F of Sec. 3) and an optional -i*delta prescription as in eq. (7).
 *
 * Conventions for every entry point:
 *   - Every function returns a qmc_status; nothing throws across the ABI.
 *   - Arguments are validated on the host before any device call; on an
 *     argument error nothing is launched and the outputs are untouched.
 *   - Input pointers are host pointers, borrowed for the duration of the
 *     call only (the library copies what it keeps).  Output pointers are
 *     caller-owned host memory.
 *   - A plan owns its device memory (allocated at create, freed at destroy).
 *     A plan must not be used from two host threads at once; separate plans
 *     may run concurrently on separate streams.
 *   - qmc_last_error() returns a thread-local message for the last failure.
 */
#ifndef QMC_H
#define QMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qmc_plan_s *qmc_plan_t;

typedef enum {
    QMC_OK = 0,
    QMC_EINVAL = 1,        /* invalid argument */
    QMC_EUNSUPPORTED = 2,  /* valid but outside what this build supports */
    QMC_ENOMEM = 3,        /* device or host allocation failed */
    QMC_EDEVICE = 4,       /* HIP runtime error; detail in qmc_last_error() */
    QMC_ENONFINITE = 5,    /* a per-shift sum is not finite; means/errors set to NaN */
    QMC_ECONTOUR = 6       /* a deformed contour reaches Im(F - i delta) > 0 at some points
                              (Sec. 3); the result is filled in, contour_crossed > 0 */
} qmc_status;

/* Periodising transforms, eqs. (4) and (5).  QMC_T_TENT is the same map as
   the baker's transform, read as a modification of the lattice (Sec. 2). */
typedef enum {
    QMC_T_NONE = 0,
    QMC_T_KOROBOV = 1,  /* weight alpha in 1..6 */
    QMC_T_BAKER = 2,
    QMC_T_TENT = 2,
    /* Sidi's sin^m transform, m = alpha in 1..6: w(x) = sin^m(pi x) / T_m,
       T_m the integral of sin^m over [0, 1]; one of the other periodising
       substitutions Sec. 2 refers to.  Compiled for QMC_F_CONST,
       QMC_F_GENZ_PRODUCT_PEAK and the specialised sector kernels. */
    QMC_T_SIDI = 3
} qmc_transform_kind;

typedef struct {
    int32_t kind;   /* qmc_transform_kind */
    int32_t alpha;  /* Korobov weight or Sidi order; ignored otherwise */
} qmc_transform;

/* Integrand families f(z), z in [0,1]^d. */
typedef enum {
    QMC_F_CONST = 0,              /* qmc_const_params */
    QMC_F_TRIG = 1,               /* qmc_trig_params */
    QMC_F_P2KERNEL = 2,           /* prod_i (1 + 2 pi^2 B2(z_i)); params NULL */
    QMC_F_GENZ_PRODUCT_PEAK = 3,  /* prod_i 1/(a_i^-2 + (z_i - u_i)^2) */
    QMC_F_GENZ_OSCILLATORY = 4,   /* cos(2 pi u_1 + sum_i a_i z_i) */
    QMC_F_GENZ_GAUSSIAN = 5,      /* exp(-sum_i a_i^2 (z_i - u_i)^2) */
    QMC_F_GENZ_CONTINUOUS = 6,    /* exp(-sum_i a_i |z_i - u_i|) */
    QMC_F_GENZ_CORNER_PEAK = 7,   /* (1 + sum_i a_i z_i)^-(d+1) */
    QMC_F_SECTOR = 8              /* qmc_sector_params */
} qmc_family;

typedef struct {
    double c;
} qmc_const_params;

/* f = c0 + sum_t c[t] cos(2 pi h_t . z + phi[t]); h row-major (n_terms, d). */
typedef struct {
    uint32_t n_terms;
    double c0;
    const int64_t *h;
    const double *c;
    const double *phi;
} qmc_trig_params;

/* Genz parameters, length d each. */
typedef struct {
    const double *a;
    const double *u;
} qmc_genz_params;

/* Sector integrand  prod_i z_i^nu_i * U(z)^pow_u * (F(z) - i delta_im)^pow_f,
   U(z) = sum_t coef_u[t] prod_i z_i^exp_u[t*d+i]  (row-major (n_u, d)), F alike.
   Exponents and nu are 0..2; a monomial may have total degree <= 12.
   Real form (is_complex = 0) needs U > 0 and F > 0 on the domain; complex form
   uses the principal branch.  pow_u, pow_f, delta_im are plain doubles;
   EUNSUPPORTED for a complex sector with |pow_f| > 1e5. */
typedef struct {
    uint32_t n_u, n_f;
    const double *coef_u;
    const uint8_t *exp_u;
    const double *coef_f;
    const uint8_t *exp_f;
    const uint8_t *nu;
    double pow_u, pow_f;
    double delta_im;
    int32_t is_complex;
    /* Expansion in a regulator e (qmc_integrate_orders): with n_orders >= 2
       the exponents become pow_u + eps_u e and pow_f + eps_f e and the
       integrand's coefficients of e^0 .. e^(n_orders-1) are integrated in one
       pass; order k is f L^k / k!, L = eps_u ln U + eps_f ln(F - i delta).
       n_orders <= 4; 0 or 1 is the plain integrand. */
    uint32_t n_orders;
    double eps_u, eps_f;
    /* Contour deformation (Sec. 3), deform_lambda != 0: the integrand is
       evaluated at z_k = x_k - i lambda x_k (1 - x_k) dF/dx_k (x) (x the
       transformed point) and multiplied by det(dz/dx); the faces of the cube
       stay fixed, and F(z) gains a negative imaginary part to first order, so
       a sector whose F changes sign inside the cube is integrated with the
       -i0 prescription (delta_im may be 0).  The result is complex whatever
       is_complex says; delta_im applies when is_complex != 0.  Needs the
       specialised kernel (jit mode 1 or 2); EUNSUPPORTED in control
       variates, in batches other than QMC_BATCH_SPECIALISED, and for
       |pow_u| or |pow_f| > 1e5.  0 = none. */
    double deform_lambda;
} qmc_sector_params;

/* Result of eqs. (2)-(3).  err = sqrt(sigma^2); complex integrands carry
   separate errors for the real and imaginary parts. */
typedef struct {
    double mean_re, mean_im;
    double err_re, err_im;
    int32_t is_complex;
    int32_t used_cv;  /* 1 when a control-variate estimate was returned */
    /* Contour-deformed sectors: the fraction of the points (over all
       shifts) at which the deformed F(z) - i delta has a positive imaginary
       part, counted in the same pass as the estimate; 0 otherwise. */
    double contour_crossed;
} qmc_result;

/* Launch shape of the lattice kernel.  shift_tile is the number of shifts
   each thread evaluates per lattice point (1, 2, 4 or 8); blocks_per_cu sets
   the grid size (workgroups of 256 threads per compute unit and per shift
   tile).  Zero fields mean "use the tuned or default choice". */
typedef struct {
    uint32_t shift_tile;
    uint32_t blocks_per_cu;
} qmc_launch;

/* Create a plan for the rule of eq. (2).
   d       dimension, 1..16
   n       number of lattice points, 2..2^31
   g       generating vector, length d; every g_i mod n must be nonzero
   m       number of shifts, >= 2 (eq. (3) divides by m - 1)
   shifts  m*d doubles, row-major (shift k is shifts[k*d .. k*d+d-1]), each in [0,1)
   t       periodising transform
   Errors: EINVAL on a bad argument, EUNSUPPORTED for d > 16, n > 2^31 or a
   Korobov weight above 6, ENOMEM / EDEVICE from the device. */
qmc_status qmc_plan_create(uint32_t d, uint64_t n, const uint64_t *g, uint32_t m,
                           const double *shifts, qmc_transform t, qmc_plan_t *out);

/* Run the plan's kernels on this HIP stream (a hipStream_t; NULL = default). */
qmc_status qmc_plan_set_stream(qmc_plan_t plan, void *hip_stream);

/* Fix the launch shape for later calls (zero fields restore the default). */
qmc_status qmc_plan_set_launch(qmc_plan_t plan, const qmc_launch *cfg);

/* How sector integrands are evaluated: 0 = interpret the sparse polynomial
   tables in the kernel; 1 (default) = compile a kernel specialised to the
   exponent structure on first use (hipRTC; 0.1-1 s, cached per structure
   for the process) and fall back to the tables if compilation fails; 2 =
   always specialise and return EUNSUPPORTED if that fails.  Results agree
   to rounding either way.  With the environment variable QMC_JIT_CACHE
   naming a directory, compiled kernels are also stored there (one file per
   library build, architecture and source) and loaded by later processes
   instead of being compiled again.  With QMC_JIT_DUMP naming a directory,
   the source of every kernel compiled is written there for inspection. */
qmc_status qmc_plan_set_jit(qmc_plan_t plan, int32_t mode);

/* Launch shape of the plan's last estimate: shift_tile = tile used,
   blocks_per_cu = workgroups per shift tile along the lattice points;
   used_jit (nullable) = 1 if it ran a specialised sector kernel. */
qmc_status qmc_plan_get_launch(qmc_plan_t plan, qmc_launch *cfg, int32_t *used_jit);

/* Evaluate eqs. (2)-(3) for the integrand (family, params).
   params     the family's parameter struct (NULL for QMC_F_P2KERNEL)
   out        mean and error
   per_shift  nullable; receives Q_k for k = 0..m-1 (real) or 2m doubles
              (re, im interleaved) for a complex sector integrand.
   Errors: EINVAL for a bad family/params, ENONFINITE if any Q_k is not
   finite (then means and errors are NaN), EDEVICE on a HIP error.  A sector
   with deform_lambda != 0 returns ECONTOUR when the deformed contour is on
   the wrong side of the cut (Im(F(z) - i delta) > 0) at any lattice point:
   out and per_shift are still filled, out->contour_crossed gives the
   fraction, and the value is not the -i0 integral (Sec. 3). */
qmc_status qmc_integrate(qmc_plan_t plan, qmc_family family, const void *params, qmc_result *out,
                         double *per_shift);

/* Device time of the lattice kernels launched through this plan since the
   last reset, measured with HIP events on the plan's stream.  Timing is off
   until qmc_plan_set_timing(plan, 1).  A batch (qmc_integrate_batch) whose
   first plan has timing on adds its device time (its kernels on the batch
   stream, from the launch to the end of the last one) to that plan. */
qmc_status qmc_plan_set_timing(qmc_plan_t plan, int32_t enable);
qmc_status qmc_plan_kernel_time(qmc_plan_t plan, double *total_ms, uint64_t *launches, int32_t reset);

/* Exact lattice indices idx_{j,i} = (j g_i) mod n for j = j_lo .. j_lo+count-1
   (j counts from 0, i.e. j = (paper's j) - 1), written row-major into idx_out
   (count*d uint32), produced by the same index walk the lattice kernel runs.
   sums_out (nullable, 2*d uint64) receives, over all n points, sum_j idx and
   sum_j idx^2 (mod 2^64) per dimension.  count <= 2^24. */
qmc_status qmc_lattice_dump(qmc_plan_t plan, uint64_t j_lo, uint64_t count, uint32_t *idx_out,
                            uint64_t *sums_out);

/* Korobov generating vector g_i = a^i mod n, i = 0..d-1. */
qmc_status qmc_korobov_vector(uint64_t n, uint32_t d, uint64_t a, uint64_t *g);

/* P_2 criterion P2(g) = -1 + (1/n) sum_j prod_i (1 + 2 pi^2 B2({j g_i / n}))
   for the Korobov vector of every candidate multiplier, evaluated on the GPU
   as an unshifted lattice rule; returns the minimiser (ties: smaller P2, then
   smaller a).  p2_all (nullable) receives all ncand values.  The generating
   vector itself is not fixed by the paper (Sec. 2 only names it); this is
   the standard worst-case-error choice.  For odd n, and for even n when
   every candidate is odd, the sum runs over j <= n/2 and is doubled less the
   self-mirrored terms j = 0 and (even n) j = n/2: the point n - j mirrors
   the point j, and B2(1 - x) = B2(x).  n <= 2^31, d <= 16, ncand <= 4096. */
qmc_status qmc_korobov_search(uint64_t n, uint32_t d, const uint64_t *cand, uint32_t ncand,
                              uint64_t *a_best, double *p2_best, double *p2_all);

/* Many independent estimates in one launch: plan p of `count` plans is
   evaluated with family and params[p].  All plans must share the transform;
   each plan keeps its own d, n, g, m and shifts.  The work is cut into tiles
   (tile_points lattice points times one shift tile) ordered longest first,
   one work list per dimension, and run by one kernel launch per dimension:
   persistent workgroups that loop over the list, or one workgroup per tile
   taking tiles in list order (schedule).  When every plan has the same d, n
   and m and tile_points is 0, the plans instead run as instances of one
   lattice-kernel launch (with the first plan's qmc_plan_set_launch
   configuration, if any).  When use_graph is set, the launch sequence is
   captured once into a HIP graph and replayed on later calls with the same
   plans.  out receives count results.  Supported families: QMC_F_SECTOR
   (real) and the Genz families. */
typedef enum {
    QMC_BATCH_DEFAULT = 0,    /* one workgroup per tile */
    QMC_BATCH_PERSISTENT = 1, /* CUs x 8 workgroups loop over the work list */
    QMC_BATCH_PER_TILE = 2,   /* one workgroup per tile */
    /* sectors only: one launch per plan of the run-time specialised sector
       kernel (with use_graph: every plan's kernel, finalize and result copy
       captured into one HIP graph on four parallel chains and replayed by
       later calls with the same plans, exponent structures and buffers; the
       coefficients are uploaded before each replay).  Each distinct exponent
       structure is compiled once per process (hipRTC, about 0.1-0.2 s) and
       reused for every later call and coefficient set with that structure, so
       this pays when the same sectors are integrated repeatedly (new
       kinematics, new shifts); EUNSUPPORTED when a specialised kernel cannot
       be built.  The only schedule that takes contour-deformed sectors;
       ECONTOUR as in qmc_integrate when any of them crosses the cut. */
    QMC_BATCH_SPECIALISED = 3
} qmc_batch_schedule;

typedef struct {
    int32_t use_graph;         /* capture/replay through a HIP graph */
    int32_t per_plan_launches; /* 1 = one launch per plan instead (for comparison) */
    uint32_t tile_points;      /* lattice points per tile (0 = default 8192, or the
                                  instance launch for uniform batches) */
    int32_t schedule;          /* qmc_batch_schedule */
} qmc_batch_opts;

qmc_status qmc_integrate_batch(uint32_t count, const qmc_plan_t *plans, qmc_family family,
                               const void *const *params, const qmc_batch_opts *opts,
                               qmc_result *out);

/* Per-shift values Q_k of the last qmc_integrate_batch call with exactly these
   plans: per_shift[i] (nullable entries) receives m_i doubles, or 2 m_i
   interleaved (re, im) for complex sectors.  Not filled by the per-plan
   comparison mode. */
qmc_status qmc_batch_per_shift(uint32_t count, const qmc_plan_t *plans, double *const *per_shift);

/* Counters of the batch machinery since the library was loaded (all
   devices): out[0] batch contexts built (buffers, uploads and, with
   use_graph, a graph captured) for the table-driven schedules, out[1] their
   graph launches, out[2] specialised-schedule graphs captured, out[3] their
   graph launches.  A repeated qmc_integrate_batch with the same plans,
   parameters and options reuses its context and graph (until eight newer
   contexts displace it), so only the launch counts grow.  out: 4 uint64
   values, caller-owned.  Errors: EINVAL for a null out. */
qmc_status qmc_batch_stats(uint64_t *out);

/* Autotuner of the batched launch (the table-driven schedules of
   qmc_integrate_batch): times tile_points in {4096, 8192, 16384, 32768} with
   the one-workgroup-per-tile and the persistent schedule, each captured into
   a HIP graph and launched once (device time of the graph, events on the
   batch stream), and returns the fastest options in best
   (use_graph = 1) and their time in best_ms (nullable, milliseconds).  The
   arguments are those of qmc_integrate_batch; the estimates it computes are
   discarded. */
qmc_status qmc_batch_autotune(uint32_t count, const qmc_plan_t *plans, qmc_family family,
                              const void *const *params, qmc_batch_opts *best, double *best_ms);

/* Pick a launch shape for (plan, family, params) by timing candidate shapes
   on the device; the choice is stored in the plan and in the tuning cache
   file named by the QMC_TUNE_CACHE environment variable (if set).  best
   (nullable) receives the choice. */
qmc_status qmc_autotune(qmc_plan_t plan, qmc_family family, const void *params, qmc_launch *best);

/* ---------------------------------------------------------------- control
   variate.  A separable rank-R model on orthonormal shifted Legendre
   polynomials P~_k(z) = sqrt(2k+1) P_k(2z - 1), k < K:
     g(z) = sum_r c_r prod_i sum_k W[r,i,k] P~_k(z_i),   int g = sum_r c_r prod_i W[r,i,0],
   W row-major (R, d, K).  The estimate int g + Qbar[f - g] keeps eqs. (2)-(3)
   unbiased (g is fitted on an independent training lattice) and the m
   shifts judge its error.  Built for real QMC_F_SECTOR integrands with
   (R, K) in {(8,4), (8,8), (16,8), (16,12), (32,8), (32,12), (32,16), (64,12)}
   and d <= 12. */
typedef struct {
    uint32_t max_sweeps;  /* alternating least-squares sweeps (0 = 12) */
    double ridge;         /* ridge relative to the mean diagonal (0 = 1e-5) */
    double tol;           /* stop when the relative loss improves less than this */
    uint64_t seed;        /* initial-factor seed */
    uint32_t refine;      /* refinements per step against the FP64 residual (0 = 4, at most 8) */
} qmc_cv_train_opts;

typedef struct {
    uint32_t sweeps;      /* sweeps run */
    double rel_loss;      /* sum (fhat - J g)^2 / sum fhat^2 on the training set */
    double scale;         /* target scale (mean |fhat|), folded into c */
    double seconds;       /* device time of the training */
} qmc_cv_train_report;

/* Fit W and c to the integrand sampled at the n points of train_plan's
   lattice with its first shift (z, J and fhat are sampled by the GPU), by
   minimising sum_j (fhat_j - J_j g(z_j))^2 + lam |W[., i, .]|^2 with
   alternating least squares over the dimensions i.  Each step assembles its
   normal equations with BF16 MFMA (each feature rounded once, FP32
   accumulation), factorises them in FP64 and refines the solution (4 times
   by default) against the FP64 residual, whose right-hand side comes from
   the FP64 design matrix; a sweep ends by balancing each rank's factor
   norms.  lam = ridge times the mean diagonal; it must stay above the
   rounding of the assembled normal matrix for the refinement to converge.
   Training stops when a sweep improves the loss by less than tol (relative)
   and returns the factors of the lowest loss seen.

   The control variate is an addition to the paper's estimator (it does not
   appear in the paper); the estimate it feeds stays unbiased because the
   training lattice is independent of the estimation shifts.  A complex
   integrand gets one model for its real part and one for its imaginary
   part, trained in turn.  QMC_F_SECTOR only, d <= 12, (R, K) in {(8,4),
   (8,8), (16,8), (16,12), (32,8), (32,12), (32,16), (64,12)} (EUNSUPPORTED
   otherwise); ENONFINITE when the loss is not finite.  w_out: nm*R*d*K
   doubles (model-major, each (R, d, K) row-major, orthonormal-basis
   coefficients), c_out: nm*R doubles, nm = 1 (real) or 2 (complex);
   caller-owned.  rep (nullable): total sweeps, the larger relative loss,
   the real part's target scale, total device time. */
qmc_status qmc_cv_train(qmc_plan_t train_plan, qmc_family family, const void *params, uint32_t R, uint32_t K,
                        const qmc_cv_train_opts *opts, double *w_out, double *c_out, qmc_cv_train_report *rep);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): one
   estimate of eqs. (2)-(3), as qmc_plan_create + qmc_integrate +
   qmc_plan_destroy would give it, that allocates nothing on the device.
   The rule's device copies, the parameter blob, the block partial sums and
   the results live in a fixed 1 MiB device array inside the library (one
   per device, held until the process ends); its address is looked up once
   per device on the first call.  Limits of that array: m <= 64 shifts and a
   parameter blob of at most 8192 doubles (EUNSUPPORTED beyond).  It runs
   the precompiled kernels only (sector integrands use the table-driven
   kernel, never the run-time specialised one, whose code-object load
   allocates), and no expansion orders or contour deformation.  The inputs
   are host memory as for qmc_plan_create / qmc_integrate; `stream` is a
   hipStream_t (NULL: the null stream); the call returns after the stream
   has finished it.  Calls that overlap on one device share the array and
   race: serialise them.  out, per_shift: as qmc_integrate. */
qmc_status qmc_integrate_static(uint32_t d, uint64_t n, const uint64_t *g, uint32_t m, const double *shifts,
                                qmc_transform t, qmc_family family, const void *params, void *stream,
                                qmc_result *out, double *per_shift);

/* The steps of one training update, callable on their own (same kernels as
   qmc_cv_train).  Training samples are n points z (n, d) in [0,1]^d with
   the transform's Jacobian sw (n) and the weighted targets yw = fhat (n),
   all single precision, row-major.  For the dimension i being solved the
   model is linear in W[., i, .] (c = 1):
     sw_j g(z_j) = sum_{r,k} rho_j[r] phi_j[k] W[r,i,k],
     rho_j[r] = sw_j prod_{i' != i} sum_k W[r,i',k] P~_k(z_{j,i'}),  phi_j[k] = P~_k(z_{j,i}),
   so the step solves the ridge normal equations of the design matrix
   A_j[u] = rho_j[r] phi_j[k], columns u = r K + k, F = R K.  The limits are
   those of qmc_cv_train (d <= 12, the compiled (R, K) pairs, else
   EUNSUPPORTED) and n <= 2^26.  All pointers are host memory, borrowed
   for the call; the library allocates and frees its own device memory and
   runs on the current device's null stream.  Not part of the paper (the
   control variate is an addition to its estimator). */

/* Training samples of the plan's lattice with its first shift: z_out
   (n, d), sw_out (n), yw_out (n) = component `part` (0 real, 1 imaginary)
   of fhat = J f(z), each rounded from FP64 to single precision. */
qmc_status qmc_cv_samples(qmc_plan_t train_plan, qmc_family family, const void *params, uint32_t part,
                          float *z_out, float *sw_out, float *yw_out);

/* Design-matrix factors of dimension i in FP64: rho_out (n, R), phi_out
   (n, K).  w: (R, d, K) orthonormal-basis factors. */
qmc_status qmc_cv_features(uint32_t n, uint32_t d, uint32_t R, uint32_t K, uint32_t i, const float *z,
                           const float *sw, const double *w, double *rho_out, double *phi_out);

/* Normal equations of given factors rho (n, R), phi (n, K) and target y (n),
   all FP64:
     gram_out (F, F) = sum_j a~_j a~_j^T,  a~_j[u] = bf16(fl32(rho_j[r]) fl32(phi_j[k])),
   BF16 matrix-core products with FP32 accumulation over at most
   acc_len_out[0] points, then FP64 over those partial sums;
     rhs_out (F) = sum_j (rho_j[r] phi_j[k]) y_j,
   FP64 accumulation over at most acc_len_out[1] points, then FP64 over the
   partial sums.  acc_len_out (nullable): 2 values. */
qmc_status qmc_cv_normal(uint32_t n, uint32_t R, uint32_t K, const double *rho, const double *phi, const double *y,
                         double *gram_out, double *rhs_out, uint32_t *acc_len_out);

/* (G + lam I) x = b in FP64 by a blocked Cholesky factorisation on the
   device.  gram: (F, F) symmetric (the lower triangle is read), rhs: F.
   lam = ridge * trace(G) / F, multiplied by 100 at each non-positive pivot,
   at most three times; lam_out (nullable) the value used, escalations
   (nullable) how often it was raised.  x_out: F.  EINVAL on non-finite
   input or ridge <= 0, ENONFINITE when G + lam I stays indefinite. */
qmc_status qmc_cv_solve(uint32_t R, uint32_t K, const double *gram, const double *rhs, double ridge,
                        double *lam_out, double *x_out, int32_t *escalations);

/* One alternating-least-squares step for dimension i as qmc_cv_train runs
   it: FP64 features, BF16 normal matrix, FP64 solve with lam = ridge times
   the mean diagonal, then `refine` (<= 8) refinements against the FP64
   residual y - A w with y = yw / scale (the right-hand side of each from the
   FP64 design matrix, so the BF16 matrix only preconditions).  w_in: (R, d, K); w_out (R, d, K) the
   same factors with W[., i, .] replaced; lam_out (nullable) the ridge
   used. */
qmc_status qmc_cv_als_step(uint32_t n, uint32_t d, uint32_t R, uint32_t K, uint32_t i, const float *z,
                           const float *sw, const float *yw, double scale, const double *w_in, double ridge,
                           uint32_t refine, double *w_out, double *lam_out);

/* int g over [0,1]^d in closed form. */
qmc_status qmc_cv_integral(uint32_t R, uint32_t d, uint32_t K, const double *w, const double *c, double *out);

/* One pass over the plan's lattice evaluating fhat and the residual
   fhat - J g (g in FP64, W and c laid out as qmc_cv_train writes them).
   plain_out (nullable): the plain estimate of the same pass; out:
   int g + Qbar[f - g] with its error, or the plain estimate (used_cv = 0)
   when the residual's error (complex modulus) is not smaller.  per_shift
   (nullable): real integrands 2m doubles (plain Q_k, residual Q_k) per
   shift; complex ones 4m doubles (Re, Im plain, Re, Im residual). */
qmc_status qmc_integrate_cv(qmc_plan_t plan, qmc_family family, const void *params, uint32_t R, uint32_t K,
                            const double *w, const double *c, qmc_result *out, qmc_result *plain_out,
                            double *per_shift);

/* The coefficients of e^0 .. e^(n_orders-1) of a sector integrand whose
   exponents depend on a regulator e (qmc_sector_params.n_orders >= 2), all
   from one pass over the lattice: the sector functions U, F, their
   logarithms and the powers are shared between the orders.  Sector
   integrands are expanded in the dimensional regulator order by order
   (Sec. 1); the exponents' dependence on it is what the caller passes as
   eps_u, eps_f.  out: n_orders results (caller-owned); per_shift (nullable):
   m * parts doubles, per shift the orders in turn, (Re, Im) for complex.
   Needs the specialised kernel (EUNSUPPORTED with qmc_plan_set_jit(0));
   qmc_integrate rejects n_orders >= 2 with EINVAL.  With deform_lambda != 0
   every result carries the crossing fraction and the call returns ECONTOUR
   as qmc_integrate does. */
qmc_status qmc_integrate_orders(qmc_plan_t plan, qmc_family family, const void *params, qmc_result *out,
                                double *per_shift);

/* The sum of `count` sector integrals of the plan's dimension in one pass
   (Sec. 1: an integral is the sum of its sectors' contributions): every
   lattice point is evaluated once for all sectors, whose values are added
   before the per-shift sums, so eqs. (2)-(3) estimate the sum directly and
   its error accounts for the correlation between the sectors.  params:
   count sector parameter sets (all real or all complex; n_orders < 2,
   deform_lambda = 0, else EUNSUPPORTED); count <= 32.  One kernel is
   compiled per combination of exponent structures (specialised kernel
   only).  out: host result; per_shift (nullable) as qmc_integrate's. */
qmc_status qmc_integrate_sum(qmc_plan_t plan, uint32_t count, const qmc_sector_params *const *params,
                             qmc_result *out, double *per_shift);

/* Sign check of a contour deformation (Sec. 3): the fraction of the plan's
   lattice points (all m shifts, transformed as the plan says, unweighted) at
   which the deformed F(z) - i delta has a positive imaginary part, i.e. the
   contour lies on the wrong side of the -i0 prescription there.  params is
   a sector with deform_lambda != 0 (EINVAL otherwise); orders are ignored.
   fraction: host double; per_shift (nullable): m doubles, the fraction per
   shift.  A valid deformation gives 0.  Needs the specialised kernel. */
qmc_status qmc_deform_check(qmc_plan_t plan, const qmc_sector_params *params, double *fraction,
                            double *per_shift);

/* Choice of the deformation parameter on a (pilot) plan: for lambda =
   lam_max * shrink^i, i = 0 .. count-1, the sign check above runs; every
   lambda that passes it is integrated, and the one with the smallest
   estimated error sqrt(err_re^2 + err_im^2) is returned in *lam_out with its
   result in *out (all host memory).  By Cauchy's theorem every valid lambda
   gives the same integral, so the error is the criterion.  shrink in (0, 1),
   count 1..64, lam_max > 0 (EINVAL otherwise); n_orders >= 2 is EINVAL
   (select on the plain integrand); EUNSUPPORTED when no lambda passes. */
qmc_status qmc_deform_select(qmc_plan_t plan, const qmc_sector_params *params, double lam_max, double shrink,
                             uint32_t count, double *lam_out, qmc_result *out);

/* Component-by-component construction of a generating vector (rank-1
   lattices, Sec. 2; the construction is the standard one of the lattice
   literature): z_1 = 1 and, for s = 2..d, z_s is the candidate c minimising
     e_s^2(c) = -1 + (1/n) sum_{j<n} prod_{i<s} (1 + gamma_i 2 pi^2 B2({j z_i/n}))
                                     * (1 + gamma_s 2 pi^2 B2({j c/n})),
   B2(x) = x^2 - x + 1/6, the squared worst-case error of the weighted
   Korobov space of smoothness 2 (with unit weights, the P2 of
   qmc_korobov_search).  gamma: d non-negative product weights (NULL: all 1).
   cand: ncand candidates, each a unit mod n (NULL: every unit in [1, n/2]);
   values within 1e-13 (1 + e^2) of the minimum are ties (lattice symmetries
   make exact ties common: c and c^-1 in two dimensions), and ties go to the
   smaller c.  The sum over j is formed from j <= n/2 (the points j and
   n - j contribute equally) as twice that sum less the self-mirrored terms
   j = 0 and, for even n, j = n/2.  z_out: d values; e2_out: d values, e_s^2(z_s)
   after each component (host memory, caller-owned).  n in [2, 2^31],
   d <= 16; EUNSUPPORTED when candidates x n exceeds 2^44 (pass a subset).
   Runs on the current device, synchronously. */
qmc_status qmc_cbc_search(uint64_t n, uint32_t d, const double *gamma, const uint64_t *cand, uint32_t ncand,
                          uint64_t *z_out, double *e2_out);

/* Embedded (extensible) lattices in base 2 (rank-1 lattices of Sec. 2 whose
   point sets nest): with n = 2^k and g = (1, a, a^2, ...) mod 2^kmax, the
   2n-point lattice is the n-point lattice plus the same lattice with every
   shift moved by (g mod 2n) / (2n), so a ladder of sizes evaluates every
   point once.  This search scores each odd candidate a by the mean over
   k = kmin..kmax of ln P2(2^k, korobov_vector(2^k, d, a)) (qmc_korobov_search
   per rung) and returns the best (ties: smaller a).  cand: ncand odd values
   (EINVAL otherwise), ncand <= 4096; 1 <= kmin <= kmax <= 31.  score: the
   best mean log P2; p2_levels (nullable): kmax - kmin + 1 values, the best
   candidate's P2 per rung.  Host memory. */
qmc_status qmc_korobov_search_extensible(uint32_t kmin, uint32_t kmax, uint32_t d, const uint64_t *cand,
                                         uint32_t ncand, uint64_t *a_best, double *score, double *p2_levels);

/* The shifts that make the n-point lattice (n = n2 / 2, generator g) the
   odd points of the n2-point one: {shift_k + (g mod n2) / n2} per shift and
   coordinate, the construction of the embedded lattices above.  n2: a power
   of two in [2, 2^32] (EINVAL otherwise); g: d values; shifts, out: m * d
   doubles row-major, each shift in [0, 1) (EINVAL otherwise); out may alias
   shifts.  Host memory, no device call. */
qmc_status qmc_lattice_moved_shifts(uint64_t n2, uint32_t d, const uint64_t *g, uint32_t m, const double *shifts,
                                    double *out);

/* Merge of two half-lattice estimates into the estimate of their union
   (eqs. (2)-(3)): q_out = (q_a + q_b) / 2 per shift and part, then the mean
   and the error over the m shifts.  q_a, q_b, q_out: m * np doubles laid out
   as qmc_integrate's per_shift (np = 1 real, 2 complex); out: host result.
   ENONFINITE when a merged sum is not finite. */
qmc_status qmc_lattice_merge(uint32_t m, uint32_t np, const double *q_a, const double *q_b, double *q_out,
                             qmc_result *out);

/* The library's device FP64 math on count host inputs, for checking the
   functions the sector integrand uses against a host reference:
   fn = 0 logarithm (x > 0), 1 exponential: x and y hold count values;
   fn = 2 atan2: x holds count pairs (y_i, x_i), y count angles;
   fn = 3 sincos (|x| < 2^19): x count values, y count pairs (sin, cos). */
qmc_status qmc_math_eval(int32_t fn, uint64_t count, const double *x, double *y);

/* Release a plan and its device memory (NULL is ignored). */
void qmc_plan_destroy(qmc_plan_t plan);

/* Name of a status code ("unknown status" for any other value; an int so
   that any value is a valid argument). */
const char *qmc_status_string(int32_t status);
const char *qmc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* QMC_H */
