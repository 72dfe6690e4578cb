/*
 * pfista: polynomial-preconditioned FISTA for Cartesian SENSE on AMD gfx950.
 *
 * Solves  argmin_x 1/2 ||A' x - b'||^2 + lambda ||Psi x||_1   (the unconstrained
 * problem of the paper's Introduction) with Algorithm 4 of Iyer et al.,
 * "Polynomial Preconditioners for Regularized Linear Inverse Problems"
 * (arXiv 2204.10252): FISTA whose gradient A'^H(A' z - b') is multiplied by
 * p(A'^H A') for a degree-d polynomial p fitted by the L2 cost of Section 2.5
 * and applied in the nested (Horner) order of Section 2.7.
 *
 *   A  = M F S  (Section 3.2, Cartesian SENSE): S multiplies by each coil map,
 *        F is the unitary 2-D DFT (forward exponent exp(-2 pi i k n / N),
 *        DC at index 0), M keeps the sampled k-space points;
 *   A' = sqrt(inv_l) A, b' = b / ||b||  (normalisation of Section 3, with
 *        inv_l = 1/L and L an upper bound of the top eigenvalue of A^H A);
 *   Psi = orthonormal 2-D Haar transform with `haar_levels` levels; every
 *        coefficient (the coarsest approximation too) is soft-thresholded.
 *
 * Memory: every array argument is a DEVICE pointer owned by the caller unless
 * marked "host".  Complex data is complex64 (pfista_c32), row-major with x
 * fastest:
 *   image (x, y, w, z, g, ...)   [S][N][N]
 *   coil maps `sens`             [S][C][N][N]
 *   k-space `kspace`, `b`        [S][C][N][N]  natural order, zero off-mask
 *   mask, 2-D kind               uint8 [S][N][N], nonzero = sampled
 *   mask, phase-encode kind      uint8 [S][N], one flag per ky row (all kx)
 * with N = desc.n, C = desc.coils, S = desc.slices.  Complex pointers must be
 * 8-byte aligned; pfista_step needs 16-byte alignment.  `ws` is a caller-owned
 * device workspace of at least pfista_workspace_bytes() bytes; the library
 * allocates no device memory and keeps no state between calls.
 *
 * Devices: a plan or batch belongs to the device that is current when it is
 * created; every call that takes it must run with that device current (EINVAL
 * otherwise), with arrays and stream on that device.
 *
 * Streams: every call enqueues on `stream` and returns without waiting, except
 * pfista_solve, pfista_data_term and pfista_power_iteration, which wait for
 * their host-visible scalars (documented per call).  Calls sharing a
 * workspace must not overlap.
 *
 * Errors: functions return PFISTA_OK (0) or a negative pfista_status; the
 * library never aborts.  pfista_last_error() gives a per-thread message.
 */
#ifndef PFISTA_H
#define PFISTA_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  float re, im;
} pfista_c32;

typedef enum {
  PFISTA_OK = 0,
  PFISTA_EINVAL = -1,      /* null, misaligned or aliased pointer; bad size */
  PFISTA_UNSUPPORTED = -2, /* image side, levels or degree outside the supported set */
  PFISTA_EHIP = -3,        /* HIP runtime error (message kept) */
  PFISTA_DIVERGED = -4     /* non-finite or exploding objective in pfista_solve */
} pfista_status;

/* Operator kind of a plan.  2D / 1D: Cartesian sampling, `mask` as in the
 * header.  TOEPLITZ: non-Cartesian sampling (Section 3.3), whose normal
 * operator E^H E (E the non-uniform DFT of a trajectory) is applied through
 * its Toeplitz structure as a 2n x 2n circular convolution; every `mask`
 * argument of such a plan is the real kernel float [S][2n][2n] that
 * pfista_toeplitz_kernel builds (n in {64, 128, 160, 192, 256}). */
typedef enum { PFISTA_MASK_2D = 0, PFISTA_MASK_1D = 1, PFISTA_TOEPLITZ = 2 } pfista_mask_kind;

/* Problem shape.  n in {64, 128, 160, 192, 256, 320, 384, 512} (radices 2, 3,
 * 5); 1 <= haar_levels <= 4; coils >= 1; slices >= 0; slices * coils <= 65535;
 * phase-encode plans also need coils * n * n * 8 < 2^31 (the coil maps of one
 * slice, e.g. at most 1023 coils at n = 512). */
typedef struct {
  int n;
  int coils;
  int slices;
  int haar_levels;
  int mask_kind; /* pfista_mask_kind */
} pfista_desc;

typedef struct pfista_plan pfista_plan;

/* Validate `d` and build an immutable plan (host object, plus one-time upload
 * of FP64-computed twiddle tables to the current device).  Plans may be shared
 * across streams and threads.  Returns EINVAL / UNSUPPORTED on a bad desc. */
int pfista_plan_create(pfista_plan **out, const pfista_desc *d);
void pfista_plan_destroy(pfista_plan *p);

/* Workspace size in bytes needed by every call on this plan (including
 * pfista_solve at any degree <= 8): one complex64 per (slice, coil, pixel),
 * five images, and small FP64 scratch; phase-encode plans add one more
 * complex64 per (slice, coil, pixel), where pfista_solve keeps the packed coil
 * maps its loop reads (see pfista_pack_coil_maps). */
size_t pfista_workspace_bytes(const pfista_plan *p);

/* Normal operator (the paper's A^H A, Section 2.7 counts these):
 *   y = alpha * A^H A x + beta * w      (A un-normalised; pass alpha = inv_l
 *                                        for the normalised operator)
 * w may be NULL (beta ignored) or equal to y; y must not overlap x.
 * Arithmetic: FP32 complex, FP32 accumulation over coils in a fixed order
 * (bitwise deterministic). */
int pfista_normal_apply(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask,
                        const pfista_c32 *x, pfista_c32 *y, float alpha, const pfista_c32 *w,
                        float beta, void *ws, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * operation as pfista_normal_apply, with its transform buffer in the library's
 * own static device array of PFISTA_STATIC_SCRATCH_BYTES (32 MiB) instead of a
 * caller workspace; it calls no allocating routine.  Each GPU holds one such
 * array for the life of the process, shared by every call on that GPU: calls
 * that overlap on one GPU (other streams, other threads) race.  The array's
 * contents are left over from the last call; every element a call reads, it
 * has written first.  EINVAL when the plan's transform buffer (S * C * n^2
 * complex values, twice that for Toeplitz plans) exceeds the array. */
#define PFISTA_STATIC_SCRATCH_BYTES (32u << 20)
int pfista_normal_apply_noalloc(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask,
                                const pfista_c32 *x, pfista_c32 *y, float alpha,
                                const pfista_c32 *w, float beta, hipStream_t stream);

/* Polynomial preconditioner (Section 2.7, nested evaluation):
 *   out = p(N') g,  N' = inv_l * A^H A,  p(z) = sum_{i=0..degree} coef[i] z^i,
 * evaluated as h = coef[d] g; h = coef[i] g + N' h for i = d-1 .. 0, i.e.
 * `degree` normal applies.  coef: HOST array of degree+1 doubles (rounded to
 * FP32 for the kernels).  out must not overlap g.  0 <= degree <= 8. */
int pfista_poly_apply(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask,
                      double inv_l, const double *coef, int degree, const pfista_c32 *g,
                      pfista_c32 *out, void *ws, hipStream_t stream);

/* Coil maps of a phase-encode plan in the layout its one-pass operator
 * (Section 2.7's A^H A with F^H M F acting along the phase-encode axis only)
 * reads fastest: `packed` receives the same S * C * N * N complex values,
 * reordered so that every load of the operator's coil loop is one contiguous
 * 1 KB run per wavefront.  The order is internal to this library version: the
 * only valid uses of `packed` are the *_packed calls below on a plan of the
 * same desc.  Cost: one read and one write of the coil maps.  `packed` (device,
 * 16-byte aligned, caller-owned) must not overlap `sens`.  UNSUPPORTED for
 * 2-D and Toeplitz plans. */
int pfista_pack_coil_maps(const pfista_plan *p, const pfista_c32 *sens, pfista_c32 *packed,
                          hipStream_t stream);

/* pfista_normal_apply and pfista_poly_apply of a phase-encode plan with the
 * coil maps given packed (from pfista_pack_coil_maps): the same arithmetic in
 * the same order, so bitwise the same results.  UNSUPPORTED for other plans;
 * `packed` must be 16-byte aligned.  pfista_solve packs the maps into its
 * workspace by itself when it runs at least 12 normal applies
 * (max_iter * (degree + 1), plus power_iters when inv_l = 0); shorter solves
 * read them in place, with the same results. */
int pfista_normal_apply_packed(const pfista_plan *p, const pfista_c32 *packed, const uint8_t *mask,
                               const pfista_c32 *x, pfista_c32 *y, float alpha, const pfista_c32 *w,
                               float beta, void *ws, hipStream_t stream);
int pfista_poly_apply_packed(const pfista_plan *p, const pfista_c32 *packed, const uint8_t *mask,
                             double inv_l, const double *coef, int degree, const pfista_c32 *g,
                             pfista_c32 *out, void *ws, hipStream_t stream);

/* Fused proximal and momentum step of Algorithm 4 (prox of Section 2.1):
 *   x_new = Psi^H soft(Psi (z - pg), lambda)
 *   z_new = x_new + beta_k (x_new - x_old)
 * and red[0] = sum |soft(Psi(z - pg))| (= ||Psi x_new||_1), red[1] =
 * ||x_new - x_old||^2, red[2] = ||x_new||^2, accumulated in FP64 (red: device,
 * 3 doubles).  Outputs may alias inputs element for element (in-place update of
 * x and z is allowed).  Complex soft-threshold: w (1 - lambda/|w|) where
 * |w| > lambda, else 0.  16-byte aligned pointers required. */
int pfista_step(const pfista_plan *p, const pfista_c32 *z, const pfista_c32 *pg,
                const pfista_c32 *x_old, pfista_c32 *x_new, pfista_c32 *z_new, float lambda,
                float beta_k, double *red, void *ws, hipStream_t stream);

/* Forward model: kspace = M F (S x), zero off-mask.  Cartesian plans only
 * (UNSUPPORTED for Toeplitz plans, as are pfista_adjoint and pfista_data_term:
 * their data lives off the grid, see pfista_nudft_*). */
int pfista_forward(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask,
                   const pfista_c32 *x, pfista_c32 *kspace, void *ws, hipStream_t stream);

/* Adjoint: y = alpha * A^H kspace = alpha * sum_c conj(S_c) F^H (M kspace_c). */
int pfista_adjoint(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask,
                   const pfista_c32 *kspace, pfista_c32 *y, float alpha, void *ws,
                   hipStream_t stream);

/* Data term 1/2 || sqrt(inv_l) A x - b_scale * b ||^2 from the k-space
 * residual, reduced in FP64.  Waits for the stream; *out is HOST. */
int pfista_data_term(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask,
                     const pfista_c32 *b, const pfista_c32 *x, double inv_l, double b_scale,
                     double *out, void *ws, hipStream_t stream);

/* Power iteration for the top eigenvalue of A^H A (the normalisation scalar
 * of Section 3): v <- N v / ||N v|| for `iters` steps; *lam_max (HOST) =
 * ||N v|| of the last step.  v: device image, the start vector on entry (if
 * NULL, an internal SplitMix64-seeded vector in the workspace is used) and the
 * last iterate on exit.  Waits for the stream. */
int pfista_power_iteration(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask,
                           pfista_c32 *v, int iters, double *lam_max, void *ws,
                           hipStream_t stream);

/* L2-optimal coefficients of Section 2.5 (minimise int_0^1 (1 - z q(z))^2 dz),
 * ascending powers, into HOST coef[0..degree]; exact integer sums through the
 * shifted-Legendre kernel, one final rounding.  0 <= degree <= 8. */
int pfista_poly_coefficients(int degree, double *coef);

/* Per-pass timing of the normal operator (y = A^H A x): each kernel pass is
 * launched `reps` times back to back between two HIP events on `stream`; HOST
 * pass_ms[k] receives the average duration (ms) of pass k and *npasses their
 * count: 4 for a 2-D mask (row transforms; column transform pair with the mask;
 * inverse rows + coil combine; inverse rows + coil combine fused with the next
 * apply's forward rows, as in the polynomial chain), 1 for a phase-encode mask.
 * pass_ms must hold 4 floats.  Synchronous.  For profiling: y ends up holding
 * the result of the last timed pass, not a defined function of x. */
int pfista_profile_normal(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask,
                          const pfista_c32 *x, pfista_c32 *y, int reps, float *pass_ms, int *npasses,
                          void *ws, hipStream_t stream);

/* Weighted L2 design of Section 2.5 with the weight w(z) = z^alpha
 * (alpha > -1; alpha = 0 is pfista_poly_coefficients): minimise
 * int_0^1 z^alpha (1 - z q(z))^2 dz.  HOST coef[0..degree], ascending powers;
 * long-double Gaussian elimination of the moment system.  0 <= degree <= 8. */
int pfista_poly_coefficients_weighted(int degree, double alpha, double *coef);

/* L-infinity design of Section 2.5 for a known smallest eigenvalue mu in (0, 1)
 * of the normalised A^H A: p(z) = (1 - r(z)) / z with
 * r(z) = T_(d+1)((1 + mu - 2z)/(1 - mu)) / T_(d+1)((1 + mu)/(1 - mu)).
 * HOST coef[0..degree], ascending powers.  0 <= degree <= 8. */
int pfista_poly_coefficients_chebyshev(int degree, double mu, double *coef);

/* Launch-shape candidates of the normal-operator chain (2-D masks), which a
 * solve (pfista_params.tune), the unrolled passes (pfista_unroll_params.tune) or
 * a batch group (pfista_batch_params.tune) can be forced to with tune = k + 1: candidate k uses radix schedule k % 2 (0:
 * default, 1: twice the lanes per transform), fuses the Horner row passes
 * unless (k / 2) % 2, and multiplies the rows per coil-combine block by
 * 2^(k / 4).  Every candidate computes the same operator. */
#define PFISTA_TUNE_CANDIDATES 12

typedef struct {
  double lambda;       /* l1 weight in normalised units */
  double inv_l;        /* 1/L > 0; 0: estimate L = 1.01 * power iteration */
  int power_iters;     /* power-iteration steps when inv_l == 0 (e.g. 30) */
  int degree;          /* polynomial degree d >= 0 (d + 1 normal applies/iter) */
  const double *coef;  /* HOST, degree+1 coefficients; NULL: L2-optimal fit.
                          Plain FISTA (Algorithm 2) is degree 0, coef = {1}. */
  int max_iter;        /* iterations to run (>= 0) */
  int check_every;     /* host check / history interval, 1..4096 */
  double tol;          /* stop when ||x_k+1 - x_k|| <= tol ||x_k+1|| at a check; 0 off */
  double f_stop;       /* stop when F(x_k) <= f_stop at a check; 0 off */
  int eval_objective;  /* evaluate F(x_k) at each check (one residual pass) */
  int k0;              /* resume: iterations already done; x_io, z_io hold x_k0, z_k0 */
  int graph_iters;     /* > 0: replay the loop as a HIP graph of this many
                          iterations (needs a non-default stream); 0: launches */
  int momentum;        /* 1: FISTA momentum (Algorithms 2 and 4); 0: none, i.e.
                          PGD / PPGD (Algorithms 1 and 3) */
  double bnorm;        /* Toeplitz plans: ||b|| of the non-Cartesian data (> 0);
                          their `b` argument is the image A^H b [S][N][N].
                          Ignored by Cartesian plans (they compute ||b||). */
  int tune;            /* launch shape of the loop (2-D masks): 0 default; -1 tune
                          (times every candidate of PFISTA_TUNE_CANDIDATES on this
                          solve's chain once, cached per device architecture and
                          plan shape, persisted in $PFISTA_TUNE_CACHE if set);
                          k >= 1 candidate k - 1 */
} pfista_params;

typedef struct {
  int iters;              /* iterations run in this call */
  int status;             /* pfista_status of the run */
  double objective;       /* last evaluated F (NaN if none) */
  double rel_change;      /* ||x_k - x_k-1|| / ||x_k|| at the last check */
  double l1;              /* ||Psi x_k||_1 at the last check */
  double inv_l;           /* 1/L used */
  double bnorm;           /* ||b|| */
  long long normal_applies; /* A^H A applications in the loop */
  int candidate;          /* launch shape used */
  double tune_us;         /* with tune == -1: the tuned shape's time of one chain
                             (measured now or read from the cache); else 0 */
  double loop_ms;         /* device time of the iteration loop: HIP events on
                             `stream` from before the first iteration to after
                             the last check (set-up excluded); 0 if no iteration */
} pfista_report;

/* Algorithm 4 on the caller's stream.  Setup (FP64 ||b||, optional power
 * iteration, exact coefficients, A'^H b') then max_iter iterations
 *   g = N' z - A'^H b';  pg = p(N') g;  x, z <- pfista_step(z, pg, x, beta_k),
 * beta_k = k / (k + 3), x_0 = z_0 = 0 unless resuming (k0 > 0).  The stream is
 * synchronised only at checks (every check_every iterations) and on return.
 * x_io: device image, output x_k (input x_k0 when resuming).  z_io: device
 * image for the momentum point (may be NULL when k0 == 0).  history (HOST,
 * nullable): F(x) after each check, ceil(max_iter / check_every) doubles, when
 * eval_objective.  Returns DIVERGED (and stops) on a non-finite value or an
 * objective above 10 F(0) = 5.  Toeplitz plans: `b` is the image A^H b and
 * params.bnorm = ||b||; the data term at checks is evaluated through the
 * normal equations, <x, N'x> - 2 Re <x, A'^H b'> + 1 (one more apply). */
int pfista_solve(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask,
                 const pfista_c32 *b, const pfista_params *prm, pfista_c32 *x_io,
                 pfista_c32 *z_io, double *history, pfista_report *rep, void *ws,
                 hipStream_t stream);

/* ---------------------------------------------------------------- non-Cartesian
 * Trajectories are float [S][J][2] (kx, ky) in cycles per field of view
 * (|k| <= n/2); the non-uniform DFT of slice s is
 *   (E v)_j = (1/n) sum_(y,x) v[y][x] exp(-2 pi i (kx_j x + ky_j y) / n),
 * which on integer points is the unitary DFT of the Cartesian model.  The
 * Toeplitz kernel is
 *   K[ky][kx] = (1/n^2) sum_j w_j D(kx_j/n - kx/(2n)) D(ky_j/n - ky/(2n)),
 *   D(u) = sin((2n - 1) pi u) / sin(pi u),
 * the 2n-point DFT of the difference kernel of E^H W E (W = diag(w), w = 1
 * when `weights` is NULL), so that for a Toeplitz plan
 *   A'^H A' x = inv_l sum_c conj(S_c) crop(IDFT(K DFT(pad(S_c x)))).
 * All three calls are set-up work (FP64 sums, O(J n^2) per slice), enqueued
 * on `stream`; plan must be a Toeplitz plan; errors EINVAL on NULL, J < 1. */
/* kern: device float [S][2n][2n]; weights: device float [S][J] or NULL. */
int pfista_toeplitz_kernel(const pfista_plan *p, const float *traj, const float *weights, int J,
                           float *kern, hipStream_t stream);
/* kdata[s][c][j] = (E (S_c x_s))_j: device [S][C][J] from x [S][N][N]. */
int pfista_nudft_forward(const pfista_plan *p, const pfista_c32 *sens, const float *traj, int J,
                         const pfista_c32 *x, pfista_c32 *kdata, hipStream_t stream);
/* y[s] = sum_c conj(S_c) E^H kdata[s][c]: the image A^H b a Toeplitz solve takes. */
int pfista_nudft_adjoint(const pfista_plan *p, const pfista_c32 *sens, const float *traj, int J,
                         const pfista_c32 *kdata, pfista_c32 *y, hipStream_t stream);

/* ------------------------------------------------------------ differentiation
 * Algorithm 4 unrolled for a fixed iteration count K from x_0 = z_0 = 0,
 * viewed as a map (lambda, c_0..c_d) -> x_K, and its reverse-mode derivative
 * (for learning the threshold and the polynomial of Section 2.5 from data).
 * The backward pass is hand-written: the prox pulls back through the Haar
 * transform (orthonormal: its pull-back is its inverse) and the complex soft
 * threshold (on its support the radial part of the cotangent passes unchanged
 * and the tangential part is scaled by 1 - lambda/|u|; d w / d lambda =
 * -u/|u|); the polynomial p(N') pulls back through the powers N'^i v_bar,
 * i = 1..d, which also give dL/dc_i = -Re <N'^i v_bar, g_k> (N' is
 * Hermitian).  Complex cotangents are real gradients packed as complex
 * numbers (dL/dRe + i dL/dIm).  Iterates are checkpointed every ckpt_every
 * iterations; the backward pass recomputes one segment at a time. */
typedef struct {
  double lambda;       /* >= 0 */
  double inv_l;        /* 1/L > 0 */
  int degree;          /* d >= 0 */
  const double *coef;  /* HOST, degree+1 coefficients; NULL: L2-optimal fit */
  int iters;           /* K >= 1 */
  int ckpt_every;      /* >= 1 (values above K act as K) */
  int momentum;        /* 1: FISTA momentum; 0: PGD / PPGD */
  int tune;            /* launch shape, as pfista_params.tune (0 default, -1 tuned
                          and cached, k >= 1 candidate k - 1); pass the same
                          value to the forward and the backward pass */
} pfista_unroll_params;

/* Device bytes of the checkpoint buffer filled by the forward pass and read
 * by the backward pass: A'^H b' and (x_k, z_k) every ckpt_every iterations. */
size_t pfista_unroll_ckpt_bytes(const pfista_plan *p, const pfista_unroll_params *prm);
/* Device workspace of both passes (the plan's workspace plus the segment
 * store, 3 * ckpt_every images, and d + 6 images of cotangents). */
size_t pfista_unroll_workspace_bytes(const pfista_plan *p, const pfista_unroll_params *prm);
/* x_out (device image) = x_K; fills ckpt.  Waits once for ||b||. */
int pfista_unroll_forward(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask,
                          const pfista_c32 *b, const pfista_unroll_params *prm, pfista_c32 *x_out,
                          void *ckpt, void *ws, hipStream_t stream);
/* Given x_bar = dL/dx_K (device image) and the forward's ckpt (same plan,
 * sens, mask and params), writes grad (HOST, degree + 2 doubles):
 * dL/dlambda, dL/dc_0 .. dL/dc_d.  Waits for the result. */
int pfista_unroll_backward(const pfista_plan *p, const pfista_c32 *sens, const uint8_t *mask,
                           const pfista_unroll_params *prm, const pfista_c32 *x_bar,
                           const void *ckpt, double *grad, void *ws, hipStream_t stream);

/* ------------------------------------------------------------------ batches
 * A batch is a list of independent slices of uneven shape (image side, coil
 * count, Haar levels), each its own problem of the form above with its own
 * normalisation (inv_l_s, ||b_s||, Section 3) and its own lambda_s, all run
 * for the same iterations with one polynomial.  (The Cartesian experiment of
 * Section 3.2 reconstructs 2-D slices of a many-slice volume; every slice is an
 * independent instance of the problem.)  2-D masks only.  Slices with the same
 * image side and levels
 * form a group; each kernel launch covers a whole group, whatever its slices'
 * coil counts.  Every group gets its own launch shape from a tuner that times
 * the candidate radix schedules and coil-combine shapes on the device. */
typedef struct {
  int n;           /* image side (as pfista_desc.n) */
  int coils;       /* >= 1 */
  int haar_levels; /* 1..4 */
} pfista_slice_desc;

typedef struct pfista_batch pfista_batch;

/* Validate and group `count` slices (HOST array); count >= 0, at most 65535
 * coil images per group.  chunk_bytes > 0 caps the coil-map bytes of a group
 * (a slice larger than the cap forms a group of its own): a group's loop then
 * keeps its coil maps and transform buffer inside the GPU's last-level cache
 * (256 MB Infinity Cache on MI355X) across the passes of an iteration;
 * 0 groups every slice of an image side and level count together.  Returns
 * EINVAL / UNSUPPORTED on a bad slice. */
int pfista_batch_create(pfista_batch **out, const pfista_slice_desc *slices, int count,
                        size_t chunk_bytes);
void pfista_batch_destroy(pfista_batch *b);
/* Device workspace for pfista_batch_solve: about three times the coil-map
 * bytes of all slices (normalised copies of maps and data, transform buffer)
 * plus five images per slice. */
size_t pfista_batch_workspace_bytes(const pfista_batch *b);
/* Number of groups (entries of the group report). */
int pfista_batch_groups(const pfista_batch *b);

typedef struct {
  int degree;          /* as pfista_params */
  const double *coef;  /* HOST, degree+1 coefficients; NULL: L2-optimal fit */
  int max_iter;        /* iterations (all slices run the same count) */
  int check_every;     /* 1..4096 */
  double tol;          /* stop when every slice's relative change <= tol at a check; 0 off */
  int eval_objective;  /* per-slice F(x_k) at each check */
  int power_iters;     /* power-iteration steps for slices whose inv_l is 0 */
  int graph_iters;     /* > 0: replay the loop as one HIP graph of this many
                          iterations over all groups (non-default stream) */
  int momentum;        /* 1: FISTA momentum; 0: PGD / PPGD */
  int streams;         /* 1: groups one after another on `stream`; k > 1: groups
                          spread over k concurrent branches (forked from and
                          joined back into `stream`) */
  int tune;            /* -1: tune every group (cached per device architecture,
                          image side, slice and coil counts, degree; the file
                          named by PFISTA_TUNE_CACHE, if set, persists the
                          choices); 0: default shape; k >= 1: candidate k - 1 */
} pfista_batch_params;

typedef struct {
  double objective;  /* F_s(x) at the last check (NaN without eval_objective) */
  double rel_change; /* ||x_k - x_k-1|| / ||x_k|| at the last check */
  double l1;         /* ||Psi x_k||_1 */
  double inv_l;      /* 1/L_s used */
  double bnorm;      /* ||b_s|| */
} pfista_slice_report;

typedef struct {
  int n;             /* image side */
  int haar_levels;
  int slices;        /* slices in the group */
  int coil_images;   /* sum of their coil counts */
  int candidate;     /* launch shape used (see PFISTA_TUNE_CANDIDATES) */
  double chain_us;   /* tuner's time of one gradient + polynomial chain (0 if not timed) */
} pfista_group_report;

typedef struct {
  int iters;
  int status;
  long long normal_applies; /* per slice */
} pfista_batch_report;

/* Algorithm 4 on every slice of the batch.  sens, mask, kspace, x_out: HOST
 * arrays of `count` device pointers, slice s's coil maps [C_s][n_s][n_s],
 * 2-D mask uint8 [n_s][n_s], k-space data [C_s][n_s][n_s] and output image
 * [n_s][n_s] (x_k in normalised units; x_out may not alias the inputs).
 * lambda: HOST [count].  inv_l: HOST [count] (0 entries are estimated by
 * power iteration) or NULL (all estimated).  Setup folds sqrt(inv_l_s) into a
 * copy of the coil maps and 1/||b_s|| into a copy of the data, so the loop is
 * the single-slice loop with per-slice thresholds.  slice_rep (HOST [count]),
 * group_rep (HOST [pfista_batch_groups]) and rep may be NULL.  Synchronises
 * at setup, at checks and on return.  DIVERGED if any slice's values turn
 * non-finite or its objective exceeds 5. */
int pfista_batch_solve(const pfista_batch *b, const pfista_c32 *const *sens,
                       const uint8_t *const *mask, const pfista_c32 *const *kspace,
                       const double *lambda, const double *inv_l,
                       const pfista_batch_params *prm, pfista_c32 *const *x_out,
                       pfista_slice_report *slice_rep, pfista_group_report *group_rep,
                       pfista_batch_report *rep, void *ws, hipStream_t stream);

/* Message of the last failed call on this thread ("" if none). */
const char *pfista_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PFISTA_H */
