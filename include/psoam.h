/*
 * psoam.h -- C ABI of the MI355X (gfx950) hot path of the one-step
 * photo-switching optoacoustic reconstruction (arXiv 2510.23739).
 *
 * The library applies the forward model A = H S and its adjoint, the
 * proximal maps of the one-step regulariser (anisotropic TV, l1, x >= 0) and
 * the proximal-gradient solver with FISTA momentum, all as HIP kernels.
 *
 * Conventions shared by every entry point
 *  - Device pointers are HIP device memory on the current device; the caller
 *    allocates and frees them.  Host pointers are named so below.
 *  - Every call is enqueued on the given stream (a hipStream_t passed as
 *    void*, NULL = the null stream) and returns before the work finishes,
 *    except where a call states it synchronises.
 *  - All external arrays are float32, C-contiguous:
 *        c  concentrations  [S][Ny][Nx][Nz]
 *        y  A-scans         [K][Ny][Nx][Nt]
 *  - Return value: PSOAM_OK or one of the error codes; no exception crosses
 *    the ABI.  psoam_last_error() gives the message of the last failure on
 *    the calling thread.
 *  - A plan is immutable after creation except for its internal scratch
 *    buffers, so calls that share a plan must not overlap in time (they
 *    serialise naturally when issued on one stream).
 */
#ifndef PSOAM_H
#define PSOAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PSOAM_OK = 0,
  PSOAM_EINVAL = 1,       /* bad argument: null pointer, size, shape, option */
  PSOAM_EUNSUPPORTED = 2, /* valid request the library does not implement */
  PSOAM_EHIP = 3,         /* a HIP runtime call failed (message has the HIP error) */
  PSOAM_ENOMEM = 4,       /* device allocation failed */
  PSOAM_EDIVERGED = 5     /* a FP64 reduction of the solver was not finite */
};

/* Arithmetic of the acoustic contraction (H and its adjoint).  FP32 runs
 * float32 matrix cores; BF16/FP16 round both operands to 16 bits and
 * accumulate in float32; the _SPLIT forms add the low-order parts of both
 * operands (three products per tile) for about 16 significant bits.
 * FP16 operands are written times a power of two chosen on the device for
 * every operand, from an FP32 max-abs reduction of what is converted (the
 * switched concentrations, the A-scans of an adjoint) or from a bound that
 * holds for every element (the solver's residual: max over t of the sum of
 * |h| times the largest switched value, plus max |p|), so that the largest
 * value lands at or below 2^14: inputs in any units neither overflow FP16
 * nor lose precision to its subnormal range (values down to 2^-28 of the
 * largest keep 11 significant bits).  Inputs with an infinite element give
 * non-finite results, as in FP32.
 * BF16 rounds the impulse-response table with error feedback along dy (for
 * each dx, sample and depth, the rounding error of an entry is added to the
 * next entry inside the band before it is rounded), so that the table's
 * errors cancel in sums over neighbouring lateral offsets.
 * BF16_REFINED is BF16 plus the low-order BF16 part of the impulse-response
 * table for the columns (z, jdy, jdx) that carry most of the table's
 * rounding error: the fewest columns, by decreasing squared rounding error,
 * whose squared errors sum to at least 90% of the table's, chosen in FP64 at
 * plan creation.  Those corrections run as extra matrix-core tiles on the
 * same operand windows; H and H^T use the same columns, so they stay exact
 * transposes of each other. */
typedef enum {
  PSOAM_FP32 = 0,
  PSOAM_BF16 = 1,
  PSOAM_FP16 = 2,
  PSOAM_BF16_SPLIT = 3,
  PSOAM_FP16_SPLIT = 4,
  PSOAM_BF16_REFINED = 5
} psoam_prec;

/* Geometry of one reconstruction. */
typedef struct {
  int32_t nx, ny, nz;      /* voxel grid = scan grid laterally */
  int32_t n_species;       /* S, 1..8 */
  int32_t n_pulses;        /* K, switching pulses per cycle, >= 1 */
  int32_t nt;              /* samples per A-scan */
  int32_t f;               /* lateral footprint of the impulse response, odd; R = (f-1)/2 */
  int32_t phi_per_voxel;   /* 0: phi is [Nz]; 1: phi is [Ny][Nx][Nz] */
  int32_t separable;       /* 1: separable fast form (requires gamma = 0): with a
                              fluence-independent rate S_v[k][s] = phi_v T[k][s],
                              T[k][s] = a_s + b_s exp(-k / tau_s), so
                              A c = sum_s T[:, s] (x) H(phi c_s) and the
                              contraction runs over the S species instead of
                              the K pulses; results equal the general form's
                              up to rounding.  0: general form. */
} psoam_geom;

/* Photo-physics of the species (Sec. 2.1.2, eqs. epsilon, final-H):
 *   S_v[k][s] = phi_v * (a[s] + b[s] * exp(-k * phi_v^gamma / tau[s]))
 * a = OFF-state extinction, b = ON minus OFF extinction, tau = switching
 * time constant in pulses; gamma = 1 is the fluence-dependent rate of the
 * paper, gamma = 0 a fluence-independent one. */
typedef struct {
  double a[8];
  double b[8];
  double tau[8];
  double gamma;
} psoam_species;

typedef struct psoam_plan psoam_plan;

/* Build a plan: validates the geometry, packs the banded impulse response
 * into matrix-core tiles for both H and its adjoint, and allocates the
 * padded operand buffers (zeroed borders) the kernels read.
 *
 * The acoustic operator of one pulse (Sec. 2.1.4, eqs. q-above-1d,
 * q-below-1d, acoustic-temporal-conv; discretised in Sec. 2.2.3):
 *   y[k][iy][ix][t] = sum_{jdy,jdx in [0,F)} sum_z h[z][jdy][jdx][t] *
 *                     b[k][iy+jdy-R][ix+jdx-R][z],   b = S c,
 * with voxels outside the grid and samples outside [0, Nt) absent.
 * h is given banded: h[z][jdy][jdx][t0 + j] = sir_taps[z][jdy][jdx][j] for
 * j < sir_w, zero elsewhere by definition.
 *
 * phi, sir_t0, sir_taps are HOST pointers, read during the call only:
 *   phi       float [Nz] or [Ny][Nx][Nz] (fluence, > 0)
 *   sir_t0    int32 [Nz][F][F]
 *   sir_taps  float [Nz][F][F][sir_w]
 * The call synchronises `stream` (uploads finish before it returns).
 * Errors: EINVAL (null pointer, non-positive size, even f, n_species outside
 * 1..8, sir_w outside 1..64, non-finite table entry, non-positive phi or
 * tau), EUNSUPPORTED (prec not built), ENOMEM, EHIP. *out is NULL on error. */
int psoam_plan_create(const psoam_geom* g, const psoam_species* sp, const float* phi,
                      const int32_t* sir_t0, const float* sir_taps, int32_t sir_w,
                      int32_t prec, void* stream, psoam_plan** out);

/* Free everything the plan owns (waits for the device first).  NULL is a no-op. */
int psoam_plan_destroy(psoam_plan* plan);

/* Geometry the plan was built with (host copy). */
int psoam_plan_geom(const psoam_plan* plan, psoam_geom* g);

/* y = A c = H S c  (eq. full-forward).  c: device [S][Ny][Nx][Nz] float,
 * y: device [K][Ny][Nx][Nt] float, 16-byte aligned, overwritten.  c and y
 * must not alias.  EINVAL: null plan or pointer, misaligned y. */
int psoam_apply_A(const psoam_plan* plan, const float* c, float* y, void* stream);

/* c = A^T y = S^T H^T y.  y: device [K][Ny][Nx][Nt], c: device
 * [S][Ny][Nx][Nz], overwritten.  y and c must not alias.
 * EINVAL: null plan or pointer. */
int psoam_apply_AT(const psoam_plan* plan, const float* y, float* c, void* stream);

/* Proximal map of thresh*||.||_1 (eqs. reg-tv-l1-one, prox), elementwise on
 * n device floats: x = sign(z) max(|z| - thresh, 0), or max(z - thresh, 0)
 * when nonneg != 0 (adds the indicator of x >= 0).  x may alias z.
 * EINVAL: n < 0, thresh < 0 or not finite, null pointer with n > 0. */
int psoam_prox_l1(float* x, const float* z, int64_t n, float thresh, int32_t nonneg,
                  void* stream);

/* Bytes of workspace psoam_prox_tv needs for this plan's grid. */
size_t psoam_prox_tv_ws_bytes(const psoam_plan* plan);

/* Proximal map of theta * TV, TV = sum over species of the l1 norms of the
 * forward differences along y, x and z with a zero last difference (eq.
 * reg-tv-l1-one, anisotropic, extended to 3D), computed by n_inner steps of
 * the accelerated projected gradient on the dual (Alg. alg:prox-inner with
 * L = grad, step 1/eig_max(grad^T grad), cold start u = 0):
 *   u <- clip(eta + grad(z - grad^T eta)/mu, -theta, theta), FISTA momentum,
 *   x  = z - grad^T u, then max(x, 0) if nonneg != 0.
 * x, z: device [S][Ny][Nx][Nz] float (may alias).  ws: device, at least
 * psoam_prox_tv_ws_bytes(plan) bytes, 256-byte aligned.
 * EINVAL: theta < 0 or not finite, n_inner < 0, null pointers. */
int psoam_prox_tv(const psoam_plan* plan, float* x, const float* z, float theta,
                  int32_t n_inner, int32_t nonneg, void* ws, void* stream);

/* psoam_prox_tv for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same dual iteration and result, bit for bit, with its three dual
 * buffers in a static device array of the library instead of a workspace.
 * Limit: S*Ny*Nx*Nz <= 3728256 species-voxels (the array holds 128 MiB on
 * every GPU the library runs on, until the process ends); larger grids get
 * EINVAL and use psoam_prox_tv.  The call allocates nothing; its first call
 * on a device looks up the array's device address (hipGetSymbolAddress).
 * The current device must be the plan's (EINVAL otherwise).  Every call on
 * a GPU shares that GPU's array: calls that overlap in time on one GPU (two
 * streams, two threads, two plans) race and must be ordered by the caller.
 * Arguments and other errors as psoam_prox_tv. */
int psoam_prox_tv_noalloc(const psoam_plan* plan, float* x, const float* z, float theta,
                          int32_t n_inner, int32_t nonneg, void* stream);

/* Bytes of workspace psoam_prox_r3 needs for this plan's grid and pulses. */
size_t psoam_prox_r3_ws_bytes(const psoam_plan* plan);

/* Proximal map of the full one-step regulariser (eq. reg-tv-l1-one):
 *   theta_tv TV(x) + theta_tvs sum_k TV((S x)^k) + theta_l1 |x|_1, x >= 0,
 * by n_inner steps of the paper's dual iteration on the stacked operator
 * L = [grad; grad S; I] (Alg. alg:prox-inner, eq. prox-dual), duals rescaled
 * per block so their boxes are theta_b, from zero duals:
 *   w   = z - (grad^T e1 + S^T grad^T e2 + e3)
 *   u1' = clip(e1 + s1 grad w), u2' = clip(e2 + s2 grad(S w)),
 *   u3' = clip(e3 + s3 w),   e = u' + beta (u' - u)  (FISTA weights)
 *   x   = max(z - (grad^T u1 + S^T grad^T u2 + u3), 0)
 * with s_b = theta_b^2 / sum_b' theta_b'^2 m_b', m = {mu, mu max_v |S_v|^2,
 * 1}, mu = eig_max(grad^T grad): the step 1/eig_max(L^T L) with eig_max
 * replaced by that upper bound.  As printed, the duals are projected onto
 * their boxes only and the sign constraint enters through the final clamp.
 * x, z: device [S][Ny][Nx][Nz] float (may alias).  ws: device, at least
 * psoam_prox_r3_ws_bytes(plan) bytes, 256-byte aligned.
 * EINVAL: a threshold < 0 or not finite, n_inner < 0, null pointers. */
int psoam_prox_r3(const psoam_plan* plan, float* x, const float* z, float theta_tv,
                  float theta_tvs, float theta_l1, int32_t n_inner, void* ws, void* stream);

/* Options of psoam_solve (Alg. alg:prox-outer and alg:prox-inner). */
typedef struct {
  double lambda_tv;        /* weight of TV(c) (lambda_1 of eq. reg-tv-l1-one) */
  double lambda_l1;        /* weight of ||c||_1 (lambda_2 of eq. reg-tv-l1-one) */
  int32_t k1;              /* outer iterations (maximum), >= 0 */
  int32_t k2;              /* inner dual iterations of the TV prox, >= 0 */
  double eps1;             /* relative objective change stop; 0 disables */
  double eps2;             /* relative momentum-iterate change stop; 0 disables */
  double alpha1;           /* step; <= 0: 1/(1.01 * power-iteration estimate) */
  int32_t n_power;         /* power iterations when alpha1 <= 0 (e.g. 30).  The
                              estimate rises towards eig_max(A^T A) from below,
                              so with few steps the step can exceed
                              1/eig_max by a few percent where the top
                              eigenvalues lie close together (the iteration
                              stays stable; FISTA's O(1/k^2) bound assumes it
                              does not); more steps close the gap */
  int32_t literal_momentum;/* 0: (t_k - 1)/t_{k+1}; 1: printed (t_k - 1)/(t_k + 1) */
  int32_t warm_inner;      /* 0: cold dual start every outer step; 1: warm */
  const float* v0;         /* device [S][Ny][Nx][Nz] power start, or NULL (constant) */
  double* trace;           /* host, k1 doubles: F(c_{k+1}) per iteration, or NULL */
  double lambda_tvs;       /* weight of sum_k TV((S c)^k) (lambda_3 of eq.
                              reg-tv-l1-one); > 0 selects the full
                              regulariser's prox (psoam_prox_r3; warm_inner
                              does not apply to it) */
  int32_t device_stop;     /* 0: the stopping tests and the trace read FP64
                              scalars on the host every iteration (the solve
                              synchronises per iteration); 1: they run on the
                              device: a one-thread kernel after each
                              iteration takes the same decisions in the same
                              FP64 arithmetic and sets a device flag that
                              every later kernel of the solve checks first
                              (and returns), so the iterations are enqueued
                              without host reads (and psoam_solve_batch
                              captures them into graphs); the trace is
                              copied to the host at the end */
} psoam_solve_opts;

typedef struct {
  int32_t iterations;      /* outer iterations performed */
  int32_t status;          /* PSOAM_OK or PSOAM_EDIVERGED */
  double alpha1;           /* step used */
  double lambda_max;       /* power-iteration estimate (0 if alpha1 was given) */
  double objective;        /* F(c) at exit if computed (trace or eps1), else NaN */
} psoam_solve_stats;

/* Solve eq. one-step:
 *   c = argmin_{c >= 0} 1/2 |A c - p|^2 + lambda_tv TV(c) + lambda_l1 |c|_1
 *                       + lambda_tvs sum_k TV((S c)^k)
 * by Alg. alg:prox-outer: c_{k+1} = prox(xi_k - alpha1 A^T(A xi_k - p)),
 * xi_{k+1} = c_{k+1} + beta_k (c_{k+1} - c_k).  With lambda_tvs = 0 the prox
 * is the TV dual iteration followed by max(. - alpha1 lambda_l1, 0) (exact
 * for that regulariser); with lambda_tvs > 0 it is psoam_prox_r3's stacked
 * dual iteration at thresholds alpha1 * lambda.
 * p: device [K][Ny][Nx][Nt]; c: device [S][Ny][Nx][Nz], initial guess on
 * entry (zeros for the paper's start), result on exit.  st: host, may be
 * NULL.  Synchronises the stream when it needs host scalars (power
 * iteration result, stopping tests and trace unless device_stop) and at exit.
 * With eps1 > 0 or a trace, the data term of F(c_{k+1}) comes from A c_{k+1}
 * = (A xi_{k+1} + beta_k A c_k) / (1 + beta_k), formed in the epilogue of
 * the next iteration's H (A is linear), not from a second H apply; this
 * needs a y-sized FP32 array the plan allocates once (4 K Ny Nx Nt bytes).
 * The separable and factorised plans evaluate F directly.
 * EINVAL: bad options; EDIVERGED: non-finite reduction (c holds the last
 * finite iterate). */
int psoam_solve(const psoam_plan* plan, const float* p, float* c, const psoam_solve_opts* o,
                psoam_solve_stats* st, void* stream);

/* ---- the two-step method (the paper's comparison, Sec. two-step approach) --
 * Step 1, acoustic inversion (eq. acoustic-inverse with R1 of eq. reg-tv):
 *   b = argmin_{b >= 0} 1/2 |H b - p|^2 + nu_1 sum_k TV(b^k)
 * with a plan from psoam_plan_create_acoustic and psoam_solve (lambda_tv =
 * nu_1, lambda_l1 = 0): the plan's "species" are the K pulse volumes and its
 * switching is the identity.  Step 2, unmixing (eq. unmixing with R2 of eq.
 * reg-unmixing):
 *   c = argmin_{c >= 0} 1/2 |S c - b|^2 + nu_2 |c|_1 + nu_3 TV(c)
 * with psoam_unmix on a plan of the species (the same FISTA and prox as
 * psoam_solve, with the per-voxel S in place of A). */

/* Plan of the acoustic operator alone on K pulse volumes: y[k] = H b[k],
 * b: device [K][Ny][Nx][Nz] as the "concentrations" of psoam_apply_A /
 * psoam_solve, y: [K][Ny][Nx][Nt].  g->n_species, phi_per_voxel and
 * separable are ignored (set to K, 0, 0).  Same table arguments and errors
 * as psoam_plan_create. */
int psoam_plan_create_acoustic(const psoam_geom* g, const int32_t* sir_t0, const float* sir_taps,
                               int32_t sir_w, int32_t prec, void* stream, psoam_plan** out);

/* ---- the factorised acoustic operator (Sec. 2.2.3 "Acoustic Model": eqs.
 * q-above-final, q-below-final, discrete-upper-circle, discrete-lower-circle,
 * acoustic-temporal-conv; App. E) ----
 * The paper's own discretisation of one acoustic process: the signal at
 * sample t is the initial pressure times the spatial response image eta,
 * summed with unit weight over the voxels that the delay sphere of t
 * crosses, then convolved in time with the electrical impulse response v:
 *   q[k][iy][ix][t] = sum_{(z,jdy,jdx) in Shell(t)} eta[z][jdy][jdx] *
 *                     b[k][iy+jdy-R][ix+jdx-R][z],          b = S c
 *   y[k][iy][ix][t] = sum_j v[j] q[k][iy][ix][t - j + eir_origin]
 * Shell(t): radius rho_t = |t - t_focus| * dr voxel pitches around the
 * focal point (scan position, z_focus).  For t < t_focus the voxels whose
 * centre depth is < z_focus, for t >= t_focus those with centre depth
 * >= z_focus; of these, the voxels whose box (one pitch wide) meets the
 * sphere: nearest box point at distance <= rho_t <= farthest box point.
 * Distances use the box coordinates max(|o| - 1/2, 0) and |o| + 1/2 of each
 * offset o (dy, dx, z - z_focus), squared and summed in the order y, x, z,
 * in double precision.  Samples outside [0, Nt) and voxels outside the grid
 * are absent. */
typedef struct {
  double dr;            /* radius step per time sample, voxel pitches (c0 dt / pitch), > 0 */
  double z_focus;       /* focal depth in voxel units (voxel centres at 0 .. Nz-1) */
  int32_t t_focus;      /* sample of radius 0 */
  int32_t n_eir;        /* taps of v, 1..32 */
  int32_t eir_origin;   /* index of v's zero-lag tap, 0 .. n_eir-1 */
} psoam_shell;

/* Plan of A = V Lambda S with the factorised acoustic operator above in
 * place of the banded H; every other entry point (psoam_apply_A/AT,
 * psoam_solve, psoam_solve_batch, the prox calls) takes it like any plan.
 * The shell sums run on the matrix cores as a narrow band (each voxel
 * column meets a few consecutive samples), the convolution as a separate
 * pass over the A-scans; the plan owns one extra [K][Ny][Nx][Nt] buffer.
 * HOST pointers, read during the call only:
 *   phi  float [Nz] or [Ny][Nx][Nz];  spr  float [Nz][F][F] (eta);
 *   eir  float [n_eir] (v).
 * g->separable must be 0.  Synchronises `stream`.
 * Errors: EINVAL (null pointer, bad size or shell parameter, non-finite
 * eta or v; the psoam_plan_create checks), EUNSUPPORTED (nt > 4096, a shell
 * band wider than 64 samples, i.e. dr too small, or separable = 1), ENOMEM,
 * EHIP.  *out is NULL on error. */
int psoam_plan_create_factorised(const psoam_geom* g, const psoam_species* sp, const float* phi,
                                 const float* spr, const float* eir, const psoam_shell* sh,
                                 int32_t prec, void* stream, psoam_plan** out);

/* Unmixing step: psoam_solve's iteration with the per-voxel switching S of
 * `plan` in place of A: gradient S^T (S xi - b) voxel by voxel, the same
 * prox (lambda_tv = nu_3 on TV(c), lambda_l1 = nu_2), step alpha1 or the
 * power-iteration estimate of eig_max(S^T S).  b: device [K][Ny][Nx][Nz]
 * (e.g. step 1's result); c: device [S][Ny][Nx][Nz], initial guess in,
 * result out.  lambda_tvs must be 0.  Errors as psoam_solve. */
int psoam_unmix(const psoam_plan* plan, const float* b, float* c, const psoam_solve_opts* o,
                psoam_solve_stats* st, void* stream);

/* n independent solves (plans of different shapes and pulse counts allowed)
 * as one batch, the batched family of reconstructions of the same method
 * (Alg. alg:prox-outer per problem).  Arrays of length n; opts/st arrays
 * too (st may be NULL).  Same result per problem as psoam_solve.
 * Execution: every problem runs on a stream of its own (default priority);
 * the power iterations run concurrently, then each problem's pairs of outer
 * iterations are captured into a HIP graph (the FISTA step state kept on the
 * device) and replayed on its stream; an odd last iteration runs uncaptured.
 * Stopping tests and traces run inside the captured iterations when the
 * problem sets device_stop (its kernels return at once after its test
 * fires).  Problems that need host decisions inside the loop (eps1 > 0,
 * eps2 > 0 or a trace without device_stop), warm_inner, k1 < 2, and every
 * problem when a plan appears twice in the batch (plans own their operand
 * buffers), are solved one after another on the caller's stream instead.  The call
 * synchronises the streams it creates; results are ordered before later
 * work on `stream`.  EINVAL: bad arguments (checked for all problems before
 * any work); EHIP: stream, event or graph call failed; EDIVERGED as for
 * psoam_solve. */
int psoam_solve_batch(int32_t n, const psoam_plan* const* plans, const float* const* p,
                      float* const* c, const psoam_solve_opts* o, psoam_solve_stats* st,
                      void* stream);

/* ---- diagnostics (timing and profiling; not steps of the method) ---- */

/* Work figures of a plan's band contraction, per position and per pulse:
 * useful_macs = nonzero band entries h[z][jdy][jdx][t] with t in [0, Nt)
 * (the algorithmic multiply-adds of one A-scan of one pulse);
 * chunks = packed matrix-core tiles of the kernel the plan launches (the
 * run-packed tiles when the LDS-staged kernel is used); executed_macs =
 * chunks times the tile size (16 x 32 for 16-bit, 16 x 4 for FP32).
 * dir 0: H, dir 1: H^T. */
typedef struct {
  int64_t useful_macs[2];
  int64_t chunks[2];
  int64_t executed_macs[2];
  int64_t operand_bytes[2];  /* padded operand buffer of H (0) and H^T (1) */
  int64_t lds_bytes[2];      /* LDS per workgroup of the staged kernel, 0 if not used */
  int32_t lds_rows[2];       /* output rows per workgroup of the staged kernel */
} psoam_plan_info;

int psoam_plan_stats(const psoam_plan* plan, psoam_plan_info* info);

/* Launch only the band-contraction kernel of H (dir 0: writes y) or of
 * S^T H^T (dir 1: writes c) on the padded operand the plan holds from its
 * last apply, on `stream`.  Used to time that kernel alone; its output
 * equals the matching apply's only after that apply ran on the same input. */
int psoam_band_only(const psoam_plan* plan, int32_t dir, float* out, void* stream);

/* What psoam_plan_create_tuned chose and measured. */
typedef struct {
  int32_t h_rows;        /* output rows per workgroup of the staged H kernel (0: not staged) */
  int32_t ht_rows;       /* the same for S^T H^T */
  int32_t ht_shift;      /* sample shift of the 16-bit H^T operand (0 or 4) */
  int32_t candidates;    /* launch shapes timed (0: nothing to tune, or taken from a cache) */
  int32_t from_cache;    /* 1: the choice came from this process's cache, 2: from the disk cache */
  double h_ms, ht_ms;    /* kernel times of the choice (residual form of H; S^T H^T) */
  double h_ms_default, ht_ms_default;  /* the same for the plan's own rules' choice */
  int32_t h_loaders;     /* loader waves beside H's eight contracting waves (0 or 4) */
  int32_t tv_tile[4];    /* tile of the TV dual step: y, x, z extent and threads per block */
  double tv_ms, tv_ms_default;  /* one TV dual step with the chosen / the default tile */
  int32_t fp32_runs[2];  /* FP32 plans: 1 when H (H^T) runs the run-packed kernel, 0 per-tile */
} psoam_tune_report;

/* psoam_plan_create with the launch shapes chosen by measurement: for a
 * 16-bit plan of the general form it builds the plan the built-in rules
 * choose and the alternatives that fit (4, 8 or 12 output rows per workgroup
 * for H, with or without four loader waves at 8 rows; 4, 8 or 12 rows and
 * operand shift 0 or 4 for H^T; 12 rows for one-part operands only), for an
 * FP32 plan the one with the per-tile instead
 * of the run-packed kernel, times each band kernel's solver form on `stream`
 * (HIP events, one warm-up and three timed launches on the zeroed operands),
 * times the TV dual step on the plan's grid with each tile shape of the
 * kernel's list (8x8x32 with 512 threads, 4x8x32/256, 4x16x32/512,
 * 4x8x64/512, 8x8x32/1024; one warm-up and ten steps), and returns the plan
 * with the fastest H, H^T and TV step.  Rows, loader waves and TV tiles do
 * not change results (the same products and sums in the same order);
 * another H^T operand shift or the other FP32 kernel can regroup the band's
 * entries and so the summation order (rounding-level differences).  The
 * choice is cached per process and on disk, keyed by the device
 * (architecture and compute units), the geometry, the precision and a hash
 * of the impulse-response table; the disk cache is the file named by the
 * environment variable PSOAM_TUNE_CACHE (empty: no disk cache), else
 * $HOME/.cache/psoam/tune.txt, one line per choice, appended after each
 * tuning (a file that cannot be read or written is skipped silently).  A
 * call served from a cache only builds the plan.  Separable plans have
 * nothing to tune and are built directly.  For callers who create a plan
 * once and apply it many times: tuning builds up to seven plans (about
 * 0.25 s at 128 x 128 x 64).  `report` may be null.  Errors as
 * psoam_plan_create; synchronises `stream`. */
int psoam_plan_create_tuned(const psoam_geom* g, const psoam_species* sp, const float* phi,
                            const int32_t* sir_t0, const float* sir_taps, int32_t sir_w,
                            int32_t prec, void* stream, psoam_plan** out,
                            psoam_tune_report* report);

/* Message of the last failing call on this thread ("" if none). */
const char* psoam_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PSOAM_H */
