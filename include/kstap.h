/*
 * kstap.h - C ABI of the per-pixel Kronecker STAP library for AMD MI355X (gfx950).
 *
 * The library implements, for every pixel of a multichannel SAR frame, the
 * Kron-STAP clutter-cancellation pass of Greenewald, Zelnio & Hero,
 * "Kronecker STAP and SAR GMTI" (SPIE 2016):
 *   - the sample covariance S of the pixel's n training snapshots
 *     (Sec. 1.1, Eq. (2)), with the snapshot vector x = vec(X^T) of Sec. 2;
 *   - the low-rank Kronecker fit S ~ A (x) B by LR-Kron (Sec. 4, Algorithm 2,
 *     on the rearrangement of Algorithm 1), rank(A) <= r_a, and B truncated
 *     to rank r_b once at the end (Sec. 4, relaxation after Eq. (17));
 *   - the Kron-STAP projector F = (I - U_A U_A^H) (x) (I - U_B U_B^H)
 *     (Sec. 5, Eq. (25)) used as the filter w = F d (Eq. (23));
 *   - the normalised output statistic T = max_h |d^H F x|^2 / (d^H F d) over
 *     spatial steerings h with d = h (x) b_s (Sec. 6.3, Eq. (26)), which
 *     equals ||F_A X conj(F_B b_s)||^2 / (b_s^H F_B b_s); and D = (T > tau).
 *
 * Conventions shared by every entry point
 *   - Frames are complex64 (interleaved re, im float pairs) in DEVICE memory,
 *     laid out x[p][H][W][q] (q fastest): channel i, pixel (r, c) owns the q
 *     consecutive azimuth samples x[i][r][c][0..q-1].
 *   - Pixel (r, c) is processed iff every training offset (r+dr, c+dc) of the
 *     stencil lies inside the frame (its "valid region"); elsewhere T = 0 and
 *     D = 0.
 *   - Every call returns a stap_status.  Nothing throws, aborts or exits
 *     across the ABI.  On error, stap_last_error() returns a message
 *     (thread-local, valid until the next call on the same thread).
 *   - Argument checks happen on the host before anything is enqueued.  Calls
 *     that take a `hip_stream` (a hipStream_t, NULL = the default stream) only
 *     enqueue work and return; errors that happen on the device surface at the
 *     caller's next synchronisation.
 *   - Non-finite input samples give T = NaN and D = 0 for the affected pixels;
 *     that is not an error.  An all-zero training set gives T = 0.
 *   - The caller owns every buffer passed in and keeps it alive until the
 *     enqueued work has completed.
 */
#ifndef KSTAP_H_
#define KSTAP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  STAP_OK = 0,
  STAP_ERR_INVALID_ARG = 1,   /* a pointer, size or configuration value is out of range */
  STAP_ERR_UNSUPPORTED = 2,   /* valid, but no kernel is built for this (p, q, precision) */
  STAP_ERR_OUT_OF_MEMORY = 3, /* a host or device allocation failed */
  STAP_ERR_DEVICE = 4,        /* the HIP runtime reported an error */
  STAP_ERR_BUSY = 5,          /* admission refused (serving): retry later */
  STAP_ERR_INTERNAL = 6
} stap_status;

typedef enum {
  STAP_PREC_FP32 = 0,   /* covariance on FP32 MFMA, everything else FP32 (eta terms FP64) */
  STAP_PREC_BF16X3 = 1, /* covariance as three BF16 MFMA products (hi*hi + hi*lo + lo*hi) with
                           FP32 accumulation; eigensolves and normalisation in FP64 */
  STAP_PREC_FP32_FP64 = 2 /* covariance on FP32 MFMA as full sums (no sliding-window update),
                             eigensolves and normalisation in FP64: for frames with point
                             scatterers far above the clutter; built for p = 3, q in {8, 16},
                             r_b <= 4 (other shapes: UNSUPPORTED) */
} stap_precision;

typedef enum {
  STAP_STAT_GLRT = 0,   /* T maximised over the spatial steering h (Sec. 6.3) */
  STAP_STAT_FIXED = 1   /* T for the single spatial steering h_steer */
} stap_stat_mode;

typedef enum {
  STAP_FILTER_KRON = 0,      /* Kron-STAP projector (I - U_A U_A^H) (x) (I - U_B U_B^H), Sec. 5, Eq. (25) */
  STAP_FILTER_CLASSICAL = 1  /* classical joint projector I - U_A U_A^H (x) U_B U_B^H, Sec. 5, Eq. (24) */
} stap_filter;

/* Detector configuration.  Fill with stap_config_default(), then override. */
typedef struct {
  int32_t p;              /* channels, 1 <= p <= 8 */
  int32_t q;              /* azimuth samples per pixel, 2 <= q <= 32, p*q <= 128 */
  int32_t n;              /* training snapshots per pixel, 1 <= n <= 256 */
  const int32_t* stencil; /* host, n (dr, dc) pairs, |dr|,|dc| <= 64, no (0,0), no repeats;
                             NULL = default stencil (below).  Copied by stap_plan_create. */
  int32_t window;         /* default stencil: square window side W (even); 0 = smallest even
                             W >= 10 with W*W - guard*guard >= n */
  int32_t guard;          /* default stencil: odd side of the excluded centre block (3) */
  int32_t r_a;            /* rank of the space factor, 1 <= r_a <= min(p, 4) */
  int32_t r_b;            /* rank of the time factor, 0 <= r_b <= min(q, 8); 0 means F_B = I */
  double eps;             /* LR-Kron stop: |eta_k - eta_{k-1}| <= eps; <= 0: run max_iter */
  int32_t min_iter;       /* >= 1 */
  int32_t max_iter;       /* >= min_iter, <= 1000 */
  int32_t stat_mode;      /* stap_stat_mode */
  const float* b_steer;   /* host, q complex (re, im pairs) temporal steering; NULL = all ones */
  const float* h_steer;   /* host, p complex spatial steering; required for STAP_STAT_FIXED */
  double tau;             /* > 0: threshold used as given; else from pfa */
  double pfa;             /* tau = upper-tail pfa quantile of Gamma(p - r_a, 1), the null law
                             of T under white noise; 0 < pfa < 1 */
  int32_t precision;      /* stap_precision */
  int32_t filter;         /* stap_filter.  The classical filter's statistic,
                             ||F_A X b*||^2/||b||^2 + ||P_A X conj(F_B b)||^2/(b^H F_B b),
                             is Gamma(p, 1) under white noise, so its default tau is
                             that quantile */
  int32_t nbank;          /* 0: the temporal steering b_steer.  1 <= M <= 64: a bank of
                             M Doppler bins b_m[k] = exp(2 pi j ((m k) mod M) / M)
                             (the steering vectors d_i of Sec. 6.3); T is the maximum
                             over the bank (D = T > tau with the single-bin tau) */
  int32_t passes;         /* K >= 1 registered passes stacked into the p channels,
                             pass k in channels k*p/K .. (k+1)*p/K - 1 (Sec. 3); K > 1
                             needs p % K == 0 and the Kron-STAP filter; use r_a = K */
} stap_config;

/* Default stencil: offsets (dr, dc) of the window [-W/2, W/2-1]^2 minus the
 * centred guard x guard block, ordered by (dr^2 + dc^2, dr, dc); the first n
 * are used.  (The paper trains on "representative range bins", Sec. 1.1; the
 * window rule is this library's choice.) */

typedef struct stap_plan_s stap_plan_t;

/* Fills *cfg with defaults: p=3, q=16, n=200, stencil=NULL, window=0,
 * guard=3, r_a=1, r_b=4, eps=1e-6, min_iter=2, max_iter=50, GLRT, b_steer=NULL,
 * h_steer=NULL, tau=0, pfa=1e-4, FP32, Kron-STAP filter, nbank=0, passes=1.
 * Errors: INVALID_ARG if cfg is NULL. */
stap_status stap_config_default(stap_config* cfg);

/* Validates *cfg, builds the stencil, computes tau, and copies every host
 * array.  Host only: no device memory is allocated and nothing is launched,
 * so a plan may be used on any device and from several streams at once.
 * Errors: INVALID_ARG (bad value), UNSUPPORTED (no kernel for p, q, precision),
 * OUT_OF_MEMORY. */
stap_status stap_plan_create(const stap_config* cfg, stap_plan_t** out);

/* The same call under the short name of the stap_plan / stap_run pair. */
stap_status stap_plan(const stap_config* cfg, stap_plan_t** out);

/* Frees a plan (NULL is accepted).  The plan must not be in use by work that
 * is still enqueued. */
stap_status stap_plan_destroy(stap_plan_t* plan);

/* Plan facts: threshold tau, window side, and the stencil extent
 * (min/max dr, min/max dc).  Any output pointer may be NULL. */
stap_status stap_plan_info(const stap_plan_t* plan, double* tau, int32_t* window,
                           int32_t* dr_min, int32_t* dr_max, int32_t* dc_min, int32_t* dc_max);

/* Copies the plan's stencil (n (dr, dc) pairs) into host memory `out`
 * (2*n int32).  Errors: INVALID_ARG. */
stap_status stap_plan_stencil(const stap_plan_t* plan, int32_t* out);

/* Half-open valid region [r0, r1) x [c0, c1) of an H x W frame: the pixels
 * whose whole training stencil (the range bins of Sec. 1.1) lies in the frame; empty
 * (r0 == r1 or c0 == c1) if the stencil does not fit.  Errors: INVALID_ARG. */
stap_status stap_valid_region(const stap_plan_t* plan, int32_t H, int32_t W,
                              int32_t* r0, int32_t* r1, int32_t* c0, int32_t* c1);

/* The order in which stap_run visits an H x W frame (host only; for mapping
 * work ranges to pixels and for checking the sliding-window bookkeeping).
 * For the positions first .. first + count - 1 of the tiled order (4 x 4
 * pixel units in stripes 64 pixels high, a snake inside each unit; the order
 * has ceil(H/4) * ceil(W/4) * 16 positions), writes pix[2i], pix[2i+1] =
 * (r, c), or (-1, -1) for a position past the frame's edge, and move[i] = the
 * one-pixel move (0 right, 1 left, 2 down) from the previous position whose
 * covariance this position's may update, or -1 where a sliding-window chain
 * starts (every 16 positions, every 64 for p*q > 64).  move may be NULL.
 * Errors: INVALID_ARG (NULL, negative sizes, range outside the order). */
stap_status stap_plan_order(const stap_plan_t* plan, int32_t H, int32_t W, int64_t first, int64_t count,
                            int32_t* pix, int32_t* move);

/* Training vectors that enter (add) and leave (rem) the stencil on a
 * one-pixel move (0 right, 1 left, 2 down), as (dr, dc) offsets from the new
 * pixel: the plan's sliding-window update.  *nadd = *nrem = -1 if the plan
 * always takes the full sum (a list would exceed 48 entries).  add / rem
 * (room for 2 * 48 int32 each) may be NULL to query the counts.
 * Errors: INVALID_ARG. */
stap_status stap_plan_moves(const stap_plan_t* plan, int32_t move, int32_t* nadd, int32_t* nrem, int32_t* add,
                            int32_t* rem);

/* Whole-frame pass: for every valid pixel, the sample covariance of Eq. (2)
 * (Sec. 1.1) over the plan's training stencil, LR-Kron (Sec. 4, Algorithm 2,
 * on the rearrangement of Algorithm 1, started from Eqs. (18)-(19)), the
 * rank-r_a / rank-r_b subspaces of the factors, the statistic of Eq. (25)
 * (Sec. 5; Eq. (26) of Sec. 6.3 for the GLRT over h), and D = T > tau.
 * x: device complex64 [p][H][W][q]; T: device float [H][W];
 * D: device uint8 [H][W] or NULL.  Every element of T (and D) is written.
 * 1 <= H, W and p*H*W*q < 2^31.  Enqueued on hip_stream (hipStream_t).
 * Errors: INVALID_ARG, UNSUPPORTED, DEVICE (launch failed). */
stap_status stap_run(const stap_plan_t* plan, const void* x, int32_t H, int32_t W,
                     float* T, uint8_t* D, void* hip_stream);

/* Optional outputs of stap_run_ex beside T and D (device buffers, NULL = not
 * written).  Pixels outside the valid region get 0 in every output; pixels
 * with non-finite data get NaN in the float outputs. */
typedef struct {
  float* T;        /* [H][W], required */
  uint8_t* D;      /* [H][W] */
  float* E;        /* [H][W] enhancement image (Sec. 6.3): T divided by channel 0's SAR
                      intensity |sum_k X[0,k] conj(b_k)|^2 / ||b||^2 at the selected
                      steering; 0 where that intensity is 0 */
  uint8_t* bin;    /* [H][W] Doppler bin of the maximum (first maximiser; 0 without a bank) */
  float* Tpass;    /* [K][H][W] per-pass images (passes K > 1): the energy of pass k's
                      channels of F_A X conj(F_B b), over b^H F_B b (Sec. 3, Sec. 6.4) */
  float* C;        /* [K-1][H][W] non-coherent change images sqrt(Tpass_k) - sqrt(Tpass_0),
                      k = 1..K-1 (Sec. 6.4) */
} stap_outputs;

/* Whole-frame pass with the optional outputs above; otherwise as stap_run.
 * Errors: INVALID_ARG (also Tpass or C requested from a one-pass plan),
 * UNSUPPORTED, DEVICE. */
stap_status stap_run_ex(const stap_plan_t* plan, const void* x, int32_t H, int32_t W,
                        const stap_outputs* out, void* hip_stream);

/* LR-Kron on one large covariance (the single-covariance estimation the
 * paper times, Sec. 6.1: a few training snapshots, many azimuth samples).
 * Algorithm 2 (Sec. 4) with the stop rule of the plan configuration, on the
 * rearrangement (Algorithm 1) of S = (1/n) sum_m x_m x_m^H, x_m = vec(X_m^T)
 * (Eq. (2)); the time factor is not truncated (r_b = q, as in the timing
 * experiment).  S and R are never formed: R(S) = (1/n) sum_m conj(X_m) (x) X_m,
 * so each iteration works on the n^2 Gram blocks X_m X_m'^H.
 *   X     device complex64 [n][p][q] (snapshot m, channel i, sample k)
 *   A     device complex64 [p][p], row-major: the final space factor A-hat
 *   B     device complex64 [q][q], row-major, or NULL: the final time factor
 *         B-hat = vec^-1(R^T conj(a) / ||a||^2)
 *   stats device double [4], or NULL: eta, iterations, ||R||_F, ||b||
 * Limits: 1 <= p <= 8, 2 <= q <= 16384, n >= 1, n * p <= 64, 1 <= r_a <= p.
 * Allocates nothing; enqueued on hip_stream.
 * Errors: INVALID_ARG, DEVICE. */
typedef struct {
  int32_t n, p, q, r_a;
  double eps;
  int32_t min_iter, max_iter;
} stap_lrk_config;

stap_status stap_lrkron(const stap_lrk_config* cfg, const void* X, float* A, float* B, double* stats,
                        void* hip_stream);

/* Size of the static work area of stap_run_noalloc, per device (bytes). */
#define STAP_NOALLOC_MAX_BYTES (128u << 20)

/* stap_run for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same whole-frame pass with the same arguments, results and errors, but the
 * call allocates nothing.  The mixed path's split planes (8 bytes per complex
 * sample of x) go to a static work area of STAP_NOALLOC_MAX_BYTES that each
 * device holds from the library's first use on it until the process ends
 * (FP32 plans need no work area).  A frame whose planes exceed it is refused
 * with INVALID_ARG before anything is enqueued.  Every call on one device
 * shares that device's area and it keeps the last call's contents: calls that
 * overlap on one device (concurrent streams, or host threads without
 * ordering) race and must be serialised by the caller; calls on one stream
 * are ordered.  Errors: INVALID_ARG, UNSUPPORTED, DEVICE. */
stap_status stap_run_noalloc(const stap_plan_t* plan, const void* x, int32_t H, int32_t W,
                             float* T, uint8_t* D, void* hip_stream);

/* Per-pixel probe: the same computation for a list of pixels, with the
 * intermediate results (the subspaces of the LR-Kron factors of Sec. 4,
 * Algorithm 2, its residual eta and iteration count, and Eq. (25)'s T).  All pointers are device memory:
 *   pix   int32 [npix][2] (r, c)   (pixels outside the valid region get T = 0,
 *                                   eta = 0, iters = 0, zero bases)
 *   UA    complex64 [npix][p][r_a]  orthonormal basis of the space subspace
 *   UB    complex64 [npix][q][r_b]  orthonormal basis of the time subspace
 *   eta   float [npix]              last LR-Kron relative residual
 *   iters int32 [npix]              LR-Kron iterations run
 *   T     float [npix]
 * Any of UA, UB, eta, iters may be NULL.  Plans with a statistic variant
 * (classical filter, Doppler bank, several passes) are refused with
 * UNSUPPORTED.  Errors: INVALID_ARG, UNSUPPORTED, DEVICE. */
typedef struct {
  float* UA;
  float* UB;
  float* eta;
  int32_t* iters;
  float* T;
} stap_probe_out;

stap_status stap_probe(const stap_plan_t* plan, const void* x, int32_t H, int32_t W,
                       const int32_t* pix, int32_t npix, const stap_probe_out* out,
                       void* hip_stream);

/* Unstructured low-rank STAP baseline (LR-STAP), the classical method the
 * Kronecker filters are compared with (Sec. 1; its filter is the
 * unstructured counterpart of the joint projector of Eq. (24)): per pixel of
 * a list, the sample covariance S of Eq. (2) over the plan's training
 * stencil, the eigenvectors U of its r largest eigenvalues, the filter
 * F = I - U U^H and the statistic max over spatial steerings h of
 * |d^H F x|^2 / (d^H F d), d = h (x) b_s, with the plan's temporal steering
 * (the pseudo-inverse form: eigenvalues of E^H F E at or below
 * 1e-12 ||b_s||^2 dropped).  Under white noise the statistic is Gamma(p, 1).
 *   r         rank; < 0: r_a * r_b of the plan (the rank of A (x) B);
 *             0 <= r <= min(8, p q)
 *   max_iter  subspace iterations (each: S times the p q x r basis, then
 *             Gram-Schmidt twice), >= 1; 0: 300
 *   tol       stop when the squared sines of the principal angles between
 *             successive bases sum to at most tol^2; <= 0: 1e-7
 * S is summed in FP32, the iteration, the Rayleigh-Ritz ordering of U and
 * the statistic run in FP64.  All pointers are device memory:
 *   pix   int32 [npix][2] (r, c)   (pixels outside the valid region get
 *                                   T = 0, zero U and lam, iters = 0)
 *   T     float [npix]
 *   U     complex64 [npix][p q][r], columns ordered by decreasing eigenvalue,
 *         rows in the vec(X^T) order (index i q + k), or NULL
 *   lam   float [npix][r]: the Rayleigh-Ritz eigenvalues, decreasing, or NULL
 *   iters int32 [npix]: iterations run (max_iter when not converged), or NULL
 * Limits: p q <= 64, the plan's single temporal steering and GLRT statistic
 * (plans with the fixed-steering statistic, a Doppler bank or several
 * passes are refused with UNSUPPORTED).  Enqueued on hip_stream; allocates
 * nothing.  Errors: INVALID_ARG, UNSUPPORTED, DEVICE. */
typedef struct {
  int32_t r;
  int32_t max_iter;
  double tol;
} stap_lrstap_config;

stap_status stap_lrstap_probe(const stap_plan_t* plan, const stap_lrstap_config* cfg, const void* x,
                              int32_t H, int32_t W, const int32_t* pix, int32_t npix, float* T, float* U,
                              float* lam, int32_t* iters, void* hip_stream);

/* Output SINR loss of per-pixel filters (Sec. 5): for filter F and target
 * steering d, SINR_out = |w^H d|^2 / (w^H Sigma w) with w = F d (Eqs. (21),
 * (23), |alpha| = 1), divided by the optimum d^H Sigma^-1 d reached by
 * F = Sigma^-1 (Eq. (22)); the loss lies in [0, 1] and is 0 where w = 0.
 * The true clutter-plus-noise covariance of the SIRV model (Eqs. (5), (9))
 * is Sigma = tau2 A (x) B + sigma2 I with A = UA diag(lamA) UA^H and
 * B = UB diag(lamB) UB^H; UA and UB must have orthonormal columns (the
 * optimum uses the Woodbury identity on that basis).  Steerings are all
 * pairs d = a (x) b of a_grid [na][p] and b_grid [nb][q].
 * Filters per pixel: KRON (I - P_A) (x) (I - P_B) (Eq. (25)) and CLASSICAL
 * I - P_A (x) P_B (Eq. (24)) from bases UA [npix][p][r_a] and
 * UB [npix][q][r_b] (as stap_probe writes them); LRSTAP I - U U^H from
 * U [npix][p q][r] (as stap_lrstap_probe writes it).  All arrays are device
 * memory, complex64 interleaved except lamA and lamB (double); output
 * loss float [npix][na][nb].  Limits: 1 <= p <= 8, p q <= 64, sigma2 > 0,
 * tau2 >= 0.  Allocates nothing.  Errors: INVALID_ARG, DEVICE. */
typedef enum { STAP_SINR_KRON = 0, STAP_SINR_CLASSICAL = 1, STAP_SINR_LRSTAP = 2 } stap_sinr_filter;

typedef struct {
  int32_t p, q;
  int32_t ra, rb;
  const float* UA;
  const double* lamA;
  const float* UB;
  const double* lamB;
  double sigma2, tau2;
} stap_true_cov;

typedef struct {
  int32_t filter;   /* stap_sinr_filter */
  int32_t npix;
  int32_t r_a, r_b, r;
  const float* UA;
  const float* UB;
  const float* U;
} stap_filter_set;

stap_status stap_sinr_loss(const stap_true_cov* cov, const stap_filter_set* filters, const float* a_grid,
                           int32_t na, const float* b_grid, int32_t nb, float* loss, void* hip_stream);

/* Batched uneven tiles (tiles may differ in p, q, n, ranks, steering,
 * precision and size; each has its own plan, frame and outputs).  Every tile
 * gets stap_run's per-pixel computation: Eq. (2) of Sec. 1.1, Algorithm 2 of
 * Sec. 4 and Eq. (25) of Sec. 5.
 *
 * stap_batch_create validates every tile, uploads a tile table to device
 * memory it owns, numbers the work items (runs of `pix_per_item` consecutive
 * positions of one tile's tiled pixel order, rounded up to a multiple of 16)
 * longest tile first within each kernel class, and
 * builds one HIP graph: a counter-reset kernel node followed, as parallel
 * branches, by one persistent kernel node per kernel class present; every
 * workgroup of a persistent kernel pops work items from a device counter until
 * the queue is empty.  pix_per_item = 0 takes, per kernel class, the tuned
 * entry of the tuning cache for the current device (else 16 positions and a
 * grid of compute units x 8); pix_per_item > 0 applies to every class.  Results are bitwise equal to
 * stap_run on each tile alone.  The frames and outputs named by the tiles must
 * stay valid while the batch is launched.  Must be called with the device that
 * will run the batch current.  Tiles whose plan has a statistic variant
 * (classical filter, Doppler bank, several passes) are refused with
 * UNSUPPORTED (those run through stap_run_ex).
 * Errors: INVALID_ARG, UNSUPPORTED, OUT_OF_MEMORY, DEVICE. */
typedef struct {
  const stap_plan_t* plan;
  const void* x;
  int32_t H, W;
  float* T;
  uint8_t* D;
} stap_tile;

typedef struct stap_batch_s stap_batch_t;

stap_status stap_batch_create(const stap_tile* tiles, int32_t ntiles, int32_t pix_per_item, stap_batch_t** out);

/* One hipGraphLaunch of the captured graph on hip_stream (asynchronous). */
stap_status stap_batch_launch(stap_batch_t* batch, void* hip_stream);

/* Autotuner: for every kernel class of the batch, alone, times (synchronously,
 * on hip_stream, with direct launches) work items of {16, 32, 64, 128}
 * positions and persistent grids of {1, 2, 4} x (compute units x 8)
 * workgroups, keeps each class's fastest, rebuilds the graph, and records the
 * choices in the tuning cache (stap_tune_record) keyed by (device
 * architecture, p, q, r_b bound, precision).  best_ppb / best_grid_mult
 * report the slowest class's choice, best_ms the sum of the classes' times;
 * any may be NULL. */
stap_status stap_batch_tune(stap_batch_t* batch, void* hip_stream, int32_t* best_ppb, int32_t* best_grid_mult,
                            double* best_ms);

/* Kernel class `cls` (0 .. classes-1) of a batch: its p, q, r_b bound (4 or
 * 8), precision, work-item size and grid multiplier.  Any output may be NULL.
 * Errors: INVALID_ARG. */
stap_status stap_batch_class_info(const stap_batch_t* batch, int32_t cls, int32_t* p, int32_t* q,
                                  int32_t* rb_bound, int32_t* precision, int32_t* pix_per_item,
                                  int32_t* grid_mult);

/* The tuning cache (host only).  Entries are keyed by (architecture, p, q,
 * r_b bound, precision), with r_b mapped to its bound (<= 4 -> 4, else 8).
 * When the environment variable KSTAP_TUNE_CACHE names a file, the cache is
 * read from it (again whenever it changes) and every recorded entry rewrites
 * it (JSON, written to a temporary file and renamed), so tuned choices carry
 * over to later processes; stap_batch_create with pix_per_item = 0 takes each
 * class's entry for the current device.  arch = NULL means the current
 * device's architecture (e.g. "gfx950").
 * stap_tune_lookup: *found = 1 and the entry, or *found = 0 and the defaults
 *   (16, 1).  Errors: INVALID_ARG (found is NULL).
 * stap_tune_record: pix_per_item a multiple of 16 in [16, 4096], grid_mult
 *   in [1, 64]; ms is informative.  Errors: INVALID_ARG (also: the file
 *   cannot be written). */
stap_status stap_tune_lookup(const char* arch, int32_t p, int32_t q, int32_t r_b, int32_t precision,
                             int32_t* pix_per_item, int32_t* grid_mult, int32_t* found);
stap_status stap_tune_record(const char* arch, int32_t p, int32_t q, int32_t r_b, int32_t precision,
                             int32_t pix_per_item, int32_t grid_mult, double ms);

/* Batch facts: total pixels, kernel classes present, and the first class's
 * work-item size and grid multiplier (every class's: stap_batch_class_info).
 * Any output pointer may be NULL. */
stap_status stap_batch_info(const stap_batch_t* batch, int64_t* pixels, int32_t* classes, int32_t* pix_per_item,
                            int32_t* grid_mult);

/* Frees the batch and its device memory; waits for nothing (launched work
 * must have completed).  NULL is accepted. */
stap_status stap_batch_destroy(stap_batch_t* batch);

/* One-shot form: create, launch on hip_stream, synchronise hip_stream,
 * destroy. */
stap_status stap_run_batch(const stap_tile* tiles, int32_t ntiles, void* hip_stream);

/* Serving with continuous batching: frames arriving over time get
 * stap_run's per-pixel computation (Eq. (2) of Sec. 1.1, Algorithm 2 of
 * Sec. 4, Eq. (25) of Sec. 5).
 *
 * A server owns an HBM arena of hbm_budget_bytes (allocated on the current
 * device at creation), a copy stream, a compute stream and a worker thread.
 * Frames are admitted in arrival order as soon as their device buffers
 * (input unless x_on_device, T, D) fit in the arena and fewer than
 * max_inflight frames are active; their host-to-device copies overlap the
 * running computation.  Each scheduling step processes a fair-share slice of
 * every active frame, about step_pixels pixels in total (0 = 2^20), in one
 * persistent launch per kernel class, so frames that arrive while others are
 * on the GPU join at the next step.  Results are bitwise equal to stap_run on
 * the frame alone.  Host frames in pinned memory give asynchronous copies.
 * Errors of create: INVALID_ARG, OUT_OF_MEMORY, DEVICE. */
typedef struct stap_server_s stap_server_t;

stap_status stap_server_create(size_t hbm_budget_bytes, int32_t max_inflight, int64_t step_pixels,
                               stap_server_t** out);

/* Queues one frame.  x: complex64 [p][H][W][q], host memory (or device memory
 * if x_on_device != 0); T_host: float [H][W] and D_host: uint8 [H][W] (or
 * NULL), host memory written when the frame completes.  x, T_host and D_host
 * must stay valid until stap_server_wait returns for the ticket.  For a
 * device-resident x, hip_stream is the stream whose work produces x: the
 * call records an event on it and the server reads x only after the work
 * enqueued there before the call (NULL = the default stream); host frames
 * ignore it and must be complete at the call.  Returns at once with a
 * ticket.  Plans with a statistic variant are refused with UNSUPPORTED.
 * Errors: INVALID_ARG, UNSUPPORTED, BUSY (the frame can never fit in the
 * budget), DEVICE. */
stap_status stap_server_submit(stap_server_t* server, const stap_plan_t* plan, const void* x, int32_t H, int32_t W,
                               int32_t x_on_device, float* T_host, uint8_t* D_host, void* hip_stream,
                               uint64_t* ticket);

/* Waits until the frame's results are in T_host / D_host (timeout_ms < 0:
 * no limit) and releases the ticket.  latency_s: submit to results in host
 * memory.  Errors: INVALID_ARG (unknown ticket), BUSY (timed out; the ticket
 * stays valid), DEVICE (the frame failed). */
stap_status stap_server_wait(stap_server_t* server, uint64_t ticket, int32_t timeout_ms, double* latency_s);

/* Latency percentiles of the frames completed so far, and completed pixels
 * per second between the first submission and the last completion. */
stap_status stap_server_stats(stap_server_t* server, double* p50_s, double* p99_s, double* pixels_per_s,
                              int64_t* frames_done);

/* Finishes every queued frame, then frees the server.  Tickets not yet waited
 * for are released.  NULL is accepted. */
stap_status stap_server_destroy(stap_server_t* server);

/* Library version string and the HIP device architecture the code object
 * was built for. */
const char* stap_version(void);

/* Thread-local text of the last error on this thread ("" if none). */
const char* stap_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* KSTAP_H_ */
