// Internal interface between the host runtime (kstap_api.cpp) and the HIP
// kernels (kstap_device.h and the kstap_kern_*.hip instantiations).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kstap {

constexpr int kMaxP = 8;
constexpr int kMaxQ = 32;
constexpr int kMaxN = 256;
constexpr int kMaxRA = 4;
constexpr int kMaxRB = 8;
constexpr int kMaxDelta = 48;   // training vectors entering (or leaving) on a one-pixel move

// Everything a launch needs, passed by value as the kernel argument
// (about 2.7 KB; the kernarg segment allows 4 KB).
struct KParams {
  const float2* x;        // frame, complex64 [p][H][W][q]
  const uint32_t* xs;     // mixed path: BF16 split of x, hi plane then lo plane, one packed pair per sample
  float* T;               // run: [H][W];  probe: [npix]
  uint8_t* D;             // run: [H][W] or null
  int32_t H, W;
  int32_t n, r_a, r_b;
  int32_t min_iter, max_iter;
  int32_t stat_mode;
  double eps;
  float tau;
  float bs_norm2;         // ||b_s||^2
  float h_norm2;          // ||h||^2
  int32_t r0, r1, c0, c1; // valid region, half-open
  int32_t st_min;         // smallest stencil offset (dr*W + dc)*q, in complex samples
  uint32_t rec_bytes;     // bytes a training-vector buffer record spans from the window origin
  int32_t pix_per_block;  // run: consecutive tiled-order positions per workgroup
  int32_t nlogical;       // run: workgroups that carry pixels (grid is rounded up to 8)
  int64_t range_first;    // persistent: tiled-order position range [range_first, range_end)
  int64_t range_end;
  // probe
  const int32_t* pix;     // [npix][2]
  int32_t npix;
  float2* UA;             // [npix][p][r_a]
  float2* UB;             // [npix][q][r_b]
  float* eta;             // [npix]
  int32_t* iters;         // [npix]
  // statistic variants (run mode outputs beyond T and D)
  int32_t filter;         // 0: Kron-STAP projector (Sec. 5, Eq. (25)); 1: classical joint projector (Eq. (24))
  int32_t nbank;          // 0: the temporal steering b_s; M > 0: the M-bin Doppler bank (Sec. 6.3)
  int32_t passes;         // K registered passes stacked in the p channels (Sec. 3), >= 1
  float* E;               // enhancement image [H][W] or null (Sec. 6.3)
  uint8_t* bin;           // bank bin of the maximum [H][W] or null
  float* Tpass;           // per-pass images [K][H][W] or null (passes > 1)
  float* C;               // change images against pass 0 [K-1][H][W] or null (passes > 1; Sec. 6.4)
  float2 b_s[kMaxQ];
  float2 h_s[kMaxP];
  int16_t st[2 * kMaxN];  // stencil (dr, dc)
  // sliding-window update (run mode): for a one-pixel move m (kMoveRight,
  // kMoveLeft, kMoveDown) from the previous pixel's S, add the nadd[m]
  // vectors dadd[m] and remove the nrem[m] vectors drem[m], offsets relative
  // to the new pixel; nadd[0] < 0: always the full sum
  int32_t nadd[3], nrem[3];
  int16_t dadd[3][2 * kMaxDelta];
  int16_t drem[3][2 * kMaxDelta];
};

static_assert(sizeof(KParams) <= 4096, "KParams is passed as a kernel argument");

// LR-Kron on one large covariance given by its n training snapshots
// (stap_lrkron): snapshots X[n][p][q], outputs A[p][p], B[q][q] (or null),
// stats[4] = eta, iterations, ||R||_F, ||b|| (or null).
struct LrkParams {
  int32_t n, p, q, r_a;
  int32_t min_iter, max_iter;
  double eps;
  float2* A;
  float2* B;
  double* stats;
};
int launch_lrkron(const float2* X, const LrkParams& prm, hipStream_t stream);

// Unstructured low-rank STAP baseline on a pixel list (stap_lrstap_probe):
// per pixel the sample covariance over the plan's stencil, its top-r
// eigenvectors by subspace iteration, and the statistic of the projector
// I - U U^H.
constexpr int kLrsMaxPQ = 64;
constexpr int kLrsMaxR = 8;
struct LrsParams {
  const float2* x;        // frame, complex64 [p][H][W][q]
  int32_t H, W, p, q, n, r;
  int32_t max_iter;
  double tol;
  int32_t r0, r1, c0, c1; // valid region, half-open
  double bs_norm2;
  float2 b_s[kMaxQ];
  int16_t st[2 * kMaxN];
  const int32_t* pix;     // [npix][2]
  int32_t npix;
  float* T;               // [npix]
  float2* U;              // [npix][pq][r] or null
  float* lam;             // [npix][r] or null
  int32_t* iters;         // [npix] or null
};
int launch_lrstap(const LrsParams& prm, hipStream_t stream);

// Output SINR loss of per-pixel filters against a true covariance given in
// factored form (stap_sinr_loss).
struct SinrParams {
  int32_t kind;           // 0: (I - P_A) (x) (I - P_B); 1: I - P_A (x) P_B; 2: I - U U^H
  int32_t p, q, npix;
  int32_t r_a, r_b, r;
  const float2* UA;       // [npix][p][r_a]
  const float2* UB;       // [npix][q][r_b]
  const float2* U;        // [npix][pq][r]
  int32_t ra_t, rb_t;
  const float2* UA_t;     // [p][ra_t], orthonormal columns
  const double* lamA_t;   // [ra_t]
  const float2* UB_t;     // [q][rb_t], orthonormal columns
  const double* lamB_t;   // [rb_t]
  double sigma2, tau2;
  const float2* a_grid;   // [na][p]
  const float2* b_grid;   // [nb][q]
  int32_t na, nb;
  float* loss;            // [npix][na][nb]
};
int launch_sinr(const SinrParams& prm, hipStream_t stream);

enum Mode { kModeRun = 0, kModeProbe = 1 };
enum Move { kMoveRight = 0, kMoveLeft = 1, kMoveDown = 2 };

// Tiled visiting order of a frame's pixels.  The frame is cut into 4 x 4
// pixel units; units are grouped into horizontal stripes 16 units (64 pixels)
// high and, inside a stripe, taken column of units by column of units, top to
// bottom.  Inside a unit the order is a snake: row 0 left to right, row 1
// right to left, and so on, so that every position after a unit's first is a
// one-pixel move (right, left or down) from the one before it.  Position
// pos = 16 * unit + 4 * (row in unit) + k, column k (even rows) or 3 - k (odd
// rows).  A run of consecutive positions therefore covers a compact patch of
// the frame, so the training windows of the workgroups that are in flight on
// one XCD at the same time overlap and their snapshots are served from its L2
// instead of being fetched again.  Positions past the right or bottom edge of
// the frame map to no pixel.
constexpr int kUnit = 4;
constexpr int kStripeUnits = 16;

__host__ __device__ inline int64_t tiled_positions(int H, int W) {
  const int64_t nbr = (H + kUnit - 1) / kUnit, nbc = (W + kUnit - 1) / kUnit;
  return nbr * nbc * (kUnit * kUnit);
}

// Pixel (r, c) at position pos; false if the position lies outside the frame.
__host__ __device__ inline bool tiled_pixel(int64_t pos, int H, int W, int* r, int* c) {
  const int nbr = (H + kUnit - 1) / kUnit, nbc = (W + kUnit - 1) / kUnit;
  const int64_t u = pos / (kUnit * kUnit);
  const int k = int(pos - u * (kUnit * kUnit));
  const int64_t per_stripe = int64_t(kStripeUnits) * nbc;
  const int s = int(u / per_stripe);
  const int within = int(u - int64_t(s) * per_stripe);
  const int rows = (nbr - kStripeUnits * s < kStripeUnits) ? nbr - kStripeUnits * s : kStripeUnits;
  const int cb = within / rows, rb = within - cb * rows;
  const int row = k / kUnit, j = k % kUnit;
  *r = (kStripeUnits * s + rb) * kUnit + row;
  *c = cb * kUnit + ((row & 1) ? kUnit - 1 - j : j);
  return *r < H && *c < W;
}

// Sliding-window chains: every position but a chain's first is a one-pixel
// move from the position before it, so its covariance can be updated from
// that pixel's.  A chain spans one unit for the narrow kernels (16 positions:
// short runs keep many workgroups in flight) and four units down one column
// of units for the wide kernels (64: a wide pixel's full sum costs more).
// Narrow runs of 64 positions take a quarter of the full sums, but the ~256
// workgroups in flight on one XCD then cover four times the pixels, whose
// training windows no longer fit in that XCD's L2: on a 2048 x 2048 p=3 q=16
// frame its misses grew from 2.0 to 28 GB per launch for a 1.5 % shorter run.
// Runs of positions given to a workgroup start on a chain, so the chains, and
// the results, are the same for every decomposition of a frame.
constexpr int kChainNarrow = kUnit * kUnit;
constexpr int kChainWide = 4 * kUnit * kUnit;

// The move that reaches position pos from pos - 1, or -1 if pos starts a chain
// (or follows a unit at the bottom of a column of units).  Inside a unit the
// snake makes every step a move; a unit's first pixel lies directly below the
// previous unit's last one (row 3, column 0) unless the unit starts a column
// of its stripe.
__host__ __device__ inline int tiled_move(int64_t pos, int H, int W, int chain) {
  if (pos % chain == 0) return -1;
  const int k = int(pos % (kUnit * kUnit));
  if (k != 0) {
    if (k % kUnit == 0) return kMoveDown;
    return ((k / kUnit) & 1) ? kMoveLeft : kMoveRight;
  }
  const int nbr = (H + kUnit - 1) / kUnit, nbc = (W + kUnit - 1) / kUnit;
  const int64_t u = pos / (kUnit * kUnit);
  const int64_t per_stripe = int64_t(kStripeUnits) * nbc;
  const int s = int(u / per_stripe);
  const int within = int(u - int64_t(s) * per_stripe);
  const int rows = (nbr - kStripeUnits * s < kStripeUnits) ? nbr - kStripeUnits * s : kStripeUnits;
  return (within % rows == 0) ? -1 : kMoveDown;
}

// One built kernel: (p, q, r_b bound, precision) and its launchers.  The
// tables live in the translation units that instantiate the kernels.
struct Entry {
  int p, q, rbm, prec;
  bool planes;   // reads the split planes of the mixed path (narrow kernels, PREC 1)
  int (*fn)(int mode, const KParams& prm, hipStream_t stream);
  int (*persist)(const KParams* descs, const int32_t* order, const int64_t* prefix, int nt, int ppb,
                 unsigned long long* counter, int grid, hipStream_t stream);   // null: no persistent form
  const void* persist_fn;
};

// Returns true if a kernel is built for (p, q, r_b bound, precision).
bool kernel_available(int p, int q, int r_b, int precision);

// True if that kernel reads the split planes (KParams::xs) of the mixed path:
// 2 * 4 bytes per complex sample of the frame, filled by launch_split.
bool kernel_needs_planes(int p, int q, int r_b, int precision);

// (p, q, r_b bound, precision) of a kernel class; false if out of range.
bool class_shape(int cls, int* p, int* q, int* rbm, int* prec);

// Enqueues the fused per-pixel kernel.  Returns a hipError_t value.
int launch_pixels(int p, int q, int precision, int mode, const KParams& prm, hipStream_t stream);

// Kernel class id of (p, q, r_b, precision), -1 if none is built.
int kernel_class(int p, int q, int r_b, int precision);

// Work queues of a persistent launch: the work items are cut into kQueues
// contiguous ranges, one per XCD; a workgroup takes items from its own XCD's
// range first (so the workgroups in flight on one XCD share training windows
// in its L2), then from the others'.  A launch needs kQueues zeroed counters.
constexpr int kQueues = 8;

// Enqueues the persistent batched kernel of class `cls` over the tiles
// descs[order[j]], j < nt, whose work items (runs of ppb pixels) are numbered
// by prefix[] (device arrays); counter: kQueues device work counters (zero).
int launch_persistent(int cls, const KParams* descs, const int32_t* order, const int64_t* prefix, int nt, int ppb,
                      unsigned long long* counter, int grid, hipStream_t stream);

// Mixed path: for the n complex samples of x writes the packed BF16 pairs
// xs[i] = hi = bf16(x[i]) and xs[n + i] = lo = bf16(x[i] - hi).  Returns a
// hipError_t value.  split_kernel(): its handle (arguments: x, xs, n) for
// explicit graph nodes, launched with split_grid(n) blocks of 256 threads.
int launch_split(const float2* x, uint32_t* xs, int64_t n, hipStream_t stream);
const void* split_kernel();
inline unsigned split_grid(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return unsigned(b < 256 * 32 ? (b > 0 ? b : 1) : 256 * 32);
}

// Zeroes n device counters with a kernel (no memset node in graphs).
int launch_reset(unsigned long long* counters, int n, hipStream_t stream);

// Host handles of the persistent kernel of class `cls` (arguments: descs,
// order, prefix, nt, ppb, counter) and of the counter-reset kernel
// (arguments: counters, n), for explicit graph nodes.
const void* persistent_kernel(int cls);
const void* reset_kernel();

}  // namespace kstap
