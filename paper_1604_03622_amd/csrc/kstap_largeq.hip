// LR-Kron on one large covariance (Sec. 6.1: p channels, q up to thousands of
// azimuth samples, a few training snapshots), without forming S or R.
//
// For S = (1/n) sum_m x_m x_m^H with x_m = vec(X_m^T) (Eq. (2)), Algorithm 1
// maps every rank-one term to a Kronecker product of the snapshot with its
// conjugate: R(x_m x_m^H)[a p + b][l q + k] = conj(X_m[a][l]) X_m[b][k], so
// R(S) = (1/n) sum_m conj(X_m) (x) X_m.  Both half-steps of Algorithm 2 then
// reduce to p x p algebra on the n^2 Gram blocks G_mm' = X_m X_m'^H:
//   B = c sum_m X_m^T conj(A) conj(X_m),  c = 1 / (n ||A||^2)
//   R conj(b) = c sum_{m,m'} G_m'm A G_mm'
//   ||b||^2 = c^2 Re sum_{m,m'} tr(A G_mm' A G_m'm)
//   ||R||^2 = (1/n^2) sum_{m,m'} |tr G_m'm|^2
// and eta follows from ||R - a b^T||^2 = ||R||^2 - 2 Re(a^H R conj(b)) +
// ||a||^2 ||b||^2.  The only q^2-sized work is writing the final time factor
// B-hat, a rank-np product (kernel lrk_emit_b).
//
// lrk_solve: one workgroup.  All eight waves accumulate the Gram matrix of the
// n p snapshot rows (FP64 sums of FP32 products, in LDS) and the row sums that
// give the initialiser of Eq. (18); wave 0 then runs the iterations in FP64
// with its lanes over (m, m') pairs and EIG_{r_a} by cyclic Jacobi rotations
// (lane k updates row and column k), with no workgroup barrier.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kstap_internal.h"

namespace kstap {
namespace {

constexpr int kLrkMaxRows = 64;   // n * p
constexpr int kLrkMaxP = 8;

struct dc {
  double x, y;
};
__device__ __forceinline__ dc mk(double x, double y) { return dc{x, y}; }
__device__ __forceinline__ dc add(dc a, dc b) { return mk(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ dc sub(dc a, dc b) { return mk(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ dc mul(dc a, dc b) { return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ dc cj(dc a) { return mk(a.x, -a.y); }
__device__ __forceinline__ dc scl(dc a, double s) { return mk(a.x * s, a.y * s); }
__device__ __forceinline__ double ab2(dc a) { return a.x * a.x + a.y * a.y; }

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Wave-local LDS exchange: a wavefront's LDS operations complete in issue
// order, so only the compiler has to be kept from moving accesses across.
__device__ __forceinline__ void lane_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Eigen-decomposition of the Hermitian p x p matrix H (LDS, overwritten) by
// cyclic Jacobi rotations, run by one wavefront with lane k < p updating row
// and column k; V (LDS) receives the eigenvectors as columns, lam (LDS) the
// eigenvalues (unsorted).  Each rotation U = D [c s; -s c] on the pair (a, b),
// D = diag(1, e^{-i phi}) making H[a][b] real, zeroes H[a][b]: H <- U^H H U.
__device__ void jacobi_herm(dc* H, dc* V, double* lam, int p, int lane) {
  if (lane < p)
    for (int j = 0; j < p; ++j) V[lane * p + j] = mk(lane == j ? 1.0 : 0.0, 0.0);
  lane_sync();
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0, tot = 0;
    for (int i = 0; i < p; ++i)
      for (int j = 0; j < p; ++j) {
        tot += ab2(H[i * p + j]);
        if (i != j) off += ab2(H[i * p + j]);
      }
    if (off <= 1e-30 * tot) break;   // uniform: every lane reads the same LDS values
    for (int a = 0; a < p - 1; ++a)
      for (int b = a + 1; b < p; ++b) {
        const dc hab = H[a * p + b];
        const double r = sqrt(ab2(hab));
        if (r <= 1e-300 * sqrt(tot)) continue;
        const dc e = scl(hab, 1.0 / r);   // e^{i phi}
        const double tau = (H[b * p + b].x - H[a * p + a].x) / (2.0 * r);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + t * t), sn = t * c;
        const dc ec = cj(e);
        lane_sync();
        if (lane < p) {   // columns: H <- H U, V <- V U
          const int k = lane;
          const dc ha = H[k * p + a], hb = H[k * p + b];
          H[k * p + a] = sub(scl(ha, c), scl(mul(ec, hb), sn));
          H[k * p + b] = add(scl(ha, sn), scl(mul(ec, hb), c));
          const dc va = V[k * p + a], vb = V[k * p + b];
          V[k * p + a] = sub(scl(va, c), scl(mul(ec, vb), sn));
          V[k * p + b] = add(scl(va, sn), scl(mul(ec, vb), c));
        }
        lane_sync();
        if (lane < p) {   // rows: H <- U^H H
          const int k = lane;
          const dc ha = H[a * p + k], hb = H[b * p + k];
          H[a * p + k] = sub(scl(ha, c), scl(mul(e, hb), sn));
          H[b * p + k] = add(scl(ha, sn), scl(mul(e, hb), c));
        }
        lane_sync();
        if (lane == 0) {
          H[a * p + b] = mk(0, 0);
          H[b * p + a] = mk(0, 0);
          H[a * p + a].y = 0;
          H[b * p + b].y = 0;
        }
        lane_sync();
      }
  }
  if (lane < p) lam[lane] = H[lane * p + lane].x;
  lane_sync();
}

constexpr int kSolveThreads = 512;
constexpr int kSolveWaves = kSolveThreads / 64;
constexpr int kChunk = 128;   // samples per staged chunk (64 rows x 128 x 8 bytes = 64 KB)

// P: channels, a compile-time constant so that the p x p matrices of the
// iteration live in registers.
template <int P>
__global__ __launch_bounds__(kSolveThreads) void lrk_solve(const float2* __restrict__ X, LrkParams prm) {
  constexpr int p = P;
  const int n = prm.n, q = prm.q, np = n * p;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  __shared__ dc sG[kLrkMaxRows * kLrkMaxRows];   // Gram of the snapshot rows
  __shared__ dc sRow[kLrkMaxRows];               // row sums
  __shared__ dc sA[kLrkMaxP * kLrkMaxP], sAp[kLrkMaxP * kLrkMaxP];
  __shared__ dc sH[kLrkMaxP * kLrkMaxP], sV[kLrkMaxP * kLrkMaxP], sM[kLrkMaxP * kLrkMaxP];
  __shared__ double sLam[kLrkMaxP];
  __shared__ float2 sX[kLrkMaxRows * kChunk];    // staged samples of every snapshot row

  // ---- Gram matrix (upper triangle) and row sums, FP64 sums of FP32 products.
  // The snapshot rows are staged through LDS in chunks of kChunk samples
  // (coalesced loads by the whole workgroup); entry e of the Gram (or a row
  // sum) belongs to wave e % 8, whose lanes split the chunk's samples and add
  // the chunk's sum into the LDS entry.
  const int ntri = np * (np + 1) / 2, nent = ntri + np;
  for (int e = tid; e < np * np; e += kSolveThreads) sG[e] = mk(0, 0);
  for (int e = tid; e < np; e += kSolveThreads) sRow[e] = mk(0, 0);
  for (int k0 = 0; k0 < q; k0 += kChunk) {
    const int len = min(kChunk, q - k0);
    __syncthreads();   // the previous chunk is consumed (and the sums above zeroed)
    for (int e = tid; e < np * kChunk; e += kSolveThreads) {
      const int u = e / kChunk, k = e - (e / kChunk) * kChunk;
      sX[u * kChunk + k] = (k < len) ? X[int64_t(u) * q + k0 + k] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    for (int e = wave; e < nent; e += kSolveWaves) {
      int u, v;
      const bool rowsum = e >= ntri;
      if (rowsum) {
        u = v = e - ntri;
      } else {
        // e -> (u, v), u <= v, row-major over the upper triangle
        u = 0;
        int rem = e;
        while (rem >= np - u) {
          rem -= np - u;
          ++u;
        }
        v = u + rem;
      }
      double sr = 0, si = 0;
      for (int k = lane; k < len; k += 64) {
        const float2 a = sX[u * kChunk + k];
        if (rowsum) {
          sr += double(a.x);
          si += double(a.y);
        } else {
          const float2 b = sX[v * kChunk + k];   // a * conj(b)
          sr += double(a.x) * double(b.x) + double(a.y) * double(b.y);
          si += double(a.y) * double(b.x) - double(a.x) * double(b.y);
        }
      }
      sr = wave_sum(sr);
      si = wave_sum(si);
      if (lane == 0) {   // one writer per entry
        if (rowsum) {
          sRow[u] = add(sRow[u], mk(sr, si));
        } else {
          sG[u * np + v] = add(sG[u * np + v], mk(sr, si));
          if (v != u) sG[v * np + u] = add(sG[v * np + u], mk(sr, -si));
        }
      }
    }
  }
  __syncthreads();
  // ---- the iterations: wave 0 alone, lanes over (m, m') pairs
  if (wave != 0) return;

  auto G = [&](int m, int mm, int i, int j) -> dc { return sG[(m * p + i) * np + mm * p + j]; };
  const int npair = n * n;

  // ||R||^2 = ||S||^2 = (1/n^2) sum_{m,m'} |tr G_m'm|^2
  double nr = 0;
  for (int t = lane; t < npair; t += 64) {
    const int m = t / n, mm = t - (t / n) * n;
    dc tr = mk(0, 0);
    for (int i = 0; i < p; ++i) tr = add(tr, G(mm, m, i, i));
    nr += ab2(tr);
  }
  const double normR2 = wave_sum(nr) / (double(n) * n);

  // initialiser (Eq. (18)): A0 = (1/(n q^2)) sum_m s_m s_m^H, s_m the row sums;
  // fallback R vec(I_q) = (1/n) sum_m G_mm when ||A0|| is negligible.
  // Lane e < p^2 holds entry (e / p, e % p).
  {
    double an = 0;
    if (lane < p * p) {
      const int i = lane / p, j = lane - (lane / p) * p;
      dc s = mk(0, 0);
      for (int m = 0; m < n; ++m) s = add(s, mul(sRow[m * p + i], cj(sRow[m * p + j])));
      sA[lane] = scl(s, 1.0 / (double(n) * q * q));
      an = ab2(sA[lane]);
    }
    an = wave_sum(an);
    if (an <= 1e-24 * normR2 && lane < p * p) {
      const int i = lane / p, j = lane - (lane / p) * p;
      dc s = mk(0, 0);
      for (int m = 0; m < n; ++m) s = add(s, G(m, m, i, j));
      sA[lane] = scl(s, 1.0 / n);
    }
    lane_sync();
  }

  double eta = 0, eta_prev = INFINITY, bn2 = 0;
  int iters = 0;
  const bool zero = !(normR2 > 0.0);
  while (!zero) {
    double an2 = 0;
    for (int e = 0; e < P * P; ++e) an2 += ab2(sA[e]);
    const double c = 1.0 / (double(n) * an2);
    // M = sum G_m'm A G_mm' and tb = Re sum tr(A G_mm' A G_m'm), one row i of
    // M at a time: each lane accumulates its pairs' contributions to row i,
    // the row is summed over the wave into LDS (few live registers at any P)
    double tb = 0;
    for (int i = 0; i < P; ++i) {
      dc out[P];
#pragma unroll
      for (int j = 0; j < P; ++j) out[j] = mk(0, 0);
      for (int t = lane; t < npair; t += 64) {
        const int m = t / n, mm = t - (t / n) * n;
        dc r1[P];   // row i of G_m'm A
#pragma unroll
        for (int k = 0; k < P; ++k) {
          dc s = mk(0, 0);
#pragma unroll
          for (int l = 0; l < P; ++l) s = add(s, mul(G(mm, m, i, l), sA[l * P + k]));
          r1[k] = s;
        }
#pragma unroll
        for (int j = 0; j < P; ++j) {
          dc s = mk(0, 0);
#pragma unroll
          for (int k = 0; k < P; ++k) s = add(s, mul(r1[k], G(m, mm, k, j)));
          out[j] = add(out[j], s);
        }
        // row i of A G_mm' against column i of A G_m'm
#pragma unroll
        for (int j = 0; j < P; ++j) {
          dc t2 = mk(0, 0), t3 = mk(0, 0);
#pragma unroll
          for (int k = 0; k < P; ++k) {
            t2 = add(t2, mul(sA[i * P + k], G(m, mm, k, j)));
            t3 = add(t3, mul(sA[j * P + k], G(mm, m, k, i)));
          }
          tb += mul(t2, t3).x;
        }
      }
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const dc v = mk(wave_sum(out[j].x), wave_sum(out[j].y));
        if (lane == 0) sM[i * P + j] = v;
      }
    }
    tb = wave_sum(tb);
    lane_sync();
    bn2 = c * c * tb;                           // ||b||^2
    const double sa = c / (double(n) * bn2);    // A' = R conj(b) / ||b||^2 = sa M
    // EIG_{r_a} of the Hermitian part of A'
    if (lane < p * p) {
      const int i = lane / p, j = lane - (lane / p) * p;
      sAp[lane] = scl(sM[lane], sa);
      sH[lane] = scl(add(scl(sM[i * p + j], sa), cj(scl(sM[j * p + i], sa))), 0.5);
    }
    lane_sync();
    jacobi_herm(sH, sV, sLam, p, lane);
    // the r_a largest algebraic eigenvalues (uniform selection on every lane)
    dc anew = mk(0, 0);
    {
      unsigned used = 0;
      const int i = lane / p, j = lane - (lane / p) * p;
      for (int r = 0; r < prm.r_a; ++r) {
        int best = -1;
        for (int k = 0; k < p; ++k)
          if (!((used >> k) & 1u) && (best < 0 || sLam[k] > sLam[best])) best = k;
        used |= 1u << best;
        if (lane < p * p) anew = add(anew, scl(mul(sV[i * p + best], cj(sV[j * p + best])), sLam[best]));
      }
    }
    lane_sync();
    double na = 0, cross = 0;
    if (lane < p * p) {
      sA[lane] = anew;
      na = ab2(anew);
      cross = mul(cj(anew), sAp[lane]).x;
    }
    na = wave_sum(na);
    cross = wave_sum(cross);
    lane_sync();
    ++iters;
    // eta^2 = (||R||^2 - 2 ||b||^2 Re<A, A'> + ||A||^2 ||b||^2) / ||R||^2
    const double r2 = normR2 - 2.0 * bn2 * cross + na * bn2;
    const double e = sqrt(fmax(r2, 0.0) / normR2);
    eta = e;
    const bool stop =
        iters >= prm.max_iter || (prm.eps > 0.0 && iters >= prm.min_iter && fabs(e - eta_prev) <= prm.eps);
    if (stop) break;
    eta_prev = e;
  }
  if (lane < p * p) prm.A[lane] = zero ? make_float2(0.f, 0.f) : make_float2(float(sA[lane].x), float(sA[lane].y));
  if (lane == 0 && prm.stats) {
    prm.stats[0] = zero ? 0.0 : eta;
    prm.stats[1] = double(iters);
    prm.stats[2] = sqrt(normR2);
    prm.stats[3] = zero ? 0.0 : sqrt(bn2);
  }
}

// Final time factor B-hat[k][l] = c sum_{m, j} W_m[k][j] conj(X_m[j][l]) with
// W_m = X_m^T conj(A) (q x p) and c = 1 / (n ||A||^2): a rank-np product,
// bound by writing q^2 complex values.  64 x 64 outputs per 256-thread block,
// each thread 4 rows x 4 columns (columns strided by 16 so that each store
// instruction writes 16 consecutive entries per row).  The LDS operands are
// sized for the actual n p (dynamic shared memory), so that many blocks share
// a compute unit and keep enough stores in flight.
constexpr int kTile = 64;
__global__ __launch_bounds__(256) void lrk_emit_b(const float2* __restrict__ X, LrkParams prm) {
  const int n = prm.n, p = prm.p, q = prm.q, np = n * p;
  extern __shared__ float2 dyn[];
  float2* const sW = dyn;                        // [kTile][np + 1]: W for the tile's rows k
  float2* const sXc = dyn + kTile * (np + 1);    // [np][kTile + 1]: conj(X) for the tile's columns l
  __shared__ float2 sAc[kLrkMaxP * kLrkMaxP];
  __shared__ float sC;
  const int tid = threadIdx.x;
  const int k0 = blockIdx.y * kTile, l0 = blockIdx.x * kTile;
  if (tid < p * p) sAc[tid] = make_float2(prm.A[tid].x, -prm.A[tid].y);   // conj(A)
  if (tid == 0) {
    float an = 0.f;
    for (int e = 0; e < p * p; ++e) an += prm.A[e].x * prm.A[e].x + prm.A[e].y * prm.A[e].y;
    sC = an > 0.f ? 1.f / (float(n) * an) : 0.f;
  }
  // conj(X) rows for the tile's columns (coalesced over l)
  for (int e = tid; e < np * kTile; e += 256) {
    const int u = e / kTile, ll = e - (e / kTile) * kTile;
    const int l = l0 + ll;
    const float2 x = (l < q) ? X[int64_t(u) * q + l] : make_float2(0.f, 0.f);
    sXc[u * (kTile + 1) + ll] = make_float2(x.x, -x.y);
  }
  __syncthreads();
  // W[k][(m, j)] = sum_i X_m[i][k] conj(A)[i][j], consecutive threads over k
  for (int e = tid; e < kTile * np; e += 256) {
    const int u = e / kTile, kk = e - (e / kTile) * kTile;
    const int m = u / p, j = u - (u / p) * p;
    const int k = k0 + kk;
    float2 sum = make_float2(0.f, 0.f);
    if (k < q) {
      for (int i = 0; i < p; ++i) {
        const float2 x = X[(int64_t(m) * p + i) * q + k];
        const float2 a = sAc[i * p + j];
        sum.x += x.x * a.x - x.y * a.y;
        sum.y += x.x * a.y + x.y * a.x;
      }
    }
    sW[kk * (np + 1) + u] = sum;
  }
  __syncthreads();
  const int tx = tid & 15, ty = tid >> 4;   // columns tx + 16 c, rows ty + 16 r
  float2 acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = make_float2(0.f, 0.f);
  for (int u = 0; u < np; ++u) {
    float2 w[4], x[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) w[r] = sW[(ty + 16 * r) * (np + 1) + u];
#pragma unroll
    for (int c = 0; c < 4; ++c) x[c] = sXc[u * (kTile + 1) + tx + 16 * c];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        acc[r][c].x = fmaf(w[r].x, x[c].x, fmaf(-w[r].y, x[c].y, acc[r][c].x));
        acc[r][c].y = fmaf(w[r].x, x[c].y, fmaf(w[r].y, x[c].x, acc[r][c].y));
      }
  }
  const float cs = sC;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int k = k0 + ty + 16 * r;
    if (k >= q) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int l = l0 + tx + 16 * c;
      if (l < q) prm.B[int64_t(k) * q + l] = make_float2(acc[r][c].x * cs, acc[r][c].y * cs);
    }
  }
}

}  // namespace

int launch_lrkron(const float2* X, const LrkParams& prm, hipStream_t stream) {
  if (prm.n * prm.p > kLrkMaxRows || prm.p > kLrkMaxP || prm.p < 1 || prm.q < 1) return hipErrorInvalidValue;
  switch (prm.p) {
    case 1: hipLaunchKernelGGL(lrk_solve<1>, dim3(1), dim3(kSolveThreads), 0, stream, X, prm); break;
    case 2: hipLaunchKernelGGL(lrk_solve<2>, dim3(1), dim3(kSolveThreads), 0, stream, X, prm); break;
    case 3: hipLaunchKernelGGL(lrk_solve<3>, dim3(1), dim3(kSolveThreads), 0, stream, X, prm); break;
    case 4: hipLaunchKernelGGL(lrk_solve<4>, dim3(1), dim3(kSolveThreads), 0, stream, X, prm); break;
    case 5: hipLaunchKernelGGL(lrk_solve<5>, dim3(1), dim3(kSolveThreads), 0, stream, X, prm); break;
    case 6: hipLaunchKernelGGL(lrk_solve<6>, dim3(1), dim3(kSolveThreads), 0, stream, X, prm); break;
    case 7: hipLaunchKernelGGL(lrk_solve<7>, dim3(1), dim3(kSolveThreads), 0, stream, X, prm); break;
    default: hipLaunchKernelGGL(lrk_solve<8>, dim3(1), dim3(kSolveThreads), 0, stream, X, prm); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !prm.B) return e;
  const unsigned t = unsigned((prm.q + kTile - 1) / kTile);
  const int np = prm.n * prm.p;
  const size_t lds = sizeof(float2) * (size_t(kTile) * (np + 1) + size_t(np) * (kTile + 1));
  hipLaunchKernelGGL(lrk_emit_b, dim3(t, t), dim3(256), lds, stream, X, prm);
  return hipGetLastError();
}

}  // namespace kstap
