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
// give the initialiser of Eq. (18); the iterations then run in FP64 with the
// threads over (m, m') pairs and EIG_{r_a} by cyclic Jacobi rotations.
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

// C = A * B for p x p row-major matrices
__device__ __forceinline__ void matmul(const dc* A, const dc* B, dc* C, int p) {
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < p; ++j) {
      dc s = mk(0, 0);
      for (int k = 0; k < p; ++k) s = add(s, mul(A[i * p + k], B[k * p + j]));
      C[i * p + j] = s;
    }
}

// Eigen-decomposition of a Hermitian p x p matrix H (overwritten) by cyclic
// Jacobi rotations; V receives the eigenvectors as columns, lam the
// eigenvalues (unsorted).
__device__ void jacobi_herm(dc* H, dc* V, double* lam, int p) {
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < p; ++j) V[i * p + j] = mk(i == j ? 1.0 : 0.0, 0.0);
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0, tot = 0;
    for (int i = 0; i < p; ++i)
      for (int j = 0; j < p; ++j) {
        tot += ab2(H[i * p + j]);
        if (i != j) off += ab2(H[i * p + j]);
      }
    if (off <= 1e-30 * tot) break;
    for (int a = 0; a < p - 1; ++a)
      for (int b = a + 1; b < p; ++b) {
        const dc hab = H[a * p + b];
        const double r = sqrt(ab2(hab));
        if (r <= 1e-300) continue;
        // D = diag(1, e^{-i phi}) makes the (a, b) entry real (= r); a real
        // rotation [c s; -s c] then zeroes it: U = D [c s; -s c]
        const dc e = scl(hab, 1.0 / r);   // e^{i phi}
        const double tau = (H[b * p + b].x - H[a * p + a].x) / (2.0 * r);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        const dc ec = cj(e);               // e^{-i phi}
        // columns: H <- H U, V <- V U
        for (int k = 0; k < p; ++k) {
          const dc ha = H[k * p + a], hb = H[k * p + b];
          H[k * p + a] = sub(scl(ha, c), scl(mul(ec, hb), s));
          H[k * p + b] = add(scl(ha, s), scl(mul(ec, hb), c));
          const dc va = V[k * p + a], vb = V[k * p + b];
          V[k * p + a] = sub(scl(va, c), scl(mul(ec, vb), s));
          V[k * p + b] = add(scl(va, s), scl(mul(ec, vb), c));
        }
        // rows: H <- U^H H
        for (int k = 0; k < p; ++k) {
          const dc ha = H[a * p + k], hb = H[b * p + k];
          H[a * p + k] = sub(scl(ha, c), scl(mul(e, hb), s));
          H[b * p + k] = add(scl(ha, s), scl(mul(e, hb), c));
        }
        H[a * p + b] = mk(0, 0);
        H[b * p + a] = mk(0, 0);
        H[a * p + a].y = 0;
        H[b * p + b].y = 0;
      }
  }
  for (int i = 0; i < p; ++i) lam[i] = H[i * p + i].x;
}

constexpr int kSolveThreads = 512;
constexpr int kSolveWaves = kSolveThreads / 64;

// Sums a double over the workgroup (every thread gets the total).
__device__ __forceinline__ double block_sum(double v, double* red) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  v = wave_sum(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0;
  for (int w = 0; w < kSolveWaves; ++w) t += red[w];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(kSolveThreads) void lrk_solve(const float2* __restrict__ X, LrkParams prm) {
  const int n = prm.n, p = prm.p, q = prm.q, np = n * p;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  __shared__ dc sG[kLrkMaxRows * kLrkMaxRows];   // Gram of the snapshot rows
  __shared__ dc sRow[kLrkMaxRows];               // row sums
  __shared__ dc sA[kLrkMaxP * kLrkMaxP], sAp[kLrkMaxP * kLrkMaxP];
  __shared__ double sRed[kSolveWaves];
  __shared__ double sScal[4];

  // ---- Gram matrix (upper triangle) and row sums, FP64 sums of FP32 products
  const int ntri = np * (np + 1) / 2, nent = ntri + np;
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
    const float2* xu = X + int64_t(u) * q;
    const float2* xv = X + int64_t(v) * q;
    double sr = 0, si = 0;
    for (int k = lane; k < q; k += 64) {
      const float2 a = xu[k];
      if (rowsum) {
        sr += double(a.x);
        si += double(a.y);
      } else {
        const float2 b = xv[k];   // a * conj(b)
        sr += double(a.x) * double(b.x) + double(a.y) * double(b.y);
        si += double(a.y) * double(b.x) - double(a.x) * double(b.y);
      }
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (lane == 0) {
      if (rowsum) {
        sRow[u] = mk(sr, si);
      } else {
        sG[u * np + v] = mk(sr, si);
        sG[v * np + u] = mk(sr, -si);
      }
    }
  }
  __syncthreads();

  auto G = [&](int m, int mm, int i, int j) -> dc { return sG[(m * p + i) * np + mm * p + j]; };
  const int npair = n * n;

  // ||R||^2 = ||S||^2 = (1/n^2) sum_{m,m'} |tr G_m'm|^2
  double nr = 0;
  for (int t = tid; t < npair; t += kSolveThreads) {
    const int m = t / n, mm = t - (t / n) * n;
    dc tr = mk(0, 0);
    for (int i = 0; i < p; ++i) tr = add(tr, G(mm, m, i, i));
    nr += ab2(tr);
  }
  const double normR2 = block_sum(nr, sRed) / (double(n) * n);

  // initialiser (Eq. (18)): A0 = (1/(n q^2)) sum_m s_m s_m^H, s_m the row sums;
  // fallback R vec(I_q) = (1/n) sum_m G_mm when ||A0|| is negligible
  if (tid == 0) {
    double an = 0;
    for (int i = 0; i < p; ++i)
      for (int j = 0; j < p; ++j) {
        dc s = mk(0, 0);
        for (int m = 0; m < n; ++m) s = add(s, mul(sRow[m * p + i], cj(sRow[m * p + j])));
        sA[i * p + j] = scl(s, 1.0 / (double(n) * q * q));
        an += ab2(sA[i * p + j]);
      }
    if (an <= 1e-24 * normR2) {
      for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j) {
          dc s = mk(0, 0);
          for (int m = 0; m < n; ++m) s = add(s, G(m, m, i, j));
          sA[i * p + j] = scl(s, 1.0 / n);
        }
    }
  }
  __syncthreads();

  double eta = 0, eta_prev = INFINITY, bn2 = 0;
  int iters = 0;
  const bool zero = !(normR2 > 0.0);   // uniform over the workgroup
  while (!zero) {
    double an2 = 0;
    for (int e = 0; e < p * p; ++e) an2 += ab2(sA[e]);
    const double c = 1.0 / (double(n) * an2);
    // M = sum G_m'm A G_mm',  tb = Re sum tr(A G_mm' A G_m'm)
    dc M[kLrkMaxP * kLrkMaxP];
    for (int e = 0; e < p * p; ++e) M[e] = mk(0, 0);
    double tb = 0;
    for (int t = tid; t < npair; t += kSolveThreads) {
      const int m = t / n, mm = t - (t / n) * n;
      dc g1[kLrkMaxP * kLrkMaxP], g2[kLrkMaxP * kLrkMaxP], T1[kLrkMaxP * kLrkMaxP], T2[kLrkMaxP * kLrkMaxP];
      for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j) {
          g1[i * p + j] = G(mm, m, i, j);   // G_m'm
          g2[i * p + j] = G(m, mm, i, j);   // G_mm'
        }
      matmul(g1, sA, T1, p);                // G_m'm A
      for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j) {
          dc s = mk(0, 0);
          for (int k = 0; k < p; ++k) s = add(s, mul(T1[i * p + k], g2[k * p + j]));
          M[i * p + j] = add(M[i * p + j], s);
        }
      matmul(sA, g2, T2, p);                // A G_mm'
      // tr(A G_mm' A G_m'm) = sum_ij T2[i][j] (A G_m'm)[j][i]
      for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j) {
          dc s = mk(0, 0);
          for (int k = 0; k < p; ++k) s = add(s, mul(sA[j * p + k], g1[k * p + i]));
          tb += mul(T2[i * p + j], s).x;
        }
    }
    for (int e = 0; e < p * p; ++e) M[e] = mk(block_sum(M[e].x, sRed), block_sum(M[e].y, sRed));
    tb = block_sum(tb, sRed);
    bn2 = c * c * tb;                           // ||b||^2
    const double sa = c / (double(n) * bn2);    // A' = R conj(b) / ||b||^2 = sa M
    if (tid == 0) {
      for (int e = 0; e < p * p; ++e) sAp[e] = scl(M[e], sa);
      // EIG_{r_a} of the Hermitian part
      dc Hm[kLrkMaxP * kLrkMaxP], Vm[kLrkMaxP * kLrkMaxP];
      double lam[kLrkMaxP];
      for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j)
          Hm[i * p + j] = scl(add(sAp[i * p + j], cj(sAp[j * p + i])), 0.5);
      jacobi_herm(Hm, Vm, lam, p);
      bool used[kLrkMaxP];
      for (int i = 0; i < p; ++i) used[i] = false;
      for (int e = 0; e < p * p; ++e) sA[e] = mk(0, 0);
      for (int r = 0; r < prm.r_a; ++r) {   // largest algebraic eigenvalues first
        int best = -1;
        for (int i = 0; i < p; ++i)
          if (!used[i] && (best < 0 || lam[i] > lam[best])) best = i;
        used[best] = true;
        for (int i = 0; i < p; ++i)
          for (int j = 0; j < p; ++j)
            sA[i * p + j] = add(sA[i * p + j], scl(mul(Vm[i * p + best], cj(Vm[j * p + best])), lam[best]));
      }
      double na = 0, cross = 0;
      for (int e = 0; e < p * p; ++e) {
        na += ab2(sA[e]);
        cross += mul(cj(sA[e]), sAp[e]).x;
      }
      sScal[0] = na;
      sScal[1] = cross;
    }
    __syncthreads();
    ++iters;
    // eta^2 = (||R||^2 - 2 ||b||^2 Re<A, A'> + ||A||^2 ||b||^2) / ||R||^2
    const double r2 = normR2 - 2.0 * bn2 * sScal[1] + sScal[0] * bn2;
    const double e = sqrt(fmax(r2, 0.0) / normR2);
    eta = e;
    const bool stop =
        iters >= prm.max_iter || (prm.eps > 0.0 && iters >= prm.min_iter && fabs(e - eta_prev) <= prm.eps);
    __syncthreads();   // sScal is rewritten by the next iteration
    if (stop) break;
    eta_prev = e;
  }
  if (tid == 0) {
    for (int e = 0; e < p * p; ++e)
      prm.A[e] = zero ? make_float2(0.f, 0.f) : make_float2(float(sA[e].x), float(sA[e].y));
    if (prm.stats) {
      prm.stats[0] = zero ? 0.0 : eta;
      prm.stats[1] = double(iters);
      prm.stats[2] = sqrt(normR2);
      prm.stats[3] = zero ? 0.0 : sqrt(bn2);
    }
  }
}

// Final time factor B-hat[k][l] = c sum_{m, j} W_m[k][j] conj(X_m[j][l]) with
// W_m = X_m^T conj(A) (q x p) and c = 1 / (n ||A||^2): a rank-np product,
// bound by writing q^2 complex values.  64 x 64 outputs per 256-thread block,
// each thread 4 rows x 4 columns (columns strided by 16 so that each store
// instruction writes 16 consecutive entries per row).
constexpr int kTile = 64;
__global__ __launch_bounds__(256) void lrk_emit_b(const float2* __restrict__ X, LrkParams prm) {
  const int n = prm.n, p = prm.p, q = prm.q, np = n * p;
  __shared__ float2 sW[kTile][kLrkMaxRows + 1];   // W for the tile's rows k
  __shared__ float2 sX[kLrkMaxRows][kTile + 1];   // conj(X) rows for the tile's columns l
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
  __syncthreads();
  // W[k][(m, j)] = sum_i X_m[i][k] conj(A)[i][j]
  for (int e = tid; e < kTile * np; e += 256) {
    const int kk = e / np, u = e - (e / np) * np;
    const int m = u / p, j = u - (u / p) * p;
    const int k = k0 + kk;
    float2 s = make_float2(0.f, 0.f);
    if (k < q) {
      for (int i = 0; i < p; ++i) {
        const float2 x = X[(int64_t(m) * p + i) * q + k];
        const float2 a = sAc[i * p + j];
        s.x += x.x * a.x - x.y * a.y;
        s.y += x.x * a.y + x.y * a.x;
      }
    }
    sW[kk][u] = s;
  }
  for (int e = tid; e < np * kTile; e += 256) {
    const int u = e / kTile, ll = e - (e / kTile) * kTile;
    const int l = l0 + ll;
    const float2 x = (l < q) ? X[int64_t(u) * q + l] : make_float2(0.f, 0.f);
    sX[u][ll] = make_float2(x.x, -x.y);
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
    for (int r = 0; r < 4; ++r) w[r] = sW[ty + 16 * r][u];
#pragma unroll
    for (int c = 0; c < 4; ++c) x[c] = sX[u][tx + 16 * c];
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
  hipLaunchKernelGGL(lrk_solve, dim3(1), dim3(kSolveThreads), 0, stream, X, prm);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !prm.B) return e;
  const unsigned t = unsigned((prm.q + kTile - 1) / kTile);
  hipLaunchKernelGGL(lrk_emit_b, dim3(t, t), dim3(256), 0, stream, X, prm);
  return hipGetLastError();
}

}  // namespace kstap
