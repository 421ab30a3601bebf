// Robustness evaluation kernels.
//
// lrstap_probe: the unstructured low-rank STAP baseline the Kronecker
// methods are compared with (Sec. 1): per pixel of a list, the sample
// covariance S of Eq. (2) over the plan's training stencil, the
// eigenvectors U of its r largest eigenvalues, the filter F = I - U U^H and
// the statistic max_h |d^H F x|^2 / (d^H F d), d = h (x) b, of that filter.
// One 64-lane workgroup per pixel: the lanes own entries of the upper
// triangle of S (FP32 sums of the training vectors staged through LDS), then
// rows of the pq x r iterate (FP64) of a subspace iteration orthonormalised
// by classical Gram-Schmidt with reorthogonalisation; a Rayleigh-Ritz step
// orders the basis by eigenvalue.
//
// sinr_loss: the output SINR of Eq. (21) (|alpha| = 1) of the filter
// w = F d (Eq. (23)) of each pixel, for every steering d = a (x) b of two
// grids, divided by the optimum d^H Sigma^-1 d of Eq. (22), with the true
// covariance Sigma = tau2 A (x) B + sigma2 I given by orthonormal factor
// bases: w^H Sigma w = sigma2 ||w||^2 + tau2 sum_ij lamA_i lamB_j
// |(uA_i (x) uB_j)^H w|^2 and, by the Woodbury identity, d^H Sigma^-1 d =
// (||d||^2 - sum_ij c_ij / (c_ij + sigma2) |(uA_i (x) uB_j)^H d|^2) / sigma2
// with c_ij = tau2 lamA_i lamB_j.  One 64-lane workgroup per (pixel,
// steering), lane = entry of the pq vector.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kstap_internal.h"
#include "kstap_small_eig.h"

namespace kstap {
namespace {

using namespace small;

constexpr int kStageVec = 16;                                        // training vectors per staged chunk
constexpr int kEnt = (kLrsMaxPQ * (kLrsMaxPQ + 1) / 2 + 63) / 64;    // upper-triangle entries per lane

__device__ __forceinline__ dc cd(float2 a) { return mk(double(a.x), double(a.y)); }
__device__ __forceinline__ dc wsum(dc a) { return mk(wave_sum_dpp(a.x), wave_sum_dpp(a.y)); }

// Fixed start block of the subspace iteration: small deterministic complex
// entries (no clutter subspace is orthogonal to them in practice).
__device__ __forceinline__ dc start_entry(int i, int k) {
  const unsigned h = (unsigned(i) * 2654435761u) ^ (unsigned(k + 1) * 40503u);
  return mk(double(int(h % 17u)) - 7.5, double(int((h >> 8) % 13u)) - 5.75);
}

// Orthonormalises the columns y[0..r) of a pq x r block held by rows (lane =
// row; lanes >= pq hold zeros): classical Gram-Schmidt, each column projected
// twice.
__device__ __forceinline__ void cgs2(dc (&y)[kLrsMaxR], int r) {
#pragma unroll
  for (int k = 0; k < kLrsMaxR; ++k) {
    if (k < r) {
#pragma unroll
      for (int pass = 0; pass < 2; ++pass) {
        dc c[kLrsMaxR];
#pragma unroll
        for (int j = 0; j < kLrsMaxR; ++j)
          if (j < k) c[j] = wsum(mul(cj(y[j]), y[k]));
#pragma unroll
        for (int j = 0; j < kLrsMaxR; ++j)
          if (j < k) y[k] = sub(y[k], mul(y[j], c[j]));
      }
      const double nrm = sqrt(wave_sum_dpp(ab2(y[k])));
      y[k] = nrm > 0.0 ? scl(y[k], 1.0 / nrm) : mk(0, 0);
    }
  }
}

__global__ __launch_bounds__(64) void lrstap_probe(const LrsParams prm) {
  const int lane = threadIdx.x;
  const int p = prm.p, q = prm.q, pq = p * q, n = prm.n, r = prm.r;
  const int H = prm.H, W = prm.W;
  __shared__ float2 sS[kLrsMaxPQ * kLrsMaxPQ];    // S, full Hermitian, row-major
  __shared__ float2 sX[kStageVec * kLrsMaxPQ];    // staged training vectors
  __shared__ dc sV[kLrsMaxPQ * kLrsMaxR];         // current basis, row-major
  __shared__ dc sW[(kLrsMaxR + 1) * 64];          // per-lane terms of segmented sums; Ritz vectors
  __shared__ dc sSm[kLrsMaxR];                    // Ritz values
  __shared__ dc sC[64];                           // C[k][a] on k p + a (r p <= 64)
  __shared__ dc sU[8];                            // u[a]
  __shared__ double sLamG[8];                     // eigenvalues of G

  const int ntri = pq * (pq + 1) / 2;
  const int ri = lane / (q > 0 ? q : 1), rk = lane - ri * q;   // row lane = ri q + rk
  const bool row = lane < pq;

  for (int t = blockIdx.x; t < prm.npix; t += gridDim.x) {
    const int pr = prm.pix[2 * t], pc = prm.pix[2 * t + 1];
    const bool valid = pr >= prm.r0 && pr < prm.r1 && pc >= prm.c0 && pc < prm.c1;
    if (!valid) {   // T = 0, zero basis, zero eigenvalues, no iterations
      if (lane == 0) {
        prm.T[t] = 0.f;
        if (prm.iters) prm.iters[t] = 0;
      }
      if (prm.U && row)
        for (int k = 0; k < r; ++k) prm.U[(int64_t(t) * pq + lane) * r + k] = make_float2(0.f, 0.f);
      if (prm.lam && lane < r) prm.lam[int64_t(t) * r + lane] = 0.f;
      continue;
    }
    // ---- S = (1/n) sum_m x_m x_m^H (Eq. (2)), x_m = vec(X_m^T); this lane's
    // entries (u, v), u <= v, of the upper triangle, row-major
    int ent[kEnt];
    int ne = 0;
#pragma unroll
    for (int j = 0; j < kEnt; ++j) {
      const int e = lane + 64 * j;
      ent[j] = 0;
      if (e < ntri) {
        int u = 0, rem = e;
        while (rem >= pq - u) {
          rem -= pq - u;
          ++u;
        }
        ent[j] = (u << 8) | (u + rem);
        ne = j + 1;
      }
    }
    float2 acc[kEnt];
#pragma unroll
    for (int j = 0; j < kEnt; ++j) acc[j] = make_float2(0.f, 0.f);
    for (int m0 = 0; m0 < n; m0 += kStageVec) {
      const int nv = min(kStageVec, n - m0);
      __syncthreads();
      for (int e = lane; e < nv * pq; e += 64) {
        const int v = e / pq, j = e - v * pq, i = j / q, k = j - i * q;
        const int m = m0 + v;
        const int rr = pr + prm.st[2 * m], cc = pc + prm.st[2 * m + 1];
        sX[v * pq + j] = prm.x[((int64_t(i) * H + rr) * W + cc) * q + k];
      }
      __syncthreads();
      for (int v = 0; v < nv; ++v) {
#pragma unroll
        for (int j = 0; j < kEnt; ++j) {
          if (j < ne) {
            const float2 a = sX[v * pq + (ent[j] >> 8)], b = sX[v * pq + (ent[j] & 0xff)];   // a conj(b)
            acc[j].x = fmaf(a.x, b.x, fmaf(a.y, b.y, acc[j].x));
            acc[j].y = fmaf(a.y, b.x, fmaf(-a.x, b.y, acc[j].y));
          }
        }
      }
    }
    __syncthreads();
    const float inv_n = 1.f / float(n);
#pragma unroll
    for (int j = 0; j < kEnt; ++j) {
      if (j < ne) {
        const int u = ent[j] >> 8, v = ent[j] & 0xff;
        const float2 s = make_float2(acc[j].x * inv_n, acc[j].y * inv_n);
        sS[u * pq + v] = s;
        if (v != u) sS[v * pq + u] = make_float2(s.x, -s.y);
      }
    }
    __syncthreads();

    // ---- top-r subspace: V <- orth(S V), starting from orth(S Z)
    dc y[kLrsMaxR];
    auto apply_s = [&]() {   // y = S V, V read from sV
#pragma unroll
      for (int k = 0; k < kLrsMaxR; ++k) y[k] = mk(0, 0);
      if (row) {
        for (int j = 0; j < pq; ++j) {
          const dc s = cd(sS[lane * pq + j]);
#pragma unroll
          for (int k = 0; k < kLrsMaxR; ++k)
            if (k < r) y[k] = add(y[k], mul(s, sV[j * kLrsMaxR + k]));
        }
      }
    };
    if (row)
      for (int k = 0; k < r; ++k) sV[lane * kLrsMaxR + k] = start_entry(lane, k);
    __syncthreads();
    apply_s();
    cgs2(y, r);
    int it = 0;
    for (; it < prm.max_iter; ++it) {
      __syncthreads();
      if (row)
#pragma unroll
        for (int k = 0; k < kLrsMaxR; ++k)
          if (k < r) sV[lane * kLrsMaxR + k] = y[k];
      __syncthreads();
      apply_s();
      cgs2(y, r);
      // sum of squared sines of the principal angles between the previous
      // basis (still in sV) and the new one: r - ||Vold^H Vnew||_F^2
      double s2 = 0;
#pragma unroll
      for (int j = 0; j < kLrsMaxR; ++j)
#pragma unroll
        for (int k = 0; k < kLrsMaxR; ++k)
          if (j < r && k < r) s2 += ab2(wsum(mul(cj(row ? sV[lane * kLrsMaxR + j] : mk(0, 0)), y[k])));
      if (double(r) - s2 <= prm.tol * prm.tol) {
        ++it;
        break;
      }
    }
    // ---- Rayleigh-Ritz: M = V^H S V, its eigenvectors order the basis
    __syncthreads();
    if (row)
#pragma unroll
      for (int k = 0; k < kLrsMaxR; ++k)
        if (k < r) sV[lane * kLrsMaxR + k] = y[k];
    __syncthreads();
    dc v_row[kLrsMaxR];
#pragma unroll
    for (int k = 0; k < kLrsMaxR; ++k) v_row[k] = y[k];
    apply_s();   // y = S V
    const int RE = (r + 1) / 2 * 2;
    dc mentry = mk(0, 0);
#pragma unroll
    for (int j = 0; j < kLrsMaxR; ++j)
#pragma unroll
      for (int k = 0; k < kLrsMaxR; ++k)
        if (j < r && k < r) {
          const dc m = wsum(mul(cj(v_row[j]), y[k]));
          if (lane == j * RE + k) mentry = m;
        }
    {
      // Hermitian part, in the Jacobi lane layout (entry (j, k) on lane j RE + k)
      const int jj = lane / (RE > 0 ? RE : 1), kk = lane - jj * RE;
      const dc mt = shd(mentry, kk * RE + jj);
      dc h = (jj < r && kk < r && lane < RE * RE) ? scl(add(mentry, cj(mt)), 0.5) : mk(0, 0), zv;
      if (r > 0) jacobi_par_n(h, zv, lane, r);
      // eigenvalues (diagonal lanes) to sSm[k], vectors to sW[j][k]
      __syncthreads();
      if (jj < r && kk < r && lane < RE * RE) {
        sW[jj * kLrsMaxR + kk] = zv;
        if (jj == kk) sSm[jj] = h;
      }
      __syncthreads();
    }
    // order by decreasing eigenvalue (uniform selection), U = V Q
    {
      unsigned used = 0;
      dc urow[kLrsMaxR];
#pragma unroll
      for (int k = 0; k < kLrsMaxR; ++k) {
        urow[k] = mk(0, 0);
        if (k < r) {
          int best = -1;
          for (int c = 0; c < r; ++c)
            if (!((used >> c) & 1u) && (best < 0 || sSm[c].x > sSm[best].x)) best = c;
          used |= 1u << best;
#pragma unroll
          for (int j = 0; j < kLrsMaxR; ++j)
            if (j < r) urow[k] = add(urow[k], mul(v_row[j], sW[j * kLrsMaxR + best]));
          if (prm.lam && lane == 0) prm.lam[int64_t(t) * r + k] = float(sSm[best].x);
        }
      }
      if (prm.U && row)
#pragma unroll
        for (int k = 0; k < kLrsMaxR; ++k)
          if (k < r) prm.U[(int64_t(t) * pq + lane) * r + k] = make_float2(float(urow[k].x), float(urow[k].y));
#pragma unroll
      for (int k = 0; k < kLrsMaxR; ++k) v_row[k] = urow[k];
    }

    // ---- statistic of F = I - U U^H: u = E^H F x, G = E^H F E = ||b||^2 I - C^H C, C = U^H E
    const dc xt = row ? cd(prm.x[((int64_t(ri) * H + pr) * W + pc) * q + rk]) : mk(0, 0);
    dc fx = xt;
#pragma unroll
    for (int k = 0; k < kLrsMaxR; ++k)
      if (k < r) fx = sub(fx, mul(v_row[k], wsum(mul(cj(v_row[k]), xt))));
    const dc bconj = row ? mk(prm.b_s[rk].x, -prm.b_s[rk].y) : mk(0, 0);
    __syncthreads();
    sW[lane] = mul(bconj, fx);   // terms of u[a] = sum_l conj(b_l) (F x)[a q + l]
#pragma unroll
    for (int k = 0; k < kLrsMaxR; ++k)   // terms of C[k][a] = sum_l conj(U[a q + l][k]) b_l
      if (k < r) sW[(k + 1) * 64 + lane] = cj(mul(v_row[k], bconj));
    __syncthreads();
    // u[a] on lane a, C[k][a] on lane k p + a
    if (lane < p) {
      dc sm = mk(0, 0);
      for (int l = 0; l < q; ++l) sm = add(sm, sW[lane * q + l]);
      sU[lane] = sm;
    }
    if (lane < r * p) {
      const int k = lane / p, a = lane - k * p;
      dc sm = mk(0, 0);
      for (int l = 0; l < q; ++l) sm = add(sm, sW[(k + 1) * 64 + a * q + l]);
      sC[lane] = sm;
    }
    __syncthreads();
    const int PE = (p + 1) / 2 * 2;
    const int ga = lane / PE, gb = lane - ga * PE;
    const bool gin = ga < p && gb < p && lane < PE * PE;
    dc g = mk(0, 0);
    if (gin) {
      g = mk(ga == gb ? prm.bs_norm2 : 0.0, 0.0);
      for (int k = 0; k < r; ++k) g = sub(g, mul(cj(sC[k * p + ga]), sC[k * p + gb]));
    }
    // Hermitian part of G
    const dc gt = shd(g, gb * PE + ga);
    g = gin ? scl(add(g, cj(gt)), 0.5) : mk(0, 0);
    dc gv;
    jacobi_par_n(g, gv, lane, p);
    // T = sum over eigenpairs (lam > 1e-12 ||b||^2) of |w^H u|^2 / lam
    const dc term = gin ? mul(cj(gv), sU[ga]) : mk(0, 0);   // conj(W[row][col]) u[row]
    __syncthreads();
    sW[lane] = term;
    if (gin && ga == gb) sLamG[ga] = g.x;   // eigenvalue of column ga
    __syncthreads();
    double tval = 0;
    if (lane < p) {
      dc c = mk(0, 0);
      for (int a = 0; a < p; ++a) c = add(c, sW[a * PE + lane]);
      const double lam = sLamG[lane];
      if (lam > 1e-12 * prm.bs_norm2) tval = ab2(c) / lam;
    }
    tval = wave_sum_dpp(tval);
    if (lane == 0) {
      prm.T[t] = float(tval);
      if (prm.iters) prm.iters[t] = it;
    }
  }
}

__global__ __launch_bounds__(64) void sinr_loss(const SinrParams prm) {
  const int lane = threadIdx.x;
  const int p = prm.p, q = prm.q, pq = p * q;
  const bool act = lane < pq;
  const int i = act ? lane / q : 0, k = act ? lane - (lane / q) * q : 0;
  const int per = prm.na * prm.nb;
  const int64_t total = int64_t(prm.npix) * per;
  for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
    const int pix = int(t / per), rem = int(t - int64_t(pix) * per), ia = rem / prm.nb, ib = rem - ia * prm.nb;
    const dc ai = cd(prm.a_grid[ia * p + i]), bk = cd(prm.b_grid[ib * q + k]);
    const dc d = act ? mul(ai, bk) : mk(0, 0);
    dc w;
    if (prm.kind == 2) {   // I - U U^H
      const float2* U = prm.U + int64_t(pix) * pq * prm.r;
      w = d;
      for (int j = 0; j < prm.r; ++j) {
        const dc u = act ? cd(U[lane * prm.r + j]) : mk(0, 0);
        w = sub(w, mul(u, wsum(mul(cj(u), d))));
      }
    } else {   // P_A a and P_B b, every lane for its own (i, k)
      const float2* UA = prm.UA + int64_t(pix) * p * prm.r_a;
      const float2* UB = prm.UB + int64_t(pix) * q * prm.r_b;
      dc pa = mk(0, 0), pb = mk(0, 0);
      for (int j = 0; j < prm.r_a; ++j) {
        dc c = mk(0, 0);
        for (int l = 0; l < p; ++l) c = add(c, mul(cj(cd(UA[l * prm.r_a + j])), cd(prm.a_grid[ia * p + l])));
        pa = add(pa, mul(cd(UA[i * prm.r_a + j]), c));
      }
      for (int j = 0; j < prm.r_b; ++j) {
        dc c = mk(0, 0);
        for (int l = 0; l < q; ++l) c = add(c, mul(cj(cd(UB[l * prm.r_b + j])), cd(prm.b_grid[ib * q + l])));
        pb = add(pb, mul(cd(UB[k * prm.r_b + j]), c));
      }
      if (prm.kind == 0)
        w = mul(sub(ai, pa), sub(bk, pb));    // ((I - P_A) a) (x) ((I - P_B) b)
      else
        w = sub(mul(ai, bk), mul(pa, pb));    // a (x) b - (P_A a) (x) (P_B b)
      if (!act) w = mk(0, 0);
    }
    const double num = ab2(wsum(mul(cj(w), d)));
    double den = prm.sigma2 * wave_sum_dpp(ab2(w));
    double opt = wave_sum_dpp(ab2(d));
    for (int a = 0; a < prm.ra_t; ++a) {
      const dc ua = act ? cd(prm.UA_t[i * prm.ra_t + a]) : mk(0, 0);
      for (int b = 0; b < prm.rb_t; ++b) {
        const dc ub = cd(prm.UB_t[k * prm.rb_t + b]);
        const dc uab = mul(ua, ub);
        const double c = prm.tau2 * prm.lamA_t[a] * prm.lamB_t[b];
        den += c * ab2(wsum(mul(cj(uab), w)));
        opt -= c / (c + prm.sigma2) * ab2(wsum(mul(cj(uab), d)));
      }
    }
    opt /= prm.sigma2;
    if (lane == 0) prm.loss[t] = (den > 0.0 && opt > 0.0) ? float(num / (den * opt)) : 0.f;
  }
}

}  // namespace

int launch_lrstap(const LrsParams& prm, hipStream_t stream) {
  if (prm.p * prm.q > kLrsMaxPQ || prm.r < 0 || prm.r > kLrsMaxR || prm.p > 8) return hipErrorInvalidValue;
  if (prm.npix <= 0) return hipSuccess;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int grid = prm.npix < cus * 8 ? prm.npix : cus * 8;
  hipLaunchKernelGGL(lrstap_probe, dim3(grid), dim3(64), 0, stream, prm);
  return hipGetLastError();
}

int launch_sinr(const SinrParams& prm, hipStream_t stream) {
  if (prm.p * prm.q > 64) return hipErrorInvalidValue;
  const int64_t total = int64_t(prm.npix) * prm.na * prm.nb;
  if (total <= 0) return hipSuccess;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int64_t cap = int64_t(cus) * 32;
  hipLaunchKernelGGL(sinr_loss, dim3(unsigned(total < cap ? total : cap)), dim3(64), 0, stream, prm);
  return hipGetLastError();
}

}  // namespace kstap
