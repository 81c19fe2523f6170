// Small dense FP64 linear algebra done by the 64 lanes of ONE wave of a
// workgroup (matrices of order M <= 8 held in LDS).  Only wave 0 calls these
// functions; lanes synchronise with wave_sync() (the wave executes in
// lock-step, so a wave-scope fence on the LDS traffic is all that is needed).
// The caller follows with __syncthreads() before other waves read results.
#pragma once

#include "rcscm_internal.h"

namespace rcscm {

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zmulc(double2 a, double2 b) {  // conj(a) b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ bool zfinite(double2 v) { return isfinite(v.x) && isfinite(v.y); }

// 1/p in FP64 for p > 0: the hardware estimate refined by two Newton-Raphson
// steps r <- r + r (1 - p r), each of which doubles the number of correct bits.
__device__ __forceinline__ double rcp_f64_nr(double p) {
  double r = __builtin_amdgcn_rcp(p);
  r = fma(r, fma(-p, r, 1.0), r);
  return fma(r, fma(-p, r, 1.0), r);
}

// In-place inverse of a Hermitian positive-definite M x M matrix by
// Gauss-Jordan elimination without pivoting (stable for HPD matrices: every
// pivot is a positive Schur-complement diagonal).  aug is LDS [M][2M]:
// [A | I] on entry, [I | A^{-1}] on exit.  Lane t < M*M of wave 0 updates
// entry (t / M, t % M) of both halves in each of the M elimination steps;
// every step reads all it needs in one batch of LDS loads, then writes.
// Returns false (and continues with a clamped pivot) when a pivot is <= tol;
// *pivprod receives the product of the pivots (= det A).
template <int M>
__device__ bool gj_inverse_hpd_wave(double2 (*aug)[2 * M], double tol, double* pivprod) {
  const int t = threadIdx.x;
  const int i = t / M, j = t % M;
  const bool on = t < M * M;
  bool ok = true;
  double prod = 1.0;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    double p = aug[k][k].x;
    double2 f = make_double2(0.0, 0.0), r1 = f, r2 = f, a1 = f, a2 = f;
    if (on) {
      f = aug[i][k];
      r1 = aug[k][j];
      r2 = aug[k][M + j];
      a1 = aug[i][j];
      a2 = aug[i][M + j];
    }
    if (!(p > tol)) {
      ok = false;
      p = fmax(tol, 1e-300);
    }
    prod *= p;
    const double ip = rcp_f64_nr(p);
    wave_sync();  // every lane's reads of this step precede any write
    if (on) {
      const double2 n1 = make_double2(r1.x * ip, r1.y * ip);
      const double2 n2 = make_double2(r2.x * ip, r2.y * ip);
      if (i == k) {
        aug[k][j] = n1;
        aug[k][M + j] = n2;
      } else {
        const double2 d1 = zmul(f, n1), d2 = zmul(f, n2);
        aug[i][j] = make_double2(a1.x - d1.x, a1.y - d1.y);
        aug[i][M + j] = make_double2(a2.x - d2.x, a2.y - d2.y);
      }
    }
    wave_sync();
  }
  *pivprod = prod;
  return ok;
}

// Entry (i, j) of the inverse of a Hermitian positive-definite M x M matrix A
// (M <= 4) for lane t < M*M of wave 0, (i, j) = (t / M, t % M).  a is LDS
// [M][2M] with A in its left half on entry; the right half is overwritten.
// Every lane of the wave factorises A = L D L^H (L unit lower triangular, D
// real diagonal; no pivoting, stable for HPD matrices) in its own registers,
// so the M dependent pivot steps need no LDS round trip.  Lane 0 then stores
// X = L^{-1} (below the diagonal) and 1/D (on it) in the right half, and lane
// (i, j) forms (A^{-1})_ij = sum_{m >= max(i, j)} conj(X_mi) X_mj / d_m
// (X_mm = 1), which is exactly Hermitian in (i, j).  Returns false (and
// continues with a clamped pivot) when a pivot is <= tol; *pivprod receives
// the product of the pivots (= det A).
template <int M>
__device__ bool ldl_inverse_hpd_wave(double2 (*a)[2 * M], double tol, double* pivprod,
                                     double2* inv_ij) {
  static_assert(M <= 4, "registers hold the whole factorisation");
  const int t = threadIdx.x;
  const int i = t / M, j = t % M;
  double2 A[M][M];
#pragma unroll
  for (int r = 0; r < M; ++r)
#pragma unroll
    for (int c = 0; c <= r; ++c) A[r][c] = a[r][c];  // lower triangle (a broadcast read)
  double2 Lm[M][M];
  double d[M], id[M];
  bool ok = true;
  double prod = 1.0;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    double dk = A[k][k].x;
#pragma unroll
    for (int m = 0; m < k; ++m) dk -= (Lm[k][m].x * Lm[k][m].x + Lm[k][m].y * Lm[k][m].y) * d[m];
    if (!(dk > tol)) {
      ok = false;
      dk = fmax(tol, 1e-300);
    }
    prod *= dk;
    d[k] = dk;
    id[k] = rcp_f64_nr(dk);
#pragma unroll
    for (int r = k + 1; r < M; ++r) {
      double2 v = A[r][k];
#pragma unroll
      for (int m = 0; m < k; ++m) {
        const double2 p = zmul(Lm[r][m], zconj(Lm[k][m]));
        v.x -= p.x * d[m];
        v.y -= p.y * d[m];
      }
      Lm[r][k] = make_double2(v.x * id[k], v.y * id[k]);
    }
  }
  // X = L^{-1}: X_rr = 1, X_rc = -(L_rc + sum_{c < m < r} L_rm X_mc) for r > c
  double2 X[M][M];
#pragma unroll
  for (int c = 0; c < M; ++c)
#pragma unroll
    for (int r = c + 1; r < M; ++r) {
      double2 v = Lm[r][c];
#pragma unroll
      for (int m = c + 1; m < r; ++m) {
        const double2 p = zmul(Lm[r][m], X[m][c]);
        v.x += p.x;
        v.y += p.y;
      }
      X[r][c] = make_double2(-v.x, -v.y);
    }
  if (t == 0) {
#pragma unroll
    for (int r = 0; r < M; ++r) {
      a[r][M + r] = make_double2(id[r], 0.0);
#pragma unroll
      for (int c = 0; c < r; ++c) a[r][M + c] = X[r][c];
    }
  }
  wave_sync();
  double2 acc = make_double2(0.0, 0.0);
  if (t < M * M) {
    const int lo = i > j ? i : j;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      if (m < lo) continue;
      const double im = a[m][M + m].x;
      const double2 xi = m == i ? make_double2(1.0, 0.0) : a[m][M + i];
      const double2 xj = m == j ? make_double2(1.0, 0.0) : a[m][M + j];
      const double2 p = zmulc(xi, xj);  // conj(X_mi) X_mj
      acc.x += p.x * im;
      acc.y += p.y * im;
    }
  }
  *inv_ij = acc;
  *pivprod = prod;
  return ok;
}

}  // namespace rcscm
