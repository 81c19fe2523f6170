// Naive EM update (Sec. II-B-2, eqs. (13)-(20)) on gfx950: the comparator.
//
// One iteration is two launches per microphone count:
//   naive_a   (per chunk of bins)  E-step with one M x M factorisation per bin
//             and the r^h update:
//               R~    = R' + lambda~ b b^H                          eq. (13)
//               Sigma = r~h a a^H + r~u R~ = L L^H  (float Cholesky) eq. (14)
//               p = L^{-1} a, w = L^{-1} x, Y = L^{-1} R~
//               h^    = r~h - r~h^2 |p|^2 + r~h^2 |w^H p|^2          eq. (15)
//               U^    = r~u R~ - r~u^2 Y^H Y + r~u^2 (Y^H w)(Y^H w)^H eq. (16)
//               r^h   = (h^ + beta) / (alpha + 2)                    eq. (17)
//             U^ is stored packed (M real diagonal entries, then the
//             upper triangle) and the chunk's sum of b^H U^ b / r~u is
//             written as a partial sum for eq. (18).
//   naive_b   (per chunk)  lambda = mean of the partial sums (eq. (18)),
//             R = R' + lambda b b^H (eq. (19)) and R^{-1} by FP64
//             Gauss-Jordan elimination, then r^u = tr(R^{-1} U^) / M    eq. (20)
// No step uses the pseudoinverse of R' or the Sherman-Morrison identity.
#include "accel_common.h"
#include "small_linalg.h"

namespace rcscm {

namespace {

constexpr int kNT = 256;

struct cf {
  float x, y;
};
__device__ __forceinline__ cf cmk(float x, float y) { return cf{x, y}; }
__device__ __forceinline__ cf operator+(cf a, cf b) { return cf{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cf operator-(cf a, cf b) { return cf{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cf cmul(cf a, cf b) {
  return cf{fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x)};
}
__device__ __forceinline__ cf cmulc(cf a, cf b) {  // conj(a) b
  return cf{fmaf(a.x, b.x, a.y * b.y), fmaf(a.x, b.y, -a.y * b.x)};
}
__device__ __forceinline__ cf cscale(cf a, float s) { return cf{a.x * s, a.y * s}; }
__device__ __forceinline__ float cabs2(cf a) { return fmaf(a.x, a.x, a.y * a.y); }

// E-step of one bin (eqs. (13)-(16)) at (r~h, r~u) = (h, u), with R~ = R' +
// lambda~ b b^H in sRt: factorises Sigma, calls onU(m, n, U^_mn) for every
// m <= n and returns h^ (eq. (15)).  bad is set when a pivot of the Cholesky
// factorisation is not positive.
template <int M, class OnU>
__device__ __forceinline__ float naive_estep(const cf (&sRt)[M][M], const cf (&sa)[M],
                                             const cf (&xv)[M], float h, float u, bool& bad,
                                             OnU&& onU) {
  // lower triangle of Sigma, then Cholesky in place (real diagonal)
  cf L[M][M];
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      const cf aa = cmulc(sa[j], sa[i]);  // a_i conj(a_j)
      L[i][j] = cmk(fmaf(h, aa.x, u * sRt[i][j].x), fmaf(h, aa.y, u * sRt[i][j].y));
    }
  float dinv[M];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    float d = L[j][j].x;
#pragma unroll
    for (int k = 0; k < j; ++k) d -= cabs2(L[j][k]);
    bad = bad || !(d > 0.0f);
    const float is = rsqrtf(fmaxf(d, 1e-37f));
    L[j][j] = cmk(d * is, 0.0f);
    dinv[j] = is;
#pragma unroll
    for (int i = j + 1; i < M; ++i) {
      cf s = L[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) s = s - cmul(L[i][k], cmk(L[j][k].x, -L[j][k].y));
      L[i][j] = cscale(s, is);
    }
  }
  // forward substitutions with L
  auto fwd = [&](const cf* v, cf* y) {
#pragma unroll
    for (int i = 0; i < M; ++i) {
      cf s = v[i];
#pragma unroll
      for (int k = 0; k < i; ++k) s = s - cmul(L[i][k], y[k]);
      y[i] = cscale(s, dinv[i]);
    }
  };
  cf p[M], w[M];
  fwd(sa, p);
  fwd(xv, w);
  cf Y[M][M];  // Y[:, n] = L^{-1} R~[:, n]
#pragma unroll
  for (int n = 0; n < M; ++n) {
    cf col[M], yc[M];
#pragma unroll
    for (int i = 0; i < M; ++i) col[i] = sRt[i][n];
    fwd(col, yc);
#pragma unroll
    for (int i = 0; i < M; ++i) Y[i][n] = yc[i];
  }
  float pp = 0.0f;
  cf wp = cmk(0.0f, 0.0f);
#pragma unroll
  for (int i = 0; i < M; ++i) {
    pp += cabs2(p[i]);
    wp = wp + cmulc(w[i], p[i]);
  }
  const float hh = h - h * h * pp + h * h * cabs2(wp);

  cf v[M];  // Y^H w = R~ Sigma^{-1} x
#pragma unroll
  for (int m = 0; m < M; ++m) {
    cf s = cmk(0.0f, 0.0f);
#pragma unroll
    for (int k = 0; k < M; ++k) s = s + cmulc(Y[k][m], w[k]);
    v[m] = s;
  }
  const float u2 = u * u;
#pragma unroll
  for (int m = 0; m < M; ++m) {
#pragma unroll
    for (int n = m; n < M; ++n) {
      cf yy = cmk(0.0f, 0.0f);
#pragma unroll
      for (int k = 0; k < M; ++k) yy = yy + cmulc(Y[k][m], Y[k][n]);
      const cf vv = cmul(v[m], cmk(v[n].x, -v[n].y));
      onU(m, n, cmk(fmaf(u, sRt[m][n].x, u2 * (vv.x - yy.x)),
                    fmaf(u, sRt[m][n].y, u2 * (vv.y - yy.y))));
    }
  }
  return hh;
}

// R~ = R' + lambda~ b b^H of the row into LDS (float), with a and b.
template <int M>
__device__ __forceinline__ void naive_row_model(const RowSpatialF* S, float lam_t, cf (&sRt)[M][M],
                                                cf (&sa)[M], cf (&sb)[M]) {
  const int t = threadIdx.x;
  if (t < M * M) {
    const int i = t / M, j = t % M;
    const float2 r = S->Rp[i * MAXM + j];
    const float2 bi = S->b[i], bj = S->b[j];
    const cf bb = cmul(cmk(bi.x, bi.y), cmk(bj.x, -bj.y));
    sRt[i][j] = cmk(fmaf(lam_t, bb.x, r.x), fmaf(lam_t, bb.y, r.y));
  }
  if (t < M) {
    sa[t] = cmk(S->a[t].x, S->a[t].y);
    sb[t] = cmk(S->b[t].x, S->b[t].y);
  }
}

// First launch of a naive iteration.  STORE: U^ goes to uhat packed (M real
// diagonal entries, then the (m < n) pairs; element-major), r^h is updated in
// place.  Otherwise nothing of U^ is stored: the second launch recomputes it,
// and r~h is kept in uhat[bin] (the first nbins floats) for that.
template <int M, bool STORE>
__global__ __launch_bounds__(kNT) void naive_a_kernel(
    const ChunkInfo* __restrict__ chunks, const RowInfo* __restrict__ rows,
    const RowSpatialF* __restrict__ rsf, const float2* __restrict__ x, float* __restrict__ rh,
    const float* __restrict__ ru, const float* __restrict__ lam, float* __restrict__ uhat,
    long long nbins, uint64_t* __restrict__ part, float inv_a2, float beta_a2,
    unsigned* __restrict__ status) {
  const ChunkInfo ck = chunks[blockIdx.x];
  const RowInfo ri = rows[ck.row];
  const int t = threadIdx.x;
  __shared__ cf sRt[M][M];  // R~ = R' + lambda~ b b^H
  __shared__ cf sa[M], sb[M];
  __shared__ uint64_t red[kNT / 64];
  RCSCM_DASSERT(ri.M == M);
  RCSCM_DASSERT(ck.start >= 0 && ck.len >= 1 && ck.start + ck.len <= ri.J);
  RCSCM_DASSERT(ri.bin_off + ck.start + ck.len <= nbins);
  naive_row_model<M>(rsf + ck.row, lam[ck.row], sRt, sa, sb);
  __syncthreads();

  LamAcc<0> acc;
  bool bad = false;
  for (int jj = t; jj < ck.len; jj += kNT) {
    const long long bin = ri.bin_off + ck.start + jj;
    const float2* xp = x + ri.x_off + (long long)(ck.start + jj) * M;
    cf xv[M];
#pragma unroll
    for (int m = 0; m < M; ++m) xv[m] = cmk(xp[m].x, xp[m].y);
    const float h = rh[bin], u = ru[bin];
    float bUb = 0.0f;
    int e = M;
    const float hh = naive_estep<M>(sRt, sa, xv, h, u, bad, [&](int m, int n, cf U) {
      if (m == n) {
        if constexpr (STORE) uhat[(long long)m * nbins + bin] = U.x;
        bUb = fmaf(cabs2(sb[m]), U.x, bUb);
      } else {
        if constexpr (STORE) {
          uhat[(long long)e * nbins + bin] = U.x;
          uhat[(long long)(e + 1) * nbins + bin] = U.y;
        }
        e += 2;
        // 2 Re(conj(b_m) U_mn b_n)
        const cf t1 = cmul(cmulc(sb[m], U), sb[n]);
        bUb = fmaf(2.0f, t1.x, bUb);
      }
    });
    if constexpr (!STORE) uhat[bin] = h;
    rh[bin] = fmaf(hh, inv_a2, beta_a2);
    acc.add(bUb * frcp(u));
  }
  acc = wave_allreduce<0>(acc);
  if ((t & 63) == 0) red[t >> 6] = acc.pack();
  __syncthreads();
  if (t == 0) {
    LamAcc<0> tot;
#pragma unroll
    for (int w2 = 0; w2 < kNT / 64; ++w2) tot.combine(LamAcc<0>::unpack(red[w2]));
    part[ck.part] = tot.pack();
  }
  if (bad) atomicOr(status + ck.row, ST_NONFINITE_STATE);
}

// R^{-1} = (R' + lambda b b^H)^{-1} (eq. (19)) by FP64 Gauss-Jordan in LDS on
// wave 0, rounded to float into sR (row-major).
template <int M>
__device__ __forceinline__ void naive_rinv(const RowConstD* D, float l, float2* sR,
                                           double2 (*aug)[2 * M]) {
  const int t = threadIdx.x;
  const int i = t / M, j = t % M;
  if (t < 64) {  // R^{-1} by wave 0
    if (t < M * M) {
      const double2 bb = zmul(D->b[i], zconj(D->b[j]));
      const double2 rp = D->Rp[i * MAXM + j];
      aug[i][j] = make_double2(rp.x + (double)l * bb.x, rp.y + (double)l * bb.y);
      aug[i][M + j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    }
    wave_sync();
    double det;
    gj_inverse_hpd_wave<M>(aug, 0.0, &det);
    if (t < M * M) sR[t] = make_float2((float)aug[i][M + j].x, (float)aug[i][M + j].y);
  }
}

// lambda = mean of the partial sums (eq. (18)), R^{-1} = (R' + lambda b b^H)^{-1}
// (eq. (19)) by FP64 Gauss-Jordan in LDS (every workgroup of the row does it;
// the first one stores lambda), then r^u = tr(R^{-1} U^) / M per bin (eq. (20)).
template <int M>
__global__ __launch_bounds__(kNT) void naive_b_kernel(const ChunkInfo* __restrict__ chunks,
                                                      const RowInfo* __restrict__ rows,
                                                      const RowConstD* __restrict__ rcd,
                                                      const uint64_t* __restrict__ part,
                                                      float* __restrict__ lam,
                                                      float* __restrict__ ru,
                                                      const float* __restrict__ uhat,
                                                      long long nbins,
                                                      unsigned* __restrict__ status) {
  const ChunkInfo ck = chunks[blockIdx.x];
  const RowInfo ri = rows[ck.row];
  const RowConstD* D = rcd + ck.row;
  const int t = threadIdx.x;
  RCSCM_DASSERT(ri.M == M);
  RCSCM_DASSERT(ck.start >= 0 && ck.len >= 1 && ck.start + ck.len <= ri.J);
  RCSCM_DASSERT(ri.bin_off + ck.start + ck.len <= nbins);
  __shared__ double2 aug[M][2 * M];
  __shared__ float2 sR[M * M];
  const float l = wave_sum_packed<0>(part + ri.part_off, ri.nparts).mean(1.0 / (double)ri.J);
  if (ck.start == 0 && t == 0) {
    lam[ck.row] = l;
    if (!(l > 0.0f) || !isfinite(l)) atomicOr(status + ck.row, ST_LAM_NONPOS);
  }
  naive_rinv<M>(D, l, sR, aug);
  __syncthreads();
  bool bad = false;
  for (int jj = t; jj < ck.len; jj += kNT) {
    const long long bin = ri.bin_off + ck.start + jj;
    // U^'s entries in the order the E-step forms them: (m, m), then (m, n > m)
    float tr = 0.0f;
    int e = M;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      tr = fmaf(sR[m * M + m].x, uhat[(long long)m * nbins + bin], tr);
#pragma unroll
      for (int n = m + 1; n < M; ++n) {
        const float ur = uhat[(long long)e * nbins + bin];
        const float ui = uhat[(long long)(e + 1) * nbins + bin];
        e += 2;
        // 2 Re(Rinv[n][m] U[m][n])
        const float2 r = sR[n * M + m];
        tr = fmaf(2.0f, fmaf(r.x, ur, -r.y * ui), tr);
      }
    }
    const float v = tr * (1.0f / (float)M);
    ru[bin] = v;
    bad = bad || !isfinite(v);
  }
  if (bad) atomicOr(status + ck.row, ST_NONFINITE_STATE);
}

// Second launch without a stored U^: lambda from the partial sums (eq. (18)),
// R^{-1} of the new lambda (eq. (19)), then per bin the E-step of the first
// launch again, at the same (r~h, r~u, lambda~) and with the same arithmetic,
// so U^ is the value the first launch had; r^u = tr(R^{-1} U^) / M (eq. (20))
// is accumulated from its entries without storing them.  lambda~ is read from
// lam_old, the new lambda written to lam_new (the host swaps the two).
template <int M>
__global__ __launch_bounds__(kNT) void naive_b_recompute_kernel(
    const ChunkInfo* __restrict__ chunks, const RowInfo* __restrict__ rows,
    const RowSpatialF* __restrict__ rsf, const RowConstD* __restrict__ rcd,
    const uint64_t* __restrict__ part, const float* __restrict__ lam_old,
    float* __restrict__ lam_new, const float2* __restrict__ x, const float* __restrict__ rh_old,
    float* __restrict__ ru, unsigned* __restrict__ status) {
  const ChunkInfo ck = chunks[blockIdx.x];
  const RowInfo ri = rows[ck.row];
  const int t = threadIdx.x;
  __shared__ cf sRt[M][M];
  __shared__ cf sa[M], sb[M];
  __shared__ double2 aug[M][2 * M];
  __shared__ float2 sR[M * M];
  RCSCM_DASSERT(ri.M == M);
  RCSCM_DASSERT(ck.start >= 0 && ck.len >= 1 && ck.start + ck.len <= ri.J);
  naive_row_model<M>(rsf + ck.row, lam_old[ck.row], sRt, sa, sb);
  const float l = wave_sum_packed<0>(part + ri.part_off, ri.nparts).mean(1.0 / (double)ri.J);
  if (ck.start == 0 && t == 0) {
    lam_new[ck.row] = l;
    if (!(l > 0.0f) || !isfinite(l)) atomicOr(status + ck.row, ST_LAM_NONPOS);
  }
  naive_rinv<M>(rcd + ck.row, l, sR, aug);
  __syncthreads();
  bool bad = false, bad_e = false;
  for (int jj = t; jj < ck.len; jj += kNT) {
    const long long bin = ri.bin_off + ck.start + jj;
    const float2* xp = x + ri.x_off + (long long)(ck.start + jj) * M;
    cf xv[M];
#pragma unroll
    for (int m = 0; m < M; ++m) xv[m] = cmk(xp[m].x, xp[m].y);
    const float h = rh_old[bin], u = ru[bin];
    // the same order and arithmetic as the trace of the stored form
    float tr = 0.0f;
    naive_estep<M>(sRt, sa, xv, h, u, bad_e, [&](int m, int n, cf U) {
      if (m == n) {
        tr = fmaf(sR[m * M + m].x, U.x, tr);
      } else {
        // 2 Re(Rinv[n][m] U[m][n])
        const float2 r = sR[n * M + m];
        tr = fmaf(2.0f, fmaf(r.x, U.x, -r.y * U.y), tr);
      }
    });
    const float v = tr * (1.0f / (float)M);
    ru[bin] = v;
    bad = bad || !isfinite(v);
  }
  if (bad) atomicOr(status + ck.row, ST_NONFINITE_STATE);
}

}  // namespace

void launch_naive_a(hipStream_t s, int M, bool store_u, int nchunks, const ChunkInfo* chunks,
                    const RowInfo* rows, const RowSpatialF* rsf, const float2* x, float* rh,
                    const float* ru, const float* lam, float* uhat, long long nbins,
                    uint64_t* part, float alpha, float beta, unsigned* status) {
  if (nchunks <= 0) return;
  const float inv_a2 = (float)(1.0 / ((double)alpha + 2.0));
  const float beta_a2 = (float)((double)beta / ((double)alpha + 2.0));
#define RCSCM_NA(MM)                                                                         \
  case MM:                                                                                   \
    if (store_u)                                                                             \
      hipLaunchKernelGGL((naive_a_kernel<MM, true>), dim3(nchunks), dim3(kNT), 0, s, chunks, \
                         rows, rsf, x, rh, ru, lam, uhat, nbins, part, inv_a2, beta_a2,      \
                         status);                                                            \
    else                                                                                     \
      hipLaunchKernelGGL((naive_a_kernel<MM, false>), dim3(nchunks), dim3(kNT), 0, s,        \
                         chunks, rows, rsf, x, rh, ru, lam, uhat, nbins, part, inv_a2,       \
                         beta_a2, status);                                                   \
    break;
  switch (M) {
    RCSCM_NA(2)
    RCSCM_NA(3)
    RCSCM_NA(4)
    RCSCM_NA(5)
    RCSCM_NA(6)
    RCSCM_NA(7)
    RCSCM_NA(8)
    default: break;
  }
#undef RCSCM_NA
}

void launch_naive_b(hipStream_t s, int M, int nchunks, const ChunkInfo* chunks,
                    const RowInfo* rows, const RowConstD* rcd, const uint64_t* part, float* lam,
                    float* ru, const float* uhat, long long nbins, unsigned* status) {
  if (nchunks <= 0) return;
#define RCSCM_NB(MM)                                                                           \
  case MM:                                                                                     \
    hipLaunchKernelGGL(naive_b_kernel<MM>, dim3(nchunks), dim3(kNT), 0, s, chunks, rows, rcd, \
                       part, lam, ru, uhat, nbins, status);                                    \
    break;
  switch (M) {
    RCSCM_NB(2)
    RCSCM_NB(3)
    RCSCM_NB(4)
    RCSCM_NB(5)
    RCSCM_NB(6)
    RCSCM_NB(7)
    RCSCM_NB(8)
    default: break;
  }
#undef RCSCM_NB
}

void launch_naive_b_recompute(hipStream_t s, int M, int nchunks, const ChunkInfo* chunks,
                              const RowInfo* rows, const RowSpatialF* rsf, const RowConstD* rcd,
                              const uint64_t* part, const float* lam_old, float* lam_new,
                              const float2* x, const float* rh_old, float* ru,
                              unsigned* status) {
  if (nchunks <= 0) return;
#define RCSCM_NBR(MM)                                                                      \
  case MM:                                                                                 \
    hipLaunchKernelGGL(naive_b_recompute_kernel<MM>, dim3(nchunks), dim3(kNT), 0, s, chunks, \
                       rows, rsf, rcd, part, lam_old, lam_new, x, rh_old, ru, status);       \
    break;
  switch (M) {
    RCSCM_NBR(2)
    RCSCM_NBR(3)
    RCSCM_NBR(4)
    RCSCM_NBR(5)
    RCSCM_NBR(6)
    RCSCM_NBR(7)
    RCSCM_NBR(8)
    default: break;
  }
#undef RCSCM_NBR
}

}  // namespace rcscm
