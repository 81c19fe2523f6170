// Rank-(M-1) SCM of the diffuse noise from a demixing matrix, and the
// paper's initialisation of r^u and lambda (Sec. II-B-1 eq. (11); Sec. II-B-3
// eqs. (22), (23)), in FP64.
//
// With W_i = (w_1 ... w_M)^H, y_ij = W_i x_ij and A_i = W_i^{-1} = (a_1 ... a_M):
//   eq. (11)  R'_i = (1/J) sum_j A diag(|y_1|^2, .., 0 at n_h, .., |y_M|^2) A^H
//                  = sum_{m != n_h} p_m a_m a_m^H,   p_m = (1/J) sum_j |y_m,ij|^2
//   b_i = w_{n_h} / |w_{n_h}|   (W A = I, so R' w_{n_h} = 0: the null vector)
//   a_i = a_{n_h}               (the target's steering vector)
//   eqs. (22)-(23): y^(u) = A (y with the n_h-th entry zeroed) lies in
//   range(R') = span{a_m, m != n_h}; for R' = B P B^H with B of full column
//   rank, (R')^+ = B^{+H} P^{-1} B^+, hence
//   r^u_0 = (1/M) y^(u)H (R')^+ y^(u) = (1/M) sum_{m != n_h} |y_m|^2 / p_m
//   lambda_0 = min nonzero eigenvalue of R' = min eigenvalue of the
//   (M-1) x (M-1) Gram matrix P^{1/2} B^H B P^{1/2} (multisection on a
//   positive-definiteness test, one shift per lane).
// Launches: for M <= kBpFusedMaxM and rows of up to kBpFusedMaxJ frames one
// bp_fused per row (all of the below in one workgroup); otherwise bp_power
// (per chunk: partial sums of |y_m|^2), bp_row (per row: A = W^{-1} by
// Gauss-Jordan with partial pivoting, a, R', b, lambda_0) and bp_ru (per
// chunk: r^u_0).
#include "accel_common.h"
#include "small_linalg.h"

namespace rcscm {

namespace {

constexpr int kBpNT = 256;

template <int M>
__global__ __launch_bounds__(kBpNT) void bp_power_kernel(const ChunkInfo* __restrict__ chunks,
                                                         const RowInfo* __restrict__ rows,
                                                         const float2* __restrict__ x,
                                                         const double2* __restrict__ W,
                                                         double* __restrict__ part) {
  const ChunkInfo ck = chunks[blockIdx.x];
  const RowInfo ri = rows[ck.row];
  const int t = threadIdx.x;
  __shared__ double2 sW[M][M];
  __shared__ double red[M][kBpNT / 64];
  if (t < M * M) sW[t / M][t % M] = W[ri.rp_off + t];
  __syncthreads();
  double acc[M];
#pragma unroll
  for (int m = 0; m < M; ++m) acc[m] = 0.0;
  for (int jj = t; jj < ck.len; jj += kBpNT) {
    const float2* xp = x + ri.x_off + (long long)(ck.start + jj) * M;
    double xr[M], xi[M];
#pragma unroll
    for (int n = 0; n < M; ++n) {
      const float2 v = xp[n];
      xr[n] = v.x;
      xi[n] = v.y;
    }
    asm volatile("" ::: "memory");  // keep W in LDS (re-read per bin)
#pragma unroll
    for (int m = 0; m < M; ++m) {
      double yr = 0.0, yi = 0.0;
#pragma unroll
      for (int n = 0; n < M; ++n) {
        yr = fma(sW[m][n].x, xr[n], fma(-sW[m][n].y, xi[n], yr));
        yi = fma(sW[m][n].x, xi[n], fma(sW[m][n].y, xr[n], yi));
      }
      acc[m] = fma(yr, yr, fma(yi, yi, acc[m]));
    }
  }
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const double s = wave_sum_d(acc[m]);
    if ((t & 63) == 0) red[m][t >> 6] = s;
  }
  __syncthreads();
  if (t < M) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kBpNT / 64; ++w) s += red[t][w];
    part[(long long)ck.part * MAXM + t] = s;
  }
}

// Smallest eigenvalue of a Hermitian N x N matrix (N <= 7) by cyclic complex
// True when G - s I is positive definite: every pivot of its LDL^H
// factorisation (no square roots; unit lower L) is positive. For a positive
// definite matrix the factorisation is backward stable, so the answer is
// exact up to rounding of order eps |G| at the boundary s = lambda_min.
template <int N>
__device__ __forceinline__ bool shifted_pd(const double2 (&G)[N][N], double s) {
  double2 L[N][N];
  double d[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    double dk = G[k][k].x - s;
#pragma unroll
    for (int j = 0; j < k; ++j) dk -= d[j] * (L[k][j].x * L[k][j].x + L[k][j].y * L[k][j].y);
    if (!(dk > 0.0)) return false;
    d[k] = dk;
    const double inv = 1.0 / dk;
#pragma unroll
    for (int i = k + 1; i < N; ++i) {
      double2 v = G[i][k];
#pragma unroll
      for (int j = 0; j < k; ++j) {
        const double2 u = zmul(L[i][j], zconj(L[k][j]));  // L_ij conj(L_kj) d_j
        v.x -= u.x * d[j];
        v.y -= u.y * d[j];
      }
      L[i][k] = make_double2(v.x * inv, v.y * inv);
    }
  }
  return true;
}

// Smallest eigenvalue of the N x N Hermitian positive semidefinite G, by
// multisection over the 64 lanes of the wave (all of them must call it):
// G - s I is positive definite exactly when s < lambda_min. The bracket starts
// at [0, min_k G_kk] (no diagonal entry of a Hermitian matrix lies below its
// smallest eigenvalue); in each round lane l tests
// s_l = lo + (hi - lo)(l + 1)/65, and the first lane whose test fails gives
// the bracket 65 times narrower.
template <int N>
__device__ double min_eig_multisection(const double2 (*Gs)[MAXM]) {
  if constexpr (N == 1) {
    return Gs[0][0].x;
  } else {
    double2 G[N][N];
#pragma unroll
    for (int p = 0; p < N; ++p)
#pragma unroll
      for (int q = 0; q < N; ++q) G[p][q] = Gs[p][q];
    double lo = 0.0, hi = G[0][0].x;
#pragma unroll
    for (int k = 1; k < N; ++k) hi = fmin(hi, G[k][k].x);
    if (!(hi > 0.0)) return hi;
    const int lane = threadIdx.x & 63;
    for (int round = 0; round < 16 && hi - lo > 1e-10 * hi; ++round) {
      const double w = (hi - lo) * (1.0 / 65.0);
      const bool pd = shifted_pd<N>(G, lo + w * (double)(lane + 1));
      const unsigned long long fail = __ballot(!pd);
      if (fail == 0ull) {  // every shift lies below lambda_min
        lo = lo + w * 64.0;
      } else {
        const int f = __ffsll(fail) - 1;  // first shift at or above lambda_min
        hi = lo + w * (double)(f + 1);
        lo = lo + w * (double)f;
      }
    }
    return 0.5 * (lo + hi);
  }
}

// LDS of the per-row step.
template <int M>
struct BpRowLDS {
  double2 aug[M][2 * M];
  double sp[M];  // source powers p_m, set by the caller
  int spiv;
  double2 G[MAXM][MAXM];
  unsigned sflag;  // cleared by the caller
};

// The per-row step, run by the 64 lanes of one wave once S.sp holds the
// source powers: A = W^{-1} by Gauss-Jordan with partial pivoting, then a, R',
// b and lambda_0.
template <int M>
__device__ void bp_row_wave(BpRowLDS<M>& S, int row, const RowInfo& ri,
                            const double2* __restrict__ W, int nh, double2* __restrict__ a_out,
                            double2* __restrict__ rp_out, double2* __restrict__ b_out,
                            float* __restrict__ lam0_out, unsigned* __restrict__ status) {
  const int t = threadIdx.x & 63;
  const int i = t / M, j = t % M;
  const bool ent = t < M * M;
  if (ent) {
    S.aug[i][j] = W[ri.rp_off + t];
    S.aug[i][M + j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  wave_sync();
  // Gauss-Jordan with partial pivoting: aug = [W | I] -> [I | W^{-1}]
  for (int k = 0; k < M; ++k) {
    if (t == 0) {
      int best = k;
      double bm = -1.0;
      for (int r = k; r < M; ++r) {
        const double m2 = S.aug[r][k].x * S.aug[r][k].x + S.aug[r][k].y * S.aug[r][k].y;
        if (m2 > bm) {
          bm = m2;
          best = r;
        }
      }
      if (!(bm > 0.0)) S.sflag |= ST_NOT_PSD;  // singular demixing matrix
      S.spiv = best;
    }
    wave_sync();
    const int pr = S.spiv;
    if (pr != k && t < 2 * M) {  // swap rows k and pr
      const double2 tmp = S.aug[k][t];
      S.aug[k][t] = S.aug[pr][t];
      S.aug[pr][t] = tmp;
    }
    wave_sync();
    const double2 pv = S.aug[k][k];
    const double pm = pv.x * pv.x + pv.y * pv.y;
    const double2 ip = pm > 0.0 ? make_double2(pv.x / pm, -pv.y / pm) : make_double2(0.0, 0.0);
    double2 f = make_double2(0.0, 0.0), r1 = f, r2 = f;
    if (ent) {
      f = S.aug[i][k];
      r1 = S.aug[k][j];
      r2 = S.aug[k][M + j];
    }
    wave_sync();
    if (ent) {
      const double2 n1 = zmul(r1, ip), n2 = zmul(r2, ip);
      if (i == k) {
        S.aug[k][j] = n1;
        S.aug[k][M + j] = n2;
      } else {
        const double2 d1 = zmul(f, n1), d2 = zmul(f, n2);
        S.aug[i][j] = make_double2(S.aug[i][j].x - d1.x, S.aug[i][j].y - d1.y);
        S.aug[i][M + j] = make_double2(S.aug[i][M + j].x - d2.x, S.aug[i][M + j].y - d2.y);
      }
    }
    wave_sync();
  }
  // A = W^{-1} = aug[:, M:]; column m of A is aug[.][M + m]
  if (ent) {  // R' = sum_{m != nh} p_m a_m a_m^H
    double2 sum = make_double2(0.0, 0.0);
#pragma unroll
    for (int m = 0; m < M; ++m) {
      if (m == nh) continue;
      const double2 v = zmul(S.aug[i][M + m], zconj(S.aug[j][M + m]));
      sum.x += S.sp[m] * v.x;
      sum.y += S.sp[m] * v.y;
    }
    rp_out[ri.rp_off + t] = sum;
  }
  if (t < M) {
    a_out[ri.a_off + t] = S.aug[t][M + nh];
    // b = w_nh / |w_nh|, w_nh = conj of row nh of W
    double nw = 0.0;
#pragma unroll
    for (int n = 0; n < M; ++n) {
      const double2 v = W[ri.rp_off + nh * M + n];
      nw += v.x * v.x + v.y * v.y;
    }
    const double2 w = W[ri.rp_off + nh * M + t];
    const double inw = nw > 0.0 ? 1.0 / sqrt(nw) : 0.0;
    b_out[ri.a_off + t] = make_double2(w.x * inw, -w.y * inw);
  }
  if (lam0_out != nullptr) {
    // Gram matrix of the noise steering vectors, weighted by sqrt(p)
    const int n1 = M - 1;
    if (t < n1 * n1) {
      const int k = t / n1, l = t % n1;
      const int mk = k < nh ? k : k + 1, ml = l < nh ? l : l + 1;
      double2 sum = make_double2(0.0, 0.0);
#pragma unroll
      for (int r = 0; r < M; ++r) {
        const double2 v = zmulc(S.aug[r][M + mk], S.aug[r][M + ml]);
        sum.x += v.x;
        sum.y += v.y;
      }
      const double w = sqrt(S.sp[mk] * S.sp[ml]);
      S.G[k][l] = make_double2(w * sum.x, w * sum.y);
    }
    wave_sync();
    const double lmin = min_eig_multisection<M - 1>(S.G);
    if (t == 0) lam0_out[row] = (float)lmin;
  }
  wave_sync();
  if (t == 0 && S.sflag) atomicOr(status + row, S.sflag);
}

template <int M>
__global__ __launch_bounds__(64) void bp_row_kernel(const int* __restrict__ row_list,
                                                    const RowInfo* __restrict__ rows,
                                                    const double2* __restrict__ W,
                                                    const int* __restrict__ target,
                                                    const double* __restrict__ part,
                                                    double2* __restrict__ a_out,
                                                    double2* __restrict__ rp_out,
                                                    double2* __restrict__ b_out,
                                                    double* __restrict__ p_out,
                                                    float* __restrict__ lam0_out,
                                                    unsigned* __restrict__ status) {
  const int row = row_list[blockIdx.x];
  const RowInfo ri = rows[row];
  const int t = threadIdx.x;
  __shared__ BpRowLDS<M> S;
  if (t == 0) S.sflag = 0u;
  if (t < M) {  // p_m = mean_j |y_m|^2
    double sum = 0.0;
    for (int k = 0; k < ri.nparts; ++k) sum += part[(long long)(ri.part_off + k) * MAXM + t];
    S.sp[t] = sum / (double)ri.J;
    p_out[(long long)row * MAXM + t] = S.sp[t];
  }
  bp_row_wave<M>(S, row, ri, W, target[row], a_out, rp_out, b_out, lam0_out, status);
}

template <int M>
__global__ __launch_bounds__(kBpNT) void bp_ru_kernel(const ChunkInfo* __restrict__ chunks,
                                                      const RowInfo* __restrict__ rows,
                                                      const float2* __restrict__ x,
                                                      const double2* __restrict__ W,
                                                      const int* __restrict__ target,
                                                      const double* __restrict__ p,
                                                      float* __restrict__ ru0) {
  const ChunkInfo ck = chunks[blockIdx.x];
  const RowInfo ri = rows[ck.row];
  const int t = threadIdx.x;
  const int nh = target[ck.row];
  __shared__ double2 sW[M][M];
  __shared__ double sip[M];
  if (t < M * M) sW[t / M][t % M] = W[ri.rp_off + t];
  if (t < M) {
    const double pm = p[(long long)ck.row * MAXM + t];
    sip[t] = (t != nh && pm > 0.0) ? 1.0 / pm : 0.0;
  }
  __syncthreads();
  for (int jj = t; jj < ck.len; jj += kBpNT) {
    const float2* xp = x + ri.x_off + (long long)(ck.start + jj) * M;
    double xr[M], xi[M];
#pragma unroll
    for (int n = 0; n < M; ++n) {
      const float2 v = xp[n];
      xr[n] = v.x;
      xi[n] = v.y;
    }
    asm volatile("" ::: "memory");  // keep W in LDS (re-read per bin)
    double e = 0.0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      double yr = 0.0, yi = 0.0;
#pragma unroll
      for (int n = 0; n < M; ++n) {
        yr = fma(sW[m][n].x, xr[n], fma(-sW[m][n].y, xi[n], yr));
        yi = fma(sW[m][n].x, xi[n], fma(sW[m][n].y, xr[n], yi));
      }
      e = fma(fma(yr, yr, yi * yi), sip[m], e);
    }
    ru0[ri.bin_off + ck.start + jj] = (float)(e / (double)M);
  }
}

// The whole back-projection of one row in one workgroup (rows of up to
// kBpFusedMaxJ frames): the source powers over the row's frames, then wave 0
// runs the per-row step while every wave forms r^u_0 from a second pass over
// the row's x (which the first pass left in L2; the second pass needs only W
// and 1/p_m, so it does not wait for wave 0).
template <int M>
__global__ __launch_bounds__(kBpNT) void bp_fused_kernel(
    const int* __restrict__ row_list, const RowInfo* __restrict__ rows,
    const float2* __restrict__ x, const double2* __restrict__ W, const int* __restrict__ target,
    double2* __restrict__ a_out, double2* __restrict__ rp_out, double2* __restrict__ b_out,
    double* __restrict__ p_out, float* __restrict__ ru0, float* __restrict__ lam0_out,
    unsigned* __restrict__ status) {
  const int row = row_list[blockIdx.x];
  const RowInfo ri = rows[row];
  const int t = threadIdx.x;
  const int nh = target[row];
  __shared__ double2 sW[M][M];
  __shared__ double red[M][kBpNT / 64];
  __shared__ double sip[M];
  __shared__ BpRowLDS<M> S;
  if (t < M * M) sW[t / M][t % M] = W[ri.rp_off + t];
  if (t == 0) S.sflag = 0u;
  __syncthreads();
  double acc[M];
#pragma unroll
  for (int m = 0; m < M; ++m) acc[m] = 0.0;
  for (int jj = t; jj < ri.J; jj += kBpNT) {  // p_m: sum over frames of |y_m|^2
    const float2* xp = x + ri.x_off + (long long)jj * M;
    double xr[M], xi[M];
#pragma unroll
    for (int n = 0; n < M; ++n) {
      const float2 v = xp[n];
      xr[n] = v.x;
      xi[n] = v.y;
    }
    asm volatile("" ::: "memory");  // keep W in LDS (re-read per bin)
#pragma unroll
    for (int m = 0; m < M; ++m) {
      double yr = 0.0, yi = 0.0;
#pragma unroll
      for (int n = 0; n < M; ++n) {
        yr = fma(sW[m][n].x, xr[n], fma(-sW[m][n].y, xi[n], yr));
        yi = fma(sW[m][n].x, xi[n], fma(sW[m][n].y, xr[n], yi));
      }
      acc[m] = fma(yr, yr, fma(yi, yi, acc[m]));
    }
  }
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const double w = wave_sum_d(acc[m]);
    if ((t & 63) == 0) red[m][t >> 6] = w;
  }
  __syncthreads();
  if (t < M) {
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < kBpNT / 64; ++w) sum += red[t][w];
    const double pm = sum / (double)ri.J;
    S.sp[t] = pm;
    p_out[(long long)row * MAXM + t] = pm;
    sip[t] = (t != nh && pm > 0.0) ? 1.0 / pm : 0.0;
  }
  __syncthreads();
  if (t < 64) bp_row_wave<M>(S, row, ri, W, nh, a_out, rp_out, b_out, lam0_out, status);
  if (ru0 == nullptr) return;
  for (int jj = t; jj < ri.J; jj += kBpNT) {  // r^u_0 = (1/M) sum_{m != n_h} |y_m|^2 / p_m
    const float2* xp = x + ri.x_off + (long long)jj * M;
    double xr[M], xi[M];
#pragma unroll
    for (int n = 0; n < M; ++n) {
      const float2 v = xp[n];
      xr[n] = v.x;
      xi[n] = v.y;
    }
    asm volatile("" ::: "memory");
    double e = 0.0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      double yr = 0.0, yi = 0.0;
#pragma unroll
      for (int n = 0; n < M; ++n) {
        yr = fma(sW[m][n].x, xr[n], fma(-sW[m][n].y, xi[n], yr));
        yi = fma(sW[m][n].x, xi[n], fma(sW[m][n].y, xr[n], yi));
      }
      e = fma(fma(yr, yr, yi * yi), sip[m], e);
    }
    ru0[ri.bin_off + jj] = (float)(e / (double)M);
  }
}

}  // namespace

void launch_backproject(hipStream_t s, int M, int nchunks_m, const ChunkInfo* chunks_m,
                        int nrows_m, const int* rows_m_list, const RowInfo* rows, const float2* x,
                        const double2* W, const int* target, double* part, double* p,
                        double2* a_out, double2* rp_out, double2* b_out, float* ru0,
                        float* lam0, unsigned* status, int stage) {
  switch (M) {
#define RCSCM_BP(MM)                                                                           \
  case MM:                                                                                     \
    if (stage == 0 && nchunks_m > 0)                                                           \
      hipLaunchKernelGGL(bp_power_kernel<MM>, dim3(nchunks_m), dim3(kBpNT), 0, s, chunks_m,    \
                         rows, x, W, part);                                                    \
    if (stage == 1 && nrows_m > 0)                                                             \
      hipLaunchKernelGGL(bp_row_kernel<MM>, dim3(nrows_m), dim3(64), 0, s, rows_m_list, rows,   \
                         W, target,                                                            \
                         part, a_out, rp_out, b_out, p, lam0, status);                        \
    if (stage == 2 && nchunks_m > 0 && ru0 != nullptr)                                         \
      hipLaunchKernelGGL(bp_ru_kernel<MM>, dim3(nchunks_m), dim3(kBpNT), 0, s, chunks_m, rows, \
                         x, W, target, p, ru0);                                                \
    if (stage == 3 && nrows_m > 0)                                                             \
      hipLaunchKernelGGL(bp_fused_kernel<MM>, dim3(nrows_m), dim3(kBpNT), 0, s, rows_m_list,    \
                         rows, x, W, target, a_out, rp_out, b_out, p, ru0, lam0, status);       \
    break;
    RCSCM_BP(2)
    RCSCM_BP(3)
    RCSCM_BP(4)
    RCSCM_BP(5)
    RCSCM_BP(6)
    RCSCM_BP(7)
    RCSCM_BP(8)
#undef RCSCM_BP
    default: break;
  }
}

}  // namespace rcscm
