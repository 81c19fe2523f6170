// First-stage accelerated EM update (Algorithm 1) on gfx950.
//
// Sherman-Morrison (eqs. (24)-(25)) removes the per-bin inverse, but every
// iteration still inverts R~_i = R' + lambda~ b b^H and R_i = R' + lambda b b^H
// once per frequency and evaluates quadratic forms with them per bin:
//   rho~aa = a^H R~^{-1} a,  rho~ax = a^H R~^{-1} x                 eqs. (28), (30)
//   gamma~ = r~h / (r~u + r~h rho~aa)                               eq. (34)
//   r^h    = (gamma~ (r~u + gamma~ |rho~ax|^2) + beta) / (alpha+2)  eq. (39)
//   lambda = mean_j (gamma~ |sigma^ab|^2 + |sigma^bx - gamma~ conj(sigma^ab) rho~ax|^2 / r~u)   eq. (43)
//   rho^aa, rho^ax, rho^xx with R^{-1}                               eqs. (27), (29), (31)
//   r^u    = (gamma~ rho^aa (r~u + gamma~|rho~ax|^2) + rho^xx
//             - 2 gamma~ Re[rho~ax conj(rho^ax)]) / M                eq. (45)
// One workgroup per row keeps x (and sigma^bx, r^h, r^u) of its frames in
// registers for all K iterations; wave 0 inverts R_i in FP64 once per
// iteration (Gauss-Jordan in LDS; R~ of the next iteration is the same matrix,
// so its inverse is reused); the per-bin work is float, O(M^2) per bin for
// rho^xx.  x must stay valid (the context borrows it).
#include "accel_common.h"
#include "small_linalg.h"

namespace rcscm {

namespace {

constexpr int kFirstNT = 256;

template <int M>
__device__ void row_inverse_wave(const RowConstD* D, double lam, double2 (*aug)[2 * M],
                                 float2 (*Rinv)[M], float2* d, float* rho_aa) {
  // R = R' + lam b b^H, R^{-1} into Rinv (float), d = R^{-1} a, rho_aa = a^H d
  const int t = threadIdx.x;
  const int i = t / M, j = t % M;
  if (t < M * M) {
    const double2 bb = zmul(D->b[i], zconj(D->b[j]));
    const double2 rp = D->Rp[i * MAXM + j];
    aug[i][j] = make_double2(rp.x + lam * bb.x, rp.y + lam * bb.y);
    aug[i][M + j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  wave_sync();
  double det;
  gj_inverse_hpd_wave<M>(aug, 0.0, &det);
  if (t < M * M) Rinv[i][j] = make_float2((float)aug[i][M + j].x, (float)aug[i][M + j].y);
  double2 dv = make_double2(0.0, 0.0);
  if (t < M) {
#pragma unroll
    for (int n = 0; n < M; ++n) {
      const double2 p = zmul(aug[t][M + n], D->a[n]);
      dv.x += p.x;
      dv.y += p.y;
    }
    d[t] = make_float2((float)dv.x, (float)dv.y);
  }
  const double2 ad = (t < M) ? zmulc(D->a[t], dv) : make_double2(0.0, 0.0);
  const double raa = wave_sum_d(ad.x);
  if (t == 0) *rho_aa = (float)raa;
}

template <int M, int BPL>
__global__ __launch_bounds__(kFirstNT) void first_stage_kernel(
    const int* __restrict__ row_list, const RowInfo* __restrict__ rows,
    const RowConstF* __restrict__ rcf, const RowConstD* __restrict__ rcd,
    const float2* __restrict__ x, float* __restrict__ rh, float* __restrict__ ru,
    float* __restrict__ lam, float inv_a2, float beta_a2, int K, unsigned* __restrict__ status) {
  constexpr int NW = kFirstNT / 64;
  const int row = row_list[blockIdx.x];
  const RowInfo ri = rows[row];
  const RowConstF rc = rcf[row];
  const RowConstD* D = rcd + row;
  const int J = ri.J;
  const long long base = ri.bin_off;
  const int t = threadIdx.x;
  RCSCM_DASSERT(ri.M == M && J >= 1 && J <= kFirstNT * BPL);
  const double invJ = 1.0 / (double)J;

  __shared__ double2 aug[M][2 * M];
  __shared__ float2 sRi[M][M];
  __shared__ float2 sd[M];
  __shared__ float sraa;
  __shared__ uint64_t red[2][NW];
  __shared__ float2 sb[M];
  if (t < M) sb[t] = make_float2((float)D->b[t].x, (float)D->b[t].y);

  float2 xv[BPL][M];
  float sbr[BPL], sbi[BPL], vrh[BPL], vru[BPL];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < BPL; ++q) {
    const int j = t + q * kFirstNT;
    float br = 0.f, bi = 0.f;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      xv[q][m] = (j < J) ? x[ri.x_off + (long long)j * M + m] : make_float2(0.f, 0.f);
      // sigma^bx = b^H x   (eq. (33))
      br = fmaf(sb[m].x, xv[q][m].x, fmaf(sb[m].y, xv[q][m].y, br));
      bi = fmaf(sb[m].x, xv[q][m].y, fmaf(-sb[m].y, xv[q][m].x, bi));
    }
    sbr[q] = br;
    sbi[q] = bi;
    vrh[q] = (j < J) ? rh[base + j] : 1.f;
    vru[q] = (j < J) ? ru[base + j] : 1.f;
  }
  float lam_t = lam[row];
  // R~^{-1} of the first iteration; later iterations reuse the R^{-1} of the
  // previous one (R~_{k+1} = R' + lambda_k b b^H = R_k)
  if (K > 0 && t < 64) row_inverse_wave<M>(D, (double)lam_t, aug, sRi, sd, &sraa);
  __syncthreads();

  for (int k = 0; k < K; ++k) {
    const float rho_aa_t = sraa;
    float g[BPL], rxr[BPL], rxi[BPL];
    LamAcc<0> acc;
#pragma unroll
    for (int q = 0; q < BPL; ++q) {
      float pr = 0.f, pi = 0.f;  // rho~ax = d~^H x
#pragma unroll
      for (int m = 0; m < M; ++m) {
        pr = fmaf(sd[m].x, xv[q][m].x, fmaf(sd[m].y, xv[q][m].y, pr));
        pi = fmaf(sd[m].x, xv[q][m].y, fmaf(-sd[m].y, xv[q][m].x, pi));
      }
      const float h = vrh[q], u = vru[q];
      const float gg = h * frcp(fmaf(h, rho_aa_t, u));
      const float r2 = fmaf(pr, pr, pi * pi);
      vrh[q] = fmaf(gg * fmaf(gg, r2, u), inv_a2, beta_a2);
      // e = sigma^bx - gamma~ conj(sigma^ab) rho~ax
      const float wr = gg * pr, wi = gg * pi;
      const float er = sbr[q] - fmaf(rc.sab_re, wr, rc.sab_im * wi);
      const float ei = sbi[q] - fmaf(rc.sab_re, wi, -rc.sab_im * wr);
      if (t + q * kFirstNT < J) acc.add(fmaf(gg, rc.sab2, fmaf(er, er, ei * ei) * frcp(u)));
      g[q] = gg;
      rxr[q] = pr;
      rxi[q] = pi;
    }
    acc = wave_allreduce<0>(acc);
    if ((t & 63) == 0) red[k & 1][t >> 6] = acc.pack();
    __syncthreads();
    const float lam_n = slots_sum<0, NW>(red[k & 1]).mean(invJ);
    // R^{-1} with the new lambda
    if (t < 64) row_inverse_wave<M>(D, (double)lam_n, aug, sRi, sd, &sraa);
    __syncthreads();
    const float rho_aa = sraa;
#pragma unroll
    for (int q = 0; q < BPL; ++q) {
      float ar = 0.f, ai = 0.f;  // rho^ax = d^H x
#pragma unroll
      for (int m = 0; m < M; ++m) {
        ar = fmaf(sd[m].x, xv[q][m].x, fmaf(sd[m].y, xv[q][m].y, ar));
        ai = fmaf(sd[m].x, xv[q][m].y, fmaf(-sd[m].y, xv[q][m].x, ai));
      }
      float rxx = 0.f;  // rho^xx = x^H R^{-1} x
#pragma unroll
      for (int p = 0; p < M; ++p) {
        float yr = 0.f, yi = 0.f;
#pragma unroll
        for (int n = 0; n < M; ++n) {
          const float2 r = sRi[p][n];
          yr = fmaf(r.x, xv[q][n].x, fmaf(-r.y, xv[q][n].y, yr));
          yi = fmaf(r.x, xv[q][n].y, fmaf(r.y, xv[q][n].x, yi));
        }
        rxx = fmaf(xv[q][p].x, yr, fmaf(xv[q][p].y, yi, rxx));
      }
      const float gg = g[q];
      const float u = vru[q];
      const float r2 = fmaf(rxr[q], rxr[q], rxi[q] * rxi[q]);
      const float cross = fmaf(rxr[q], ar, rxi[q] * ai);  // Re[rho~ax conj(rho^ax)]
      vru[q] = (gg * rho_aa * fmaf(gg, r2, u) + rxx - 2.0f * gg * cross) * rc.invM;
    }
    lam_t = lam_n;
    // sd, sraa now hold R~^{-1} of the next iteration; wave 0 rewrites them
    // only after that iteration's frame-sum barrier
  }
  bool bad = false;
#pragma unroll
  for (int q = 0; q < BPL; ++q) {
    const int j = t + q * kFirstNT;
    if (j < J) {
      rh[base + j] = vrh[q];
      ru[base + j] = vru[q];
      bad = bad || !isfinite(vrh[q]) || !isfinite(vru[q]) || !(vru[q] > 0.0f);
    }
  }
  if (t == 0) {
    lam[row] = lam_t;
    if (!(lam_t > 0.0f) || !isfinite(lam_t)) atomicOr(status + row, ST_LAM_NONPOS);
  }
  if (bad) atomicOr(status + row, ST_NONFINITE_STATE);
}

template <int M>
void first_launch_m(hipStream_t s, int bpl, int nrows, const int* row_list, const RowInfo* rows,
                    const RowConstF* rcf, const RowConstD* rcd, const float2* x, float* rh,
                    float* ru, float* lam, float inv_a2, float beta_a2, int K,
                    unsigned* status) {
#define RCSCM_FS(B)                                                                            \
  case B:                                                                                      \
    hipLaunchKernelGGL((first_stage_kernel<M, B>), dim3(nrows), dim3(kFirstNT), 0, s, row_list, \
                       rows, rcf, rcd, x, rh, ru, lam, inv_a2, beta_a2, K, status);            \
    break;
  switch (bpl) {
    RCSCM_FS(1)
    RCSCM_FS(2)
    RCSCM_FS(4)
    RCSCM_FS(8)
    RCSCM_FS(16)
    default: break;
  }
#undef RCSCM_FS
}

}  // namespace

int first_stage_bpl(int J) {
  for (int b : {1, 2, 4, 8, 16})
    if (b * kFirstNT >= J) return b;
  return -1;
}

void launch_first_stage(hipStream_t s, int M, int bpl, int nrows, const int* row_list,
                        const RowInfo* rows, const RowConstF* rcf, const RowConstD* rcd,
                        const float2* x, float* rh, float* ru, float* lam, float alpha,
                        float beta, int K, unsigned* status) {
  if (nrows <= 0 || K <= 0) return;
  const float inv_a2 = (float)(1.0 / ((double)alpha + 2.0));
  const float beta_a2 = (float)((double)beta / ((double)alpha + 2.0));
  switch (M) {
    case 2: first_launch_m<2>(s, bpl, nrows, row_list, rows, rcf, rcd, x, rh, ru, lam, inv_a2, beta_a2, K, status); break;
    case 3: first_launch_m<3>(s, bpl, nrows, row_list, rows, rcf, rcd, x, rh, ru, lam, inv_a2, beta_a2, K, status); break;
    case 4: first_launch_m<4>(s, bpl, nrows, row_list, rows, rcf, rcd, x, rh, ru, lam, inv_a2, beta_a2, K, status); break;
    case 5: first_launch_m<5>(s, bpl, nrows, row_list, rows, rcf, rcd, x, rh, ru, lam, inv_a2, beta_a2, K, status); break;
    case 6: first_launch_m<6>(s, bpl, nrows, row_list, rows, rcf, rcd, x, rh, ru, lam, inv_a2, beta_a2, K, status); break;
    case 7: first_launch_m<7>(s, bpl, nrows, row_list, rows, rcf, rcd, x, rh, ru, lam, inv_a2, beta_a2, K, status); break;
    case 8: first_launch_m<8>(s, bpl, nrows, row_list, rows, rcf, rcd, x, rh, ru, lam, inv_a2, beta_a2, K, status); break;
    default: break;
  }
}

}  // namespace rcscm
