// Per-frequency FP64 setup (one workgroup of 64 lanes per row).
//
// For each (utterance, frequency) row, from a_i, R'_i, b_i (complex128):
//   1. b <- b / ||b||   (warning bit if ||b|| was not 1 within 1e-6);
//   2. null check ||R' b|| <= 1e-6 ||R'||_F  (b must span the null space of
//      the rank-(M-1) SCM, Sec. II-B-1);
//   3. R' <- P R' P with P = I - b b^H, Hermitised (removes rounding in R'b);
//   4. A = R' + s b b^H, s = tr(R')/(M-1), Cholesky A = C C^H in FP64.  Since
//      R' b = 0 and ||b|| = 1, A^{-1} = (R')^+ + b b^H / s, which is the
//      pseudoinverse expansion of eq. (26) read the other way;
//   5. G = C^{-1} P, so F = G^H satisfies F F^H = P A^{-1} P = (R')^+;
//   6. g = G a, tau^(aa) = |g|^2 (eq. (46)), c = (R')^+ a = G^H g,
//      sigma^(ab) = a^H b (eq. (32)), log pdet(R') = log det A - log s.
#include "rcscm_internal.h"

namespace rcscm {

namespace {

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ inline bool finite2(double2 v) { return isfinite(v.x) && isfinite(v.y); }

__global__ __launch_bounds__(64) void setup_kernel(const RowInfo* __restrict__ rows,
                                                   const double2* __restrict__ a_in,
                                                   const double2* __restrict__ rp_in,
                                                   const double2* __restrict__ b_in,
                                                   RowConstD* __restrict__ rcd,
                                                   RowConstF* __restrict__ rcf,
                                                   RowSpatialF* __restrict__ rsf,
                                                   unsigned* __restrict__ status) {
  const int r = blockIdx.x;
  const int t = threadIdx.x;
  const RowInfo ri = rows[r];
  const int M = ri.M;
  const int MM = M * M;

  __shared__ double2 sR[MAXM][MAXM];   // R', then projected R'
  __shared__ double2 sA[MAXM][MAXM];   // work matrix
  __shared__ double2 sL[MAXM][MAXM];   // Cholesky factor C (lower)
  __shared__ double2 sLi[MAXM][MAXM];  // C^{-1}
  __shared__ double2 sG[MAXM][MAXM];   // G = C^{-1} P
  __shared__ double2 sa[MAXM], sb[MAXM], sy[MAXM], sv[MAXM], sg[MAXM];
  __shared__ double sd[4];
  __shared__ unsigned sflag;

  if (t == 0) sflag = 0u;
  if (t < M) {
    sa[t] = a_in[ri.a_off + t];
    sb[t] = b_in[ri.a_off + t];
  }
  if (t < MM) sR[t / M][t % M] = rp_in[ri.rp_off + t];
  __syncthreads();

  if (t == 0) {
    bool fin = true;
    double nb2 = 0.0, nr2 = 0.0;
    for (int m = 0; m < M; ++m) {
      fin = fin && finite2(sa[m]) && finite2(sb[m]);
      nb2 += sb[m].x * sb[m].x + sb[m].y * sb[m].y;
    }
    for (int i = 0; i < M; ++i)
      for (int j = 0; j < M; ++j) {
        fin = fin && finite2(sR[i][j]);
        nr2 += sR[i][j].x * sR[i][j].x + sR[i][j].y * sR[i][j].y;
      }
    unsigned f = 0u;
    if (!fin) f |= ST_NONFINITE_IN;
    const double nb = sqrt(nb2);
    if (!(nb > 0.0) || !fin) f |= ST_NOT_NULL;
    else if (fabs(nb - 1.0) > 1e-6) f |= ST_B_NOT_UNIT;
    sd[0] = (nb > 0.0 && fin) ? 1.0 / nb : 0.0;
    sd[1] = sqrt(nr2);
    sflag = f;
  }
  __syncthreads();
  if (t < M) sb[t] = make_double2(sb[t].x * sd[0], sb[t].y * sd[0]);
  __syncthreads();

  // y = R' b
  if (t < M) {
    double2 acc = make_double2(0.0, 0.0);
    for (int n = 0; n < M; ++n) {
      const double2 p = cmul(sR[t][n], sb[n]);
      acc.x += p.x;
      acc.y += p.y;
    }
    sy[t] = acc;
  }
  __syncthreads();
  if (t == 0) {
    double ny2 = 0.0;
    double2 be = make_double2(0.0, 0.0);  // b^H R' b
    for (int m = 0; m < M; ++m) {
      ny2 += sy[m].x * sy[m].x + sy[m].y * sy[m].y;
      const double2 p = cmulc(sb[m], sy[m]);
      be.x += p.x;
      be.y += p.y;
    }
    if (!(sqrt(ny2) <= 1e-6 * sd[1])) sflag |= ST_NOT_NULL;
    sd[2] = be.x;
  }
  __syncthreads();
  // projected R'_ij = R_ij - b_i conj(y_j) - y_i conj(b_j) + (b^H R' b) b_i conj(b_j)
  if (t < MM) {
    const int i = t / M, j = t % M;
    const double2 bi_yj = cmul(sb[i], cconj(sy[j]));
    const double2 yi_bj = cmul(sy[i], cconj(sb[j]));
    const double2 bi_bj = cmul(sb[i], cconj(sb[j]));
    sA[i][j] = make_double2(sR[i][j].x - bi_yj.x - yi_bj.x + sd[2] * bi_bj.x,
                            sR[i][j].y - bi_yj.y - yi_bj.y + sd[2] * bi_bj.y);
  }
  __syncthreads();
  if (t < MM) {  // Hermitise
    const int i = t / M, j = t % M;
    sR[i][j] = make_double2(0.5 * (sA[i][j].x + sA[j][i].x), 0.5 * (sA[i][j].y - sA[j][i].y));
  }
  __syncthreads();
  if (t == 0) {
    double tr = 0.0;
    for (int m = 0; m < M; ++m) tr += sR[m][m].x;
    sd[3] = (tr > 0.0) ? tr / (double)(M - 1) : 1.0;  // scale s of the b b^H term
  }
  __syncthreads();
  // A = R' + s b b^H (full), L = 0
  if (t < MM) {
    const int i = t / M, j = t % M;
    const double2 bb = cmul(sb[i], cconj(sb[j]));
    sA[i][j] = make_double2(sR[i][j].x + sd[3] * bb.x, sR[i][j].y + sd[3] * bb.y);
    sL[i][j] = make_double2(0.0, 0.0);
    sLi[i][j] = make_double2(0.0, 0.0);
  }
  __syncthreads();
  if (t == 0) {
    double dmax = 0.0;
    for (int m = 0; m < M; ++m) dmax = fmax(dmax, sA[m][m].x);
    sd[1] = dmax;
  }
  __syncthreads();
  // right-looking Cholesky of A
  for (int k = 0; k < M; ++k) {
    if (t == 0) {
      double d = sA[k][k].x;
      if (!(d > 1e-13 * sd[1])) {
        sflag |= ST_NOT_PSD;
        d = fmax(1e-13 * sd[1], 1e-300);
      }
      const double l = sqrt(d);
      sL[k][k] = make_double2(l, 0.0);
      sd[0] = 1.0 / l;
    }
    __syncthreads();
    if (t > k && t < M) sL[t][k] = make_double2(sA[t][k].x * sd[0], sA[t][k].y * sd[0]);
    __syncthreads();
    if (t < MM) {
      const int i = t / M, j = t % M;
      if (j > k && i >= j) {
        const double2 p = cmul(sL[i][k], cconj(sL[j][k]));
        sA[i][j].x -= p.x;
        sA[i][j].y -= p.y;
      }
    }
    __syncthreads();
  }
  // C^{-1}: column j by forward substitution (lane j)
  if (t < M) {
    const int j = t;
    for (int i = j; i < M; ++i) {
      double2 acc = make_double2(i == j ? 1.0 : 0.0, 0.0);
      for (int k = j; k < i; ++k) {
        const double2 p = cmul(sL[i][k], sLi[k][j]);
        acc.x -= p.x;
        acc.y -= p.y;
      }
      const double inv = 1.0 / sL[i][i].x;
      sLi[i][j] = make_double2(acc.x * inv, acc.y * inv);
    }
  }
  __syncthreads();
  // v = C^{-1} b
  if (t < M) {
    double2 acc = make_double2(0.0, 0.0);
    for (int n = 0; n < M; ++n) {
      const double2 p = cmul(sLi[t][n], sb[n]);
      acc.x += p.x;
      acc.y += p.y;
    }
    sv[t] = acc;
  }
  __syncthreads();
  // G = C^{-1} - v b^H
  if (t < MM) {
    const int i = t / M, j = t % M;
    const double2 p = cmul(sv[i], cconj(sb[j]));
    sG[i][j] = make_double2(sLi[i][j].x - p.x, sLi[i][j].y - p.y);
  }
  __syncthreads();
  // g = G a
  if (t < M) {
    double2 acc = make_double2(0.0, 0.0);
    for (int n = 0; n < M; ++n) {
      const double2 p = cmul(sG[t][n], sa[n]);
      acc.x += p.x;
      acc.y += p.y;
    }
    sg[t] = acc;
  }
  __syncthreads();

  RowConstD* D = rcd + r;
  RowSpatialF* S = rsf + r;
  if (t < MM) {
    const int i = t / M, j = t % M;
    D->G[i * MAXM + j] = sG[i][j];
    D->Rp[i * MAXM + j] = sR[i][j];
    S->Rp[i * MAXM + j] = make_float2((float)sR[i][j].x, (float)sR[i][j].y);
  }
  if (t < M) {
    // c = G^H g
    double2 acc = make_double2(0.0, 0.0);
    for (int n = 0; n < M; ++n) {
      const double2 p = cmulc(sG[n][t], sg[n]);
      acc.x += p.x;
      acc.y += p.y;
    }
    D->c[t] = acc;
    D->g[t] = sg[t];
    D->b[t] = sb[t];
    D->a[t] = sa[t];
    S->a[t] = make_float2((float)sa[t].x, (float)sa[t].y);
    S->b[t] = make_float2((float)sb[t].x, (float)sb[t].y);
  }
  if (t == 0) {
    double taa = 0.0, ld = 0.0;
    double2 sab = make_double2(0.0, 0.0);
    for (int m = 0; m < M; ++m) {
      taa += sg[m].x * sg[m].x + sg[m].y * sg[m].y;
      const double2 p = cmulc(sa[m], sb[m]);
      sab.x += p.x;
      sab.y += p.y;
      ld += 2.0 * log(sL[m][m].x);
    }
    D->t_aa = taa;
    D->s_ab = sab;
    D->logpdet = ld - log(sd[3]);
    RowConstF F;
    F.t_aa = (float)taa;
    F.sab_re = (float)sab.x;
    F.sab_im = (float)sab.y;
    F.sab2 = (float)(sab.x * sab.x + sab.y * sab.y);
    F.inv_t_aa = (taa > 0.0) ? (float)(1.0 / taa) : 0.0f;
    F.invM = (float)(1.0 / (double)M);
    F.invJ = (float)(1.0 / (double)ri.J);
    F.pad = 0.0f;
    rcf[r] = F;
    status[r] |= sflag;
  }
}

}  // namespace

void launch_setup(hipStream_t s, int nrows, const RowInfo* rows, const double2* a,
                  const double2* Rp, const double2* b, RowConstD* rcd, RowConstF* rcf,
                  RowSpatialF* rsf, unsigned* status) {
  if (nrows <= 0) return;
  hipLaunchKernelGGL(setup_kernel, dim3(nrows), dim3(64), 0, s, rows, a, Rp, b, rcd, rcf, rsf,
                     status);
}

}  // namespace rcscm
