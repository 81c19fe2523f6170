// Per-row FP64 setup and per-bin FP64 precomputation, shared by the init
// kernel (rcscm_init) and the fused single-launch kernel (rcscm_run).
//
// Setup of a row (Algorithm 2, before the loop; eqs. (26), (32), (46)),
// from a_i, R'_i, b_i in complex128:
//   1. b <- b / ||b||   (warning bit if ||b|| was not 1 within 1e-6);
//   2. null check ||R' b|| <= 1e-6 ||R'||_F (b spans the null space of the
//      rank-(M-1) SCM, Sec. II-B-1);
//   3. R' <- P R' P, P = I - b b^H, Hermitised (removes the rounding in R'b);
//   4. A = R' + s b b^H with s = tr(R')/(M-1) is Hermitian positive definite
//      and, because R' b = 0 and ||b|| = 1, A^{-1} = (R')^+ + b b^H / s -
//      the pseudoinverse expansion of eq. (26) with lambda = s.  A^{-1} comes
//      from a lane-parallel Gauss-Jordan elimination (M steps), so
//      (R')^+ = A^{-1} - b b^H / s and log pdet(R') = log det A - log s;
//   5. c = (R')^+ a, tau^(aa) = a^H c, sigma^(ab) = a^H b.
// Precomputation of one bin (eqs. (33), (47), (48)), in FP64 from the
// complex64 x:
//   tau^ax = c^H x,  sigma^bx = b^H x,  tau^xx = x^H (R')^+ x,
//   nu     = tau^xx - |tau^ax|^2 / tau^aa  (>= 0; the FP64 difference is exact
//            to ~1e-16 tau^xx, far below the float rounding of the stored nu).
#pragma once

#include "accel_common.h"
#include "small_linalg.h"

namespace rcscm {

template <int M>
struct SetupLDS {
  double2 sR[M][M];       // R', then the projected R'
  double2 sQ[M][M];       // (R')^+
  double2 aug[M][2 * M];  // Gauss-Jordan work array
  double2 sa[M], sb[M], sy[M], sc[M];
  double taa, sab_re, sab_im, logpdet;
  unsigned flags;
};

// Row setup by wave 0 (lanes t < 64).  Lane t < M*M owns entry
// (t / M, t % M); sums over lanes are uniform DPP reductions.
template <int M>
__device__ void row_setup_wave(const double2* __restrict__ Rp, const double2* __restrict__ a,
                               const double2* __restrict__ b, const RowInfo& ri,
                               SetupLDS<M>& L) {
  const int t = threadIdx.x;
  const int i = t / M, j = t % M;
  const bool ent = t < M * M;
  double2 r = make_double2(0.0, 0.0), av = r, bv = r;
  if (ent) r = Rp[ri.rp_off + t];
  if (t < M) {
    av = a[ri.a_off + t];
    bv = b[ri.a_off + t];
  }
  const bool fin = zfinite(r) && zfinite(av) && zfinite(bv);
  const double nbad = wave_sum_d(fin ? 0.0 : 1.0);
  const double nr2 = wave_sum_d(r.x * r.x + r.y * r.y);
  const double nb2 = wave_sum_d(bv.x * bv.x + bv.y * bv.y);
  unsigned f = 0u;
  const double nb = sqrt(nb2);
  if (nbad > 0.0) f |= ST_NONFINITE_IN;
  if (!(nb > 0.0) || nbad > 0.0)
    f |= ST_NOT_NULL;
  else if (fabs(nb - 1.0) > 1e-6)
    f |= ST_B_NOT_UNIT;
  const double inb = (nb > 0.0 && nbad == 0.0) ? 1.0 / nb : 0.0;
  bv = make_double2(bv.x * inb, bv.y * inb);
  if (ent) L.sR[i][j] = r;
  if (t < M) {
    L.sa[t] = av;
    L.sb[t] = bv;
  }
  wave_sync();
  double2 y = make_double2(0.0, 0.0);  // y = R' b
  if (t < M) {
#pragma unroll
    for (int n = 0; n < M; ++n) {
      const double2 p = zmul(L.sR[t][n], L.sb[n]);
      y.x += p.x;
      y.y += p.y;
    }
    L.sy[t] = y;
  }
  const double ny2 = wave_sum_d(y.x * y.x + y.y * y.y);
  const double be = wave_sum_d(zmulc(bv, y).x);  // b^H R' b
  if (!(sqrt(ny2) <= 1e-6 * sqrt(nr2))) f |= ST_NOT_NULL;
  wave_sync();
  double2 pr = make_double2(0.0, 0.0);  // P R' P = R' - b y^H - y b^H + (b^H R' b) b b^H
  if (ent) {
    const double2 byj = zmul(L.sb[i], zconj(L.sy[j]));
    const double2 ybj = zmul(L.sy[i], zconj(L.sb[j]));
    const double2 bbj = zmul(L.sb[i], zconj(L.sb[j]));
    pr = make_double2(r.x - byj.x - ybj.x + be * bbj.x, r.y - byj.y - ybj.y + be * bbj.y);
    L.aug[i][j] = pr;
  }
  wave_sync();
  double2 rhm = make_double2(0.0, 0.0);  // Hermitised
  if (ent) {
    const double2 pt = L.aug[j][i];
    rhm = make_double2(0.5 * (pr.x + pt.x), 0.5 * (pr.y - pt.y));
  }
  const double tr = wave_sum_d((ent && i == j) ? rhm.x : 0.0);
  const double s = tr > 0.0 ? tr / (double)(M - 1) : 1.0;
  wave_sync();
  if (ent) {
    L.sR[i][j] = rhm;
    const double2 bb = zmul(L.sb[i], zconj(L.sb[j]));
    L.aug[i][j] = make_double2(rhm.x + s * bb.x, rhm.y + s * bb.y);
    L.aug[i][M + j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  wave_sync();
  double pivprod = 1.0;
  // A = R' + s b b^H has trace tr + s; a pivot below 1e-13 of it means rank(R') < M-1
  const bool pd = gj_inverse_hpd_wave<M>(L.aug, 1e-13 * (tr + s), &pivprod);
  double2 q = make_double2(0.0, 0.0);  // (R')^+ = A^{-1} - b b^H / s
  if (ent) {
    const double2 bb = zmul(L.sb[i], zconj(L.sb[j]));
    q = make_double2(L.aug[i][M + j].x - bb.x / s, L.aug[i][M + j].y - bb.y / s);
    L.sQ[i][j] = q;
  }
  wave_sync();
  if (ent) {
    const double2 qt = L.sQ[j][i];
    q = make_double2(0.5 * (q.x + qt.x), 0.5 * (q.y - qt.y));
  }
  wave_sync();
  if (ent) L.sQ[i][j] = q;
  wave_sync();
  double2 cc = make_double2(0.0, 0.0);  // c = (R')^+ a
  if (t < M) {
#pragma unroll
    for (int n = 0; n < M; ++n) {
      const double2 p = zmul(L.sQ[t][n], L.sa[n]);
      cc.x += p.x;
      cc.y += p.y;
    }
    L.sc[t] = cc;
  }
  const double taa = fmax(wave_sum_d(zmulc(av, cc).x), 0.0);
  const double2 ab = zmulc(av, bv);
  const double sabr = wave_sum_d(ab.x), sabi = wave_sum_d(ab.y);
  if (!pd) f |= ST_NOT_PSD;
  if (t == 0) {
    L.taa = taa;
    L.sab_re = sabr;
    L.sab_im = sabi;
    L.logpdet = log(pivprod) - log(s);  // log pdet(R') = log det A - log s
    L.flags = f;
  }
}

template <int M>
__device__ __forceinline__ RowConstF row_const_f(const SetupLDS<M>& L, const RowInfo& ri) {
  RowConstF F;
  F.t_aa = (float)L.taa;
  F.sab_re = (float)L.sab_re;
  F.sab_im = (float)L.sab_im;
  F.sab2 = (float)(L.sab_re * L.sab_re + L.sab_im * L.sab_im);
  F.inv_t_aa = L.taa > 0.0 ? (float)(1.0 / L.taa) : 0.0f;
  F.invM = (float)(1.0 / (double)M);
  F.invJ = (float)(1.0 / (double)ri.J);
  F.pad = 0.0f;
  return F;
}

// Row constants from the setup (call after the setup and a barrier; threads
// t < M*M, t < M and t == 0 write their parts).  Also sets the row's initial
// lambda and its status word.
template <int M>
__device__ void write_row_constants(const SetupLDS<M>& L, int row, const RowInfo& ri,
                                    RowConstD* __restrict__ rcd, RowConstF* __restrict__ rcf,
                                    RowSpatialF* __restrict__ rsf, const float* __restrict__ lam0,
                                    float lam_c, float* __restrict__ lam,
                                    unsigned* __restrict__ status) {
  const int t = threadIdx.x;
  const int i = t / M, j = t % M;
  RowConstD* D = rcd + row;
  RowSpatialF* S = rsf + row;
  if (t < M * M) {
    D->Q[i * MAXM + j] = L.sQ[i][j];
    D->Rp[i * MAXM + j] = L.sR[i][j];
    S->Rp[i * MAXM + j] = make_float2((float)L.sR[i][j].x, (float)L.sR[i][j].y);
  }
  if (t < M) {
    D->c[t] = L.sc[t];
    D->b[t] = L.sb[t];
    D->a[t] = L.sa[t];
    S->a[t] = make_float2((float)L.sa[t].x, (float)L.sa[t].y);
    S->b[t] = make_float2((float)L.sb[t].x, (float)L.sb[t].y);
  }
  if (t == 0) {
    D->t_aa = L.taa;
    D->s_ab = make_double2(L.sab_re, L.sab_im);
    D->logpdet = L.logpdet;
    rcf[row] = row_const_f<M>(L, ri);
    const float l = lam0 ? lam0[row] : lam_c;
    lam[row] = l;
    unsigned f = L.flags;
    if (!(l > 0.0f) || !isfinite(l)) f |= ST_NONFINITE_STATE;
    status[row] = f;
  }
}

// Loads the M complex64 observations of one bin (16-byte pairs when aligned).
template <int M>
__device__ __forceinline__ void load_x(const float2* __restrict__ xp, bool al4, float2 (&xv)[M]) {
  if (al4) {
    const float4* xp4 = reinterpret_cast<const float4*>(xp);
#pragma unroll
    for (int m = 0; m < M / 2; ++m) {
      const float4 v = xp4[m];
      xv[2 * m] = make_float2(v.x, v.y);
      xv[2 * m + 1] = make_float2(v.z, v.w);
    }
  } else {
#pragma unroll
    for (int m = 0; m < M; ++m) xv[m] = xp[m];
  }
}

// tau^ax, sigma^bx, nu of one bin (FP64), from x and the row setup in LDS.
template <int M>
__device__ __forceinline__ void precompute_bin(const float2 (&xv)[M], const SetupLDS<M>& L,
                                               double inv_taa, float4& ts, float& nu,
                                               bool& bad) {
  double xr[M], xi[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    xr[m] = xv[m].x;
    xi[m] = xv[m].y;
  }
  // keep (R')^+ in LDS (re-read per bin) rather than 4 M^2 registers
  asm volatile("" ::: "memory");
  // tau^xx = sum_p Q_pp |x_p|^2 + 2 Re sum_{p<n} conj(x_p) Q_pn x_n
  double txx = 0.0;
#pragma unroll
  for (int p = 0; p < M; ++p) {
    txx = fma(L.sQ[p][p].x, fma(xr[p], xr[p], xi[p] * xi[p]), txx);
    double ur = 0.0, ui = 0.0;  // sum_{n>p} Q_pn x_n
#pragma unroll
    for (int n = p + 1; n < M; ++n) {
      const double2 qq = L.sQ[p][n];
      ur = fma(qq.x, xr[n], fma(-qq.y, xi[n], ur));
      ui = fma(qq.x, xi[n], fma(qq.y, xr[n], ui));
    }
    txx = fma(2.0, fma(xr[p], ur, xi[p] * ui), txx);  // 2 Re(conj(x_p) u)
  }
  double tar = 0.0, tai = 0.0, sbr = 0.0, sbi = 0.0;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    tar = fma(L.sc[m].x, xr[m], fma(L.sc[m].y, xi[m], tar));
    tai = fma(L.sc[m].x, xi[m], fma(-L.sc[m].y, xr[m], tai));
    sbr = fma(L.sb[m].x, xr[m], fma(L.sb[m].y, xi[m], sbr));
    sbi = fma(L.sb[m].x, xi[m], fma(-L.sb[m].y, xr[m], sbi));
  }
  nu = (float)fmax(txx - (tar * tar + tai * tai) * inv_taa, 0.0);
  ts = make_float4((float)tar, (float)tai, (float)sbr, (float)sbi);
  bad = bad || !isfinite(txx) || !isfinite(sbr) || !isfinite(sbi);
}

}  // namespace rcscm
