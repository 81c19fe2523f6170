// Per-row FP64 setup and per-bin FP64 precomputation, shared by the init
// kernel (rcscm_init) and the fused single-launch kernel (rcscm_run).
//
// Setup of a row (Algorithm 2, before the loop; eqs. (26), (32), (46)),
// from a_i, R'_i, b_i in complex128:
//   1. b <- b / ||b||   (warning bit if ||b|| was not 1 within 1e-6);
//   2. null check ||R' b|| <= 1e-6 ||R'||_F (b spans the null space of the
//      rank-(M-1) SCM, Sec. II-B-1);
//   3. R' <- P R' P, P = I - b b^H, Hermitised (removes the rounding in R'b);
//   4. A = R' + s b b^H, s the power of two within a factor of two of
//      tr(R')/(M-1) (so s b b^H and b b^H / s are exact), is Hermitian positive definite
//      and, because R' b = 0 and ||b|| = 1, A^{-1} = (R')^+ + b b^H / s -
//      the pseudoinverse expansion of eq. (26) with lambda = s.  A^{-1} comes
//      from an LDL^H factorisation in registers for M <= 4, else from a
//      lane-parallel Gauss-Jordan elimination (M steps), so
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
  double2 sR[M][M];       // projected, Hermitised R'
  double2 sQ[M][M];       // (R')^+
  double2 aug[M][2 * M];  // Gauss-Jordan work array
  double2 sa[M], sb[M], sc[M];
  double2 sbr[M], syr[M];  // b as given and R' b with it
  double taa, inv_taa, sab_re, sab_im, det_a, shift;
  unsigned flags;
};

// The setup's inputs as held by the lanes of wave 0: lane t < M*M holds
// R'[t / M][t % M] and R'[t % M][t / M], lane t < M holds a[t] and b[t]
// (the other lanes hold copies of entry 0, which the setup leaves out).
struct SetupIn {
  double2 r, rt, av, bv;
};

// Issues the setup's loads, so a kernel can put them ahead of its own loads in
// the memory queue.  Only wave 0 loads; every lane of it does, lanes beyond the
// matrix (t >= M*M) and beyond the vectors (t >= M) loading entry 0 again, so
// the loads are straight-line code and a later wait for them need not also
// wait for loads issued after them.  row_setup_wave masks those duplicates.
template <int M>
__device__ __forceinline__ SetupIn row_setup_load(const double2* __restrict__ Rp,
                                                  const double2* __restrict__ a,
                                                  const double2* __restrict__ b,
                                                  const RowInfo& ri) {
  const int t = threadIdx.x;
  SetupIn in;
  in.r = in.rt = in.av = in.bv = make_double2(0.0, 0.0);
  if (t < 64) {  // uniform per wave
    const int e = t < M * M ? t : 0;
    const int m = t < M ? t : 0;
    in.r = Rp[ri.rp_off + e];
    in.rt = Rp[ri.rp_off + (e % M) * M + e / M];
    in.av = a[ri.a_off + m];
    in.bv = b[ri.a_off + m];
  }
  return in;
}

// 1/sqrt(v) for v > 0: the hardware estimate refined by two Newton-Raphson
// steps y <- y (3 - v y^2) / 2, each of which doubles the number of correct bits.
__device__ __forceinline__ double rsqrt_f64_nr(double v) {
  double y = __builtin_amdgcn_rsq(v);
  y = y * fma(-0.5 * v, y * y, 1.5);
  return y * fma(-0.5 * v, y * y, 1.5);
}

// Row setup by wave 0 (lanes t < 64) from its loaded inputs.  Lane t < M*M
// owns entry (i, j) = (t / M, t % M).  Everything before the elimination
// comes from ONE batch of wave sums, on b as given (b0, ||b0|| = nb) and
// y0 = R' b0: ||b0||^2, a^H b0, tr R', b0^H R' b0, ||R' b0||^2, ||R'||_F^2.
// With b = b0 / nb, y = R' b = y0 / nb and e_b = b^H R' b,
//   P R' P (Hermitised) = (R' + R'^H)/2 - b y^H - y b^H + e_b b b^H,  P = I - b b^H,
// and its trace is tr R' - e_b, so no further sum is needed; the second and
// last sum, tau^aa = a^H (R')^+ a, runs over the lanes' entries of (R')^+
// beside the products c = (R')^+ a.
template <int M>
__device__ void row_setup_wave(const SetupIn& in, SetupLDS<M>& L) {
  const int t = threadIdx.x;
  const int i = t / M, j = t % M;
  const bool ent = t < M * M;
  const double2 r = in.r, av = in.av, b0 = in.bv;
  const bool fin = zfinite(r) && zfinite(in.rt) && zfinite(av) && zfinite(b0);
  if (ent) L.aug[i][j] = r;  // R' for the products y0 = R' b0
  if (t < M) {
    L.sa[t] = av;
    L.sbr[t] = b0;
  }
  wave_sync();
  double2 y0 = make_double2(0.0, 0.0);  // row t of R' b0
  if (t < M) {
#pragma unroll
    for (int n = 0; n < M; ++n) {
      const double2 p = zmul(L.aug[t][n], L.sbr[n]);
      y0.x += p.x;
      y0.y += p.y;
    }
    L.syr[t] = y0;
  }
  const bool vec = t < M;
  const double2 ab0 = zmulc(av, b0);  // a^H b0, lanes t < M
  double s1[8] = {fin ? 0.0 : 1.0,
                  ent ? r.x * r.x + r.y * r.y : 0.0,
                  vec ? b0.x * b0.x + b0.y * b0.y : 0.0,
                  vec ? ab0.x : 0.0,
                  vec ? ab0.y : 0.0,
                  (ent && i == j) ? r.x : 0.0,
                  zmulc(b0, y0).x,
                  y0.x * y0.x + y0.y * y0.y};
  wave_sums<8, M * M>(s1);
  const double nbad = s1[0], nr2 = s1[1], nb2 = s1[2];
  unsigned f = 0u;
  if (nbad > 0.0) f |= ST_NONFINITE_IN;
  const bool bok = nb2 > 0.0 && nbad == 0.0;
  const double inb = bok ? rsqrt_f64_nr(nb2) : 0.0;  // 1 / ||b0||
  if (!bok)
    f |= ST_NOT_NULL;
  else if (fabs(nb2 * inb - 1.0) > 1e-6)
    f |= ST_B_NOT_UNIT;
  const double inb2 = inb * inb;
  const double be = s1[6] * inb2;                     // b^H R' b
  if (!(s1[7] * inb2 <= 1e-12 * nr2)) f |= ST_NOT_NULL;  // ||R' b|| <= 1e-6 ||R'||_F
  const double tr = s1[5] - be;                       // tr P R' P
  // s: a power of two within a factor of two of tr / (M - 1), so that s b b^H
  // and b b^H / s are exact and no division is needed
  double sh = 1.0, ish = 1.0;
  if (tr > 0.0) {
    const int e = ilogb(tr * (1.0 / (double)(M - 1)));
    sh = ldexp(1.0, e);
    ish = ldexp(1.0, -e);
  }
  wave_sync();
  double2 rhm = make_double2(0.0, 0.0), bb = rhm, ai = rhm, aj = rhm;
  if (ent) {
    const double2 bi0 = L.sbr[i], bj0 = L.sbr[j], yi0 = L.syr[i], yj0 = L.syr[j];
    ai = L.sa[i];
    aj = L.sa[j];
    // b_i conj(y_j), y_i conj(b_j) and b_i conj(b_j), each scaled by 1/||b0||^2
    const double2 byj = zmul(bi0, zconj(yj0));
    const double2 ybj = zmul(yi0, zconj(bj0));
    const double2 bb0 = zmul(bi0, zconj(bj0));
    bb = make_double2(bb0.x * inb2, bb0.y * inb2);
    rhm = make_double2(0.5 * (r.x + in.rt.x) - (byj.x + ybj.x) * inb2 + be * bb.x,
                       0.5 * (r.y - in.rt.y) - (byj.y + ybj.y) * inb2 + be * bb.y);
    L.sR[i][j] = rhm;
    L.aug[i][j] = make_double2(rhm.x + sh * bb.x, rhm.y + sh * bb.y);
    L.aug[i][M + j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  if (t < M) L.sb[t] = make_double2(b0.x * inb, b0.y * inb);
  wave_sync();
  double pivprod = 1.0;
  // A = R' + s b b^H has trace tr + s; a pivot below 1e-13 of it means rank(R') < M-1
  double2 q = make_double2(0.0, 0.0);
  bool pd;
  if constexpr (M <= 4) {  // (R')^+ = A^{-1} - b b^H / s, A^{-1} exactly Hermitian
    double2 ainv;
    pd = ldl_inverse_hpd_wave<M>(L.aug, 1e-13 * (tr + sh), &pivprod, &ainv);
    if (ent) {
      q = make_double2(ainv.x - bb.x * ish, ainv.y - bb.y * ish);
      L.sQ[i][j] = q;
    }
  } else {  // (R')^+ = A^{-1} - b b^H / s, Hermitised
    pd = gj_inverse_hpd_wave<M>(L.aug, 1e-13 * (tr + sh), &pivprod);
    if (ent) {
      const double2 u = L.aug[i][M + j], v = L.aug[j][M + i];
      q = make_double2(0.5 * (u.x + v.x) - bb.x * ish, 0.5 * (u.y - v.y) - bb.y * ish);
      L.sQ[i][j] = q;
    }
  }
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
  double s2[1] = {zmulc(ai, zmul(q, aj)).x};  // conj(a_i) Q_ij a_j
  wave_sums<1, M * M>(s2);
  if (!pd) f |= ST_NOT_PSD;
  if (t == 0) {
    const double taa = fmax(s2[0], 0.0);
    L.taa = taa;
    L.inv_taa = taa > 0.0 ? rcp_f64_nr(taa) : 0.0;
    L.sab_re = s1[3] * inb;
    L.sab_im = s1[4] * inb;
    L.det_a = pivprod;  // det A; log pdet(R') = log det A - log s
    L.shift = sh;
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
  F.inv_t_aa = (float)L.inv_taa;
  F.invM = (float)(1.0 / (double)M);
  F.invJ = 1.0f / (float)ri.J;
  F.sab_abs = (float)sqrt(L.sab_re * L.sab_re + L.sab_im * L.sab_im);
  return F;
}

// Row constants from the setup (call after the setup and a barrier).  The
// stores are spread over the threads of a workgroup of NT >= 256 lanes, one
// or two per thread: Q by threads [0, M*M), R' by [64, 64 + M*M), c, b, a by
// [128, 128 + M), [160, ...), [192, ...), the scalars by thread 224.  rsf
// (the float model of the naive rule) may be null.  Also sets the row's
// initial lambda and its status word.  With rcd == null (a run that keeps no
// state) only the status word is stored: rcf and lam are then not read.
template <int M, int NT>
__device__ void write_row_constants(const SetupLDS<M>& L, int row, const RowInfo& ri,
                                    RowConstD* __restrict__ rcd, RowConstF* __restrict__ rcf,
                                    RowSpatialF* __restrict__ rsf, const float* __restrict__ lam0,
                                    float lam_c, float* __restrict__ lam,
                                    unsigned* __restrict__ status) {
  static_assert(NT >= 256 && M * M <= 64 && M <= 32, "thread map of the row constants");
  const int t = threadIdx.x;
  if (rcd == nullptr) {
    if (t == 224) {
      const float l = lam0 ? lam0[row] : lam_c;
      unsigned f = L.flags;
      if (!(l > 0.0f) || !isfinite(l)) f |= ST_NONFINITE_STATE;
      status[row] = f;
    }
    return;
  }
  RowConstD* D = rcd + row;
  RowSpatialF* S = rsf != nullptr ? rsf + row : nullptr;
  if (t < M * M) {
    const int i = t / M, j = t % M;
    D->Q[i * MAXM + j] = L.sQ[i][j];
  } else if (t >= 64 && t < 64 + M * M) {
    const int i = (t - 64) / M, j = (t - 64) % M;
    const double2 r = L.sR[i][j];
    D->Rp[i * MAXM + j] = r;
    if (S) S->Rp[i * MAXM + j] = make_float2((float)r.x, (float)r.y);
  } else if (t >= 128 && t < 128 + M) {
    D->c[t - 128] = L.sc[t - 128];
  } else if (t >= 160 && t < 160 + M) {
    const double2 v = L.sb[t - 160];
    D->b[t - 160] = v;
    if (S) S->b[t - 160] = make_float2((float)v.x, (float)v.y);
  } else if (t >= 192 && t < 192 + M) {
    const double2 v = L.sa[t - 192];
    D->a[t - 192] = v;
    if (S) S->a[t - 192] = make_float2((float)v.x, (float)v.y);
  } else if (t == 224) {
    D->t_aa = L.taa;
    D->s_ab = make_double2(L.sab_re, L.sab_im);
    D->det_a = L.det_a;
    D->shift = L.shift;
    rcf[row] = row_const_f<M>(L, ri);
    const float l = lam0 ? lam0[row] : lam_c;
    lam[row] = l;
    unsigned f = L.flags;
    if (!(l > 0.0f) || !isfinite(l)) f |= ST_NONFINITE_STATE;
    status[row] = f;
  }
}

// Loads the M complex64 observations of one bin as 8-byte values (no alignment
// test, so no branch around the loads).
template <int M>
__device__ __forceinline__ void load_x8(const float2* __restrict__ xp, float2 (&xv)[M]) {
#pragma unroll
  for (int m = 0; m < M; ++m) xv[m] = xp[m];
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
