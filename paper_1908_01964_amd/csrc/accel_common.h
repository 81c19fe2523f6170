// Device helpers of the second-stage accelerated iteration (Algorithm 2).
//
// Per bin, with the values at the start of the iteration (tilde) and the
// per-row constants tau^aa, sigma^ab:
//   rho~ax = tau^ax + sigma^ab sigma^bx / lambda~                 eq. (52)
//   gamma~ = r~h / (r~u + r~h rho~aa),  rho~aa = tau^aa + |sigma^ab|^2/lambda~  eqs. (34), (50)
//   r^h    = (gamma~ (r~u + gamma~ |rho~ax|^2) + beta) / (alpha + 2)            eq. (54)
//   e      = sigma^bx - gamma~ conj(sigma^ab) rho~ax
//   t      = gamma~ |sigma^ab|^2 + |e|^2 / r~u   (lambda <- mean_j t)          eq. (55)
// and, after the frame sum has produced the new lambda,
//   r^u    = (1/M) [ gamma~ r~u rho^aa + nu + |tau^ax - w tau^aa|^2 / tau^aa
//                    + |e|^2 / lambda ],       w = gamma~ rho~ax,
// with nu = tau^xx - |tau^ax|^2 / tau^aa from the precomputation.
// The last line equals eq. (56): with y = x - w a, the statistic of eq. (44)
// is U^ = gamma~ r~u a a^H + y y^H, and tr(R^{-1} U^) splits by the
// pseudoinverse expansion eq. (26) into gamma~ r~u rho^aa + y^H (R')^+ y +
// |b^H y|^2 / lambda, where b^H y = e and
// y^H (R')^+ y = nu + |tau^ax - w tau^aa|^2 / tau^aa.  Every term is a
// non-negative number, so no float cancellation occurs.
#pragma once

#include "rcscm_internal.h"

namespace rcscm {

__device__ __forceinline__ float frcp(float v) { return __builtin_amdgcn_rcpf(v); }

// 1/v for the per-iteration lambda: the hardware reciprocal refined by one
// Newton-Raphson step r <- r + r (1 - v r) (about 0.5 ulp for normal v > 0).
__device__ __forceinline__ float frcp_nr(float v) {
  const float r = __builtin_amdgcn_rcpf(v);
  return fmaf(r, fmaf(-v, r, 1.0f), r);
}

// Per-row quantities that depend on one value of lambda.  The *M members are
// the same quantities divided by M, used by phase B.
struct LamTerms {
  float il;      // 1 / lambda
  float rho_aa;  // tau^aa + |sigma^ab|^2 / lambda
  float sp_re;   // sigma^ab / lambda
  float sp_im;
  float sa_il;   // |sigma^ab| / lambda
  float rho_aaM;  // rho^aa / M
  float ilM;      // 1 / (M lambda)
  float itaaM;    // 1 / (M tau^aa), 0 when tau^aa == 0
};

__device__ __forceinline__ LamTerms lam_terms(const RowConstF& rc, float lam) {
  LamTerms L;
  L.il = frcp_nr(lam);
  L.rho_aa = fmaf(rc.sab2, L.il, rc.t_aa);
  L.sp_re = rc.sab_re * L.il;
  L.sp_im = rc.sab_im * L.il;
  L.sa_il = rc.sab_abs * L.il;
  L.rho_aaM = L.rho_aa * rc.invM;
  L.ilM = L.il * rc.invM;
  L.itaaM = rc.inv_t_aa * rc.invM;
  return L;
}

// Phase A of one bin: new r^h, the lambda term t, and what phase B needs.
struct PhaseA {
  float rh_new, t, cg, w_re, w_im, E;
};

// With w = gamma~ rho~ax and cg = gamma~ r~u, eq. (54) reads
// r^h = (cg + |w|^2 + beta) / (alpha + 2), and e = sigma^bx - conj(sigma^ab) w.
__device__ __forceinline__ PhaseA phase_a(const float4 ts, float rh, float ru, const RowConstF& rc,
                                          const LamTerms& Lt, float inv_a2, float beta_a2) {
  PhaseA o;
  // rho~ax = tau^ax + (sigma^ab / lambda~) sigma^bx
  const float rx_re = fmaf(Lt.sp_re, ts.z, fmaf(-Lt.sp_im, ts.w, ts.x));
  const float rx_im = fmaf(Lt.sp_re, ts.w, fmaf(Lt.sp_im, ts.z, ts.y));
  const float g = rh * frcp(fmaf(rh, Lt.rho_aa, ru));
  o.w_re = g * rx_re;
  o.w_im = g * rx_im;
  o.cg = g * ru;
  o.rh_new = fmaf(fmaf(o.w_re, o.w_re, fmaf(o.w_im, o.w_im, o.cg)), inv_a2, beta_a2);
  const float e_re = fmaf(-rc.sab_re, o.w_re, fmaf(-rc.sab_im, o.w_im, ts.z));
  const float e_im = fmaf(-rc.sab_re, o.w_im, fmaf(rc.sab_im, o.w_re, ts.w));
  o.E = fmaf(e_re, e_re, e_im * e_im);
  o.t = fmaf(g, rc.sab2, o.E * frcp(ru));
  return o;
}

// The per-bin pair (tau^ax, sigma^bx) with sigma^bx turned by the phase of
// sigma^ab: u = sigma^bx sigma^ab / |sigma^ab| (sigma^bx when sigma^ab = 0).
// With it, sigma^ab sigma^bx = |sigma^ab| u and, for any w,
// (sigma^bx - conj(sigma^ab) w) sigma^ab / |sigma^ab| = u - |sigma^ab| w, so
// rho~ax, s_hat and |e| each take one real factor instead of a complex one.
__device__ __forceinline__ float4 turn_sigma_bx(const float4 ts, const RowConstF& rc) {
  float pr = 1.0f, pi = 0.0f;
  if (rc.sab_abs > 0.0f) {
    const float ia = 1.0f / rc.sab_abs;
    pr = rc.sab_re * ia;
    pi = rc.sab_im * ia;
  }
  return make_float4(ts.x, ts.y, fmaf(ts.z, pr, -ts.w * pi), fmaf(ts.z, pi, ts.w * pr));
}

// Phase A on the turned pair ts = (tau^ax, u) (turn_sigma_bx): the same
// quantities as phase_a with
//   rho~ax = tau^ax + (|sigma^ab| / lambda~) u,
//   |e| = |u - |sigma^ab| w|.
// sab2 is |sigma^ab|^2 of the row, or 0 for a padding bin (ts = 0), whose t
// is then exactly 0 as long as r~h and r~u are finite and r~u > 0.
__device__ __forceinline__ PhaseA phase_a_turned(const float4 ts, float rh, float ru,
                                                 const RowConstF& rc, const LamTerms& Lt,
                                                 float inv_a2, float beta_a2, float sab2) {
  PhaseA o;
  const float rx_re = fmaf(Lt.sa_il, ts.z, ts.x);
  const float rx_im = fmaf(Lt.sa_il, ts.w, ts.y);
  const float g = rh * frcp(fmaf(rh, Lt.rho_aa, ru));
  o.w_re = g * rx_re;
  o.w_im = g * rx_im;
  o.cg = g * ru;
  o.rh_new = fmaf(fmaf(o.w_re, o.w_re, fmaf(o.w_im, o.w_im, o.cg)), inv_a2, beta_a2);
  const float e_re = fmaf(-rc.sab_abs, o.w_re, ts.z);
  const float e_im = fmaf(-rc.sab_abs, o.w_im, ts.w);
  o.E = fmaf(e_re, e_re, e_im * e_im);
  o.t = fmaf(g, sab2, o.E * frcp(ru));
  return o;
}

// Phase B of one bin: new r^u given the new lambda (terms Ln); nuM = nu / M.
// Reads only tau^ax from ts, so it serves both forms of the pair.
__device__ __forceinline__ float phase_b(const float4 ts, float nuM, const PhaseA& A,
                                         const RowConstF& rc, const LamTerms& Ln) {
  const float d_re = fmaf(-A.w_re, rc.t_aa, ts.x);
  const float d_im = fmaf(-A.w_im, rc.t_aa, ts.y);
  float acc = fmaf(A.cg, Ln.rho_aaM, nuM);
  acc = fmaf(fmaf(d_re, d_re, d_im * d_im), Ln.itaaM, acc);
  return fmaf(A.E, Ln.ilM, acc);
}

// ---- frame-sum accumulators for lambda --------------------------------------
// Policy 0 (F64): double per lane and across lanes.
// Policy 1 (KAHAN32): Kahan-compensated float per lane; lanes combined with a
// TwoSum tree.  State (s, c) represents s - c.

template <int LS>
struct LamAcc;

template <>
struct LamAcc<0> {
  double s;
  __device__ __forceinline__ LamAcc() : s(0.0) {}
  __device__ __forceinline__ void add(float t) { s += (double)t; }
  __device__ __forceinline__ void combine(const LamAcc& o) { s += o.s; }
  __device__ __forceinline__ uint64_t pack() const { return __double_as_longlong(s); }
  __device__ __forceinline__ static LamAcc unpack(uint64_t v) {
    LamAcc r;
    r.s = __longlong_as_double((long long)v);
    return r;
  }
  __device__ __forceinline__ float mean(double invJ) const { return (float)(s * invJ); }
  __device__ __forceinline__ static LamAcc from(float v) {
    LamAcc r;
    r.s = (double)v;
    return r;
  }
};

template <>
struct LamAcc<1> {
  float s, c;
  __device__ __forceinline__ LamAcc() : s(0.0f), c(0.0f) {}
  __device__ __forceinline__ void add(float t) {
    const float y = t - c;
    const float tt = s + y;
    c = (tt - s) - y;
    s = tt;
  }
  __device__ __forceinline__ void combine(const LamAcc& o) {
    const float ss = s + o.s;
    const float bp = ss - s;
    const float err = (s - (ss - bp)) + (o.s - bp);
    c = c + o.c - err;
    s = ss;
  }
  __device__ __forceinline__ uint64_t pack() const {
    return ((uint64_t)__float_as_uint(c) << 32) | (uint64_t)__float_as_uint(s);
  }
  __device__ __forceinline__ static LamAcc unpack(uint64_t v) {
    LamAcc r;
    r.s = __uint_as_float((unsigned)(v & 0xffffffffu));
    r.c = __uint_as_float((unsigned)(v >> 32));
    return r;
  }
  __device__ __forceinline__ float mean(double invJ) const {
    return (float)(((double)s - (double)c) * invJ);
  }
};

// ---- cross-lane sums ---------------------------------------------------------
// Rotations inside each 16-lane row by 8, 4, 2, 1 (DPP row_ror, ALU-only, no
// LDS round trip) leave the row sum in every lane of the row; the four row
// sums are then read from lanes 0, 16, 32, 48 (readlane) and added in that
// fixed order, so every lane of every wave gets the bitwise same value.
// All 64 lanes must be active.

template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
  // every lane is a valid source of the row rotations, so no old value is needed
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = dpp_i32<CTRL>(__double2loint(v));
  const int hi = dpp_i32<CTRL>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(dpp_i32<CTRL>(__float_as_int(v)));
}
// The DPP-moved value as the operand of an addition (the row rotations have a
// source in every lane; the identity 0 as the old value lets the compiler fold
// the move into the add).
template <int CTRL>
__device__ __forceinline__ float dpp_f32_add_src(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float readlane_f32(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

constexpr int kRowRor8 = 0x128, kRowRor4 = 0x124, kRowRor2 = 0x122, kRowRor1 = 0x121;

constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143;

// Sum of a float over the 64 lanes of a wave by a fixed tree, left in lane 63
// only: the row rotations by 8, 4, 2, 1 leave each 16-lane row's sum in all
// its lanes; adding lane 15 of every row into the next row leaves rows 2 + 3
// in row 3 and rows 0 + 1 in row 1, and adding lane 31 into rows 2 and 3 then
// leaves the total in row 3 (the other rows hold partial sums, unused).  Six
// additions folded with their lane moves, no lane swaps.  For non-negative
// terms the relative error is at most 6 u.
__device__ __forceinline__ float wave_sum_f32_last(float v) {
  v += dpp_f32_add_src<kRowRor8>(v);
  v += dpp_f32_add_src<kRowRor4>(v);
  v += dpp_f32_add_src<kRowRor2>(v);
  v += dpp_f32_add_src<kRowRor1>(v);
  v += dpp_f32_add_src<kRowBcast15>(v);
  v += dpp_f32_add_src<kRowBcast31>(v);
  return v;
}

template <int LS, int CTRL>
__device__ __forceinline__ LamAcc<LS> rot(const LamAcc<LS>& a);

template <>
__device__ __forceinline__ LamAcc<0> rot<0, kRowRor8>(const LamAcc<0>& a) { LamAcc<0> r; r.s = dpp_f64<kRowRor8>(a.s); return r; }
template <>
__device__ __forceinline__ LamAcc<0> rot<0, kRowRor4>(const LamAcc<0>& a) { LamAcc<0> r; r.s = dpp_f64<kRowRor4>(a.s); return r; }
template <>
__device__ __forceinline__ LamAcc<0> rot<0, kRowRor2>(const LamAcc<0>& a) { LamAcc<0> r; r.s = dpp_f64<kRowRor2>(a.s); return r; }
template <>
__device__ __forceinline__ LamAcc<0> rot<0, kRowRor1>(const LamAcc<0>& a) { LamAcc<0> r; r.s = dpp_f64<kRowRor1>(a.s); return r; }
template <int CTRL>
__device__ __forceinline__ LamAcc<1> rot1(const LamAcc<1>& a) {
  LamAcc<1> r;
  r.s = dpp_f32<CTRL>(a.s);
  r.c = dpp_f32<CTRL>(a.c);
  return r;
}
template <>
__device__ __forceinline__ LamAcc<1> rot<1, kRowRor8>(const LamAcc<1>& a) { return rot1<kRowRor8>(a); }
template <>
__device__ __forceinline__ LamAcc<1> rot<1, kRowRor4>(const LamAcc<1>& a) { return rot1<kRowRor4>(a); }
template <>
__device__ __forceinline__ LamAcc<1> rot<1, kRowRor2>(const LamAcc<1>& a) { return rot1<kRowRor2>(a); }
template <>
__device__ __forceinline__ LamAcc<1> rot<1, kRowRor1>(const LamAcc<1>& a) { return rot1<kRowRor1>(a); }

__device__ __forceinline__ LamAcc<0> readlane_acc(const LamAcc<0>& a, int lane) {
  LamAcc<0> r;
  r.s = readlane_f64(a.s, lane);
  return r;
}
__device__ __forceinline__ LamAcc<1> readlane_acc(const LamAcc<1>& a, int lane) {
  LamAcc<1> r;
  r.s = readlane_f32(a.s, lane);
  r.c = readlane_f32(a.c, lane);
  return r;
}

// Sum over the 64 lanes of a wave; the result is uniform across the wave.
template <int LS>
__device__ __forceinline__ LamAcc<LS> wave_allreduce(LamAcc<LS> a) {
  a.combine(rot<LS, kRowRor8>(a));
  a.combine(rot<LS, kRowRor4>(a));
  a.combine(rot<LS, kRowRor2>(a));
  a.combine(rot<LS, kRowRor1>(a));
  LamAcc<LS> r = readlane_acc(a, 0);
  r.combine(readlane_acc(a, 16));
  r.combine(readlane_acc(a, 32));
  r.combine(readlane_acc(a, 48));
  return r;
}

// Double sum over the 64 lanes of a wave, uniform across the wave.
__device__ __forceinline__ double wave_sum_d(double v) {
  LamAcc<0> a;
  a.s = v;
  return wave_allreduce<0>(a).s;
}

// NV independent double sums over the lanes t < LANES of a wave (the other
// lanes must hold 0), interleaved so their latencies overlap; the results are
// uniform across the wave.  For LANES <= 16 only the first DPP row is read
// (the rotations leave the row sum in each of its lanes).
template <int NV, int LANES>
__device__ __forceinline__ void wave_sums(double (&v)[NV]) {
#pragma unroll
  for (int n = 0; n < NV; ++n) v[n] += dpp_f64<kRowRor8>(v[n]);
#pragma unroll
  for (int n = 0; n < NV; ++n) v[n] += dpp_f64<kRowRor4>(v[n]);
#pragma unroll
  for (int n = 0; n < NV; ++n) v[n] += dpp_f64<kRowRor2>(v[n]);
#pragma unroll
  for (int n = 0; n < NV; ++n) v[n] += dpp_f64<kRowRor1>(v[n]);
#pragma unroll
  for (int n = 0; n < NV; ++n) {
    if constexpr (LANES <= 16) {
      v[n] = readlane_f64(v[n], 0);
    } else {
      double r = readlane_f64(v[n], 0);
      r += readlane_f64(v[n], 16);
      r += readlane_f64(v[n], 32);
      r += readlane_f64(v[n], 48);
      v[n] = r;
    }
  }
}

// Sum of n packed accumulators p[0..n), computed identically by every wave.
template <int LS>
__device__ __forceinline__ LamAcc<LS> wave_sum_packed(const uint64_t* p, int n) {
  const int lane = threadIdx.x & 63;
  LamAcc<LS> a;
  for (int k = lane; k < n; k += 64) a.combine(LamAcc<LS>::unpack(p[k]));
  return wave_allreduce<LS>(a);
}

// Sum of the NW per-wave slots of a workgroup, read by every lane in slot
// order (a uniform LDS broadcast; no cross-lane traffic).
template <int LS, int NW>
__device__ __forceinline__ LamAcc<LS> slots_sum(const uint64_t* slots) {
  LamAcc<LS> a = LamAcc<LS>::unpack(slots[0]);
#pragma unroll
  for (int w = 1; w < NW; ++w) a.combine(LamAcc<LS>::unpack(slots[w]));
  return a;
}

}  // namespace rcscm
