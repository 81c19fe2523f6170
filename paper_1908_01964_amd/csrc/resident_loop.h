// The K-iteration loop of the RESIDENT schedule (one workgroup per row, BPL
// bins per lane in registers), shared by the resident kernel and the fused
// single-launch kernel.  Per iteration: phase A over the lane's bins, the
// lambda frame sum (DPP within each wave, one LDS slot per wave, one barrier;
// the slots are double-buffered so no second barrier is needed), phase B.
// Under the F64 policy a lane adds its <= BPL terms in float, the 64 lanes of
// a wave are added in float by a fixed six-level tree, and the waves are
// combined in double: for these non-negative terms the relative error is at
// most (BPL + 5) u, u = 2^-24.  The result is the same in every lane and run.
#pragma once

#include "accel_common.h"

namespace rcscm {

// Per-lane constants of the loop: nu / M, the form phase B takes, and
// |sigma^ab|^2 per bin, and 1 / J.  A padding bin (frame t + q*NT >= J,
// ts = 0) takes 0 for the latter, so its lambda term is exactly 0 and it needs
// no mask in the frame sum, and 1 for the former, which keeps its r^u >= 1 and
// so its reciprocal finite in every iteration.
template <int BPL>
struct LoopConsts {
  float nuM[BPL], sab2q[BPL];
  double invJ;
};

template <int NT, int BPL>
__device__ __forceinline__ LoopConsts<BPL> loop_consts(const float (&vnu)[BPL],
                                                       const RowConstF& rc, int J) {
  LoopConsts<BPL> c;
  const int t = threadIdx.x;
  c.invJ = 1.0 / (double)J;
#pragma unroll
  for (int q = 0; q < BPL; ++q) {
    const bool in = t + q * NT < J;
    c.nuM[q] = in ? vnu[q] * rc.invM : 1.0f;
    c.sab2q[q] = in ? rc.sab2 : 0.0f;
  }
  return c;
}

// Iterations k0 .. k1 - 1 of resident_iterations; with CK false it has no
// checkpoint stores, with CK true it stores when ck_rh is not null.  With PRE
// the loop's constants come from lc and the lambda terms of lam_t from Lt_io,
// which receives those of the returned lambda (a segment of the loop); without
// PRE both are formed here and lc, Lt_io are not used (the whole loop, as the
// classes without priority steps compile it: forming the constants in the
// caller changed their register allocation, and the 1024-lane class at M = 8
// then spilled inside the loop).
template <int NT, int BPL, int LS, bool CK, bool PRE>
__device__ __forceinline__ float resident_loop(
    const float4 (&ts)[BPL], const float (&vnu)[BPL], const LoopConsts<BPL>& lc,
    LamTerms& Lt_io, float (&vrh)[BPL], float (&vru)[BPL], const RowConstF& rc, float lam_t,
    int row, int J, long long base, int k0, int k1, float inv_a2, float beta_a2,
    uint64_t (*red)[NT / 64], float* __restrict__ ck_rh, float* __restrict__ ck_ru,
    float* __restrict__ ck_lam, long long ck_sb, int ck_sr) {
  constexpr int NW = NT / 64;
  const int t = threadIdx.x;
  const int wave = t >> 6;
  double invJ;
  float nuM[BPL], sab2q[BPL];
  if constexpr (PRE) {
    invJ = lc.invJ;
#pragma unroll
    for (int q = 0; q < BPL; ++q) {
      nuM[q] = lc.nuM[q];
      sab2q[q] = lc.sab2q[q];
    }
  } else {
    invJ = 1.0 / (double)J;
#pragma unroll
    for (int q = 0; q < BPL; ++q) {
      const bool in = t + q * NT < J;
      nuM[q] = in ? vnu[q] * rc.invM : 1.0f;
      sab2q[q] = in ? rc.sab2 : 0.0f;
    }
  }
  LamTerms Lt;
  if constexpr (PRE)
    Lt = Lt_io;
  else
    Lt = lam_terms(rc, lam_t);
  for (int k = k0; k < k1; ++k) {
    if (CK && ck_rh != nullptr) {  // checkpoint theta at the start of iteration k
#pragma unroll
      for (int q = 0; q < BPL; ++q) {
        const int j = t + q * NT;
        if (j < J) {
          ck_rh[(long long)k * ck_sb + base + j] = vrh[q];
          ck_ru[(long long)k * ck_sb + base + j] = vru[q];
        }
      }
      if (t == 0) ck_lam[(long long)k * ck_sr + row] = lam_t;
    }
    LamAcc<LS> acc;
    PhaseA A[BPL];
    float tsum;  // F64 policy: the lane's <= BPL terms in float
#pragma unroll
    for (int q = 0; q < BPL; ++q) {
      A[q] = phase_a_turned(ts[q], vrh[q], vru[q], rc, Lt, inv_a2, beta_a2, sab2q[q]);
      if constexpr (LS == 0) {
        tsum = q == 0 ? A[q].t : tsum + A[q].t;
      } else if (t + q * NT < J) {
        acc.add(A[q].t);
      }
      vrh[q] = A[q].rh_new;
    }
    if constexpr (LS == 0) {
      const float v = wave_sum_f32_last(tsum);
      if ((t & 63) == 63) red[k & 1][wave] = LamAcc<0>::from(v).pack();
    } else {
      acc = wave_allreduce<LS>(acc);
      if ((t & 63) == 0) red[k & 1][wave] = acc.pack();
    }
    __syncthreads();
    const float lam_n = slots_sum<LS, NW>(red[k & 1]).mean(invJ);
    const LamTerms Ln = lam_terms(rc, lam_n);
#pragma unroll
    for (int q = 0; q < BPL; ++q) vru[q] = phase_b(ts[q], nuM[q], A[q], rc, Ln);
    lam_t = lam_n;
    Lt = Ln;
  }
  if constexpr (PRE) Lt_io = Lt;
  return lam_t;
}

// The K iterations, as one loop or, with FAIR, as four segments of it.  With
// FAIR and fair set, the wave's issue priority falls from 3 to 0 from one
// segment to the next.  The SIMDs otherwise favour the oldest waves, so of two
// or three rows sharing a CU the first would finish well ahead and the last
// would run its final iterations alone, one wave per SIMD, with every latency
// of the iteration exposed; a row that has fallen behind now keeps a higher
// priority until it catches up.  The priority changes between segments, not
// inside the loop body (a test there cost most of the gain), and the segments
// share the loop's constants and lambda terms (forming them again at every
// segment cost half of it).
template <int NT, int BPL, int LS, bool CK, bool FAIR>
__device__ __forceinline__ float resident_segments(
    const float4 (&ts)[BPL], const float (&vnu)[BPL], float (&vrh)[BPL], float (&vru)[BPL],
    const RowConstF& rc, float lam_t, int row, int J, long long base, int K, float inv_a2,
    float beta_a2, uint64_t (*red)[NT / 64], float* __restrict__ ck_rh,
    float* __restrict__ ck_ru, float* __restrict__ ck_lam, long long ck_sb, int ck_sr,
    bool fair) {
  if constexpr (!FAIR) {
    const LoopConsts<BPL> unused{};
    LamTerms unused_lt{};
    return resident_loop<NT, BPL, LS, CK, false>(ts, vnu, unused, unused_lt, vrh, vru, rc, lam_t,
                                                 row, J, base, 0, K, inv_a2, beta_a2, red, ck_rh,
                                                 ck_ru, ck_lam, ck_sb, ck_sr);
  } else {
    const LoopConsts<BPL> lc = loop_consts<NT, BPL>(vnu, rc, J);  // once for all segments
    LamTerms Lt = lam_terms(rc, lam_t);
    for (int seg = 0; seg < 4; ++seg) {
      if (fair) {
        if (seg == 0) __builtin_amdgcn_s_setprio(3);
        if (seg == 1) __builtin_amdgcn_s_setprio(2);
        if (seg == 2) __builtin_amdgcn_s_setprio(1);
        if (seg == 3) __builtin_amdgcn_s_setprio(0);
      }
      lam_t = resident_loop<NT, BPL, LS, CK, true>(ts, vnu, lc, Lt, vrh, vru, rc, lam_t, row, J,
                                                   base, (seg * K) / 4, ((seg + 1) * K) / 4,
                                                   inv_a2, beta_a2, red, ck_rh, ck_ru, ck_lam,
                                                   ck_sb, ck_sr);
    }
    return lam_t;
  }
}

// Runs K iterations in place on (vrh, vru); returns the final lambda.  ts
// holds each bin's turned pair (tau^ax, u) of turn_sigma_bx.  Bins with frame
// index t + q*NT >= J do not enter the frame sum.  When ck_rh is not null,
// theta at the start of every iteration is stored (checkpoints).  Up to four
// bins per lane the test is made once, outside the loop (a test per iteration
// cost 1.7 % of the fused launch at M = 4, I = 513, J = 1000, K = 20); with
// eight, two copies of the loop raised the register count past the
// occupancy steps (256 x 8: 108 -> 130 VGPRs, 1024 x 8: spills), so the test
// stays inside.  FAIR compiles the segmented form (resident_segments), whose
// priority steps fair switches on; without it the loop is the plain one.
template <int NT, int BPL, int LS, bool FAIR>
__device__ __forceinline__ float resident_iterations(
    const float4 (&ts)[BPL], const float (&vnu)[BPL], float (&vrh)[BPL], float (&vru)[BPL],
    const RowConstF& rc, float lam_t, int row, int J, long long base, int K, float inv_a2,
    float beta_a2, uint64_t (*red)[NT / 64], float* __restrict__ ck_rh,
    float* __restrict__ ck_ru, float* __restrict__ ck_lam, long long ck_sb, int ck_sr,
    bool fair) {
  if (BPL > 4 || ck_rh != nullptr)
    return resident_segments<NT, BPL, LS, true, FAIR>(ts, vnu, vrh, vru, rc, lam_t, row, J, base,
                                                      K, inv_a2, beta_a2, red, ck_rh, ck_ru,
                                                      ck_lam, ck_sb, ck_sr, fair);
  return resident_segments<NT, BPL, LS, false, FAIR>(ts, vnu, vrh, vru, rc, lam_t, row, J, base,
                                                     K, inv_a2, beta_a2, red, nullptr, nullptr,
                                                     nullptr, 0, 0, fair);
}

// Wiener-filter estimate s_hat = gamma rho^ax of one bin at (r^h, r^u) and
// the lambda terms L (posterior mean of s, inside eq. (15)), from the turned
// pair ts = (tau^ax, u): rho^ax = tau^ax + (|sigma^ab| / lambda) u.
__device__ __forceinline__ float2 s_hat_of(const float4 ts, float rh, float ru, const LamTerms& L) {
  const float rx_re = fmaf(L.sa_il, ts.z, ts.x);
  const float rx_im = fmaf(L.sa_il, ts.w, ts.y);
  const float g = rh / fmaf(rh, L.rho_aa, ru);
  return make_float2(g * rx_re, g * rx_im);
}

}  // namespace rcscm
