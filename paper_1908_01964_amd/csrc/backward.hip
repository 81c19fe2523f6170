// Adjoint of the differentiable path: K accelerated iterations (Algorithm 2)
// from (r^h_0, r^u_0, lambda_0), the Wiener-filter extraction
// s_hat = gamma rho^ax at the final state, and the per-bin precomputation of
// tau^ax, sigma^bx, nu from x.
//
// Complex adjoints follow torch's convention z_bar = dL/dRe z + i dL/dIm z:
//   z = c w (c const)    -> w_bar += conj(c) z_bar
//   r = |z|^2            -> z_bar += 2 z r_bar
//   z = r w (r real)     -> w_bar += r z_bar,  r_bar += Re(conj(w) z_bar)
//
// One workgroup per row (the RESIDENT layout of the forward), bins in
// registers.  For k = K-1 .. 0 the iteration is recomputed from the
// checkpoint theta_k and reversed.  lambda couples the bins of a row twice
// per iteration, so each reversed iteration needs two frame sums:
//   #1: d lambda_{k+1}/d(everything after it) through r^u_{k+1}
//       (r^u uses the new lambda): sum_j u_bar_j/M (|e_j|^2 + |s_ab|^2 g_j u_j);
//       it completes lambda_bar_{k+1}, which reaches every bin through
//       lambda_{k+1} = mean_j t_j.
//   #2: d/d lambda_k of everything computed from it in this iteration.
// As in the forward kernels, sigma^bx is used turned by the phase p of
// sigma^ab (u = p sigma^bx, turn_sigma_bx): sigma^ab sigma^bx = |sigma^ab| u
// and p e = u - |sigma^ab| w, so the recomputed forward and its reverse take
// real factors where the printed rule has complex ones.  The reverse pass
// accumulates u_bar; sigma_bar = conj(p) u_bar before x_bar is formed.
// The two sums of a reversed iteration add a lane's terms and the 64 lanes of
// a wave in float (a fixed tree, as the forward's frame sum) and the waves in
// double; the extraction's sum runs in double throughout.
// At the end x_bar = c tau_bar' + b sigma_bar + 2 nu_bar (R')^+ x with
// c = (R')^+ a and tau_bar' = tau_bar - 2 tau^ax nu_bar / tau^aa (nu =
// tau^xx - |tau^ax|^2/tau^aa), in FP64 from the row constants.
#include <atomic>

#include "accel_common.h"

namespace rcscm {

namespace {

template <int NT>
__device__ __forceinline__ double block_sum(double v, uint64_t (*red)[NT / 64], int& phase) {
  LamAcc<0> a;
  a.s = v;
  a = wave_allreduce<0>(a);
  const int t = threadIdx.x;
  if ((t & 63) == 0) red[phase & 1][t >> 6] = a.pack();
  __syncthreads();
  const double s = slots_sum<0, NT / 64>(red[phase & 1]).s;
  ++phase;
  return s;
}

// Sum over the workgroup of a float per lane: the wave's lanes in float by a
// fixed tree, the waves in double (one LDS slot each).
template <int NT>
__device__ __forceinline__ double block_sum_f32(float v, uint64_t (*red)[NT / 64], int& phase) {
  v = wave_sum_f32_last(v);
  const int t = threadIdx.x;
  if ((t & 63) == 63) red[phase & 1][t >> 6] = LamAcc<0>::from(v).pack();
  __syncthreads();
  const double s = slots_sum<0, NT / 64>(red[phase & 1]).s;
  ++phase;
  return s;
}

// x_bar of the lane's bins: c T_bar' + b B_bar + 2 nu_bar (R')^+ x in FP64,
// with T_bar' = T_bar - 2 tau^ax nu_bar / tau^aa and (R')^+ (row-major M x M),
// c, b staged in LDS (re-read per bin rather than held in registers).
template <int M, int NT, int BPL>
__device__ __forceinline__ void xbar_bins(const float2* __restrict__ xr0,
                                          float2* __restrict__ gx0, int J,
                                          const float4 (&ts)[BPL], const float (&Tbr)[BPL],
                                          const float (&Tbi)[BPL], const float (&Bbr)[BPL],
                                          const float (&Bbi)[BPL], const float (&nub)[BPL],
                                          double inv_taad, const double2* sQ, const double2* sc,
                                          const double2* sbv) {
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < BPL; ++q) {
    const int j = t + q * NT;
    if (j >= J) continue;
    const double nb = nub[q];
    const double tr = (double)Tbr[q] - 2.0 * (double)ts[q].x * nb * inv_taad;
    const double ti = (double)Tbi[q] - 2.0 * (double)ts[q].y * nb * inv_taad;
    const float2* xp = xr0 + (long long)j * M;
    float2* gp = gx0 + (long long)j * M;
    double xr[M], xi[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const float2 v = xp[m];
      xr[m] = v.x;
      xi[m] = v.y;
    }
    asm volatile("" ::: "memory");  // keep (R')^+ in LDS
#pragma unroll
    for (int m = 0; m < M; ++m) {
      double yr = 0.0, yi = 0.0;  // ((R')^+ x)_m
#pragma unroll
      for (int n = 0; n < M; ++n) {
        const double2 Qmn = sQ[m * M + n];
        yr = fma(Qmn.x, xr[n], fma(-Qmn.y, xi[n], yr));
        yi = fma(Qmn.x, xi[n], fma(Qmn.y, xr[n], yi));
      }
      const double2 c = sc[m], b = sbv[m];
      const double gr = c.x * tr - c.y * ti + b.x * Bbr[q] - b.y * Bbi[q] + 2.0 * nb * yr;
      const double gi = c.x * ti + c.y * tr + b.x * Bbi[q] + b.y * Bbr[q] + 2.0 * nb * yi;
      gp[m] = make_float2((float)gr, (float)gi);
    }
  }
}

template <int NT, int BPL>
// (up to 4 bins per lane: at least four waves per SIMD)
__global__ __launch_bounds__(NT, (BPL <= 4 ? 4 : 1)) void backward_kernel(
    const int* __restrict__ row_list, const RowInfo* __restrict__ rows,
    const RowConstF* __restrict__ rcf, const RowConstD* __restrict__ rcd,
    const float2* __restrict__ x, const float4* __restrict__ tsig, const float* __restrict__ nu,
    const float* __restrict__ ck_rh, const float* __restrict__ ck_ru,
    const float* __restrict__ ck_lam, long long sb, int sr, const float* __restrict__ rh_fin,
    const float* __restrict__ ru_fin, const float* __restrict__ lam_fin, int K, float inv_a2,
    const float2* __restrict__ grad_s, float2* __restrict__ grad_x, float* __restrict__ grad_rh0,
    float* __restrict__ grad_lam0, int fair) {
  const int row = row_list[blockIdx.x];
  const RowInfo ri = rows[row];
  const RowConstF rc = rcf[row];
  const int J = ri.J;
  const long long base = ri.bin_off;
  const int t = threadIdx.x;
  RCSCM_DASSERT(J >= 1 && J <= NT * BPL);
  RCSCM_DASSERT(K == 0 || (base + J <= sb && row < sr));
  const float S2 = rc.sab2, sab = rc.sab_abs, taa = rc.t_aa;
  const float invM = rc.invM;
  __shared__ uint64_t red[2][NT / 64];
  int phase = 0;

  float4 ts[BPL];
  // Bbr, Bbi: the gradient of the turned u (of sigma^bx only at the end)
  float Tbr[BPL], Tbi[BPL], Bbr[BPL], Bbi[BPL], nub[BPL], hb[BPL], ub[BPL];
#pragma unroll
  for (int q = 0; q < BPL; ++q) {
    const int j = t + q * NT;
    ts[q] = (j < J) ? turn_sigma_bx(tsig[base + j], rc) : make_float4(0.f, 0.f, 0.f, 0.f);
    Tbr[q] = Tbi[q] = Bbr[q] = Bbi[q] = nub[q] = hb[q] = ub[q] = 0.f;
  }

  // ---- extraction: s_hat = gamma P, P = T + |s| U / lambda, gamma = h / (u + h A)
  float lam_bar;
  {
    const float lam = lam_fin[row];
    const float il = frcp_nr(lam);
    const float A = fmaf(S2, il, taa);
    const float sil = sab * il;
    double c = 0.0;
#pragma unroll
    for (int q = 0; q < BPL; ++q) {
      const int j = t + q * NT;
      if (j >= J) continue;
      const float h = rh_fin[base + j], u = ru_fin[base + j];
      const float2 gs = grad_s[base + j];
      const float4 T = ts[q];
      const float Pr = fmaf(sil, T.z, T.x);
      const float Pi = fmaf(sil, T.w, T.y);
      const float D = fmaf(h, A, u);
      const float iD = frcp(D);
      const float gam = h * iD;
      const float gbar = Pr * gs.x + Pi * gs.y;
      const float Pbr = gam * gs.x, Pbi = gam * gs.y;
      const float Dbar = -gbar * gam * iD;
      hb[q] = fmaf(gbar, iD, Dbar * A);
      ub[q] = Dbar;
      const float Abar = Dbar * h;
      Tbr[q] += Pbr;
      Tbi[q] += Pbi;
      // U_bar += |s| il P_bar
      Bbr[q] += sil * Pbr;
      Bbi[q] += sil * Pbi;
      // il_bar += Re(conj(|s| U) P_bar)
      c += (double)(sab * fmaf(T.z, Pbr, T.w * Pbi)) + (double)(S2 * Abar);
    }
    const double ilbar = block_sum<NT>(c, red, phase);
    lam_bar = (float)(-(double)il * (double)il * ilbar);
  }

  // ---- iterations, last to first; theta_k is loaded one iteration ahead
  float nh[BPL], nu_[BPL];
  if (K > 0) {
#pragma unroll
    for (int q = 0; q < BPL; ++q) {
      const int j = t + q * NT;
      const bool on = j < J;
      nh[q] = on ? ck_rh[(long long)(K - 1) * sb + base + j] : 1.f;
      nu_[q] = on ? ck_ru[(long long)(K - 1) * sb + base + j] : 1.f;
    }
  }
  // As in the forward loop: where all rows of the launch are resident at once
  // (fair), the 256-lane classes run the reversed iterations in four segments
  // and lower the waves' priority from one to the next, so that rows sharing
  // a CU progress together; other classes run one plain loop.
  constexpr int kSeg = (NT == 256 && BPL <= 4) ? 4 : 1;
  int k = K - 1;
  for (int seg = 0; seg < kSeg; ++seg) {
    if constexpr (kSeg == 4) {
      if (fair) {
        if (seg == 0) __builtin_amdgcn_s_setprio(3);
        if (seg == 1) __builtin_amdgcn_s_setprio(2);
        if (seg == 2) __builtin_amdgcn_s_setprio(1);
        if (seg == 3) __builtin_amdgcn_s_setprio(0);
      }
    }
    const int kend = K - ((seg + 1) * K) / kSeg;  // this segment ends at iteration kend
    for (; k >= kend; --k) {
      const float lam = ck_lam[(long long)k * sr + row];
      const float lam_n = (k + 1 < K) ? ck_lam[(long long)(k + 1) * sr + row] : lam_fin[row];
      const float il = frcp_nr(lam), il_n = frcp_nr(lam_n);
      const float A = fmaf(S2, il, taa), A_n = fmaf(S2, il_n, taa);
      const float sil = sab * il;
      float vh[BPL], vu[BPL];
#pragma unroll
      for (int q = 0; q < BPL; ++q) {
        vh[q] = nh[q];
        vu[q] = nu_[q];
      }
      if (k > 0) {  // prefetch theta_{k-1}
#pragma unroll
        for (int q = 0; q < BPL; ++q) {
          const int j = t + q * NT;
          const bool on = j < J;
          nh[q] = on ? ck_rh[(long long)(k - 1) * sb + base + j] : 1.f;
          nu_[q] = on ? ck_ru[(long long)(k - 1) * sb + base + j] : 1.f;
        }
      }
      // phase-A quantities of iteration k kept for the second pass (the cheap
      // ones are recomputed there)
      constexpr bool kKeep = BPL <= 4;  // registers allow it up to 4 bins per lane
      float viD[BPL], vg[BPL], vE[BPL];
      float c1 = 0.0f;  // the lane's terms in float
#pragma unroll
      for (int q = 0; q < BPL; ++q) {
        const int j = t + q * NT;
        const float4 T = ts[q];
        const float h = vh[q], u = vu[q];
        const float Pr = fmaf(sil, T.z, T.x);
        const float Pi = fmaf(sil, T.w, T.y);
        const float iD = frcp(fmaf(h, A, u));
        const float g = h * iD;
        const float wr = g * Pr, wi = g * Pi;
        const float er = fmaf(-sab, wr, T.z), ei = fmaf(-sab, wi, T.w);
        const float E = fmaf(er, er, ei * ei);
        if constexpr (kKeep) {
          viD[q] = iD;
          vg[q] = g;
          vE[q] = E;
        }
        if (j < J) c1 += ub[q] * invM * fmaf(S2, g * u, E);
      }
      const double ilnbar = block_sum_f32<NT>(c1, red, phase);
      const float lam_n_bar = (float)((double)lam_bar - (double)il_n * (double)il_n * ilnbar);
      const float tbar = lam_n_bar * rc.invJ;

      float c2 = 0.0f;
#pragma unroll
      for (int q = 0; q < BPL; ++q) {
        const int j = t + q * NT;
        const float4 T = ts[q];
        const float h = vh[q], u = vu[q];
        const float Pr = fmaf(sil, T.z, T.x);
        const float Pi = fmaf(sil, T.w, T.y);
        const float iD = kKeep ? viD[q] : frcp(fmaf(h, A, u));
        const float g = kKeep ? vg[q] : h * iD;
        const float iu = frcp(u);
        const float R2 = Pr * Pr + Pi * Pi;
        const float Q = fmaf(g, R2, u);
        const float wr = g * Pr, wi = g * Pi;
        const float er = fmaf(-sab, wr, T.z), ei = fmaf(-sab, wi, T.w);
        const float E = kKeep ? vE[q] : fmaf(er, er, ei * ei);
        const float dr = T.x - wr * taa, di = T.y - wi * taa;
        // r^u_{k+1} = (g u A_n + nu + |d|^2 / taa + E / lambda_n) / M
        const float uu = ub[q] * invM;
        float gbar = uu * u * A_n;
        float ubar = uu * g * A_n;
        nub[q] += uu;
        const float dsc = 2.0f * uu * rc.inv_t_aa;
        const float dbr = dsc * dr, dbi = dsc * di;
        float Ebar = uu * il_n;
        // lambda_{k+1} = mean_j (g S2 + E / u)
        gbar += S2 * tbar;
        Ebar += tbar * iu;
        ubar -= E * iu * iu * tbar;
        // d = T - w taa
        Tbr[q] += dbr;
        Tbi[q] += dbi;
        float wbr = -taa * dbr, wbi = -taa * dbi;
        // E = |e|^2 ; p e = U - |s| w
        const float ebr = 2.0f * er * Ebar, ebi = 2.0f * ei * Ebar;
        Bbr[q] += ebr;
        Bbi[q] += ebi;
        wbr = fmaf(-sab, ebr, wbr);
        wbi = fmaf(-sab, ebi, wbi);
        // w = g P
        gbar += Pr * wbr + Pi * wbi;
        float Pbr = g * wbr, Pbi = g * wbi;
        // h_{k+1} = g Q / (alpha + 2) + beta / (alpha + 2)
        const float hp = hb[q] * inv_a2;
        gbar += hp * Q;
        const float Qbar = hp * g;
        // Q = u + g R2 ; R2 = |P|^2
        ubar += Qbar;
        gbar += Qbar * R2;
        Pbr += 2.0f * Pr * (Qbar * g);
        Pbi += 2.0f * Pi * (Qbar * g);
        // g = h / D ; D = u + h A
        float hbar = gbar * iD;
        const float Dbar = -gbar * g * iD;
        ubar += Dbar;
        hbar += Dbar * A;
        // P = T + |s| il U
        Tbr[q] += Pbr;
        Tbi[q] += Pbi;
        Bbr[q] = fmaf(sil, Pbr, Bbr[q]);
        Bbi[q] = fmaf(sil, Pbi, Bbi[q]);
        if (j < J) c2 += fmaf(sab, fmaf(T.z, Pbr, T.w * Pbi), S2 * Dbar * h);
        hb[q] = hbar;
        ub[q] = ubar;
      }
      const double ilbar = block_sum_f32<NT>(c2, red, phase);
      lam_bar = (float)(-(double)il * (double)il * ilbar);
    }
  }

  if (t == 0 && grad_lam0 != nullptr) grad_lam0[row] = lam_bar;

  // sigma_bar = conj(p) u_bar, p = sigma^ab / |sigma^ab| (1 when sigma^ab = 0)
  {
    float pr = 1.0f, pi = 0.0f;
    if (sab > 0.0f) {
      const float ia = 1.0f / sab;
      pr = rc.sab_re * ia;
      pi = rc.sab_im * ia;
    }
#pragma unroll
    for (int q = 0; q < BPL; ++q) {
      const float ur = Bbr[q], ui = Bbi[q];
      Bbr[q] = fmaf(pr, ur, pi * ui);
      Bbi[q] = fmaf(pr, ui, -pi * ur);
    }
  }

  // ---- precomputation: x_bar = c T_bar' + b B_bar + 2 nu_bar (R')^+ x
  const RowConstD* Dc = rcd + row;
  const int M = ri.M;
  __shared__ double2 sQ[MAXM * MAXM], sc[MAXM], sbv[MAXM];
  for (int e = t; e < M * M; e += NT) sQ[e] = Dc->Q[(e / M) * MAXM + e % M];
  if (t < M) {
    sc[t] = Dc->c[t];
    sbv[t] = Dc->b[t];
  }
  __syncthreads();
  const double taad = Dc->t_aa;
  const double inv_taad = taad > 0.0 ? 1.0 / taad : 0.0;
#pragma unroll
  for (int q = 0; q < BPL; ++q) {
    const int j = t + q * NT;
    if (j < J && grad_rh0 != nullptr) grad_rh0[base + j] = hb[q];
  }
  if (grad_x == nullptr) return;
  switch (M) {
#define RCSCM_XB(MM)                                                                         \
  case MM:                                                                                   \
    xbar_bins<MM, NT, BPL>(x + ri.x_off, grad_x + ri.x_off, J, ts, Tbr, Tbi, Bbr, Bbi, nub,    \
                           inv_taad, sQ, sc, sbv);                                           \
    break;
    RCSCM_XB(2)
    RCSCM_XB(3)
    RCSCM_XB(4)
    RCSCM_XB(5)
    RCSCM_XB(6)
    RCSCM_XB(7)
    RCSCM_XB(8)
#undef RCSCM_XB
    default: break;
  }
}

template <int NT, int BPL>
void bw_launch(hipStream_t s, int nrows, const int* row_list, const RowInfo* rows,
               const RowConstF* rcf, const RowConstD* rcd, const float2* x, const float4* tsig,
               const float* nu, const float* ck_rh, const float* ck_ru, const float* ck_lam,
               long long sb, int sr, const float* rh_fin, const float* ru_fin,
               const float* lam_fin, int K, float inv_a2, const float2* grad_s, float2* grad_x,
               float* grad_rh0, float* grad_lam0, int fair) {
  hipLaunchKernelGGL((backward_kernel<NT, BPL>), dim3(nrows), dim3(NT), 0, s, row_list, rows, rcf,
                     rcd, x, tsig, nu, ck_rh, ck_ru, ck_lam, sb, sr, rh_fin, ru_fin, lam_fin, K,
                     inv_a2, grad_s, grad_x, grad_rh0, grad_lam0, fair);
}

// Workgroups of backward_kernel<NT, BPL> one CU holds at once (0 if unknown).
template <int NT, int BPL>
int bw_blocks_per_cu() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, backward_kernel<NT, BPL>, NT, 0) !=
      hipSuccess)
    n = 0;
  return n;
}

using BwFn = void (*)(hipStream_t, int, const int*, const RowInfo*, const RowConstF*,
                      const RowConstD*, const float2*, const float4*, const float*, const float*,
                      const float*, const float*, long long, int, const float*, const float*,
                      const float*, int, float, const float2*, float2*, float*, float*, int);

#define RCSCM_BW_LIST(NT)                                                                   \
  {bw_launch<NT, 1>, bw_launch<NT, 2>, bw_launch<NT, 3>, bw_launch<NT, 4>, bw_launch<NT, 5>, \
   bw_launch<NT, 6>, bw_launch<NT, 7>, bw_launch<NT, 8>, nullptr, bw_launch<NT, 10>, nullptr, \
   bw_launch<NT, 12>, nullptr, nullptr, nullptr, bw_launch<NT, 16>}
#define RCSCM_BW_LIST_1024                                                                  \
  {bw_launch<1024, 1>, bw_launch<1024, 2>, bw_launch<1024, 3>, bw_launch<1024, 4>,          \
   bw_launch<1024, 5>, bw_launch<1024, 6>, bw_launch<1024, 7>, bw_launch<1024, 8>, nullptr, \
   nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr}

const BwFn kBw[5][16] = {RCSCM_BW_LIST(64), RCSCM_BW_LIST(128), RCSCM_BW_LIST(256),
                         RCSCM_BW_LIST(512), RCSCM_BW_LIST_1024};

int bw_class_index(int nt) {
  switch (nt) {
    case 64: return 0;
    case 128: return 1;
    case 256: return 2;
    case 512: return 3;
    case 1024: return 4;
    default: return -1;
  }
}

}  // namespace

bool backward_fair(int nt, int bpl, int nrows, int device) {
  if (nt != 256 || bpl < 1 || bpl > 4) return false;  // only these classes have the steps
  static std::atomic<int> cache[4];                   // per bpl; 0 = not yet queried
  int v = cache[bpl - 1].load(std::memory_order_relaxed);
  if (v == 0) {
    int n = 0;
    switch (bpl) {
      case 1: n = bw_blocks_per_cu<256, 1>(); break;
      case 2: n = bw_blocks_per_cu<256, 2>(); break;
      case 3: n = bw_blocks_per_cu<256, 3>(); break;
      case 4: n = bw_blocks_per_cu<256, 4>(); break;
      default: break;
    }
    v = n > 0 ? n : -1;
    cache[bpl - 1].store(v, std::memory_order_relaxed);
  }
  return v > 0 && (long long)nrows <= (long long)v * device_cu_count(device);
}

void launch_backward(hipStream_t s, int nt, int bpl, int nrows, const int* row_list,
                     const RowInfo* rows, const RowConstF* rcf, const RowConstD* rcd,
                     const float2* x, const float4* tsig, const float* nu, const float* ckpt_rh,
                     const float* ckpt_ru, const float* ckpt_lam, long long ckpt_stride_bins,
                     int ckpt_stride_rows, const float* rh_fin, const float* ru_fin,
                     const float* lam_fin, int K, float alpha, const float2* grad_s,
                     float2* grad_x, float* grad_rh0, float* grad_lam0, int fair) {
  if (nrows <= 0) return;
  const int ni = bw_class_index(nt);
  if (ni < 0 || bpl < 1 || bpl > 16 || kBw[ni][bpl - 1] == nullptr) return;
  const float inv_a2 = (float)(1.0 / ((double)alpha + 2.0));
  kBw[ni][bpl - 1](s, nrows, row_list, rows, rcf, rcd, x, tsig, nu, ckpt_rh, ckpt_ru, ckpt_lam,
                   ckpt_stride_bins, ckpt_stride_rows, rh_fin, ru_fin, lam_fin, K, inv_a2, grad_s,
                   grad_x, grad_rh0, grad_lam0, fair);
}

}  // namespace rcscm
