// rcscm_init on the device: per-row FP64 setup, per-bin FP64 precomputation
// and the initial state, in one launch per microphone count M (one
// workgroup per chunk of a row).
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
// The first chunk of the row writes these row constants, the row's status
// word and its initial lambda.
//
// Precomputation of every bin of the chunk (eqs. (33), (47), (48)), in FP64
// from the complex64 x:
//   tau^ax = c^H x,  sigma^bx = b^H x,  tau^xx = x^H (R')^+ x,
//   nu     = tau^xx - |tau^ax|^2 / tau^aa  (>= 0; the FP64 difference is exact
//            to ~1e-16 tau^xx, far below the float rounding of the stored nu),
// stored as float4 {tau^ax, sigma^bx} and float nu (20 bytes per bin), plus
// the initial r^h, r^u of the bin.  Memory-bound: 8M bytes read and 28
// written per bin; consecutive lanes on consecutive frames.
#include "accel_common.h"
#include "small_linalg.h"

namespace rcscm {

namespace {

constexpr int kInitNT = 256;

template <int M>
__global__ __launch_bounds__(kInitNT) __attribute__((amdgpu_waves_per_eu(4))) void init_kernel(
    const InitArgs A) {
  const ChunkInfo ck = A.chunks[blockIdx.x];
  const int row = ck.row;
  const RowInfo ri = A.rows[row];
  const int t = threadIdx.x;
  const bool writer = ck.start == 0;
  const int i = t / M, j = t % M;
  const bool ent = t < M * M;

  __shared__ double2 sR[M][M];      // R', then the projected R'
  __shared__ double2 sQ[M][M];      // (R')^+
  __shared__ double2 aug[M][2 * M]; // Gauss-Jordan work array
  __shared__ double2 sa[M], sb[M], sy[M], sc[M];
  __shared__ double sd[9];
  __shared__ unsigned sflag;

  // Loads of this thread's first group of bins are issued before the row
  // setup, so their HBM latency overlaps the setup's FP64 work.
  constexpr int G = M <= 4 ? 4 : (M <= 6 ? 2 : 1);
  float2 xv[G][M];
  const bool al4 = (M & 1) == 0 && (ri.x_off & 1) == 0;  // 16-byte aligned pairs of mics
  auto load_group = [&](int g0) {
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const int jj = g0 + t + q * kInitNT;
      if (jj >= ck.len) continue;
      const float2* xp = A.x + ri.x_off + (long long)(ck.start + jj) * M;
      if (al4) {
        const float4* xp4 = reinterpret_cast<const float4*>(xp);
#pragma unroll
        for (int m = 0; m < M / 2; ++m) {
          const float4 v = xp4[m];
          xv[q][2 * m] = make_float2(v.x, v.y);
          xv[q][2 * m + 1] = make_float2(v.z, v.w);
        }
      } else {
#pragma unroll
        for (int m = 0; m < M; ++m) xv[q][m] = xp[m];
      }
    }
  };
  load_group(0);

  // Row setup: wave 0 only (the other waves' x loads are already in flight).
  // Lane t < M*M owns entry (i, j) = (t / M, t % M); sums over lanes are
  // uniform DPP reductions (wave_sum_d), so the chain is a handful of rounds.
  if (t < 64) {
    double2 r = make_double2(0.0, 0.0), av = r, bv = r;
    if (ent) r = A.Rp[ri.rp_off + t];
    if (t < M) {
      av = A.a[ri.a_off + t];
      bv = A.b[ri.a_off + t];
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
    if (ent) sR[i][j] = r;
    if (t < M) {
      sa[t] = av;
      sb[t] = bv;
    }
    wave_sync();
    double2 y = make_double2(0.0, 0.0);  // y = R' b
    if (t < M) {
#pragma unroll
      for (int n = 0; n < M; ++n) {
        const double2 p = zmul(sR[t][n], sb[n]);
        y.x += p.x;
        y.y += p.y;
      }
      sy[t] = y;
    }
    const double ny2 = wave_sum_d(y.x * y.x + y.y * y.y);
    const double be = wave_sum_d(zmulc(bv, y).x);  // b^H R' b
    if (!(sqrt(ny2) <= 1e-6 * sqrt(nr2))) f |= ST_NOT_NULL;
    wave_sync();
    double2 pr = make_double2(0.0, 0.0);  // P R' P = R' - b y^H - y b^H + (b^H R' b) b b^H
    if (ent) {
      const double2 byj = zmul(sb[i], zconj(sy[j]));
      const double2 ybj = zmul(sy[i], zconj(sb[j]));
      const double2 bbj = zmul(sb[i], zconj(sb[j]));
      pr = make_double2(r.x - byj.x - ybj.x + be * bbj.x, r.y - byj.y - ybj.y + be * bbj.y);
      aug[i][j] = pr;
    }
    wave_sync();
    double2 rhm = make_double2(0.0, 0.0);  // Hermitised
    if (ent) {
      const double2 pt = aug[j][i];
      rhm = make_double2(0.5 * (pr.x + pt.x), 0.5 * (pr.y - pt.y));
    }
    const double tr = wave_sum_d((ent && i == j) ? rhm.x : 0.0);
    const double s = tr > 0.0 ? tr / (double)(M - 1) : 1.0;
    wave_sync();
    if (ent) {
      sR[i][j] = rhm;
      const double2 bb = zmul(sb[i], zconj(sb[j]));
      aug[i][j] = make_double2(rhm.x + s * bb.x, rhm.y + s * bb.y);
      aug[i][M + j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    }
    wave_sync();
    double pivprod = 1.0;
    // A = R' + s b b^H has trace tr + s; a pivot below 1e-13 of it means rank(R') < M-1
    const bool pd = gj_inverse_hpd_wave<M>(aug, 1e-13 * (tr + s), &pivprod);
    double2 q = make_double2(0.0, 0.0);  // (R')^+ = A^{-1} - b b^H / s
    if (ent) {
      const double2 bb = zmul(sb[i], zconj(sb[j]));
      q = make_double2(aug[i][M + j].x - bb.x / s, aug[i][M + j].y - bb.y / s);
      sQ[i][j] = q;
    }
    wave_sync();
    if (ent) {
      const double2 qt = sQ[j][i];
      q = make_double2(0.5 * (q.x + qt.x), 0.5 * (q.y - qt.y));
    }
    wave_sync();
    if (ent) sQ[i][j] = q;
    wave_sync();
    double2 cc = make_double2(0.0, 0.0);  // c = (R')^+ a
    if (t < M) {
#pragma unroll
      for (int n = 0; n < M; ++n) {
        const double2 p = zmul(sQ[t][n], sa[n]);
        cc.x += p.x;
        cc.y += p.y;
      }
      sc[t] = cc;
    }
    const double taa = fmax(wave_sum_d(zmulc(av, cc).x), 0.0);
    const double2 ab = zmulc(av, bv);
    const double sabr = wave_sum_d(ab.x), sabi = wave_sum_d(ab.y);
    if (!pd) f |= ST_NOT_PSD;
    if (t == 0) {
      sd[5] = taa;
      sd[6] = sabr;
      sd[7] = sabi;
      sd[8] = log(pivprod) - log(s);  // log pdet(R') = log det A - log s
      sflag = f;
    }
  }
  __syncthreads();
  const double taa = sd[5];

  if (writer) {
    RowConstD* D = A.rcd + row;
    RowSpatialF* S = A.rsf + row;
    if (ent) {
      D->Q[i * MAXM + j] = sQ[i][j];
      D->Rp[i * MAXM + j] = sR[i][j];
      S->Rp[i * MAXM + j] = make_float2((float)sR[i][j].x, (float)sR[i][j].y);
    }
    if (t < M) {
      D->c[t] = sc[t];
      D->b[t] = sb[t];
      D->a[t] = sa[t];
      S->a[t] = make_float2((float)sa[t].x, (float)sa[t].y);
      S->b[t] = make_float2((float)sb[t].x, (float)sb[t].y);
    }
    if (t == 0) {
      D->t_aa = taa;
      D->s_ab = make_double2(sd[6], sd[7]);
      D->logpdet = sd[8];
      RowConstF F;
      F.t_aa = (float)taa;
      F.sab_re = (float)sd[6];
      F.sab_im = (float)sd[7];
      F.sab2 = (float)(sd[6] * sd[6] + sd[7] * sd[7]);
      F.inv_t_aa = taa > 0.0 ? (float)(1.0 / taa) : 0.0f;
      F.invM = (float)(1.0 / (double)M);
      F.invJ = (float)(1.0 / (double)ri.J);
      F.pad = 0.0f;
      A.rcf[row] = F;
      const float l = A.lam0 ? A.lam0[row] : A.lam_c;
      A.lam[row] = l;
      unsigned f = sflag;
      if (!(l > 0.0f) || !isfinite(l)) f |= ST_NONFINITE_STATE;
      A.status[row] = f;
    }
  }

  // ---- per-bin precomputation and initial state
  const double inv_taa = taa > 0.0 ? 1.0 / taa : 0.0;
  bool bad_x = false, bad_state = false;
  for (int g0 = 0; g0 < ck.len; g0 += G * kInitNT) {
    if (g0 > 0) load_group(g0);
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const int jj = g0 + t + q * kInitNT;
      if (jj >= ck.len) continue;
      double xr[M], xi[M];
#pragma unroll
      for (int m = 0; m < M; ++m) {
        xr[m] = xv[q][m].x;
        xi[m] = xv[q][m].y;
      }
      // keep (R')^+ in LDS (re-read per bin) rather than 4 M^2 registers
      asm volatile("" ::: "memory");
      // tau^xx = sum_p Q_pp |x_p|^2 + 2 Re sum_{p<n} conj(x_p) Q_pn x_n
      double txx = 0.0;
#pragma unroll
      for (int p = 0; p < M; ++p) {
        txx = fma(sQ[p][p].x, fma(xr[p], xr[p], xi[p] * xi[p]), txx);
        double ur = 0.0, ui = 0.0;  // sum_{n>p} Q_pn x_n
#pragma unroll
        for (int n = p + 1; n < M; ++n) {
          const double2 qq = sQ[p][n];
          ur = fma(qq.x, xr[n], fma(-qq.y, xi[n], ur));
          ui = fma(qq.x, xi[n], fma(qq.y, xr[n], ui));
        }
        txx = fma(2.0, fma(xr[p], ur, xi[p] * ui), txx);  // 2 Re(conj(x_p) u)
      }
      double tar = 0.0, tai = 0.0, sbr = 0.0, sbi = 0.0;
#pragma unroll
      for (int m = 0; m < M; ++m) {
        tar = fma(sc[m].x, xr[m], fma(sc[m].y, xi[m], tar));
        tai = fma(sc[m].x, xi[m], fma(-sc[m].y, xr[m], tai));
        sbr = fma(sb[m].x, xr[m], fma(sb[m].y, xi[m], sbr));
        sbi = fma(sb[m].x, xi[m], fma(-sb[m].y, xr[m], sbi));
      }
      const double nuv = fmax(txx - (tar * tar + tai * tai) * inv_taa, 0.0);
      const long long bin = ri.bin_off + ck.start + jj;
      A.tsig[bin] = make_float4((float)tar, (float)tai, (float)sbr, (float)sbi);
      A.nu[bin] = (float)nuv;
      const float h = A.rh0 ? A.rh0[bin] : A.rh_c;
      const float u = A.ru0 ? A.ru0[bin] : A.ru_c;
      A.rh[bin] = h;
      A.ru[bin] = u;
      bad_x = bad_x || !isfinite(txx) || !isfinite(sbr) || !isfinite(sbi);
      bad_state = bad_state || !(h > 0.0f) || !(u > 0.0f) || !isfinite(h) || !isfinite(u);
    }
  }
  // per-chunk status: OR over the lanes through LDS
  __shared__ unsigned cflag;
  if (t == 0) cflag = 0u;
  __syncthreads();
  if (bad_x) atomicOr(&cflag, ST_NONFINITE_IN);
  if (bad_state) atomicOr(&cflag, ST_NONFINITE_STATE);
  __syncthreads();
  if (t == 0) A.chunk_status[ck.part] = cflag;
}

}  // namespace

void launch_init(hipStream_t s, int M, int nchunks, const InitArgs& args) {
  if (nchunks <= 0) return;
  switch (M) {
#define RCSCM_INIT(MM)                                                                   \
  case MM:                                                                               \
    hipLaunchKernelGGL(init_kernel<MM>, dim3(nchunks), dim3(kInitNT), 0, s, args); \
    break;
    RCSCM_INIT(2)
    RCSCM_INIT(3)
    RCSCM_INIT(4)
    RCSCM_INIT(5)
    RCSCM_INIT(6)
    RCSCM_INIT(7)
    RCSCM_INIT(8)
#undef RCSCM_INIT
    default: break;
  }
}

}  // namespace rcscm
