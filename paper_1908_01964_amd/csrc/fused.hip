// rcscm_run: the whole path of one row in one workgroup and one launch -
// per-row FP64 setup, per-bin FP64 precomputation into registers, K
// second-stage iterations (Algorithm 2) in registers, Wiener-filter
// extraction.  HBM traffic per bin: x (8M bytes) read once; r^h, r^u and
// s_hat (16) written once to the caller; unless the run keeps no state
// (null workspace pointers), tau^ax, sigma^bx, nu, r^h, r^u (28 bytes) are
// also stored for a later iterate/extract/objective/backward.  Wave 0 issues
// the setup's loads first; the x loads of the first bin of every lane follow
// and overlap the setup.  When the adjoint needs them, theta_k at the start
// of every iteration is stored as well (8 bytes per bin and iteration).  One
// launch per (M, workgroup size, bins per lane) class.
#include <atomic>

#include "init_common.h"
#include "resident_loop.h"

namespace rcscm {

namespace {

template <int M, int NT, int BPL>
__global__ __launch_bounds__(NT) void accel_fused_kernel(const FusedArgs A) {
  constexpr int NW = NT / 64;
  // Only the 256-lane classes compile the priority steps (FusedArgs::fair):
  // the larger ones seldom have all their rows resident at once, and keep the
  // plain loop.
  constexpr bool kFairClass = NT == 256;
  int row;
  RowInfo ri;
  if (A.lin) {  // no dependent loads before the setup's loads
    const long long b = blockIdx.x;
    row = A.lin_row0 + (int)b;
    ri.J = A.lin_J;
    ri.M = M;
    ri.x_off = A.lin_x0 + b * A.lin_J * M;
    ri.bin_off = A.lin_bin0 + b * A.lin_J;
    ri.a_off = A.lin_a0 + b * M;
    ri.rp_off = A.lin_rp0 + b * M * M;
  } else {
    row = A.row_list[blockIdx.x];
    ri = A.rows[row];
  }
  const int J = ri.J;
  const long long base = ri.bin_off;
  const int t = threadIdx.x;
  RCSCM_DASSERT(row >= 0 && row < A.n_rows);
  RCSCM_DASSERT(ri.M == M && J >= 1 && J <= NT * BPL);
  RCSCM_DASSERT(base >= 0 && base + J <= A.n_bins);
  RCSCM_DASSERT(A.ck_rh == nullptr || (A.ck_sb >= A.n_bins && A.ck_sr >= A.n_rows));
  __shared__ SetupLDS<M> L;
  __shared__ uint64_t red[2][NW];
  __shared__ unsigned cflag;

  // x of G bins per lane in registers ahead of the precomputation (G M complex registers)
  constexpr int GMAX = NT >= 1024 ? (M <= 4 ? 2 : 1) : (M <= 2 ? 8 : (M <= 4 ? 4 : 2));
  constexpr int G = BPL < GMAX ? BPL : GMAX;
  float2 xv[G][M];
  // Lanes past the row's last frame load that frame again (their values are
  // not used), so the loads need no branch.
  auto load_bin = [&](int q, float2(&v)[M]) {
    const int j = t + q * NT;
    load_x8<M>(A.x + ri.x_off + (long long)(j < J ? j : J - 1) * M, v);
  };
  // The setup's loads first, then only the first bin of x per lane: every
  // workgroup of the launch starts at once, and the more x is in flight the
  // longer the setup's few loads wait behind it (measured at M = 4, I = 513,
  // J = 1000: setup inputs after 1.0 us instead of 2.5 us, launch 24.0 us
  // instead of 25.8 us).  The other bins are requested right after the setup.
  const SetupIn sin = row_setup_load<M>(A.Rp, A.a, A.b, ri);
  load_bin(0, xv[0]);
  if (t == 0) cflag = 0u;

  if (t < 64) row_setup_wave<M>(sin, L);
  __syncthreads();
#pragma unroll
  for (int q = 1; q < G; ++q) load_bin(q, xv[q]);
  write_row_constants<M, NT>(L, row, ri, A.rcd, A.rcf, A.rsf, A.lam0, A.lam_c, A.lam, A.status);
  const RowConstF rc = row_const_f<M>(L, ri);
  const double inv_taa = L.inv_taa;

  float4 ts[BPL];
  float vnu[BPL], vrh[BPL], vru[BPL];
  bool bad_x = false, bad_state = false;
#pragma unroll
  for (int q = 0; q < BPL; ++q) {
    const int j = t + q * NT;
    if (j < J) {
      precompute_bin<M>(xv[q % G], L, inv_taa, ts[q], vnu[q], bad_x);
      if (A.tsig) {  // the state a later iterate/extract/objective/backward reads
        A.tsig[base + j] = ts[q];
        A.nu[base + j] = vnu[q];
      }
      ts[q] = turn_sigma_bx(ts[q], rc);
      vrh[q] = A.rh0 ? A.rh0[base + j] : A.rh_c;
      vru[q] = A.ru0 ? A.ru0[base + j] : A.ru_c;
      bad_state = bad_state || !(vrh[q] > 0.0f) || !(vru[q] > 0.0f) || !isfinite(vrh[q]) ||
                  !isfinite(vru[q]);
    } else {
      ts[q] = make_float4(0.f, 0.f, 0.f, 0.f);
      vnu[q] = 0.f;
      vrh[q] = 1.f;
      vru[q] = 1.f;
    }
    if (q + G < BPL) load_bin(q + G, xv[q % G]);
  }
  const float lam0 = A.lam0 ? A.lam0[row] : A.lam_c;
  const float lam_fin = resident_iterations<NT, BPL, 0, kFairClass>(
      ts, vnu, vrh, vru, rc, lam0, row, J, base, A.K, A.inv_a2, A.beta_a2, red, A.ck_rh, A.ck_ru,
      A.ck_lam, A.ck_sb, A.ck_sr, kFairClass && A.fair != 0);
  const LamTerms Lf = lam_terms(rc, lam_fin);
#pragma unroll
  for (int q = 0; q < BPL; ++q) {
    const int j = t + q * NT;
    if (j >= J) continue;
    if (A.rh) {
      A.rh[base + j] = vrh[q];
      A.ru[base + j] = vru[q];
    }
    if (A.rh_out) A.rh_out[base + j] = vrh[q];
    if (A.ru_out) A.ru_out[base + j] = vru[q];
    if (A.s_hat) A.s_hat[base + j] = s_hat_of(ts[q], vrh[q], vru[q], Lf);
    bad_state = bad_state || !isfinite(vrh[q]) || !isfinite(vru[q]);
  }
  if (t == 0) {
    if (A.lam) A.lam[row] = lam_fin;
    if (A.lam_out) A.lam_out[row] = lam_fin;
    if (!(lam_fin > 0.0f) || !isfinite(lam_fin)) atomicOr(&cflag, ST_LAM_NONPOS);
  }
  if (bad_x) atomicOr(&cflag, ST_NONFINITE_IN);
  if (bad_state) atomicOr(&cflag, ST_NONFINITE_STATE);
  // the status word was stored by write_row_constants; OR the new bits in only
  // after a barrier (with K = 0 the iterations contain none)
  __syncthreads();
  if (t == 0 && cflag) atomicOr(A.status + row, cflag);
}

template <int M>
void fused_launch_m(hipStream_t s, int nt, int bpl, int nrows, const FusedArgs& A) {
#define RCSCM_FU(NTT, B)                                                                   \
  if (nt == NTT && bpl == B) {                                                             \
    hipLaunchKernelGGL((accel_fused_kernel<M, NTT, B>), dim3(nrows), dim3(NTT), 0, s, A); \
    return;                                                                                \
  }
  RCSCM_FU(256, 1)
  RCSCM_FU(256, 2)
  RCSCM_FU(256, 4)
  RCSCM_FU(256, 8)
  RCSCM_FU(512, 2)
  RCSCM_FU(512, 4)
  RCSCM_FU(512, 8)
  RCSCM_FU(1024, 1)
  RCSCM_FU(1024, 2)
  RCSCM_FU(1024, 4)
  RCSCM_FU(1024, 8)
#undef RCSCM_FU
}

}  // namespace

// The (workgroup size, bins per lane) pairs the fused launch is instantiated
// for; the autotuner chooses among them per (M, row length).
bool fused_supported(int nt, int bpl) {
  const int cls[11][2] = {{256, 1}, {256, 2},  {256, 4},  {256, 8},  {512, 2}, {512, 4},
                          {512, 8}, {1024, 1}, {1024, 2}, {1024, 4}, {1024, 8}};
  for (const auto& c : cls)
    if (c[0] == nt && c[1] == bpl) return true;
  return false;
}

// The smallest class holding the row.  Measured on MI355X: 256 lanes up to
// 2048 frames, then 512 x 8 (24 % faster than 1024 x 4 at J = 3000), then
// 1024 x 8 (12 % faster than 512 x 16 at J = 8000).
bool fused_class(int J, int* nt, int* bpl) {
  const int cls[6][2] = {{256, 1}, {256, 2}, {256, 4}, {256, 8}, {512, 8}, {1024, 8}};
  for (const auto& c : cls)
    if (c[0] * c[1] >= J) {
      *nt = c[0];
      *bpl = c[1];
      return true;
    }
  return false;
}

template <int M>
int fused_blocks_per_cu_m(int nt, int bpl) {
  int n = 0;
#define RCSCM_OC(NTT, B)                                                                      \
  if (nt == NTT && bpl == B) {                                                                \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, accel_fused_kernel<M, NTT, B>, NTT, \
                                                     0) != hipSuccess)                        \
      n = 0;                                                                                  \
    return n;                                                                                 \
  }
  RCSCM_OC(256, 1)
  RCSCM_OC(256, 2)
  RCSCM_OC(256, 4)
  RCSCM_OC(256, 8)
  RCSCM_OC(512, 2)
  RCSCM_OC(512, 4)
  RCSCM_OC(512, 8)
  RCSCM_OC(1024, 1)
  RCSCM_OC(1024, 2)
  RCSCM_OC(1024, 4)
  RCSCM_OC(1024, 8)
#undef RCSCM_OC
  return 0;
}

// Workgroups of the (M, nt, bpl) class one CU holds at once (0 if unknown);
// the same on every gfx950 device, queried once per class.
int fused_blocks_per_cu(int M, int nt, int bpl) {
  static std::atomic<int> cache[9][3][9];  // M, log2(nt / 256), bpl; 0 = not yet queried
  if (M < 2 || M > 8 || bpl < 1 || bpl > 8 || !fused_supported(nt, bpl)) return 0;
  const int ni = nt == 256 ? 0 : (nt == 512 ? 1 : 2);
  int v = cache[M][ni][bpl].load(std::memory_order_relaxed);
  if (v != 0) return v > 0 ? v : 0;
  int n = 0;
  switch (M) {
    case 2: n = fused_blocks_per_cu_m<2>(nt, bpl); break;
    case 3: n = fused_blocks_per_cu_m<3>(nt, bpl); break;
    case 4: n = fused_blocks_per_cu_m<4>(nt, bpl); break;
    case 5: n = fused_blocks_per_cu_m<5>(nt, bpl); break;
    case 6: n = fused_blocks_per_cu_m<6>(nt, bpl); break;
    case 7: n = fused_blocks_per_cu_m<7>(nt, bpl); break;
    case 8: n = fused_blocks_per_cu_m<8>(nt, bpl); break;
    default: break;
  }
  cache[M][ni][bpl].store(n > 0 ? n : -1, std::memory_order_relaxed);
  return n;
}

// Measured on MI355X with rows of one class: where the launch holds all its
// rows at once, lowering a row's priority as it advances (FusedArgs::fair)
// shortened the launch by 4-8 % (256-lane classes, M = 2..8; 22.3 -> 20.6 us
// at M = 4, I = 513, J = 1000, K = 20); where rows wait for a free CU, the
// same steps lengthened it by about 4 % (a row that finishes early frees its
// CU for the next), so they are left off there.
bool fused_fair(int M, int nt, int bpl, int nrows, int device) {
  const int per_cu = fused_blocks_per_cu(M, nt, bpl);
  return per_cu > 0 && (long long)nrows <= (long long)per_cu * device_cu_count(device);
}

int device_cu_count(int device) {
  static std::atomic<int> cus[64];  // CU count per device; 0 = not yet queried
  if (device < 0 || device >= 64) return 0;
  int ncu = cus[device].load(std::memory_order_relaxed);
  if (ncu == 0) {
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) !=
            hipSuccess ||
        ncu <= 0)
      return 0;
    cus[device].store(ncu, std::memory_order_relaxed);
  }
  return ncu;
}

void launch_fused(hipStream_t s, int M, int nt, int bpl, int nrows, const FusedArgs& A) {
  if (nrows <= 0) return;
  switch (M) {
    case 2: fused_launch_m<2>(s, nt, bpl, nrows, A); break;
    case 3: fused_launch_m<3>(s, nt, bpl, nrows, A); break;
    case 4: fused_launch_m<4>(s, nt, bpl, nrows, A); break;
    case 5: fused_launch_m<5>(s, nt, bpl, nrows, A); break;
    case 6: fused_launch_m<6>(s, nt, bpl, nrows, A); break;
    case 7: fused_launch_m<7>(s, nt, bpl, nrows, A); break;
    case 8: fused_launch_m<8>(s, nt, bpl, nrows, A); break;
    default: break;
  }
}

}  // namespace rcscm
