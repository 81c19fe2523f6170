// Second-stage accelerated EM iteration (Algorithm 2) on gfx950.
//
// Two schedules of the same per-bin arithmetic (accel_common.h):
//
// RESIDENT: one workgroup per (utterance, frequency) row.  Each lane holds
//   BPL bins (frames j = lane + q*NT) of the row in registers - tau^ax,
//   sigma^bx, nu, r^h, r^u - for all K iterations.  Per iteration: phase A
//   over the lane's bins, the lambda frame sum (DPP rotations within each
//   wave, then one LDS slot per wave, one barrier), phase B.  HBM traffic:
//   28 bytes read and 8 bytes written per bin for the whole K loop.
//
// STREAM: rows are cut into chunks; launch k (k = 1..K+1) finishes iteration
//   k-1 and starts iteration k.  Finishing iteration k-1 needs lambda_{k-1},
//   the mean over the whole row, which launch k reads as the per-chunk
//   partial sums written by launch k-1 - so the frame-sum barrier falls on a
//   launch boundary and no workgroup ever waits for another.  Phase A of
//   iteration k-1 is recomputed from the stored state of iteration k-2
//   (cheap arithmetic) instead of storing its intermediates.  HBM traffic
//   per launch: 28 bytes read and 8 bytes written per bin.
#include <atomic>

#include "resident_loop.h"
#include "xcd_order.h"

namespace rcscm {

namespace {

// ---------------------------------------------------------------- RESIDENT --

// The classes that compile the priority steps of the loop (resident_segments):
// 256 lanes, up to four bins per lane.
template <int NT, int BPL>
constexpr bool kResFairClass = NT == 256 && BPL <= 4;

template <int NT, int BPL, int LS>
__global__ __launch_bounds__(NT) void accel_resident_kernel(
    const int* __restrict__ row_list, const RowInfo* __restrict__ rows,
    const RowConstF* __restrict__ rcf, const float4* __restrict__ tsig,
    const float* __restrict__ nu, float* __restrict__ rh, float* __restrict__ ru,
    float* __restrict__ lam, float inv_a2, float beta_a2, int K, float* __restrict__ ck_rh,
    float* __restrict__ ck_ru, float* __restrict__ ck_lam, long long ck_sb, int ck_sr,
    unsigned* __restrict__ status, int fair) {
  constexpr int NW = NT / 64;
  const int row = row_list[blockIdx.x];
  const RowInfo ri = rows[row];
  const RowConstF rc = rcf[row];
  const int J = ri.J;
  const long long base = ri.bin_off;
  const int t = threadIdx.x;
  RCSCM_DASSERT(J >= 1 && J <= NT * BPL);
  RCSCM_DASSERT(ck_rh == nullptr || (base + J <= ck_sb && row < ck_sr));

  float4 ts[BPL];
  float vnu[BPL], vrh[BPL], vru[BPL];
#pragma unroll
  for (int q = 0; q < BPL; ++q) {
    const int j = t + q * NT;
    if (j < J) {
      ts[q] = turn_sigma_bx(tsig[base + j], rc);
      vnu[q] = nu[base + j];
      vrh[q] = rh[base + j];
      vru[q] = ru[base + j];
    } else {
      ts[q] = make_float4(0.f, 0.f, 0.f, 0.f);
      vnu[q] = 0.f;
      vrh[q] = 1.f;
      vru[q] = 1.f;
    }
  }
  __shared__ uint64_t red[2][NW];
  const float lam_t = resident_iterations<NT, BPL, LS, kResFairClass<NT, BPL>>(
      ts, vnu, vrh, vru, rc, lam[row], row, J, base, K, inv_a2, beta_a2, red, ck_rh, ck_ru, ck_lam,
      ck_sb, ck_sr, fair != 0);

  bool bad = false;
#pragma unroll
  for (int q = 0; q < BPL; ++q) {
    const int j = t + q * NT;
    if (j < J) {
      rh[base + j] = vrh[q];
      ru[base + j] = vru[q];
      bad = bad || !isfinite(vrh[q]) || !isfinite(vru[q]);
    }
  }
  if (t == 0) {
    lam[row] = lam_t;
    if (!(lam_t > 0.0f) || !isfinite(lam_t)) atomicOr(status + row, ST_LAM_NONPOS);
  }
  if (bad) atomicOr(status + row, ST_NONFINITE_STATE);
}

template <int NT, int BPL, int LS>
void res_launch(hipStream_t s, int nrows, const int* row_list, const RowInfo* rows,
                const RowConstF* rcf, const float4* tsig, const float* nu, float* rh, float* ru,
                float* lam, float inv_a2, float beta_a2, int K, float* ck_rh, float* ck_ru,
                float* ck_lam, long long ck_sb, int ck_sr, unsigned* status, int fair) {
  hipLaunchKernelGGL((accel_resident_kernel<NT, BPL, LS>), dim3(nrows), dim3(NT), 0, s, row_list,
                     rows, rcf, tsig, nu, rh, ru, lam, inv_a2, beta_a2, K, ck_rh, ck_ru, ck_lam,
                     ck_sb, ck_sr, status, fair);
}

// Workgroups of accel_resident_kernel<NT, BPL, LS> one CU holds at once (0 if unknown).
template <int NT, int BPL, int LS>
int res_blocks_per_cu() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, accel_resident_kernel<NT, BPL, LS>, NT,
                                                   0) != hipSuccess)
    n = 0;
  return n;
}

using ResFn = void (*)(hipStream_t, int, const int*, const RowInfo*, const RowConstF*,
                       const float4*, const float*, float*, float*, float*, float, float, int,
                       float*, float*, float*, long long, int, unsigned*, int);

#define RCSCM_RES_BPL_LIST(NT, LS)                                                       \
  {res_launch<NT, 1, LS>, res_launch<NT, 2, LS>, res_launch<NT, 3, LS>,                  \
   res_launch<NT, 4, LS>, res_launch<NT, 5, LS>, res_launch<NT, 6, LS>,                  \
   res_launch<NT, 7, LS>, res_launch<NT, 8, LS>, nullptr, res_launch<NT, 10, LS>,        \
   nullptr, res_launch<NT, 12, LS>, nullptr, nullptr, nullptr, res_launch<NT, 16, LS>}

// 1024-lane workgroups are limited to 128 VGPRs: 10+ bins per lane would spill.
#define RCSCM_RES_BPL_LIST_1024(LS)                                                      \
  {res_launch<1024, 1, LS>, res_launch<1024, 2, LS>, res_launch<1024, 3, LS>,            \
   res_launch<1024, 4, LS>, res_launch<1024, 5, LS>, res_launch<1024, 6, LS>,            \
   res_launch<1024, 7, LS>, res_launch<1024, 8, LS>, nullptr, nullptr, nullptr, nullptr, \
   nullptr, nullptr, nullptr, nullptr}

// [lamsum][nt index][bpl-1]; nt index: 64,128,256,512,1024
const ResFn kRes[2][5][16] = {
    {RCSCM_RES_BPL_LIST(64, 0), RCSCM_RES_BPL_LIST(128, 0), RCSCM_RES_BPL_LIST(256, 0),
     RCSCM_RES_BPL_LIST(512, 0), RCSCM_RES_BPL_LIST_1024(0)},
    {RCSCM_RES_BPL_LIST(64, 1), RCSCM_RES_BPL_LIST(128, 1), RCSCM_RES_BPL_LIST(256, 1),
     RCSCM_RES_BPL_LIST(512, 1), RCSCM_RES_BPL_LIST_1024(1)}};

int nt_index(int nt) {
  switch (nt) {
    case 64: return 0;
    case 128: return 1;
    case 256: return 2;
    case 512: return 3;
    case 1024: return 4;
    default: return -1;
  }
}

// ------------------------------------------------------------------ STREAM --

constexpr int kStreamNT = 256;

// Accesses to the per-bin state. NTMP marks them non-temporal (streamed past
// the caches), for state that does not stay in the last-level cache between
// launches anyway.
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <bool NTMP>
__device__ __forceinline__ float4 ld_state(const float4* p) {
  if constexpr (NTMP) {
    const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
    return make_float4(v.x, v.y, v.z, v.w);
  } else {
    return *p;
  }
}
template <bool NTMP>
__device__ __forceinline__ float ld_state(const float* p) {
  if constexpr (NTMP) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NTMP>
__device__ __forceinline__ void st_state(float* p, float v) {
  if constexpr (NTMP) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// NU_EARLY: the state stays in the last-level cache between launches. nu is
// then requested together with the rest of the state (one memory round trip
// instead of two). Otherwise the state streams from HBM: nu is requested after
// the frame sum (a fourth concurrent stream cost more than the round trip it
// saves), and all state accesses are non-temporal.
template <int BPL, int LS, bool FINISH, bool START, bool NU_EARLY>
__global__ __launch_bounds__(kStreamNT) void accel_stream_kernel(
    const ChunkInfo* __restrict__ chunks, const RowInfo* __restrict__ rows,
    const RowConstF* __restrict__ rcf, const float4* __restrict__ tsig,
    const float* __restrict__ nu, float* __restrict__ rh, float* __restrict__ ru,
    const float* __restrict__ lam_prev, float* __restrict__ lam_new,
    const uint64_t* __restrict__ part_in, uint64_t* __restrict__ part_out, float inv_a2,
    float beta_a2, unsigned* __restrict__ status) {
  constexpr int NW = kStreamNT / 64;
  const ChunkInfo ck = chunks[xcd_local_chunk(blockIdx.x, gridDim.x)];
  const RowInfo ri = rows[ck.row];
  const RowConstF rc = rcf[ck.row];
  const long long base = ri.bin_off + ck.start;
  const int len = ck.len;
  const int t = threadIdx.x;
  const int wave = t >> 6;
  RCSCM_DASSERT(ck.start >= 0 && ck.len >= 1 && ck.start + ck.len <= ri.J);
  RCSCM_DASSERT(len <= BPL * kStreamNT);
  const double invJ = 1.0 / (double)ri.J;
  __shared__ uint64_t red[NW];

  float4 ts[BPL];
  float vrh[BPL], vru[BPL], vnu[BPL];
#pragma unroll
  for (int q = 0; q < BPL; ++q) {
    const int j = t + q * kStreamNT;
    if (j < len) {
      ts[q] = ld_state<!NU_EARLY>(tsig + base + j);
      vrh[q] = ld_state<!NU_EARLY>(rh + base + j);
      vru[q] = ld_state<!NU_EARLY>(ru + base + j);
      vnu[q] = (FINISH && NU_EARLY) ? nu[base + j] : 0.f;
    } else {
      ts[q] = make_float4(0.f, 0.f, 0.f, 0.f);
      vrh[q] = 1.f;
      vru[q] = 1.f;
      vnu[q] = 0.f;
    }
  }
  float lam_cur = lam_prev[ck.row];
  if constexpr (FINISH) {
    // lambda of the iteration being finished: mean of the row's partial sums
    const float lam_k = wave_sum_packed<LS>(part_in + ri.part_off, ri.nparts).mean(invJ);
    if (ck.start == 0 && t == 0) {
      lam_new[ck.row] = lam_k;
      if (!(lam_k > 0.0f) || !isfinite(lam_k)) atomicOr(status + ck.row, ST_LAM_NONPOS);
    }
    const LamTerms Lt = lam_terms(rc, lam_cur);
    const LamTerms Ln = lam_terms(rc, lam_k);
    bool bad = false;
#pragma unroll
    for (int q = 0; q < BPL; ++q) {
      const int j = t + q * kStreamNT;
      if (!NU_EARLY && j < len) vnu[q] = ld_state<true>(nu + base + j);
      const PhaseA A = phase_a(ts[q], vrh[q], vru[q], rc, Lt, inv_a2, beta_a2);
      vrh[q] = A.rh_new;
      vru[q] = phase_b(ts[q], vnu[q] * rc.invM, A, rc, Ln);
      if (j < len) {
        st_state<!NU_EARLY>(rh + base + j, vrh[q]);
        st_state<!NU_EARLY>(ru + base + j, vru[q]);
        bad = bad || !isfinite(vrh[q]) || !isfinite(vru[q]);
      }
    }
    if (bad) atomicOr(status + ck.row, ST_NONFINITE_STATE);
    lam_cur = lam_k;
  }
  if constexpr (START) {
    const LamTerms Lt = lam_terms(rc, lam_cur);
    LamAcc<LS> acc;
    float tsum = 0.0f;  // F64 policy: the lane's terms in float, lanes in double
#pragma unroll
    for (int q = 0; q < BPL; ++q) {
      const PhaseA A = phase_a(ts[q], vrh[q], vru[q], rc, Lt, inv_a2, beta_a2);
      const bool in = t + q * kStreamNT < len;
      if constexpr (LS == 0)
        tsum += in ? A.t : 0.0f;
      else if (in)
        acc.add(A.t);
    }
    if constexpr (LS == 0) acc.s = (double)tsum;
    acc = wave_allreduce<LS>(acc);
    if ((t & 63) == 0) red[wave] = acc.pack();
    __syncthreads();
    if (t == 0) part_out[ck.part] = slots_sum<LS, NW>(red).pack();
  }
}

template <int BPL, int LS, bool F, bool S>
void stream_launch(hipStream_t s, bool nu_early, int nchunks, const ChunkInfo* chunks,
                   const RowInfo* rows, const RowConstF* rcf, const float4* tsig,
                   const float* nu, float* rh, float* ru, const float* lam_prev,
                   float* lam_new, const uint64_t* part_in, uint64_t* part_out, float inv_a2,
                   float beta_a2, unsigned* status) {
  if (nu_early)
    hipLaunchKernelGGL((accel_stream_kernel<BPL, LS, F, S, true>), dim3(nchunks),
                       dim3(kStreamNT), 0, s, chunks, rows, rcf, tsig, nu, rh, ru, lam_prev,
                       lam_new, part_in, part_out, inv_a2, beta_a2, status);
  else
    hipLaunchKernelGGL((accel_stream_kernel<BPL, LS, F, S, false>), dim3(nchunks),
                       dim3(kStreamNT), 0, s, chunks, rows, rcf, tsig, nu, rh, ru, lam_prev,
                       lam_new, part_in, part_out, inv_a2, beta_a2, status);
}

template <int BPL, int LS>
void stream_dispatch(hipStream_t s, bool F, bool S, bool nu_early, int nchunks,
                     const ChunkInfo* chunks, const RowInfo* rows, const RowConstF* rcf,
                     const float4* tsig, const float* nu, float* rh, float* ru,
                     const float* lam_prev, float* lam_new, const uint64_t* part_in,
                     uint64_t* part_out, float inv_a2, float beta_a2, unsigned* status) {
  if (F && S)
    stream_launch<BPL, LS, true, true>(s, nu_early, nchunks, chunks, rows, rcf, tsig, nu, rh,
                                       ru, lam_prev, lam_new, part_in, part_out, inv_a2,
                                       beta_a2, status);
  else if (F)
    stream_launch<BPL, LS, true, false>(s, nu_early, nchunks, chunks, rows, rcf, tsig, nu, rh,
                                        ru, lam_prev, lam_new, part_in, part_out, inv_a2,
                                        beta_a2, status);
  else if (S)
    stream_launch<BPL, LS, false, true>(s, nu_early, nchunks, chunks, rows, rcf, tsig, nu, rh,
                                        ru, lam_prev, lam_new, part_in, part_out, inv_a2,
                                        beta_a2, status);
}

// ----------------------------------------------------------------- EXTRACT --

__global__ __launch_bounds__(256) void extract_kernel(
    const ChunkInfo* __restrict__ chunks, const RowInfo* __restrict__ rows,
    const RowConstF* __restrict__ rcf, const float4* __restrict__ tsig,
    const float* __restrict__ rh_in, const float* __restrict__ ru_in,
    const float* __restrict__ lam_in, float* __restrict__ rh_out, float* __restrict__ ru_out,
    float* __restrict__ lam_out, float2* __restrict__ s_hat) {
  const ChunkInfo ck = chunks[xcd_local_chunk(blockIdx.x, gridDim.x)];
  const RowInfo ri = rows[ck.row];
  const RowConstF rc = rcf[ck.row];
  const float lam = lam_in[ck.row];
  const LamTerms L = lam_terms(rc, lam);
  RCSCM_DASSERT(ck.start >= 0 && ck.len >= 1 && ck.start + ck.len <= ri.J);
  if (lam_out != nullptr && ck.start == 0 && threadIdx.x == 0) lam_out[ck.row] = lam;
#pragma unroll 4
  for (int jj = threadIdx.x; jj < ck.len; jj += 256) {
    const long long bin = ri.bin_off + ck.start + jj;
    const float vrh = rh_in[bin], vru = ru_in[bin];
    if (rh_out != nullptr) rh_out[bin] = vrh;
    if (ru_out != nullptr) ru_out[bin] = vru;
    // s_hat = gamma rho^ax, rho^ax = tau^ax + sigma^ab sigma^bx / lambda, in the turned form
    // the fused launch uses (the same rounding)
    if (s_hat != nullptr) s_hat[bin] = s_hat_of(turn_sigma_bx(tsig[bin], rc), vrh, vru, L);
  }
}

// --------------------------------------------------------------- OBJECTIVE --

__global__ __launch_bounds__(256) void objective_kernel(
    const ChunkInfo* __restrict__ chunks, const RowInfo* __restrict__ rows,
    const RowConstF* __restrict__ rcf, const RowConstD* __restrict__ rcd,
    const float4* __restrict__ tsig, const float* __restrict__ nu, const float* __restrict__ rh,
    const float* __restrict__ ru, const float* __restrict__ lam, double alpha, double beta,
    double* __restrict__ partial) {
  const ChunkInfo ck = chunks[blockIdx.x];
  const RowInfo ri = rows[ck.row];
  const double taa = rcd[ck.row].t_aa;
  const double2 sab = rcd[ck.row].s_ab;
  const double logpdet = log(rcd[ck.row].det_a) - log(rcd[ck.row].shift);  // log pdet(R')
  const double l = (double)lam[ck.row];
  const double M = (double)ri.M;
  const double sab2 = sab.x * sab.x + sab.y * sab.y;
  const double rho_aa = taa + sab2 / l;
  const double inv_taa = taa > 0.0 ? 1.0 / taa : 0.0;
  const double c0 = M * log(3.14159265358979323846) + log(l) + logpdet;
  double acc = 0.0;
  for (int jj = threadIdx.x; jj < ck.len; jj += blockDim.x) {
    const long long bin = ri.bin_off + ck.start + jj;
    const float4 ts = tsig[bin];
    const double h = rh[bin], u = ru[bin];
    const double tar = ts.x, tai = ts.y, sbr = ts.z, sbi = ts.w;
    const double txx = (double)nu[bin] + (tar * tar + tai * tai) * inv_taa;
    const double rax_r = tar + (sab.x * sbr - sab.y * sbi) / l;
    const double rax_i = tai + (sab.x * sbi + sab.y * sbr) / l;
    const double rxx = txx + (sbr * sbr + sbi * sbi) / l;
    const double g = h / (u + h * rho_aa);
    acc += c0 + M * log(u) + log1p(h * rho_aa / u) + (rxx - g * (rax_r * rax_r + rax_i * rax_i)) / u +
           (alpha + 1.0) * log(h) + beta / h;
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s2 = 128; s2 > 0; s2 >>= 1) {
    if ((int)threadIdx.x < s2) red[threadIdx.x] += red[threadIdx.x + s2];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

}  // namespace

bool resident_supported(int nt, int bpl) {
  const int ni = nt_index(nt);
  return ni >= 0 && bpl >= 1 && bpl <= 16 && kRes[0][ni][bpl - 1] != nullptr;
}

void launch_accel_resident(hipStream_t s, int nt, int bpl, int lamsum, int nrows,
                           const int* row_list, const RowInfo* rows, const RowConstF* rcf,
                           const float4* tsig, const float* nu, float* rh, float* ru, float* lam,
                           float alpha, float beta, int K, float* ckpt_rh, float* ckpt_ru,
                           float* ckpt_lam, long long ckpt_stride_bins, int ckpt_stride_rows,
                           unsigned* status, int fair) {
  if (nrows <= 0 || K <= 0) return;
  const float inv_a2 = (float)(1.0 / ((double)alpha + 2.0));
  const float beta_a2 = (float)((double)beta / ((double)alpha + 2.0));
  kRes[lamsum ? 1 : 0][nt_index(nt)][bpl - 1](s, nrows, row_list, rows, rcf, tsig, nu, rh, ru,
                                              lam, inv_a2, beta_a2, K, ckpt_rh, ckpt_ru,
                                              ckpt_lam, ckpt_stride_bins, ckpt_stride_rows,
                                              status, fair);
}

bool resident_fair(int nt, int bpl, int lamsum, int nrows, int device) {
  if (nt != 256 || bpl < 1 || bpl > 4) return false;  // only these classes have the steps
  static std::atomic<int> cache[2][4];                // per (policy, bpl); 0 = not yet queried
  const int ls = lamsum ? 1 : 0;
  int v = cache[ls][bpl - 1].load(std::memory_order_relaxed);
  if (v == 0) {
    int n = 0;
    switch (bpl * 2 + ls) {
      case 2: n = res_blocks_per_cu<256, 1, 0>(); break;
      case 3: n = res_blocks_per_cu<256, 1, 1>(); break;
      case 4: n = res_blocks_per_cu<256, 2, 0>(); break;
      case 5: n = res_blocks_per_cu<256, 2, 1>(); break;
      case 6: n = res_blocks_per_cu<256, 3, 0>(); break;
      case 7: n = res_blocks_per_cu<256, 3, 1>(); break;
      case 8: n = res_blocks_per_cu<256, 4, 0>(); break;
      case 9: n = res_blocks_per_cu<256, 4, 1>(); break;
      default: break;
    }
    v = n > 0 ? n : -1;
    cache[ls][bpl - 1].store(v, std::memory_order_relaxed);
  }
  return v > 0 && (long long)nrows <= (long long)v * device_cu_count(device);
}

void launch_accel_stream(hipStream_t s, int lamsum, bool finish_prev, bool start_next,
                         bool nu_early, int nchunks, const ChunkInfo* chunks,
                         const RowInfo* rows, const RowConstF* rcf, const float4* tsig,
                         const float* nu, float* rh, float* ru, const float* lam_prev,
                         float* lam_new, const uint64_t* part_in, uint64_t* part_out,
                         float alpha, float beta, int chunk_threads, unsigned* status) {
  if (nchunks <= 0) return;
  const float inv_a2 = (float)(1.0 / ((double)alpha + 2.0));
  const float beta_a2 = (float)((double)beta / ((double)alpha + 2.0));
  const int bpl = chunk_threads / kStreamNT;
#define RCSCM_STREAM_CASE(B)                                                                 \
  case B:                                                                                    \
    if (lamsum)                                                                              \
      stream_dispatch<B, 1>(s, finish_prev, start_next, nu_early, nchunks, chunks, rows, rcf, \
                            tsig, nu, rh, ru, lam_prev, lam_new, part_in, part_out, inv_a2,  \
                            beta_a2, status);                                                \
    else                                                                                     \
      stream_dispatch<B, 0>(s, finish_prev, start_next, nu_early, nchunks, chunks, rows, rcf, \
                            tsig, nu, rh, ru, lam_prev, lam_new, part_in, part_out, inv_a2,  \
                            beta_a2, status);                                                \
    break;
  switch (bpl) {
    RCSCM_STREAM_CASE(1)
    RCSCM_STREAM_CASE(2)
    RCSCM_STREAM_CASE(4)
    RCSCM_STREAM_CASE(8)
    default: break;
  }
#undef RCSCM_STREAM_CASE
}

void launch_extract(hipStream_t s, int nchunks, const ChunkInfo* chunks, const RowInfo* rows,
                    const RowConstF* rcf, const float4* tsig, const float* rh_in,
                    const float* ru_in, const float* lam_in, float* rh_out, float* ru_out,
                    float* lam_out, float2* s_hat, unsigned* status) {
  (void)status;
  if (nchunks <= 0) return;
  hipLaunchKernelGGL(extract_kernel, dim3(nchunks), dim3(256), 0, s, chunks, rows, rcf, tsig,
                     rh_in, ru_in, lam_in, rh_out, ru_out, lam_out, s_hat);
}

void launch_objective(hipStream_t s, int nchunks, const ChunkInfo* chunks, const RowInfo* rows,
                      const RowConstF* rcf, const RowConstD* rcd, const float4* tsig,
                      const float* nu, const float* rh, const float* ru, const float* lam,
                      double alpha, double beta, double* partial) {
  if (nchunks <= 0) return;
  hipLaunchKernelGGL(objective_kernel, dim3(nchunks), dim3(256), 0, s, chunks, rows, rcf, rcd,
                     tsig, nu, rh, ru, lam, alpha, beta, partial);
}

}  // namespace rcscm
