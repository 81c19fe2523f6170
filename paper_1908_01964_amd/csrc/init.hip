// rcscm_init on the device: per-row FP64 setup, per-bin FP64 precomputation
// and the initial state, in one launch per microphone count M (one
// workgroup per chunk of a row).  The arithmetic is in init_common.h.
//
// The setup's loads of a, R', b go first, then the x loads of each thread's
// first group of bins, so the x latency overlaps the setup's FP64 work.
// The first chunk of a row writes the row constants, the row's status word
// and its initial lambda; every chunk writes tau^ax, sigma^bx (float4) and
// nu (float) for its bins plus their initial r^h, r^u.  Memory-bound: 8M
// bytes read and 28 written per bin.
#include "init_common.h"
#include "xcd_order.h"

namespace rcscm {

namespace {

constexpr int kInitNT = 256;

template <int M>
__global__ __launch_bounds__(kInitNT) __attribute__((amdgpu_waves_per_eu(4))) void init_kernel(
    const InitArgs A) {
  const ChunkInfo ck = A.chunks[xcd_local_chunk(blockIdx.x, gridDim.x)];
  const int row = ck.row;
  const RowInfo ri = A.rows[row];
  const int t = threadIdx.x;
  RCSCM_DASSERT(row >= 0 && row < A.n_rows && ri.M == M);
  RCSCM_DASSERT(ck.start >= 0 && ck.len >= 1 && ck.start + ck.len <= ri.J);
  RCSCM_DASSERT(ri.bin_off >= 0 && ri.bin_off + ri.J <= A.n_bins);
  __shared__ SetupLDS<M> L;

  constexpr int G = M <= 4 ? 4 : (M <= 6 ? 2 : 1);
  float2 xv[G][M];
  const bool al4 = (M & 1) == 0 && (ri.x_off & 1) == 0;  // 16-byte aligned pairs of mics
  auto load_group = [&](int g0) {
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const int jj = g0 + t + q * kInitNT;
      if (jj < ck.len) load_x<M>(A.x + ri.x_off + (long long)(ck.start + jj) * M, al4, xv[q]);
    }
  };
  const SetupIn sin = row_setup_load<M>(A.Rp, A.a, A.b, ri);  // ahead of the x loads
  load_group(0);

  if (t < 64) row_setup_wave<M>(sin, L);
  __syncthreads();
  if (ck.start == 0)
    write_row_constants<M, kInitNT>(L, row, ri, A.rcd, A.rcf, A.rsf, A.lam0, A.lam_c, A.lam,
                                    A.status);

  const double inv_taa = L.inv_taa;
  bool bad_x = false, bad_state = false;
  for (int g0 = 0; g0 < ck.len; g0 += G * kInitNT) {
    if (g0 > 0) load_group(g0);
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const int jj = g0 + t + q * kInitNT;
      if (jj >= ck.len) continue;
      float4 ts;
      float nu;
      precompute_bin<M>(xv[q], L, inv_taa, ts, nu, bad_x);
      const long long bin = ri.bin_off + ck.start + jj;
      A.tsig[bin] = ts;
      A.nu[bin] = nu;
      const float h = A.rh0 ? A.rh0[bin] : A.rh_c;
      const float u = A.ru0 ? A.ru0[bin] : A.ru_c;
      A.rh[bin] = h;
      A.ru[bin] = u;
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
#define RCSCM_INIT(MM)                                                             \
  case MM:                                                                         \
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
