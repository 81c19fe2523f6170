// rcscm_run_noalloc: the fused single launch of rcscm_run for one utterance,
// without a context and without device allocation, for callers that cannot
// allocate (code under HIP graph capture, serving loops).
//
// The kernel is the one rcscm_run launches (accel_fused_kernel, with no
// workspace state stored); its only device memory beyond the caller's inputs
// and outputs is one status word per row.  Those words, and the summary the
// optional check reduces them to, live in `scratch`, a static device array of
// this library: each GPU holds its own copy until the process ends, and calls
// that overlap on one GPU race on it.  Every call stores the status word of
// each of its rows before any bit is ORed into it, and the summary kernel
// writes all its words, so nothing needs clearing between calls.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "host_internal.h"
#include "rcscm.h"
#include "rcscm_internal.h"

using namespace rcscm;

namespace {

// Error bits in the order rcscm_sync reports them.
constexpr unsigned kErrBits[5] = {ST_NONFINITE_IN, ST_NOT_NULL, ST_NOT_PSD, ST_NONFINITE_STATE,
                                  ST_LAM_NONPOS};
constexpr int kSummaryWords = 8;  // OR of all rows' bits, then the first row with each error bit
constexpr int kMaxRows = RCSCM_NOALLOC_MAX_ROWS;
constexpr int kMaxDevices = 64;

// [0, kMaxRows): per-row status words; then the summary.  A host-side stand-in
// in host code: only its device address (scratch_address) is passed on.
static __device__ __align__(256) unsigned scratch[kMaxRows + kSummaryWords];

std::mutex g_mu;
unsigned* g_scratch[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per
// device with that device current.
rcscm_status scratch_address(unsigned** out, std::string* msg) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *msg = std::string("hipGetDevice failed: ") + hipGetErrorString(e);
    return RCSCM_EDEVICE;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    *msg = "device index out of range for the static scratch table";
    return RCSCM_EDEVICE;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      *msg = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
      return RCSCM_EDEVICE;
    }
    g_scratch[dev] = static_cast<unsigned*>(p);
  }
  *out = g_scratch[dev];
  return RCSCM_OK;
}

// One workgroup: summary[0] = OR of st[0..n), summary[1 + k] = the first row
// whose word has kErrBits[k] (n when none).
__global__ __launch_bounds__(256) void status_summary_kernel(const unsigned* __restrict__ st,
                                                             int n, unsigned* __restrict__ summary) {
  __shared__ unsigned s_or;
  __shared__ unsigned s_first[5];
  const int t = threadIdx.x;
  if (t == 0) s_or = 0u;
  if (t < 5) s_first[t] = (unsigned)n;
  __syncthreads();
  unsigned acc = 0u;
  unsigned first[5] = {(unsigned)n, (unsigned)n, (unsigned)n, (unsigned)n, (unsigned)n};
  for (int r = t; r < n; r += 256) {
    const unsigned w = st[r];
    acc |= w;
#pragma unroll
    for (int k = 0; k < 5; ++k)
      if ((w & kErrBits[k]) && (unsigned)r < first[k]) first[k] = (unsigned)r;
  }
  if (acc) atomicOr(&s_or, acc);
#pragma unroll
  for (int k = 0; k < 5; ++k)
    if (first[k] < (unsigned)n) atomicMin(&s_first[k], first[k]);
  __syncthreads();
  if (t == 0) summary[0] = s_or;
  if (t < 5) summary[1 + t] = s_first[t];
}

rcscm_status fail(rcscm_status s, const std::string& m) {
  set_global_error(m);
  return s;
}

}  // namespace

extern "C" rcscm_status rcscm_run_noalloc(int I, int J, int M, const rcscm_params* params,
                                          void* stream, const void* x, const void* a,
                                          const void* Rp, const void* b, const float* rh0,
                                          const float* ru0, const float* lam0, int K, float* rh,
                                          float* ru, float* lam, void* s_hat, int check) {
  rcscm_params p;
  if (params)
    p = *params;
  else
    rcscm_default_params(&p);
  std::string msg;
  rcscm_status s = validate_args(1, I, &J, &M, &p, &msg);
  if (s != RCSCM_OK) return fail(s, msg);
  if (I > kMaxRows)
    return fail(RCSCM_ESHAPE, "I = " + std::to_string(I) + " exceeds RCSCM_NOALLOC_MAX_ROWS (" +
                                  std::to_string(kMaxRows) + ")");
  if (p.rule != RCSCM_RULE_ACCEL)
    return fail(RCSCM_EINVAL, "rcscm_run_noalloc runs the ACCEL rule only");
  if (p.lamsum != RCSCM_LAMSUM_F64)
    return fail(RCSCM_EINVAL, "rcscm_run_noalloc sums lambda with RCSCM_LAMSUM_F64 only");
  if (p.flags & RCSCM_FLAG_CHECKPOINT)
    return fail(RCSCM_EINVAL, "rcscm_run_noalloc keeps no checkpoints");
  int nt = 0, bpl = 0;
  if (!fused_class(J, &nt, &bpl))
    return fail(RCSCM_ESHAPE, "rcscm_run_noalloc needs J <= 8192 (one workgroup per row)");
  if (K < 0) return fail(RCSCM_ESHAPE, "K must be >= 0");
  if (!x || !a || !Rp || !b) return fail(RCSCM_EINVAL, "x, a, Rp and b must not be NULL");
  unsigned* sp = nullptr;
  s = scratch_address(&sp, &msg);
  if (s != RCSCM_OK) return fail(s, msg);

  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  FusedArgs A{};
  A.row_list = nullptr;  // linear launch: block b serves row b
  A.rows = nullptr;
  A.lin = 1;
  A.lin_row0 = 0;
  A.lin_J = J;
  A.lin_x0 = A.lin_bin0 = A.lin_a0 = A.lin_rp0 = 0;
  A.x = static_cast<const float2*>(x);
  A.a = static_cast<const double2*>(a);
  A.Rp = static_cast<const double2*>(Rp);
  A.b = static_cast<const double2*>(b);
  A.rh0 = rh0;
  A.ru0 = ru0;
  A.lam0 = lam0;
  A.rh_c = p.rh0;
  A.ru_c = p.ru0;
  A.lam_c = p.lam0;
  A.rcd = nullptr;  // no workspace state: results go to the caller's arrays only
  A.rcf = nullptr;
  A.rsf = nullptr;
  A.tsig = nullptr;
  A.nu = nullptr;
  A.rh = nullptr;
  A.ru = nullptr;
  A.lam = nullptr;
  A.status = sp;  // per-row status words in the static scratch
  A.rh_out = rh;
  A.ru_out = ru;
  A.lam_out = lam;
  A.s_hat = static_cast<float2*>(s_hat);
  A.ck_rh = A.ck_ru = A.ck_lam = nullptr;
  A.ck_sb = 0;
  A.ck_sr = 0;
  A.inv_a2 = (float)(1.0 / (p.alpha + 2.0));
  A.beta_a2 = (float)(p.beta / (p.alpha + 2.0));
  A.K = K;
  A.n_bins = (long long)I * J;
  A.n_rows = I;
  int dev = -1;
  A.fair = hipGetDevice(&dev) == hipSuccess && fused_fair(M, nt, bpl, I, dev) ? 1 : 0;
  launch_fused(st, M, nt, bpl, I, A);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RCSCM_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  if (!check) return RCSCM_OK;

  // the rows' data errors, as rcscm_sync reports them (blocks)
  unsigned* summary = sp + kMaxRows;
  hipLaunchKernelGGL(status_summary_kernel, dim3(1), dim3(256), 0, st, sp, I, summary);
  e = hipGetLastError();
  if (e != hipSuccess) return fail(RCSCM_EDEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  unsigned h[6] = {0u, 0u, 0u, 0u, 0u, 0u};
  e = hipMemcpyAsync(h, summary, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(RCSCM_EDEVICE, std::string("status read-back failed: ") + hipGetErrorString(e));
  }
  const char* what[5] = {"non-finite input", "b is not a null vector of R'",
                         "R' + b b^H is not positive definite", "non-finite or non-positive state",
                         "lambda is not positive"};
  const rcscm_status code[5] = {RCSCM_ENONFINITE, RCSCM_ENOTNULL, RCSCM_ENOTPSD, RCSCM_ENONFINITE,
                                RCSCM_ENONFINITE};
  for (int k = 0; k < 5; ++k)
    if (h[0] & kErrBits[k])
      return fail(code[k], "row " + std::to_string(h[1 + k]) + " (frequency " +
                               std::to_string(h[1 + k]) + "): " + what[k]);
  return RCSCM_OK;
}
