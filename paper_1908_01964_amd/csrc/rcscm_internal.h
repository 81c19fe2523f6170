// Internal types shared by the host code and the HIP kernels of librcscm.
// Not part of the public ABI (include/rcscm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Device-side bounds checks of a debug build (-DRCSCM_DEBUG): a failed check
// prints where it failed and stops the kernel.  Compiled out otherwise.
#ifdef RCSCM_DEBUG
#define RCSCM_DASSERT(cond)                                                        \
  do {                                                                             \
    if (!(cond)) {                                                                 \
      printf("rcscm debug check failed: %s (%s:%d, block %d, thread %d)\n", #cond, \
             __FILE__, __LINE__, (int)blockIdx.x, (int)threadIdx.x);               \
      __builtin_trap();                                                            \
    }                                                                              \
  } while (0)
#else
#define RCSCM_DASSERT(cond) ((void)0)
#endif

namespace rcscm {

constexpr int MAXM = 8;

// One (utterance, frequency) row: J frames of one frequency bin.
struct RowInfo {
  long long x_off;    // complex64 offset of x[row][j=0][m=0] in the packed x
  long long bin_off;  // offset of frame 0 in every per-bin array
  long long a_off;    // complex128 offset of a[row][0] (and b[row][0])
  long long rp_off;   // complex128 offset of R'[row][0][0]
  int J, M, utt, freq;
  int part_off;       // first partial-sum slot of this row (STREAM / NAIVE)
  int nparts;         // number of chunks of this row
};

// Work unit of the chunked kernels: bins [start, start+len) of one row.
struct ChunkInfo {
  int row, start, len, part;  // part = partial-sum slot written by this chunk
};

// Float per-row constants read by the per-bin iteration.
struct RowConstF {
  float t_aa;      // tau^(aa) = a^H (R')^+ a
  float sab_re;    // sigma^(ab) = a^H b
  float sab_im;
  float sab2;      // |sigma^(ab)|^2
  float inv_t_aa;  // 1 / tau^(aa), or 0 when tau^(aa) == 0
  float invM;      // 1 / M
  float invJ;      // 1 / J
  float sab_abs;   // |sigma^(ab)|
};

// FP64 per-row setup results (precompute, objective, adjoint).
struct RowConstD {
  double2 Q[MAXM * MAXM];  // (R')^+, Hermitian, row-major
  double2 c[MAXM];         // (R')^+ a
  double2 b[MAXM];         // unit null vector of R'
  double2 a[MAXM];         // steering vector
  double2 Rp[MAXM * MAXM]; // projected, Hermitised R' (R' b = 0), row-major
  double2 s_ab;            // a^H b
  double t_aa;             // a^H (R')^+ a
  double det_a;            // det(R' + s b b^H); pdet(R') = det_a / s
  double shift;            // s: the power of two within a factor 2 of tr(R') / (M - 1)
};

// Float spatial model for the naive rule: a, b and the projected R'.
struct RowSpatialF {
  float2 a[MAXM];
  float2 b[MAXM];
  float2 Rp[MAXM * MAXM];  // row-major, Hermitian, R' b = 0
};

// Per-row status bits written by kernels.
enum : unsigned {
  ST_B_NOT_UNIT = 1u,       // warning: ||b|| differed from 1 by > 1e-6 (normalised)
  ST_NOT_NULL = 2u,         // ||R' b|| > 1e-6 ||R'||_F, or b == 0
  ST_NOT_PSD = 4u,          // R' + s b b^H has a non-positive pivot
  ST_NONFINITE_IN = 8u,     // non-finite x, a, R' or b
  ST_NONFINITE_STATE = 16u, // non-finite r^h / r^u produced
  ST_LAM_NONPOS = 32u,      // lambda <= 0 or non-finite
};

// Kernel launchers (defined in the .hip files).

// Per-row FP64 setup + per-bin precompute + initial state, one launch per
// microphone count M over the chunks of that M.  Writes status[row] (setup
// bits, by the row's first chunk) and chunk_status[chunk] (per-chunk bits).
struct InitArgs {
  const ChunkInfo* chunks;
  const RowInfo* rows;
  const float2* x;
  const double2* a;
  const double2* Rp;
  const double2* b;
  const float* rh0;  // may be null: rh_c
  const float* ru0;  // may be null: ru_c
  const float* lam0; // may be null: lam_c
  float rh_c, ru_c, lam_c;
  RowConstD* rcd;
  RowConstF* rcf;
  RowSpatialF* rsf;
  float4* tsig;
  float* nu;
  float* rh;
  float* ru;
  float* lam;
  unsigned* status;
  unsigned* chunk_status;
  long long n_bins;  // extent of the per-bin arrays (bounds checks of a debug build)
  int n_rows;        // extent of the per-row arrays
};
void launch_init(hipStream_t s, int M, int nchunks, const InitArgs& args);

// Fused single launch (rcscm_run): setup, precompute, K iterations and
// extraction of each row in one workgroup.  Classes (nt, bpl) from fused_class.
struct FusedArgs {
  const int* row_list;
  const RowInfo* rows;
  // Linear launch: block b serves row lin_row0 + b, whose J is lin_J and
  // whose offsets are the base offsets plus b times the per-row strides
  // (rows of one utterance); the row table is then not read.
  int lin, lin_row0, lin_J;
  long long lin_x0, lin_bin0, lin_a0, lin_rp0;
  const float2* x;
  const double2* a;
  const double2* Rp;
  const double2* b;
  const float* rh0;
  const float* ru0;
  const float* lam0;
  float rh_c, ru_c, lam_c;
  RowConstD* rcd;
  RowConstF* rcf;
  RowSpatialF* rsf;
  float4* tsig;
  float* nu;
  float* rh;
  float* ru;
  float* lam;
  unsigned* status;
  float* rh_out;
  float* ru_out;
  float* lam_out;
  float2* s_hat;
  // theta at the start of every iteration for the adjoint ([k][bin], [k][row];
  // null: not kept)
  float* ck_rh;
  float* ck_ru;
  float* ck_lam;
  long long ck_sb;
  int ck_sr;
  float inv_a2, beta_a2;
  int K;
  long long n_bins;  // extent of the per-bin arrays (bounds checks of a debug build)
  int n_rows;        // extent of the per-row arrays
  // Every row of the launch is resident at once: a row's waves lower their
  // issue priority as the row advances, so that rows sharing a CU progress
  // together (fused_fair).
  int fair;
};
bool fused_class(int J, int* nt, int* bpl);
bool fused_supported(int nt, int bpl);
void launch_fused(hipStream_t s, int M, int nt, int bpl, int nrows, const FusedArgs& A);
// Whether a launch of nrows rows of one (M, nt, bpl) class on the given device
// holds all its rows at once (the class's workgroups per CU times the CU count).
bool fused_fair(int M, int nt, int bpl, int nrows, int device);
// Compute units of a device (0 if the query fails), queried once per device.
int device_cu_count(int device);

// RESIDENT schedule: rows in row_list (all with J <= nt * bpl).
bool resident_supported(int nt, int bpl);
void launch_accel_resident(hipStream_t s, int nt, int bpl, int lamsum, int nrows,
                           const int* row_list, const RowInfo* rows, const RowConstF* rcf,
                           const float4* tsig, const float* nu, float* rh, float* ru, float* lam,
                           float alpha, float beta, int K, float* ckpt_rh, float* ckpt_ru,
                           float* ckpt_lam, long long ckpt_stride_bins, int ckpt_stride_rows,
                           unsigned* status, int fair);
// Whether a RESIDENT launch of nrows rows of one (nt, bpl) class holds all its
// rows at once on the device (as fused_fair); fair then lowers the waves'
// priority as a row advances.
bool resident_fair(int nt, int bpl, int lamsum, int nrows, int device);

// STREAM schedule: one launch of stage (finish iteration k-1, start iteration k).
// nu_early: request nu with the rest of a bin's state (for state that stays in
// the last-level cache between launches).
void launch_accel_stream(hipStream_t s, int lamsum, bool finish_prev, bool start_next,
                         bool nu_early, int nchunks, const ChunkInfo* chunks,
                         const RowInfo* rows, const RowConstF* rcf, const float4* tsig,
                         const float* nu, float* rh, float* ru, const float* lam_prev,
                         float* lam_new, const uint64_t* part_in, uint64_t* part_out,
                         float alpha, float beta, int chunk_threads, unsigned* status);

void launch_extract(hipStream_t s, int nchunks, const ChunkInfo* chunks, const RowInfo* rows,
                    const RowConstF* rcf, const float4* tsig, const float* rh_in,
                    const float* ru_in, const float* lam_in, float* rh_out, float* ru_out,
                    float* lam_out, float2* s_hat, unsigned* status);

void launch_objective(hipStream_t s, int nchunks, const ChunkInfo* chunks, const RowInfo* rows,
                      const RowConstF* rcf, const RowConstD* rcd, const float4* tsig,
                      const float* nu, const float* rh, const float* ru, const float* lam,
                      double alpha, double beta, double* partial);

// NAIVE rule, one iteration = phase A launch + phase B launch per M class;
// U^ stored packed between them (store_u), or recomputed by the second launch
// (launch_naive_b_recompute; uhat then holds r~h, nbins floats).
void launch_naive_a(hipStream_t s, int M, bool store_u, int nchunks, const ChunkInfo* chunks,
                    const RowInfo* rows, const RowSpatialF* rsf, const float2* x, float* rh,
                    const float* ru, const float* lam, float* uhat, long long nbins,
                    uint64_t* part, float alpha, float beta, unsigned* status);
void launch_naive_b(hipStream_t s, int M, int nchunks, const ChunkInfo* chunks,
                    const RowInfo* rows, const RowConstD* rcd, const uint64_t* part, float* lam,
                    float* ru, const float* uhat, long long nbins, unsigned* status);
void launch_naive_b_recompute(hipStream_t s, int M, int nchunks, const ChunkInfo* chunks,
                              const RowInfo* rows, const RowSpatialF* rsf, const RowConstD* rcd,
                              const uint64_t* part, const float* lam_old, float* lam_new,
                              const float2* x, const float* rh_old, float* ru,
                              unsigned* status);

// FIRST-STAGE rule (Algorithm 1): one workgroup of 256 lanes per row, x in
// registers; bpl = first_stage_bpl(J) in {1, 2, 4, 8, 16} (-1: row too long).
int first_stage_bpl(int J);
void launch_first_stage(hipStream_t s, int M, int bpl, int nrows, const int* row_list,
                        const RowInfo* rows, const RowConstF* rcf, const RowConstD* rcd,
                        const float2* x, float* rh, float* ru, float* lam, float alpha,
                        float beta, int K, unsigned* status);

// Back-projection (eq. (11)) and initialisation (eqs. (22), (23)); stage 3:
// all of it in one workgroup per row (M <= kBpFusedMaxM and rows of at most
// kBpFusedMaxJ frames); otherwise stage 0: powers p_m per chunk, stage 1: per
// row (a, R', b, lambda_0), stage 2: r^u_0. Above M = 5 the per-row step's
// registers leave room for only two 256-lane workgroups per CU, and the
// chunked launches measured faster (I = 513, J = 1000, M = 8).
constexpr int kBpFusedMaxJ = 8192;
constexpr int kBpFusedMaxM = 5;
void launch_backproject(hipStream_t s, int M, int nchunks_m, const ChunkInfo* chunks_m,
                        int nrows_m, const int* rows_m_list, const RowInfo* rows, const float2* x,
                        const double2* W, const int* target, double* part, double* p,
                        double2* a_out, double2* rp_out, double2* b_out, float* ru0,
                        float* lam0, unsigned* status, int stage);

// Adjoint of the RESIDENT/STREAM accelerated forward (checkpointed).
void launch_backward(hipStream_t s, int nt, int bpl, int nrows, const int* row_list,
                     const RowInfo* rows, const RowConstF* rcf, const RowConstD* rcd,
                     const float2* x, const float4* tsig, const float* nu, const float* ckpt_rh,
                     const float* ckpt_ru, const float* ckpt_lam, long long ckpt_stride_bins,
                     int ckpt_stride_rows, const float* rh_fin, const float* ru_fin,
                     const float* lam_fin, int K, float alpha, const float2* grad_s,
                     float2* grad_x, float* grad_rh0, float* grad_lam0, int fair);
// Whether a backward launch of nrows rows of one (nt, bpl) class holds all its
// rows at once on the device (as fused_fair).
bool backward_fair(int nt, int bpl, int nrows, int device);

}  // namespace rcscm
