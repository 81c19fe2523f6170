/*
 * rcscm.h - C ABI of the MI355X (gfx950) library for rank-constrained
 * spatial covariance matrix (SCM) estimation (Kubo, Takamune, Kitamura,
 * Saruwatari, APSIPA 2019).
 *
 * Model (Sec. II-B-1, eqs. (2)-(10)): per frequency i and frame j,
 *     x_ij ~ N_c(0, r^h_ij a_i a_i^H + r^u_ij (R'_i + lambda_i b_i b_i^H)),
 * with a_i (target steering vector), R'_i (rank-(M-1) Hermitian PSD SCM of the
 * diffuse noise) and b_i (unit null vector of R'_i) fixed.  The library
 * estimates theta = {r^h_ij, r^u_ij, lambda_i} by the MAP-EM iteration of
 * Sec. II-B-2 and extracts the target with the multichannel Wiener filter.
 *
 * Three update rules are provided (identical iterates in exact arithmetic):
 *   RCSCM_RULE_ACCEL - the second-stage accelerated rule (Algorithm 2,
 *                      eqs. (46)-(56)): scalar work per bin, one reduction
 *                      over frames per frequency for lambda_i.
 *   RCSCM_RULE_NAIVE - the literal E-step/M-step (eqs. (13)-(20)) with an
 *                      M x M factorisation of the model covariance per bin.
 *   RCSCM_RULE_FIRST - the first-stage accelerated rule (Algorithm 1,
 *                      eqs. (27)-(45)): the inverses of R~_i and R_i per
 *                      frequency (R~ of an iteration is R of the previous
 *                      one, so one M x M inversion per iteration) and O(M^2)
 *                      quadratic forms per bin per iteration; needs
 *                      J_u <= 4096.
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers owned by the caller, unless stated
 *     otherwise.  Complex arrays are interleaved (re, im).
 *   - Work is enqueued on the stream given at create (a hipStream_t passed as
 *     void*; NULL = the legacy default stream).  Only rcscm_sync,
 *     rcscm_objective and rcscm_destroy block the host.
 *   - Errors are returned as rcscm_status; nothing throws across the ABI.
 *     Argument errors are detected on the host before any device work.
 *     Data errors found by kernels (non-null b, non-PSD R', non-finite x or
 *     state) are recorded per row on the device and returned by the next
 *     rcscm_sync.  rcscm_last_error() describes the most recent failure.
 *   - A context is not thread-safe; distinct contexts are independent.
 *
 * Batched (ragged) layout, used by rcscm_create_batch: U utterances, each
 * with I frequencies, J_u frames and M_u microphones.  Per-utterance arrays
 * are concatenated in utterance order without padding:
 *   x      complex64  sum_u I*J_u*M_u     (utterance u: [I][J_u][M_u])
 *   a, b   complex128 sum_u I*M_u         ([I][M_u])
 *   Rp     complex128 sum_u I*M_u*M_u     ([I][M_u][M_u])
 *   rh, ru, s_hat     sum_u I*J_u         ([I][J_u])
 *   lam    float      U*I                 ([U][I])
 * A single utterance (rcscm_create) is the case U = 1.
 */
#ifndef RCSCM_H
#define RCSCM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RCSCM_MAX_M 8      /* microphones per utterance: 2 <= M <= 8 */
#define RCSCM_VERSION 1

typedef struct rcscm_ctx rcscm_ctx; /* opaque; created and freed by the library */

typedef enum {
  RCSCM_OK = 0,
  RCSCM_EINVAL = -1,     /* bad scalar argument or NULL pointer                 */
  RCSCM_ESHAPE = -2,     /* bad I, J, M, U or K                                 */
  RCSCM_ENOTNULL = -3,   /* ||R'b|| > 1e-6 ||R'||_F for some row (b is not null) */
  RCSCM_ENOTPSD = -4,    /* R' + b b^H not positive definite (rank of R' < M-1) */
  RCSCM_ENONFINITE = -5, /* non-finite x, state, or a non-positive lambda        */
  RCSCM_EDEVICE = -6,    /* a HIP runtime call failed                            */
  RCSCM_ENOMEM = -7,     /* device allocation failed                             */
  RCSCM_ESTATE = -8      /* call out of order (e.g. iterate before init)         */
} rcscm_status;

typedef enum { RCSCM_RULE_NAIVE = 0, RCSCM_RULE_ACCEL = 1, RCSCM_RULE_FIRST = 2 } rcscm_rule;

/* How the K-iteration loop of the accelerated rule is executed.
 *   STREAM:   one pass over HBM per iteration (K+1 launches, the lambda
 *             reduction of iteration k is finished by launch k+1); rows are
 *             split into fixed-size chunks.  Works for any J.
 *   RESIDENT: one workgroup owns a frequency row for all K iterations and
 *             keeps its per-bin data in registers (one launch per
 *             (workgroup size, bins-per-lane) class).  Needs J_u <= 8192
 *             (J_u <= 16 * block for an explicit block below 1024).
 *   AUTO:     RESIDENT when every row fits, else STREAM.                  */
typedef enum { RCSCM_SCHED_AUTO = 0, RCSCM_SCHED_STREAM = 1, RCSCM_SCHED_RESIDENT = 2 } rcscm_sched;

/* How the per-frequency sum over frames for lambda (eqs. (18), (43), (55)) is
 * accumulated by the accelerated rule.  F64: each lane adds its (at most 16)
 * terms in float; in the RESIDENT schedule and rcscm_run's fused launch the
 * 64 lanes of a wave are then added in float by a fixed six-level tree and
 * the waves combined in double (relative error at most (bins per lane + 5) u,
 * u = 2^-24, for these non-negative terms: below 1.3e-6); the STREAM schedule
 * combines lanes, waves and chunks in double.  Either way the order is fixed,
 * so results repeat bit for bit run to run.  KAHAN32: Kahan-compensated float
 * per lane, then a compensated (TwoSum) float tree (RESIDENT and STREAM only:
 * rcscm_run then makes the three calls).  The naive and first-stage rules sum
 * in double throughout. */
typedef enum { RCSCM_LAMSUM_F64 = 0, RCSCM_LAMSUM_KAHAN32 = 1 } rcscm_lamsum;

#define RCSCM_FLAG_GRAPH       1u  /* capture the STREAM K loop in a hipGraph      */
#define RCSCM_FLAG_CHECKPOINT  2u  /* keep theta_k per iteration for rcscm_backward */
#define RCSCM_FLAG_RUN_ONLY    4u  /* rcscm_run stores its results in the caller's
                                      arrays only and keeps no state (see rcscm_run);
                                      not with RCSCM_FLAG_CHECKPOINT                */
#define RCSCM_FLAG_NAIVE_RECOMPUTE 8u /* naive rule only: the second launch of an
                                      iteration recomputes U^ (eq. (16)) from x
                                      instead of reading it back packed; same
                                      results bit for bit, 4 B per bin of workspace
                                      instead of 4 M^2, but slower on MI355X
                                      (I=513 J=1000 K=20: 1.10x the time at M=2,
                                      1.23x at M=4, 1.62x at M=8), so the stored
                                      form is the default                          */

typedef struct {
  double alpha;    /* inverse-gamma shape; default 1.1 (Table 2); needs alpha+2 > 0 */
  double beta;     /* inverse-gamma scale; default 1e-16 (Table 2); needs beta >= 0 */
  float rh0;       /* initial r^h used when rcscm_init gets rh0 == NULL; default 1   */
  float ru0;       /* initial r^u used when ru0 == NULL; default 1                   */
  float lam0;      /* initial lambda used when lam0 == NULL; default 1               */
  int rule;        /* rcscm_rule; default RCSCM_RULE_ACCEL                           */
  int schedule;    /* rcscm_sched; default RCSCM_SCHED_AUTO                          */
  int lamsum;      /* rcscm_lamsum; default RCSCM_LAMSUM_F64                         */
  int block;       /* threads per workgroup of the RESIDENT kernel: 0 (per row: the
                      smallest of 64..1024 holding the row at <= 4 bins per lane),
                      64, 128, 256, 512 or 1024                                      */
  int chunk;       /* bins per workgroup of the STREAM, init, extract and naive
                      kernels: 0 (512), 256, 512, 1024 or 2048                       */
  unsigned flags;  /* RCSCM_FLAG_* */
} rcscm_params;

/* Fills *p with the defaults above. */
void rcscm_default_params(rcscm_params* p);

/* Single utterance: I frequencies, J frames, M microphones.  Allocates the
 * device workspace (see rcscm_workspace_bytes) on the current HIP device.
 * params may be NULL (defaults).  Errors: EINVAL (alpha+2 <= 0, beta < 0,
 * non-positive or non-finite inits, bad rule/schedule/block/chunk), ESHAPE
 * (I < 1, J < 1, M < 2 or M > RCSCM_MAX_M), ENOMEM, EDEVICE.  On error *out
 * is set to NULL and nothing is allocated. */
rcscm_status rcscm_create(rcscm_ctx** out, int I, int J, int M, const rcscm_params* params,
                          void* stream);

/* Ragged batch of U utterances sharing I; J[u], M[u] are HOST arrays of
 * length U.  Same errors as rcscm_create, per utterance. */
rcscm_status rcscm_create_batch(rcscm_ctx** out, int U, int I, const int* J, const int* M,
                                const rcscm_params* params, void* stream);

/* Per-frequency setup and per-bin precomputation (Algorithm 2, before the
 * loop; eqs. (32), (33), (46)-(48) and the pseudoinverse of eq. (26)):
 *   - b is normalised and R' projected onto the orthogonal complement of b,
 *     in FP64; (R')^+ = (R' + s b b^H)^{-1} - b b^H / s with s the power of
 *     two within a factor of two of tr(R')/(M-1),
 *     the inverse by an FP64 LDL^H factorisation (M <= 4) or Gauss-Jordan
 *     elimination (M >= 5), both without pivoting (the matrix is HPD);
 *   - per bin, in FP64 from the complex64 x, then stored as float:
 *     tau^(ax) = a^H (R')^+ x, sigma^(bx) = b^H x and
 *     nu = tau^(xx) - |tau^(ax)|^2 / tau^(aa) >= 0;
 *   - the initial state from rh0/ru0/lam0.
 * One launch per microphone count.
 * x: complex64 batch layout; a, Rp, b: complex128 batch layout.
 * rh0, ru0: float batch layout [..][I][J_u] or NULL (use params->rh0/ru0);
 * lam0: float [U][I] or NULL (params->lam0).  All are read during this call's
 * stream work only; the ACCEL rule keeps no reference to x afterwards.  The
 * NAIVE and FIRST rules re-read x in every iteration: x must stay valid and
 * unchanged until the context is destroyed.  Data errors (ENOTNULL, ENOTPSD, ENONFINITE)
 * surface at the next rcscm_sync. */
rcscm_status rcscm_init(rcscm_ctx* ctx, const void* x, const void* a, const void* Rp,
                        const void* b, const float* rh0, const float* ru0, const float* lam0);

/* Runs K >= 0 further EM iterations from the current state (eqs. (13)-(20)
 * for NAIVE; Algorithm 1 for FIRST; Algorithm 2 for ACCEL).  Within an iteration r^h and lambda use
 * the values at its start; r^u uses the new lambda.  iterate(K1) followed by
 * iterate(K2) gives the same state as iterate(K1+K2) for a fixed schedule.
 * Asynchronous.  Errors: ESTATE before init, ESHAPE for K < 0. */
rcscm_status rcscm_iterate(rcscm_ctx* ctx, int K);

/* Copies the current state into rh, ru (batch layout [..][I][J_u]) and lam
 * ([U][I]) and, if s_hat != NULL, writes the Wiener-filter estimate of the
 * dry target s_hat_ij = r^h a^H Sigma^{-1} x = gamma_ij rho^(ax)_ij with
 * gamma_ij = r^h_ij / (r^u_ij + r^h_ij rho^(aa)_i) at the current state
 * (complex64, batch layout).  Any output pointer may be NULL.  Async. */
rcscm_status rcscm_extract(rcscm_ctx* ctx, float* rh, float* ru, float* lam, void* s_hat);

/* init + iterate(K) + extract in one call (same arguments and outputs as
 * those three calls).  For the ACCEL rule with every J_u <= 8192 and the F64
 * lambda sum (with RCSCM_FLAG_CHECKPOINT: under the RESIDENT schedule, and
 * theta_k is kept for rcscm_backward as iterate keeps it), each row runs its
 * whole path - FP64 setup, FP64 precomputation, K iterations, extraction -
 * in one workgroup of one launch per (M, workgroup size) class, reading x
 * once and writing the
 * results once; otherwise the three calls are made in turn.  With several
 * classes the launches are spread over up to three library-owned
 * non-blocking streams that fork from and join back into the context's
 * stream, so completion is still ordered on that stream.  The call can be
 * captured into a HIP graph on the context's stream (it enqueues launches and
 * event records/waits only); with several classes make one uncaptured call
 * first, which creates the auxiliary streams.  Leaves the
 * context in the same state as the three calls (iterate/extract/objective
 * may follow), except with RCSCM_FLAG_RUN_ONLY: then the fused launch writes
 * only the outputs (r^h, r^u, lambda, s_hat: 16 bytes per bin and 4 per row,
 * plus the 8 M bytes per bin it reads), stores no per-bin state in the
 * workspace (28 bytes per bin less), and iterate, extract, get_state,
 * objective and backward return ESTATE until the next init (rcscm_sync still
 * reports the run's data errors).  Asynchronous. */
rcscm_status rcscm_run(rcscm_ctx* ctx, const void* x, const void* a, const void* Rp,
                       const void* b, const float* rh0, const float* ru0, const float* lam0,
                       int K, float* rh, float* ru, float* lam, void* s_hat);

/* Replaces the state (device arrays in batch layout; none may be NULL).
 * Async.  Used to resume from a saved state. */
rcscm_status rcscm_set_state(rcscm_ctx* ctx, const float* rh, const float* ru, const float* lam);

/* Copies the current state theta = {r^h, r^u, lambda} (Sec. II-B-2) into
 * caller-owned device arrays rh, ru (float, batch layout [..][I][J_u]) and lam
 * (float [U][I]); none may be NULL.  The copy is bitwise the state the next
 * rcscm_iterate starts from, so rcscm_set_state with these arrays on a context
 * initialised with the same inputs resumes exactly.  Async (device-to-device
 * copies on the context's stream).  Errors: EINVAL (NULL), ESTATE before init
 * or after a RCSCM_FLAG_RUN_ONLY run. */
rcscm_status rcscm_get_state(rcscm_ctx* ctx, float* rh, float* ru, float* lam);

/* Waits for the context's stream and returns the first data error recorded
 * by a kernel since init (see rcscm_status), or OK. */
rcscm_status rcscm_sync(rcscm_ctx* ctx);

/* Negative log-posterior of the current state (the objective the MAP-EM
 * iteration cannot increase; Sec. II-B), summed over all bins, evaluated in
 * FP64 on the device from the FP32 per-bin terms:
 *   sum_ij [ M log pi + M log r^u + log lambda + log pdet(R') +
 *            log(1 + r^h rho^(aa) / r^u) + (rho^(xx) - gamma |rho^(ax)|^2) / r^u
 *            + (alpha + 1) log r^h + beta / r^h ].
 * *nlp is a HOST pointer.  Blocks. */
rcscm_status rcscm_objective(rcscm_ctx* ctx, double* nlp);

/* Reverse-mode gradient of L = sum_ij |s_hat_ij - s_target_ij|^2 through the
 * last rcscm_iterate(K) call of a context created with RCSCM_FLAG_CHECKPOINT
 * (ACCEL rule), the extraction and the per-bin precomputation.
 * x: the complex64 input given to init (read again; must be unchanged).
 * grad_s_hat: complex64 dL/dRe(s_hat) + i dL/dIm(s_hat), batch layout.
 * Outputs (any may be NULL): grad_x complex64 [..][I][J_u][M_u] in the same
 * convention (dL/dRe x + i dL/dIm x); grad_rh0 float [..][I][J_u];
 * grad_lam0 float [U][I].  The gradient w.r.t. r^u_0 is not returned.
 * Errors: ESTATE if the context has no checkpoints or was not iterated. */
rcscm_status rcscm_backward(rcscm_ctx* ctx, const void* x, const void* grad_s_hat, void* grad_x,
                            float* grad_rh0, float* grad_lam0);

/* Builds the inputs of rcscm_init from a determined separation, as the paper
 * obtains them from ILRMA (Sec. II-B-1 eq. (11); Sec. II-B-3 eqs. (22), (23)):
 *   W       complex128 [..][I][M_u][M_u] demixing matrices, row m = w_m^H
 *           (separated signals y = W x); read only;
 *   target  HOST int[U]: index n_h of the target source per utterance;
 *   a       out complex128 [..][I][M_u]: a_i = column n_h of W^{-1};
 *   Rp      out complex128 [..][I][M_u][M_u]: R'_i = (1/J) sum_j W^{-1}
 *           diag(|w_m^H x|^2 with the n_h-th entry 0) W^{-H}   (eq. (11));
 *   b       out complex128 [..][I][M_u]: w_{n_h} / |w_{n_h}|, the unit null
 *           vector of R';
 *   ru0     out float [..][I][J_u] or NULL: (1/M) y^(u)H (R')^+ y^(u) with the
 *           back-projected noise image y^(u) of eq. (23)        (eq. (22));
 *   lam0    out float [U][I] or NULL: the minimum nonzero eigenvalue of R'.
 * x as in rcscm_init.  All arithmetic is FP64 on the device.  Asynchronous
 * (after a small host-to-device copy of the target indices).  Errors: EINVAL
 * (NULL pointers, target out of range); a singular W is reported as ENOTPSD
 * by the next rcscm_sync (rcscm_init and rcscm_run reset the per-row status
 * and check the a, R', b they receive by their own tests, so call
 * rcscm_sync in between to see this error).  The initialisation of r^h from
 * the NMF factors of
 * ILRMA (eq. (21)) is the caller's (pass it to rcscm_init as rh0). */
rcscm_status rcscm_backproject(rcscm_ctx* ctx, const void* x, const void* W, const int* target,
                               void* a, void* Rp, void* b, float* ru0, float* lam0);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): rcscm_run
 * for one utterance with no context and no device allocation.  Arguments as
 * rcscm_create + rcscm_run (x, a, Rp, b, rh0, ru0, lam0, K, rh, ru, lam,
 * s_hat; params may be NULL; stream is a hipStream_t or NULL); the same
 * kernel, so the outputs are bitwise those of rcscm_run on a context with
 * the same params.  Nothing is kept: there is no state to continue from.
 * Limits (ESHAPE / EINVAL otherwise): the ACCEL rule, RCSCM_LAMSUM_F64, no
 * RCSCM_FLAG_CHECKPOINT, 1 <= J <= 8192, 1 <= I <= RCSCM_NOALLOC_MAX_ROWS.
 * Scratch: one status word per row in a static device array of the library
 * (RCSCM_NOALLOC_MAX_ROWS + 8 words, 256 KiB, per GPU, held until the process
 * ends); calls that overlap on one GPU race on it.  The first call on a
 * device looks up the array's device address, and the first with a given
 * workgroup class queries the device's CU count and the class's occupancy
 * (host-side queries, cached for the process; no device work).  check == 0:
 * the call only enqueues work on the stream (capturable); data errors are not
 * reported.
 * check != 0: the call also reduces the status words, waits for the stream
 * and returns the first data error as rcscm_sync would (ENONFINITE,
 * ENOTNULL, ENOTPSD), described by rcscm_last_error(NULL). */
#define RCSCM_NOALLOC_MAX_ROWS 65536
rcscm_status rcscm_run_noalloc(int I, int J, int M, const rcscm_params* params, void* stream,
                               const void* x, const void* a, const void* Rp, const void* b,
                               const float* rh0, const float* ru0, const float* lam0, int K,
                               float* rh, float* ru, float* lam, void* s_hat, int check);

/* Frees every device buffer of the context (after waiting for its stream). */
void rcscm_destroy(rcscm_ctx* ctx);

/* Human-readable description of the last failure on ctx (never NULL; ctx may
 * be NULL for errors from create). */
const char* rcscm_last_error(const rcscm_ctx* ctx);

/* Bytes of device workspace rcscm_create / rcscm_create_batch allocate for
 * this shape and params (params may be NULL: defaults); 0 for arguments
 * create would reject.  Allocated later, on first use, and not counted:
 * checkpoints (RCSCM_FLAG_CHECKPOINT) at the first iterate(K) or run(K),
 * 8 K bytes per bin plus 4 K bytes per row, regrown for a larger K; the
 * back-projection's scratch at the first rcscm_backproject, 64 bytes per
 * chunk plus 68 bytes per row. */
size_t rcscm_workspace_bytes(int U, int I, const int* J, const int* M, const rcscm_params* params);

/* Schedule chosen for the RESIDENT / STREAM loop after create (for tests and
 * the autotuner): writes the schedule, block size and chunk size in use. */
rcscm_status rcscm_get_schedule(const rcscm_ctx* ctx, int* schedule, int* block, int* chunk);

/* Workgroup classes of rcscm_run's fused launch, for the autotuner.  Every row
 * runs in one workgroup of nt threads holding bpl frames per lane; the cost of
 * an iteration does not depend on M (Table 1), so a class is chosen per
 * (M, row length).  table: HOST array of n entries of 4 ints
 * (M, j_max, nt, bpl); a row with M_u microphones and J_u frames takes the
 * first entry with (M == M_u or M == 0), J_u <= j_max and J_u <= nt * bpl.
 * Rows no entry matches, and every row when n == 0, take the built-in class:
 * the smallest of 256 x 1/2/4/8, 512 x 8, 1024 x 8 that holds the row.
 * Supported (nt, bpl): (256, 1/2/4/8), (512, 2/4/8), (1024, 1/2/4/8).  Waits
 * for the context's streams, then uploads the new row lists (blocks; call
 * it outside graph capture).  Results do not depend on the class except
 * through the grouping of the lambda frame sum (rounding).  Errors: EINVAL
 * (bad entry; nothing is changed). */
rcscm_status rcscm_set_run_classes(rcscm_ctx* ctx, int n, const int* table);

/* The classes rcscm_run launches for this context: *n is their number, and the
 * first min(cap, *n) are written to the HOST array table as 5 ints each
 * (M, nt, bpl, rows, J of the class's first row).  *n == 0: rcscm_run makes
 * the three calls instead (rows longer than 8192 frames, or another rule). */
rcscm_status rcscm_get_run_classes(const rcscm_ctx* ctx, int cap, int* table, int* n);

/* Library version (RCSCM_VERSION). */
int rcscm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RCSCM_H */
