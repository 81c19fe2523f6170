// Host side of the C ABI (include/rcscm.h): argument validation, row and
// chunk tables, device workspace, schedules, hipGraph capture of the STREAM
// loop, status collection.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <array>
#include <map>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "host_internal.h"
#include "rcscm.h"
#include "rcscm_internal.h"

using namespace rcscm;

namespace {

thread_local std::string g_create_error;

constexpr int kResBpl[] = {1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 16};
constexpr int kMaxResidentJ = 512 * 16;
constexpr int kDefaultChunk = 512;  // bins per chunk when params.chunk == 0

int round_up_bpl(int need) {
  for (int b : kResBpl)
    if (b >= need) return b;
  return -1;
}

struct Buffers {
  std::vector<void*> ptrs;
  ~Buffers() {
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
  }
};

}  // namespace

struct rcscm_ctx {
  int U = 0, I = 0;
  std::vector<int> J, M;
  rcscm_params p{};
  hipStream_t stream = nullptr;
  int nrows = 0;
  long long nbins = 0;
  int chunk = kDefaultChunk;
  int nchunks = 0;
  int schedule = RCSCM_SCHED_RESIDENT;
  int res_nt = 256;
  std::vector<RowInfo> h_rows;
  std::vector<ChunkInfo> h_chunks;
  // chunk ranges per microphone count (chunks sorted by M in d_chunks_m)
  std::vector<std::pair<int, int>> m_range = std::vector<std::pair<int, int>>(RCSCM_MAX_M + 1, {0, 0});
  // rows grouped by microphone count (d_rows_m)
  std::vector<std::pair<int, int>> mrow_range = std::vector<std::pair<int, int>>(RCSCM_MAX_M + 1, {0, 0});
  struct ResClass {
    int nt, bpl, count, offset;
    // the class is the only one and all its rows are resident at once: the RESIDENT and the
    // backward launch lower their waves' priority as a row advances (set_fair_flags)
    bool fair_res = false, fair_bw = false;
  };
  std::vector<ResClass> res_classes;
  std::vector<ResClass> first_classes;  // FIRST rule: nt field holds M
  struct FusedClass {
    int M, nt, bpl, count, offset;
    bool linear;  // consecutive rows of one utterance (offsets linear in the row index)
    int row0;     // first row of the class
    bool fair = false;  // as ResClass, for the fused launch
  };
  std::vector<FusedClass> fused_classes;  // rcscm_run (empty: not available)
  int fused_offset = 0;                     // the fused classes' part of d_row_list
  std::vector<std::array<int, 4>> run_table;  // (M, j_max, nt, bpl) from rcscm_set_run_classes

  Buffers mem;
  RowInfo* d_rows = nullptr;
  ChunkInfo* d_chunks = nullptr;
  ChunkInfo* d_chunks_m = nullptr;
  int* d_row_list = nullptr;
  RowConstD* d_rcd = nullptr;
  RowConstF* d_rcf = nullptr;
  RowSpatialF* d_rsf = nullptr;
  float4* d_tsig = nullptr;
  float* d_nu = nullptr;
  float* d_rh = nullptr;
  float* d_ru = nullptr;
  float* d_lam[2] = {nullptr, nullptr};
  int lam_cur = 0;
  uint64_t* d_part[2] = {nullptr, nullptr};
  unsigned* d_status = nullptr;
  double* d_objpart = nullptr;
  float* d_uhat = nullptr;
  unsigned* d_chunk_status = nullptr;
  int* d_rows_m = nullptr;
  // back-projection scratch (allocated on first use)
  double* d_bp_part = nullptr;
  double* d_bp_p = nullptr;
  int* d_bp_target = nullptr;
  std::vector<int> h_bp_target;  // the target indices d_bp_target holds (per row)
  const float2* x_borrowed = nullptr;
  // checkpoints of the last iterate() call
  float* d_ck_rh = nullptr;
  float* d_ck_ru = nullptr;
  float* d_ck_lam = nullptr;
  int ck_capacity = 0;
  int ck_K = -1;
  bool inited = false;
  bool dropped = false;  // the last rcscm_run kept no state (RCSCM_FLAG_RUN_ONLY)
  bool chunk_status_valid = false;  // chunk_status written by the last rcscm_init
  std::string err;
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;
  std::vector<hipGraph_t> graph_defs;
  // rcscm_run with several workgroup classes: the class launches are forked
  // over auxiliary streams (non-blocking, default priority) and joined back.
  int device = 0;
  std::vector<hipStream_t> aux;
  std::vector<hipEvent_t> ev_join;
  hipEvent_t ev_fork = nullptr;

  rcscm_status fail(rcscm_status s, const std::string& m) {
    err = m;
    return s;
  }
  // ESTATE for a call that needs the state: none yet, or dropped by a run-only rcscm_run.
  rcscm_status no_state(const char* what) {
    return fail(RCSCM_ESTATE, std::string(what) +
                                  (dropped ? " after a RCSCM_FLAG_RUN_ONLY run (no state kept)"
                                           : " before init"));
  }
  template <class T>
  rcscm_status alloc(T** out, size_t count, const char* what) {
    *out = nullptr;
    if (count == 0) count = 1;
    void* ptr = nullptr;
    hipError_t e = hipMalloc(&ptr, count * sizeof(T));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(e == hipErrorOutOfMemory ? RCSCM_ENOMEM : RCSCM_EDEVICE,
                  std::string("hipMalloc failed for ") + what + ": " + hipGetErrorString(e));
    }
    mem.ptrs.push_back(ptr);
    *out = static_cast<T*>(ptr);
    return RCSCM_OK;
  }
  // Frees a buffer from alloc (the caller makes sure no queued work uses it).
  template <class T>
  void release(T** p) {
    if (!*p) return;
    for (auto& q : mem.ptrs)
      if (q == static_cast<void*>(*p)) {
        (void)hipFree(q);
        q = nullptr;
      }
    *p = nullptr;
  }
};

#define RCSCM_HIP(ctx, call)                                                            \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) {                                                             \
      (void)hipGetLastError();                                                          \
      return (ctx)->fail(RCSCM_EDEVICE, std::string(#call " failed: ") + hipGetErrorString(e_)); \
    }                                                                                   \
  } while (0)

#define RCSCM_TRY(expr)            \
  do {                             \
    rcscm_status s_ = (expr);      \
    if (s_ != RCSCM_OK) return s_; \
  } while (0)

extern "C" {

void rcscm_default_params(rcscm_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->alpha = 1.1;
  p->beta = 1e-16;
  p->rh0 = 1.0f;
  p->ru0 = 1.0f;
  p->lam0 = 1.0f;
  p->rule = RCSCM_RULE_ACCEL;
  p->schedule = RCSCM_SCHED_AUTO;
  p->lamsum = RCSCM_LAMSUM_F64;
  p->block = 0;
  p->chunk = 0;
  p->flags = 0u;
}

int rcscm_version(void) { return RCSCM_VERSION; }

static rcscm_status validate(int U, int I, const int* J, const int* M, const rcscm_params* p,
                             std::string* msg);

}  // extern "C"

namespace rcscm {
rcscm_status validate_args(int U, int I, const int* J, const int* M, const rcscm_params* p,
                           std::string* msg) {
  return validate(U, I, J, M, p, msg);
}
void set_global_error(const std::string& msg) { g_create_error = msg; }
}  // namespace rcscm

extern "C" {

static rcscm_status validate(int U, int I, const int* J, const int* M, const rcscm_params* p,
                             std::string* msg) {
  if (U < 1) {
    *msg = "U must be >= 1";
    return RCSCM_ESHAPE;
  }
  if (I < 1) {
    *msg = "I must be >= 1";
    return RCSCM_ESHAPE;
  }
  if (!J || !M) {
    *msg = "J and M arrays must not be NULL";
    return RCSCM_EINVAL;
  }
  long long bins = 0;
  for (int u = 0; u < U; ++u) {
    if (J[u] < 1) {
      *msg = "J must be >= 1 (utterance " + std::to_string(u) + ")";
      return RCSCM_ESHAPE;
    }
    if (M[u] < 2 || M[u] > RCSCM_MAX_M) {
      *msg = "M must be in [2, 8] (utterance " + std::to_string(u) + ")";
      return RCSCM_ESHAPE;
    }
    bins += (long long)I * J[u];
  }
  if (bins > (1LL << 40)) {
    *msg = "too many bins";
    return RCSCM_ESHAPE;
  }
  if ((long long)U * I > (1LL << 30)) {
    *msg = "too many rows";
    return RCSCM_ESHAPE;
  }
  if (!(std::isfinite(p->alpha) && p->alpha + 2.0 > 0.0)) {
    *msg = "alpha must be finite with alpha + 2 > 0";
    return RCSCM_EINVAL;
  }
  if (!(std::isfinite(p->beta) && p->beta >= 0.0)) {
    *msg = "beta must be finite and >= 0";
    return RCSCM_EINVAL;
  }
  if (!(std::isfinite(p->rh0) && p->rh0 > 0.0f && std::isfinite(p->ru0) && p->ru0 > 0.0f &&
        std::isfinite(p->lam0) && p->lam0 > 0.0f)) {
    *msg = "scalar initial values must be finite and > 0";
    return RCSCM_EINVAL;
  }
  if (p->rule != RCSCM_RULE_NAIVE && p->rule != RCSCM_RULE_ACCEL && p->rule != RCSCM_RULE_FIRST) {
    *msg = "unknown rule";
    return RCSCM_EINVAL;
  }
  if (p->schedule < RCSCM_SCHED_AUTO || p->schedule > RCSCM_SCHED_RESIDENT) {
    *msg = "unknown schedule";
    return RCSCM_EINVAL;
  }
  if (p->lamsum != RCSCM_LAMSUM_F64 && p->lamsum != RCSCM_LAMSUM_KAHAN32) {
    *msg = "unknown lamsum";
    return RCSCM_EINVAL;
  }
  if (!(p->block == 0 || p->block == 64 || p->block == 128 || p->block == 256 ||
        p->block == 512 || p->block == 1024)) {
    *msg = "block must be 0, 64, 128, 256, 512 or 1024";
    return RCSCM_EINVAL;
  }
  if (!(p->chunk == 0 || p->chunk == 256 || p->chunk == 512 || p->chunk == 1024 ||
        p->chunk == 2048)) {
    *msg = "chunk must be 0, 256, 512, 1024 or 2048";
    return RCSCM_EINVAL;
  }
  if (p->flags & ~(RCSCM_FLAG_GRAPH | RCSCM_FLAG_CHECKPOINT | RCSCM_FLAG_RUN_ONLY |
                   RCSCM_FLAG_NAIVE_RECOMPUTE)) {
    *msg = "unknown flag bits";
    return RCSCM_EINVAL;
  }
  if ((p->flags & RCSCM_FLAG_NAIVE_RECOMPUTE) && p->rule != RCSCM_RULE_NAIVE) {
    *msg = "RCSCM_FLAG_NAIVE_RECOMPUTE applies to the naive rule only";
    return RCSCM_EINVAL;
  }
  if ((p->flags & RCSCM_FLAG_CHECKPOINT) && (p->flags & RCSCM_FLAG_RUN_ONLY)) {
    *msg = "RCSCM_FLAG_RUN_ONLY keeps no state, so it excludes RCSCM_FLAG_CHECKPOINT";
    return RCSCM_EINVAL;
  }
  int maxJ = 0;
  for (int u = 0; u < U; ++u) maxJ = J[u] > maxJ ? J[u] : maxJ;
  if ((p->schedule == RCSCM_SCHED_RESIDENT || (p->flags & RCSCM_FLAG_CHECKPOINT)) &&
      p->rule == RCSCM_RULE_ACCEL) {
    const int nt = p->block ? p->block : 1024;
    const int cap = nt == 1024 ? 8 * 1024 : nt * 16;
    if (maxJ > cap) {
      *msg = "RESIDENT schedule (or checkpoints) needs J <= 16 * block (8192 for block 1024)";
      return RCSCM_ESHAPE;
    }
  }
  if (p->rule == RCSCM_RULE_FIRST && maxJ > 16 * 256) {
    *msg = "the FIRST rule needs J <= 4096";
    return RCSCM_ESHAPE;
  }
  if ((p->flags & RCSCM_FLAG_CHECKPOINT) && p->rule != RCSCM_RULE_ACCEL) {
    *msg = "checkpoints (backward) need the ACCEL rule";
    return RCSCM_EINVAL;
  }
  return RCSCM_OK;
}

// Workgroup size of a row in the RESIDENT schedule when params.block == 0:
// the smallest workgroup that holds the row with at most 4 bins per lane
// (1024 lanes for longer rows).  Per-row sizes keep short rows of a ragged
// batch from idling most lanes of a wide workgroup.
static int auto_block(int J) {
  for (int nt : {64, 128, 256, 512, 1024})
    if (nt * 4 >= J) return nt;
  return 1024;
}

// The fused launch's class of a row: the first entry of the caller's table
// (rcscm_set_run_classes) that matches, else the built-in choice.
static bool pick_fused_class(const rcscm_ctx* c, int M, int J, int* nt, int* bpl) {
  for (const auto& e : c->run_table)
    if ((e[0] == 0 || e[0] == M) && J <= e[1] && J <= e[2] * e[3]) {
      *nt = e[2];
      *bpl = e[3];
      return true;
    }
  return fused_class(J, nt, bpl);
}

// Groups the rows into the fused launch's classes (M, nt, bpl), appending the
// rows of each class to *row_list; leaves *out empty when a row fits no class.
static void group_fused(rcscm_ctx* c, std::vector<int>* row_list,
                        std::vector<rcscm_ctx::FusedClass>* out) {
  out->clear();
  std::map<std::tuple<int, int, int>, std::vector<int>> cls;  // (M, nt, bpl)
  for (int r = 0; r < c->nrows; ++r) {
    int nt = 0, bpl = 0;
    if (!pick_fused_class(c, c->h_rows[r].M, c->h_rows[r].J, &nt, &bpl)) return;
    cls[std::make_tuple(c->h_rows[r].M, nt, bpl)].push_back(r);
  }
  for (auto& kv : cls) {
    const std::vector<int>& rl = kv.second;
    bool linear = true;
    const RowInfo& r0 = c->h_rows[rl[0]];
    for (size_t k = 1; k < rl.size() && linear; ++k) {
      const RowInfo& rk = c->h_rows[rl[k]];
      const long long kk = (long long)k;
      linear = rl[k] == rl[0] + (int)k && rk.utt == r0.utt && rk.J == r0.J && rk.M == r0.M &&
               rk.x_off == r0.x_off + kk * r0.J * r0.M && rk.bin_off == r0.bin_off + kk * r0.J &&
               rk.a_off == r0.a_off + kk * r0.M && rk.rp_off == r0.rp_off + kk * r0.M * r0.M;
    }
    out->push_back(rcscm_ctx::FusedClass{std::get<0>(kv.first), std::get<1>(kv.first),
                                         std::get<2>(kv.first), (int)rl.size(),
                                         (int)row_list->size(), linear, rl[0]});
    row_list->insert(row_list->end(), rl.begin(), rl.end());
  }
}

// The priority-step flags of the classes (fused_fair, resident_fair, backward_fair): a class
// qualifies when it is the only one of its launch kind.  The occupancy queries behind them run
// here, when the classes are formed, so that no launch (possibly under graph capture) makes them.
static void set_fair_flags(rcscm_ctx* c) {
  for (auto& cl : c->res_classes) {
    cl.fair_res = c->res_classes.size() == 1 &&
                  resident_fair(cl.nt, cl.bpl, c->p.lamsum, cl.count, c->device);
    cl.fair_bw = c->res_classes.size() == 1 && backward_fair(cl.nt, cl.bpl, cl.count, c->device);
  }
  for (auto& cl : c->fused_classes)
    cl.fair = c->fused_classes.size() == 1 &&
              fused_fair(cl.M, cl.nt, cl.bpl, cl.count, c->device);
}

static rcscm_status build_tables(rcscm_ctx* c) {
  const int U = c->U, I = c->I;
  c->nrows = U * I;
  long long xoff = 0, boff = 0, aoff = 0, rpoff = 0;
  c->h_rows.resize(c->nrows);
  int maxJ = 0;
  for (int u = 0; u < U; ++u) {
    const int J = c->J[u], M = c->M[u];
    maxJ = J > maxJ ? J : maxJ;
    for (int i = 0; i < I; ++i) {
      RowInfo& r = c->h_rows[(size_t)u * I + i];
      r.x_off = xoff + (long long)i * J * M;
      r.bin_off = boff + (long long)i * J;
      r.a_off = aoff + (long long)i * M;
      r.rp_off = rpoff + (long long)i * M * M;
      r.J = J;
      r.M = M;
      r.utt = u;
      r.freq = i;
    }
    xoff += (long long)I * J * M;
    boff += (long long)I * J;
    aoff += (long long)I * M;
    rpoff += (long long)I * M * M;
  }
  c->nbins = boff;
  // chunks (row order); the partial slot of a chunk is its index
  c->chunk = c->p.chunk ? c->p.chunk : kDefaultChunk;
  c->h_chunks.clear();
  for (int r = 0; r < c->nrows; ++r) {
    RowInfo& ri = c->h_rows[r];
    ri.part_off = (int)c->h_chunks.size();
    for (int s = 0; s < ri.J; s += c->chunk) {
      ChunkInfo ck;
      ck.row = r;
      ck.start = s;
      ck.len = (ri.J - s) < c->chunk ? (ri.J - s) : c->chunk;
      ck.part = (int)c->h_chunks.size();
      c->h_chunks.push_back(ck);
    }
    ri.nparts = (int)c->h_chunks.size() - ri.part_off;
  }
  c->nchunks = (int)c->h_chunks.size();
  // the same chunks grouped by microphone count
  std::vector<ChunkInfo> by_m;
  by_m.reserve(c->h_chunks.size());
  for (int m = 2; m <= RCSCM_MAX_M; ++m) {
    const int start = (int)by_m.size();
    for (const ChunkInfo& ck : c->h_chunks)
      if (c->h_rows[ck.row].M == m) by_m.push_back(ck);
    c->m_range[m] = {start, (int)by_m.size() - start};
  }
  // schedule
  if (c->p.rule == RCSCM_RULE_ACCEL) {
    const bool fits = maxJ <= kMaxResidentJ;
    if (c->p.flags & RCSCM_FLAG_CHECKPOINT)
      c->schedule = RCSCM_SCHED_RESIDENT;
    else if (c->p.schedule == RCSCM_SCHED_AUTO)
      c->schedule = fits ? RCSCM_SCHED_RESIDENT : RCSCM_SCHED_STREAM;
    else
      c->schedule = c->p.schedule;
  } else {
    c->schedule = RCSCM_SCHED_STREAM;
  }
  std::vector<int> row_list;
  c->res_classes.clear();
  c->res_nt = c->p.block;
  if (c->p.rule == RCSCM_RULE_ACCEL && c->schedule == RCSCM_SCHED_RESIDENT) {
    // classes of rows sharing (workgroup size, bins per lane): one launch each
    std::map<std::pair<int, int>, std::vector<int>> cls;
    for (int r = 0; r < c->nrows; ++r) {
      const int J = c->h_rows[r].J;
      const int nt = c->p.block ? c->p.block : auto_block(J);
      int bpl = round_up_bpl((J + nt - 1) / nt);
      while (bpl > 0 && !resident_supported(nt, bpl)) bpl = round_up_bpl(bpl + 1);
      if (bpl < 0) return c->fail(RCSCM_ESHAPE, "row too long for the RESIDENT schedule");
      cls[{nt, bpl}].push_back(r);
    }
    long long best_bins = -1;
    for (auto it = cls.rbegin(); it != cls.rend(); ++it) {  // widest rows first
      rcscm_ctx::ResClass rc{it->first.first, it->first.second, (int)it->second.size(),
                             (int)row_list.size()};
      row_list.insert(row_list.end(), it->second.begin(), it->second.end());
      c->res_classes.push_back(rc);
      long long bins = 0;
      for (int r : it->second) bins += c->h_rows[r].J;
      if (bins > best_bins) {
        best_bins = bins;
        c->res_nt = rc.nt;  // reported by rcscm_get_schedule: the class with most bins
      }
    }
  }
  if (c->p.rule == RCSCM_RULE_FIRST) {
    std::map<std::pair<int, int>, std::vector<int>> cls;  // (M, bins per lane)
    for (int r = 0; r < c->nrows; ++r) {
      const int bpl = first_stage_bpl(c->h_rows[r].J);
      if (bpl < 0) return c->fail(RCSCM_ESHAPE, "row too long for the FIRST rule");
      cls[{c->h_rows[r].M, bpl}].push_back(r);
    }
    for (auto& kv : cls) {
      c->first_classes.push_back(rcscm_ctx::ResClass{kv.first.first, kv.first.second,
                                                     (int)kv.second.size(), (int)row_list.size()});
      row_list.insert(row_list.end(), kv.second.begin(), kv.second.end());
    }
  }
  c->fused_offset = (int)row_list.size();
  if (c->p.rule == RCSCM_RULE_ACCEL && maxJ <= kMaxResidentJ)
    group_fused(c, &row_list, &c->fused_classes);
  set_fair_flags(c);
  if (row_list.empty()) row_list.push_back(0);
  // device copies
  RCSCM_TRY(c->alloc(&c->d_rows, c->nrows, "rows"));
  RCSCM_TRY(c->alloc(&c->d_chunks, c->nchunks, "chunks"));
  RCSCM_TRY(c->alloc(&c->d_chunks_m, c->nchunks, "chunks by M"));
  RCSCM_TRY(c->alloc(&c->d_row_list, row_list.size(), "row list"));
  std::vector<int> rows_m;
  for (int m = 2; m <= RCSCM_MAX_M; ++m) {
    const int start = (int)rows_m.size();
    for (int r = 0; r < c->nrows; ++r)
      if (c->h_rows[r].M == m) rows_m.push_back(r);
    c->mrow_range[m] = {start, (int)rows_m.size() - start};
  }
  RCSCM_TRY(c->alloc(&c->d_rows_m, rows_m.size(), "rows by M"));
  RCSCM_HIP(c, hipMemcpy(c->d_rows_m, rows_m.data(), sizeof(int) * rows_m.size(),
                         hipMemcpyHostToDevice));
  RCSCM_HIP(c, hipMemcpy(c->d_rows, c->h_rows.data(), sizeof(RowInfo) * c->nrows,
                         hipMemcpyHostToDevice));
  RCSCM_HIP(c, hipMemcpy(c->d_chunks, c->h_chunks.data(), sizeof(ChunkInfo) * c->nchunks,
                         hipMemcpyHostToDevice));
  RCSCM_HIP(c, hipMemcpy(c->d_chunks_m, by_m.data(), sizeof(ChunkInfo) * by_m.size(),
                         hipMemcpyHostToDevice));
  RCSCM_HIP(c, hipMemcpy(c->d_row_list, row_list.data(), sizeof(int) * row_list.size(),
                         hipMemcpyHostToDevice));
  return RCSCM_OK;
}

static rcscm_status alloc_workspace(rcscm_ctx* c) {
  RCSCM_TRY(c->alloc(&c->d_rcd, c->nrows, "row constants (fp64)"));
  RCSCM_TRY(c->alloc(&c->d_rcf, c->nrows, "row constants"));
  RCSCM_TRY(c->alloc(&c->d_rsf, c->nrows, "row spatial model"));
  RCSCM_TRY(c->alloc(&c->d_tsig, c->nbins, "tau/sigma"));
  RCSCM_TRY(c->alloc(&c->d_nu, c->nbins, "nu"));
  RCSCM_TRY(c->alloc(&c->d_rh, c->nbins, "r^h"));
  RCSCM_TRY(c->alloc(&c->d_ru, c->nbins, "r^u"));
  RCSCM_TRY(c->alloc(&c->d_lam[0], c->nrows, "lambda"));
  RCSCM_TRY(c->alloc(&c->d_lam[1], c->nrows, "lambda"));
  RCSCM_TRY(c->alloc(&c->d_part[0], c->nchunks, "partial sums"));
  RCSCM_TRY(c->alloc(&c->d_part[1], c->nchunks, "partial sums"));
  RCSCM_TRY(c->alloc(&c->d_status, c->nrows, "status"));
  RCSCM_TRY(c->alloc(&c->d_chunk_status, c->nchunks, "chunk status"));
  RCSCM_HIP(c, hipMemset(c->d_status, 0, sizeof(unsigned) * c->nrows));
  RCSCM_HIP(c, hipMemset(c->d_chunk_status, 0, sizeof(unsigned) * c->nchunks));
  RCSCM_TRY(c->alloc(&c->d_objpart, c->nchunks, "objective partials"));
  if (c->p.rule == RCSCM_RULE_NAIVE) {
    long long maxMM = 0;
    for (int u = 0; u < c->U; ++u) maxMM = c->M[u] * c->M[u] > maxMM ? c->M[u] * c->M[u] : maxMM;
    if (c->p.flags & RCSCM_FLAG_NAIVE_RECOMPUTE) maxMM = 1;  // r~h only
    RCSCM_TRY(c->alloc(&c->d_uhat, (size_t)(maxMM * c->nbins), "packed U^"));
  }
  return RCSCM_OK;
}

size_t rcscm_workspace_bytes(int U, int I, const int* J, const int* M,
                             const rcscm_params* params) {
  rcscm_params p;
  if (params)
    p = *params;
  else
    rcscm_default_params(&p);
  std::string msg;
  if (validate(U, I, J, M, &p, &msg) != RCSCM_OK) return 0;
  // mirrors build_tables and alloc_workspace (every buffer holds at least one element)
  auto n1 = [](long long n) { return n > 0 ? n : 1LL; };
  long long bins = 0, chunks = 0, maxMM = 0;
  int maxJ = 0;
  const long long chunk = p.chunk ? p.chunk : kDefaultChunk;
  for (int u = 0; u < U; ++u) {
    bins += (long long)I * J[u];
    chunks += (long long)I * ((J[u] + chunk - 1) / chunk);
    maxMM = M[u] * M[u] > maxMM ? M[u] * M[u] : maxMM;
    maxJ = J[u] > maxJ ? J[u] : maxJ;
  }
  const long long rows = (long long)U * I;
  // the row list: RESIDENT classes, then the fused classes (ACCEL); FIRST classes
  long long row_list = 0;
  if (p.rule == RCSCM_RULE_ACCEL) {
    const bool fits = maxJ <= kMaxResidentJ;
    const bool resident = (p.flags & RCSCM_FLAG_CHECKPOINT) ||
                          (p.schedule == RCSCM_SCHED_AUTO ? fits
                                                          : p.schedule == RCSCM_SCHED_RESIDENT);
    row_list = (resident ? rows : 0) + (fits ? rows : 0);
  } else if (p.rule == RCSCM_RULE_FIRST) {
    row_list = rows;
  }
  size_t b = 0;
  // build_tables: rows, chunks, chunks by M, row list, rows by M
  b += n1(rows) * sizeof(RowInfo) + 2 * n1(chunks) * sizeof(ChunkInfo) + n1(row_list) * sizeof(int) +
       n1(rows) * sizeof(int);
  // alloc_workspace: row constants, per-bin state, lambda x 2, partial sums x 2, status words,
  // objective partials, packed U^ (NAIVE)
  b += n1(rows) * (sizeof(RowConstD) + sizeof(RowConstF) + sizeof(RowSpatialF));
  b += n1(bins) * (sizeof(float4) + 3 * sizeof(float));
  b += 2 * n1(rows) * sizeof(float) + 2 * n1(chunks) * sizeof(uint64_t);
  b += n1(rows) * sizeof(unsigned) + n1(chunks) * sizeof(unsigned) + n1(chunks) * sizeof(double);
  if (p.rule == RCSCM_RULE_NAIVE)
    b += n1((p.flags & RCSCM_FLAG_NAIVE_RECOMPUTE ? 1 : maxMM) * bins) * sizeof(float);
  return b;
}

static rcscm_status create_impl(rcscm_ctx** out, int U, int I, const int* J, const int* M,
                                const rcscm_params* params, void* stream) {
  if (!out) {
    g_create_error = "out must not be NULL";
    return RCSCM_EINVAL;
  }
  *out = nullptr;
  rcscm_params p;
  if (params)
    p = *params;
  else
    rcscm_default_params(&p);
  std::string msg;
  rcscm_status s = validate(U, I, J, M, &p, &msg);
  if (s != RCSCM_OK) {
    g_create_error = msg;
    return s;
  }
  rcscm_ctx* c = new rcscm_ctx();
  c->U = U;
  c->I = I;
  c->J.assign(J, J + U);
  c->M.assign(M, M + U);
  c->p = p;
  c->stream = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetDevice(&c->device);
  s = build_tables(c);
  if (s == RCSCM_OK) s = alloc_workspace(c);
  if (s != RCSCM_OK) {
    g_create_error = c->err;
    delete c;
    return s;
  }
  *out = c;
  return RCSCM_OK;
}

rcscm_status rcscm_create(rcscm_ctx** out, int I, int J, int M, const rcscm_params* params,
                          void* stream) {
  return create_impl(out, 1, I, &J, &M, params, stream);
}

rcscm_status rcscm_create_batch(rcscm_ctx** out, int U, int I, const int* J, const int* M,
                                const rcscm_params* params, void* stream) {
  return create_impl(out, U, I, J, M, params, stream);
}

rcscm_status rcscm_init(rcscm_ctx* c, const void* x, const void* a, const void* Rp, const void* b,
                        const float* rh0, const float* ru0, const float* lam0) {
  if (!c) return RCSCM_EINVAL;
  if (!x || !a || !Rp || !b) return c->fail(RCSCM_EINVAL, "x, a, Rp and b must not be NULL");
  hipStream_t s = c->stream;
  c->lam_cur = 0;
  InitArgs A;
  A.rows = c->d_rows;
  A.x = static_cast<const float2*>(x);
  A.a = static_cast<const double2*>(a);
  A.Rp = static_cast<const double2*>(Rp);
  A.b = static_cast<const double2*>(b);
  A.rh0 = rh0;
  A.ru0 = ru0;
  A.lam0 = lam0;
  A.rh_c = c->p.rh0;
  A.ru_c = c->p.ru0;
  A.lam_c = c->p.lam0;
  A.rcd = c->d_rcd;
  A.rcf = c->d_rcf;
  A.rsf = c->d_rsf;
  A.tsig = c->d_tsig;
  A.nu = c->d_nu;
  A.rh = c->d_rh;
  A.ru = c->d_ru;
  A.lam = c->d_lam[c->lam_cur];
  A.status = c->d_status;
  A.chunk_status = c->d_chunk_status;
  A.n_bins = c->nbins;
  A.n_rows = c->nrows;
  for (int m = 2; m <= RCSCM_MAX_M; ++m) {
    const auto rg = c->m_range[m];
    if (rg.second == 0) continue;
    A.chunks = c->d_chunks_m + rg.first;
    launch_init(s, m, rg.second, A);
    RCSCM_HIP(c, hipGetLastError());
  }
  c->x_borrowed = static_cast<const float2*>(x);
  c->inited = true;
  c->dropped = false;
  c->chunk_status_valid = true;
  c->ck_K = -1;
  return RCSCM_OK;
}

// The MI355X last-level cache (AMD Infinity Cache): 256 MB.
constexpr double kLastLevelCacheBytes = 256.0 * 1024.0 * 1024.0;

static rcscm_status enqueue_stream_loop(rcscm_ctx* c, int K) {
  hipStream_t s = c->stream;
  const float alpha = (float)c->p.alpha, beta = (float)c->p.beta;
  // Every launch re-reads the whole per-bin state (tau^ax, sigma^bx, nu, r^h,
  // r^u: 28 B per bin); whether it stays in the last-level cache between
  // launches decides how the launch requests it.
  const bool nu_early = 28.0 * (double)c->nbins <= kLastLevelCacheBytes;
  int cur = c->lam_cur;
  for (int k = 1; k <= K + 1; ++k) {
    const bool finish = k >= 2;
    const bool start = k <= K;
    const float* lam_prev = c->d_lam[cur];
    float* lam_new = c->d_lam[cur ^ 1];
    const uint64_t* part_in = finish ? c->d_part[(k - 2) & 1] : nullptr;
    uint64_t* part_out = start ? c->d_part[(k - 1) & 1] : nullptr;
    launch_accel_stream(s, c->p.lamsum, finish, start, nu_early, c->nchunks, c->d_chunks,
                        c->d_rows, c->d_rcf, c->d_tsig, c->d_nu, c->d_rh, c->d_ru, lam_prev,
                        lam_new, part_in, part_out, alpha, beta, c->chunk, c->d_status);
    RCSCM_HIP(c, hipGetLastError());
    if (finish) cur ^= 1;
  }
  return RCSCM_OK;
}

// Checkpoint storage for K iterations (theta_k, k < K), grown on demand.
static rcscm_status ensure_checkpoints(rcscm_ctx* c, int K) {
  if (K <= c->ck_capacity) return RCSCM_OK;
  if (c->ck_capacity > 0) {  // replace the smaller buffers once queued work is done with them
    RCSCM_HIP(c, hipStreamSynchronize(c->stream));
    c->release(&c->d_ck_rh);
    c->release(&c->d_ck_ru);
    c->release(&c->d_ck_lam);
    c->ck_capacity = 0;
  }
  RCSCM_TRY(c->alloc(&c->d_ck_rh, (size_t)K * c->nbins, "checkpoints r^h"));
  RCSCM_TRY(c->alloc(&c->d_ck_ru, (size_t)K * c->nbins, "checkpoints r^u"));
  RCSCM_TRY(c->alloc(&c->d_ck_lam, (size_t)K * c->nrows, "checkpoints lambda"));
  c->ck_capacity = K;
  return RCSCM_OK;
}

rcscm_status rcscm_iterate(rcscm_ctx* c, int K) {
  if (!c) return RCSCM_EINVAL;
  if (K < 0) return c->fail(RCSCM_ESHAPE, "K must be >= 0");
  if (!c->inited) return c->no_state("iterate");
  if (K == 0) return RCSCM_OK;
  hipStream_t s = c->stream;
  const float alpha = (float)c->p.alpha, beta = (float)c->p.beta;
  if (c->p.rule == RCSCM_RULE_FIRST) {
    for (const auto& cl : c->first_classes) {
      launch_first_stage(s, cl.nt, cl.bpl, cl.count, c->d_row_list + cl.offset, c->d_rows,
                         c->d_rcf, c->d_rcd, c->x_borrowed, c->d_rh, c->d_ru,
                         c->d_lam[c->lam_cur], alpha, beta, K, c->d_status);
      RCSCM_HIP(c, hipGetLastError());
    }
    return RCSCM_OK;
  }
  if (c->p.rule == RCSCM_RULE_NAIVE) {
    const bool store_u = (c->p.flags & RCSCM_FLAG_NAIVE_RECOMPUTE) == 0;
    for (int k = 0; k < K; ++k) {
      for (int m = 2; m <= RCSCM_MAX_M; ++m) {
        const auto rg = c->m_range[m];
        if (rg.second == 0) continue;
        launch_naive_a(s, m, store_u, rg.second, c->d_chunks_m + rg.first, c->d_rows, c->d_rsf,
                       c->x_borrowed, c->d_rh, c->d_ru, c->d_lam[c->lam_cur], c->d_uhat, c->nbins,
                       c->d_part[0], alpha, beta, c->d_status);
        RCSCM_HIP(c, hipGetLastError());
      }
      for (int m = 2; m <= RCSCM_MAX_M; ++m) {
        const auto rg = c->m_range[m];
        if (rg.second == 0) continue;
        if (store_u)
          launch_naive_b(s, m, rg.second, c->d_chunks_m + rg.first, c->d_rows, c->d_rcd,
                         c->d_part[0], c->d_lam[c->lam_cur], c->d_ru, c->d_uhat, c->nbins,
                         c->d_status);
        else  // lambda~ stays readable until every chunk has rebuilt R~: new lambda to the other buffer
          launch_naive_b_recompute(s, m, rg.second, c->d_chunks_m + rg.first, c->d_rows,
                                   c->d_rsf, c->d_rcd, c->d_part[0], c->d_lam[c->lam_cur],
                                   c->d_lam[c->lam_cur ^ 1], c->x_borrowed, c->d_uhat, c->d_ru,
                                   c->d_status);
        RCSCM_HIP(c, hipGetLastError());
      }
      if (!store_u) c->lam_cur ^= 1;
    }
    return RCSCM_OK;
  }
  if (c->schedule == RCSCM_SCHED_RESIDENT) {
    float *ck_rh = nullptr, *ck_ru = nullptr, *ck_lam = nullptr;
    if (c->p.flags & RCSCM_FLAG_CHECKPOINT) {
      RCSCM_TRY(ensure_checkpoints(c, K));
      ck_rh = c->d_ck_rh;
      ck_ru = c->d_ck_ru;
      ck_lam = c->d_ck_lam;
      c->ck_K = K;
    }
    for (const auto& cl : c->res_classes) {
      const int fair = cl.fair_res ? 1 : 0;
      launch_accel_resident(s, cl.nt, cl.bpl, c->p.lamsum, cl.count, c->d_row_list + cl.offset,
                            c->d_rows, c->d_rcf, c->d_tsig, c->d_nu, c->d_rh, c->d_ru,
                            c->d_lam[c->lam_cur], alpha, beta, K, ck_rh, ck_ru, ck_lam, c->nbins,
                            c->nrows, c->d_status, fair);
      RCSCM_HIP(c, hipGetLastError());
    }
    return RCSCM_OK;
  }
  // STREAM
  if (c->p.flags & RCSCM_FLAG_GRAPH) {
    const std::pair<int, int> key{K, c->lam_cur};
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
      hipStream_t cap = nullptr;
      RCSCM_HIP(c, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
      hipGraph_t g = nullptr;
      hipStream_t saved = c->stream;
      c->stream = cap;
      hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
      rcscm_status st = RCSCM_OK;
      if (e == hipSuccess) st = enqueue_stream_loop(c, K);
      hipError_t e2 = hipStreamEndCapture(cap, &g);
      c->stream = saved;
      (void)hipStreamDestroy(cap);
      if (e != hipSuccess || e2 != hipSuccess || st != RCSCM_OK) {
        (void)hipGetLastError();
        if (g) (void)hipGraphDestroy(g);
        return c->fail(RCSCM_EDEVICE, "hipGraph capture of the iteration loop failed");
      }
      c->graph_defs.push_back(g);  // owned by the context from here on
      hipGraphExec_t ex = nullptr;
      RCSCM_HIP(c, hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
      it = c->graphs.emplace(key, ex).first;
    }
    RCSCM_HIP(c, hipGraphLaunch(it->second, s));
    c->lam_cur ^= (K & 1);
    return RCSCM_OK;
  }
  RCSCM_TRY(enqueue_stream_loop(c, K));
  c->lam_cur ^= (K & 1);
  return RCSCM_OK;
}

rcscm_status rcscm_extract(rcscm_ctx* c, float* rh, float* ru, float* lam, void* s_hat) {
  if (!c) return RCSCM_EINVAL;
  if (!c->inited) return c->no_state("extract");
  if (!rh && !ru && !lam && !s_hat) return RCSCM_OK;
  launch_extract(c->stream, c->nchunks, c->d_chunks, c->d_rows, c->d_rcf, c->d_tsig, c->d_rh,
                 c->d_ru, c->d_lam[c->lam_cur], rh, ru, lam, static_cast<float2*>(s_hat),
                 c->d_status);
  RCSCM_HIP(c, hipGetLastError());
  return RCSCM_OK;
}

rcscm_status rcscm_set_state(rcscm_ctx* c, const float* rh, const float* ru, const float* lam) {
  if (!c) return RCSCM_EINVAL;
  if (!c->inited) return c->no_state("set_state");
  if (!rh || !ru || !lam) return c->fail(RCSCM_EINVAL, "state arrays must not be NULL");
  hipStream_t s = c->stream;
  RCSCM_HIP(c, hipMemcpyAsync(c->d_rh, rh, sizeof(float) * c->nbins, hipMemcpyDeviceToDevice, s));
  RCSCM_HIP(c, hipMemcpyAsync(c->d_ru, ru, sizeof(float) * c->nbins, hipMemcpyDeviceToDevice, s));
  RCSCM_HIP(c, hipMemcpyAsync(c->d_lam[c->lam_cur], lam, sizeof(float) * c->nrows,
                              hipMemcpyDeviceToDevice, s));
  c->ck_K = -1;
  return RCSCM_OK;
}

rcscm_status rcscm_get_state(rcscm_ctx* c, float* rh, float* ru, float* lam) {
  if (!c) return RCSCM_EINVAL;
  if (!rh || !ru || !lam) return c->fail(RCSCM_EINVAL, "state arrays must not be NULL");
  if (!c->inited) return c->no_state("get_state");
  hipStream_t s = c->stream;
  RCSCM_HIP(c, hipMemcpyAsync(rh, c->d_rh, sizeof(float) * c->nbins, hipMemcpyDeviceToDevice, s));
  RCSCM_HIP(c, hipMemcpyAsync(ru, c->d_ru, sizeof(float) * c->nbins, hipMemcpyDeviceToDevice, s));
  RCSCM_HIP(c, hipMemcpyAsync(lam, c->d_lam[c->lam_cur], sizeof(float) * c->nrows,
                              hipMemcpyDeviceToDevice, s));
  return RCSCM_OK;
}

rcscm_status rcscm_sync(rcscm_ctx* c) {
  if (!c) return RCSCM_EINVAL;
  RCSCM_HIP(c, hipStreamSynchronize(c->stream));
  std::vector<unsigned> st(c->nrows), cst(c->nchunks);
  RCSCM_HIP(c, hipMemcpy(st.data(), c->d_status, sizeof(unsigned) * c->nrows,
                         hipMemcpyDeviceToHost));
  RCSCM_HIP(c, hipMemcpy(cst.data(), c->d_chunk_status, sizeof(unsigned) * c->nchunks,
                         hipMemcpyDeviceToHost));
  if (c->chunk_status_valid)
    for (int k = 0; k < c->nchunks; ++k) st[c->h_chunks[k].row] |= cst[k];
  const unsigned order[] = {ST_NONFINITE_IN, ST_NOT_NULL, ST_NOT_PSD, ST_NONFINITE_STATE,
                            ST_LAM_NONPOS};
  for (unsigned bit : order) {
    for (int r = 0; r < c->nrows; ++r) {
      if (st[r] & bit) {
        const RowInfo& ri = c->h_rows[r];
        char buf[160];
        std::snprintf(buf, sizeof(buf), "row %d (utterance %d, frequency %d): %s", r, ri.utt,
                      ri.freq,
                      bit == ST_NONFINITE_IN     ? "non-finite input"
                      : bit == ST_NOT_NULL       ? "b is not a null vector of R'"
                      : bit == ST_NOT_PSD        ? "R' + b b^H is not positive definite"
                      : bit == ST_NONFINITE_STATE ? "non-finite or non-positive state"
                                                 : "lambda is not positive");
        c->err = buf;
        switch (bit) {
          case ST_NONFINITE_IN: return RCSCM_ENONFINITE;
          case ST_NOT_NULL: return RCSCM_ENOTNULL;
          case ST_NOT_PSD: return RCSCM_ENOTPSD;
          default: return RCSCM_ENONFINITE;
        }
      }
    }
  }
  return RCSCM_OK;
}

rcscm_status rcscm_objective(rcscm_ctx* c, double* nlp) {
  if (!c || !nlp) return RCSCM_EINVAL;
  if (!c->inited) return c->no_state("objective");
  launch_objective(c->stream, c->nchunks, c->d_chunks, c->d_rows, c->d_rcf, c->d_rcd, c->d_tsig,
                   c->d_nu, c->d_rh, c->d_ru, c->d_lam[c->lam_cur], c->p.alpha, c->p.beta,
                   c->d_objpart);
  RCSCM_HIP(c, hipGetLastError());
  RCSCM_HIP(c, hipStreamSynchronize(c->stream));
  std::vector<double> part(c->nchunks);
  RCSCM_HIP(c, hipMemcpy(part.data(), c->d_objpart, sizeof(double) * c->nchunks,
                         hipMemcpyDeviceToHost));
  double sum = 0.0;
  for (double v : part) sum += v;
  *nlp = sum;
  return RCSCM_OK;
}

rcscm_status rcscm_backward(rcscm_ctx* c, const void* x, const void* grad_s_hat, void* grad_x,
                            float* grad_rh0, float* grad_lam0) {
  if (!c) return RCSCM_EINVAL;
  if (!(c->p.flags & RCSCM_FLAG_CHECKPOINT) || c->ck_K < 0 || !c->inited)
    return c->fail(RCSCM_ESTATE, "backward needs a context with checkpoints that was iterated");
  if (!x || !grad_s_hat) return c->fail(RCSCM_EINVAL, "x and grad_s_hat must not be NULL");
  for (const auto& cl : c->res_classes) {
    const int fair = cl.fair_bw ? 1 : 0;
    launch_backward(c->stream, cl.nt, cl.bpl, cl.count, c->d_row_list + cl.offset, c->d_rows,
                    c->d_rcf, c->d_rcd, static_cast<const float2*>(x), c->d_tsig, c->d_nu,
                    c->d_ck_rh, c->d_ck_ru, c->d_ck_lam, c->nbins, c->nrows, c->d_rh, c->d_ru,
                    c->d_lam[c->lam_cur], c->ck_K, (float)c->p.alpha,
                    static_cast<const float2*>(grad_s_hat), static_cast<float2*>(grad_x),
                    grad_rh0, grad_lam0, fair);
    RCSCM_HIP(c, hipGetLastError());
  }
  return RCSCM_OK;
}

rcscm_status rcscm_backproject(rcscm_ctx* c, const void* x, const void* W, const int* target,
                               void* a, void* Rp, void* b, float* ru0, float* lam0) {
  if (!c) return RCSCM_EINVAL;
  if (!x || !W || !target || !a || !Rp || !b)
    return c->fail(RCSCM_EINVAL, "x, W, target, a, Rp and b must not be NULL");
  for (int u = 0; u < c->U; ++u)
    if (target[u] < 0 || target[u] >= c->M[u])
      return c->fail(RCSCM_EINVAL, "target index out of range (utterance " + std::to_string(u) + ")");
  if (!c->d_bp_part) {
    RCSCM_TRY(c->alloc(&c->d_bp_part, (size_t)c->nchunks * MAXM, "back-projection partials"));
    RCSCM_TRY(c->alloc(&c->d_bp_p, (size_t)c->nrows * MAXM, "back-projection powers"));
    RCSCM_TRY(c->alloc(&c->d_bp_target, (size_t)c->nrows, "target indices"));
  }
  std::vector<int> tg(c->nrows);
  for (int r = 0; r < c->nrows; ++r) tg[r] = target[c->h_rows[r].utt];
  hipStream_t s = c->stream;
  if (tg != c->h_bp_target) {  // upload only when the targets change
    c->h_bp_target = tg;
    RCSCM_HIP(c, hipMemcpyAsync(c->d_bp_target, c->h_bp_target.data(), sizeof(int) * c->nrows,
                                hipMemcpyHostToDevice, s));
    RCSCM_HIP(c, hipStreamSynchronize(s));  // the host vector may change on the next call
  }
  // one fused launch per microphone count of at most kBpFusedMaxM whose rows
  // are all short enough, the three chunked stages for the others
  int maxJ[RCSCM_MAX_M + 1] = {0};
  for (const RowInfo& r : c->h_rows) maxJ[r.M] = r.J > maxJ[r.M] ? r.J : maxJ[r.M];
  for (int stage : {3, 0, 1, 2})
    for (int m = 2; m <= RCSCM_MAX_M; ++m) {
      const auto cr = c->m_range[m];
      const auto rr = c->mrow_range[m];
      const bool fused = m <= kBpFusedMaxM && maxJ[m] <= kBpFusedMaxJ;
      if (rr.second == 0 || (stage == 3) != fused) continue;
      launch_backproject(s, m, cr.second, c->d_chunks_m + cr.first, rr.second,
                         c->d_rows_m + rr.first, c->d_rows, static_cast<const float2*>(x),
                         static_cast<const double2*>(W), c->d_bp_target, c->d_bp_part, c->d_bp_p,
                         static_cast<double2*>(a), static_cast<double2*>(Rp),
                         static_cast<double2*>(b), ru0, lam0, c->d_status, stage);
      RCSCM_HIP(c, hipGetLastError());
    }
  return RCSCM_OK;
}

// Creates the auxiliary streams and events of a multi-class rcscm_run (once).
static rcscm_status ensure_aux(rcscm_ctx* c, int n) {
  if ((int)c->aux.size() >= n) return RCSCM_OK;
  int cur = 0;
  RCSCM_HIP(c, hipGetDevice(&cur));
  if (cur != c->device) RCSCM_HIP(c, hipSetDevice(c->device));
  struct Restore {  // the caller's current device, also on the error paths
    int dev, ctx_dev;
    ~Restore() {
      if (dev != ctx_dev) (void)hipSetDevice(dev);
    }
  } restore{cur, c->device};
  if (!c->ev_fork) RCSCM_HIP(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
  while ((int)c->aux.size() < n) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    RCSCM_HIP(c, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipEventDestroy(ev);
      return c->fail(RCSCM_EDEVICE, "hipStreamCreateWithFlags failed");
    }
    c->aux.push_back(st);
    c->ev_join.push_back(ev);
  }
  return RCSCM_OK;
}

rcscm_status rcscm_run(rcscm_ctx* c, const void* x, const void* a, const void* Rp, const void* b,
                       const float* rh0, const float* ru0, const float* lam0, int K, float* rh,
                       float* ru, float* lam, void* s_hat) {
  if (!c) return RCSCM_EINVAL;
  if (K < 0) return c->fail(RCSCM_ESHAPE, "K must be >= 0");
  if (!x || !a || !Rp || !b) return c->fail(RCSCM_EINVAL, "x, a, Rp and b must not be NULL");
  // with checkpoints the adjoint walks the RESIDENT classes, so the fused path
  // keeps them only under that schedule
  const bool ckpt = (c->p.flags & RCSCM_FLAG_CHECKPOINT) != 0;
  const bool fused = !c->fused_classes.empty() && c->p.lamsum == RCSCM_LAMSUM_F64 &&
                     (!ckpt || c->schedule == RCSCM_SCHED_RESIDENT);
  if (!fused) {  // the same path as separate calls
    RCSCM_TRY(rcscm_init(c, x, a, Rp, b, rh0, ru0, lam0));
    RCSCM_TRY(rcscm_iterate(c, K));
    return rcscm_extract(c, rh, ru, lam, s_hat);
  }
  c->lam_cur = 0;
  const bool keep = (c->p.flags & RCSCM_FLAG_RUN_ONLY) == 0;  // store the state for later calls
  FusedArgs A;
  A.rows = c->d_rows;
  A.x = static_cast<const float2*>(x);
  A.a = static_cast<const double2*>(a);
  A.Rp = static_cast<const double2*>(Rp);
  A.b = static_cast<const double2*>(b);
  A.rh0 = rh0;
  A.ru0 = ru0;
  A.lam0 = lam0;
  A.rh_c = c->p.rh0;
  A.ru_c = c->p.ru0;
  A.lam_c = c->p.lam0;
  A.rcd = keep ? c->d_rcd : nullptr;
  A.rcf = keep ? c->d_rcf : nullptr;
  A.rsf = nullptr;  // the fused path serves the accelerated rule only
  A.tsig = keep ? c->d_tsig : nullptr;
  A.nu = keep ? c->d_nu : nullptr;
  A.rh = keep ? c->d_rh : nullptr;
  A.ru = keep ? c->d_ru : nullptr;
  A.lam = keep ? c->d_lam[c->lam_cur] : nullptr;
  A.status = c->d_status;
  A.rh_out = rh;
  A.ru_out = ru;
  A.lam_out = lam;
  A.s_hat = static_cast<float2*>(s_hat);
  A.inv_a2 = (float)(1.0 / (c->p.alpha + 2.0));
  A.beta_a2 = (float)(c->p.beta / (c->p.alpha + 2.0));
  A.K = K;
  A.n_bins = c->nbins;
  A.n_rows = c->nrows;
  A.ck_rh = A.ck_ru = A.ck_lam = nullptr;
  A.ck_sb = 0;
  A.ck_sr = 0;
  if (ckpt) {
    RCSCM_TRY(ensure_checkpoints(c, K));
    A.ck_rh = c->d_ck_rh;
    A.ck_ru = c->d_ck_ru;
    A.ck_lam = c->d_ck_lam;
    A.ck_sb = c->nbins;
    A.ck_sr = c->nrows;
  }
  c->chunk_status_valid = false;  // the fused kernel reports through status[row] only
  // Largest class first on the context's stream; the others go round-robin to
  // up to three auxiliary streams, so the tail of one class launch overlaps
  // the next class instead of leaving CUs idle.
  const int ncls = (int)c->fused_classes.size();
  std::vector<int> order(ncls);
  for (int k = 0; k < ncls; ++k) order[k] = k;
  std::sort(order.begin(), order.end(), [&](int u, int v) {
    const auto& a = c->fused_classes[u];
    const auto& b = c->fused_classes[v];
    return (long long)a.count * a.nt * a.bpl > (long long)b.count * b.nt * b.bpl;
  });
  const int naux = std::min(3, ncls - 1);
  if (naux > 0) {
    RCSCM_TRY(ensure_aux(c, naux));
    RCSCM_HIP(c, hipEventRecord(c->ev_fork, c->stream));
    for (int k = 0; k < naux; ++k) RCSCM_HIP(c, hipStreamWaitEvent(c->aux[k], c->ev_fork, 0));
  }
  for (int oi = 0; oi < ncls; ++oi) {
    const auto& cl = c->fused_classes[order[oi]];
    hipStream_t st = oi == 0 ? c->stream : c->aux[(oi - 1) % naux];
    A.row_list = c->d_row_list + cl.offset;
    A.lin = 0;
    if (cl.linear) {
      const RowInfo& r0 = c->h_rows[cl.row0];
      A.lin = 1;
      A.lin_row0 = cl.row0;
      A.lin_J = r0.J;
      A.lin_x0 = r0.x_off;
      A.lin_bin0 = r0.bin_off;
      A.lin_a0 = r0.a_off;
      A.lin_rp0 = r0.rp_off;
    }
    A.fair = cl.fair ? 1 : 0;
    launch_fused(st, cl.M, cl.nt, cl.bpl, cl.count, A);
    RCSCM_HIP(c, hipGetLastError());
  }
  for (int k = 0; k < naux; ++k) {
    RCSCM_HIP(c, hipEventRecord(c->ev_join[k], c->aux[k]));
    RCSCM_HIP(c, hipStreamWaitEvent(c->stream, c->ev_join[k], 0));
  }
  c->x_borrowed = static_cast<const float2*>(x);
  c->inited = keep;
  c->dropped = !keep;
  c->ck_K = ckpt ? K : -1;
  return RCSCM_OK;
}

rcscm_status rcscm_set_run_classes(rcscm_ctx* c, int n, const int* table) {
  if (!c) return RCSCM_EINVAL;
  if (n < 0 || (n > 0 && !table)) return c->fail(RCSCM_EINVAL, "n must be >= 0 and table non-NULL");
  std::vector<std::array<int, 4>> t;
  for (int k = 0; k < n; ++k) {
    const int M = table[4 * k], jmax = table[4 * k + 1], nt = table[4 * k + 2],
              bpl = table[4 * k + 3];
    if (!(M == 0 || (M >= 2 && M <= RCSCM_MAX_M)) || jmax < 1 || !fused_supported(nt, bpl))
      return c->fail(RCSCM_EINVAL,
                     "run class entry " + std::to_string(k) +
                         ": M must be 0 or 2..8, j_max >= 1, and (nt, bpl) one of (256, 1/2/4/8), "
                         "(512, 2/4/8), (1024, 1/2/4/8)");
    t.push_back({M, jmax, nt, bpl});
  }
  c->run_table = t;
  if (c->fused_classes.empty()) return RCSCM_OK;  // no fused launch for this context
  std::vector<int> rl;
  std::vector<rcscm_ctx::FusedClass> cls;
  group_fused(c, &rl, &cls);
  if (cls.empty()) return c->fail(RCSCM_EDEVICE, "regrouping the fused classes failed");
  for (auto& cl : cls) cl.offset += c->fused_offset;
  // queued runs may still read the row list
  RCSCM_HIP(c, hipStreamSynchronize(c->stream));
  for (hipStream_t st : c->aux) RCSCM_HIP(c, hipStreamSynchronize(st));
  RCSCM_HIP(c, hipMemcpy(c->d_row_list + c->fused_offset, rl.data(), sizeof(int) * rl.size(),
                         hipMemcpyHostToDevice));
  c->fused_classes = cls;
  set_fair_flags(c);
  return RCSCM_OK;
}

rcscm_status rcscm_get_run_classes(const rcscm_ctx* c, int cap, int* table, int* n) {
  if (!c || !n || (cap > 0 && !table)) return RCSCM_EINVAL;
  *n = (int)c->fused_classes.size();
  for (int k = 0; k < *n && k < cap; ++k) {
    const auto& cl = c->fused_classes[k];
    table[5 * k] = cl.M;
    table[5 * k + 1] = cl.nt;
    table[5 * k + 2] = cl.bpl;
    table[5 * k + 3] = cl.count;
    table[5 * k + 4] = c->h_rows[cl.row0].J;
  }
  return RCSCM_OK;
}

rcscm_status rcscm_get_schedule(const rcscm_ctx* c, int* schedule, int* block, int* chunk) {
  if (!c) return RCSCM_EINVAL;
  if (schedule) *schedule = c->schedule;
  if (block) *block = c->res_nt;
  if (chunk) *chunk = c->chunk;
  return RCSCM_OK;
}

void rcscm_destroy(rcscm_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  for (hipStream_t st : c->aux) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  for (hipEvent_t ev : c->ev_join) (void)hipEventDestroy(ev);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  for (hipGraph_t g : c->graph_defs) (void)hipGraphDestroy(g);
  delete c;
}

const char* rcscm_last_error(const rcscm_ctx* c) {
  if (!c) return g_create_error.c_str();
  return c->err.c_str();
}

}  // extern "C"
