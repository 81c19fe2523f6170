/* Host-side checks of the C ABI that need no GPU: argument validation,
 * workspace sizing, the row/chunk/class tables that rcscm_create builds
 * before its first device allocation, and the error paths that follow when
 * no device is present.  Built with AddressSanitizer and UBSan on the host
 * code of the library (tests/test_sanitize_cpu.py); prints one line per
 * group and exits non-zero on the first wrong status. */
#include <limits.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "rcscm.h"

static int failures = 0;

static void expect(int cond, const char* what) {
  if (!cond) {
    printf("FAIL %s\n", what);
    ++failures;
  }
}

static rcscm_params params(void) {
  rcscm_params p;
  rcscm_default_params(&p);
  return p;
}

/* rcscm_create with these arguments must return want (or, for shapes the
 * validation accepts, fail cleanly at the first device call: EDEVICE or
 * ENOMEM without a GPU, OK with one). */
static void create_case(int U, int I, const int* J, const int* M, const rcscm_params* p,
                        rcscm_status want, const char* what) {
  rcscm_ctx* ctx = (rcscm_ctx*)1;
  const rcscm_status st = rcscm_create_batch(&ctx, U, I, J, M, p, NULL);
  if (want == RCSCM_OK) {
    expect(st == RCSCM_OK || st == RCSCM_EDEVICE || st == RCSCM_ENOMEM, what);
    if (st == RCSCM_OK)
      rcscm_destroy(ctx);
    else
      expect(ctx == NULL, what);
  } else {
    expect(st == want && ctx == NULL, what);
  }
  expect(strlen(rcscm_last_error(NULL)) < 4096, what);
}

int main(void) {
  expect(rcscm_version() > 0, "version");

  /* workspace sizes: valid shapes give a positive size, rejected ones 0 */
  {
    const int J1[1] = {1000}, M1[1] = {4};
    rcscm_params p = params();
    const size_t w = rcscm_workspace_bytes(1, 513, J1, M1, &p);
    expect(w >= (size_t)513 * 1000 * 28, "workspace single");
    expect(rcscm_workspace_bytes(1, 513, J1, M1, NULL) == w, "workspace NULL params");
    const int Jr[5] = {1, 257, 8192, 8193, 40000}, Mr[5] = {2, 3, 5, 7, 8};
    int rules[3] = {RCSCM_RULE_ACCEL, RCSCM_RULE_NAIVE, RCSCM_RULE_FIRST};
    int chunks[5] = {0, 256, 512, 1024, 2048};
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 5; ++c) {
        p = params();
        p.rule = rules[r];
        p.chunk = chunks[c];
        const size_t wr = rcscm_workspace_bytes(5, 17, Jr, Mr, &p);
        /* the FIRST rule rejects rows longer than 4096 frames */
        expect(r == 2 ? wr == 0 : wr > 0, "workspace ragged");
      }
    p = params();
    p.flags = RCSCM_FLAG_CHECKPOINT;
    expect(rcscm_workspace_bytes(5, 17, Jr, Mr, &p) == 0, "workspace checkpoint too long");
    p.flags = RCSCM_FLAG_RUN_ONLY;
    expect(rcscm_workspace_bytes(5, 17, Jr, Mr, &p) > 0, "workspace run-only");
    p = params();
    p.rule = RCSCM_RULE_NAIVE;
    p.flags = RCSCM_FLAG_NAIVE_RECOMPUTE;
    expect(rcscm_workspace_bytes(1, 513, J1, M1, &p) > 0, "workspace naive recompute");
    const int Jbig[1] = {INT_MAX}, Mbig[1] = {8};
    expect(rcscm_workspace_bytes(1, INT_MAX, Jbig, Mbig, NULL) == 0, "workspace too many bins");
    expect(rcscm_workspace_bytes(0, 513, J1, M1, NULL) == 0, "workspace U = 0");
    expect(rcscm_workspace_bytes(1, 513, NULL, M1, NULL) == 0, "workspace NULL J");
    printf("workspace ok\n");
  }

  /* create: every validation branch, then shapes that pass validation */
  {
    const int J1[1] = {1000}, M1[1] = {4}, M9[1] = {9}, J0[1] = {0};
    rcscm_params p = params();
    create_case(1, 0, J1, M1, &p, RCSCM_ESHAPE, "I = 0");
    create_case(1, 513, J0, M1, &p, RCSCM_ESHAPE, "J = 0");
    create_case(1, 513, J1, M9, &p, RCSCM_ESHAPE, "M = 9");
    create_case(0, 513, J1, M1, &p, RCSCM_ESHAPE, "U = 0");
    create_case(1, 513, NULL, M1, &p, RCSCM_EINVAL, "J NULL");
    p.alpha = -3.0;
    create_case(1, 513, J1, M1, &p, RCSCM_EINVAL, "alpha");
    p = params();
    p.beta = NAN;
    create_case(1, 513, J1, M1, &p, RCSCM_EINVAL, "beta");
    p = params();
    p.lam0 = 0.0f;
    create_case(1, 513, J1, M1, &p, RCSCM_EINVAL, "lam0");
    p = params();
    p.rule = 5;
    create_case(1, 513, J1, M1, &p, RCSCM_EINVAL, "rule");
    p = params();
    p.block = 96;
    create_case(1, 513, J1, M1, &p, RCSCM_EINVAL, "block");
    p = params();
    p.chunk = 100;
    create_case(1, 513, J1, M1, &p, RCSCM_EINVAL, "chunk");
    p = params();
    p.flags = 64u;
    create_case(1, 513, J1, M1, &p, RCSCM_EINVAL, "flags");
    p.flags = RCSCM_FLAG_RUN_ONLY | RCSCM_FLAG_CHECKPOINT;
    create_case(1, 513, J1, M1, &p, RCSCM_EINVAL, "run-only + checkpoint");
    p.flags = RCSCM_FLAG_NAIVE_RECOMPUTE;
    create_case(1, 513, J1, M1, &p, RCSCM_EINVAL, "recompute without naive");
    expect(rcscm_create(NULL, 4, 16, 4, NULL, NULL) == RCSCM_EINVAL, "out NULL");

    const int Jr[6] = {1, 200, 4000, 8192, 8193, 30000}, Mr[6] = {2, 4, 6, 8, 3, 5};
    int rules[3] = {RCSCM_RULE_ACCEL, RCSCM_RULE_NAIVE, RCSCM_RULE_FIRST};
    int scheds[3] = {RCSCM_SCHED_AUTO, RCSCM_SCHED_STREAM, RCSCM_SCHED_RESIDENT};
    for (int r = 0; r < 3; ++r)
      for (int s = 0; s < 3; ++s) {
        p = params();
        p.rule = rules[r];
        p.schedule = scheds[s];
        /* rows over 8192 frames: RESIDENT and FIRST reject them */
        const int too_long = (r == 0 && s == 2) || r == 2;
        create_case(6, 9, Jr, Mr, &p, too_long ? RCSCM_ESHAPE : RCSCM_OK, "ragged create");
        create_case(3, 9, Jr, Mr, &p, RCSCM_OK, "ragged create (rows <= 4096 frames)");
      }
    printf("create ok\n");
  }

  /* calls on a NULL context are rejected before any device work */
  {
    float f = 0.0f;
    int i0 = 0, i1 = 0, i2 = 0;
    double d = 0.0;
    const int tab[4] = {4, 1024, 256, 4};
    expect(rcscm_init(NULL, &f, &f, &f, &f, NULL, NULL, NULL) == RCSCM_EINVAL, "init NULL");
    expect(rcscm_iterate(NULL, 1) == RCSCM_EINVAL, "iterate NULL");
    expect(rcscm_extract(NULL, NULL, NULL, NULL, NULL) == RCSCM_EINVAL, "extract NULL");
    expect(rcscm_run(NULL, &f, &f, &f, &f, NULL, NULL, NULL, 1, NULL, NULL, NULL, NULL) ==
               RCSCM_EINVAL,
           "run NULL");
    expect(rcscm_set_state(NULL, &f, &f, &f) == RCSCM_EINVAL, "set_state NULL");
    expect(rcscm_get_state(NULL, &f, &f, &f) == RCSCM_EINVAL, "get_state NULL");
    expect(rcscm_sync(NULL) == RCSCM_EINVAL, "sync NULL");
    expect(rcscm_objective(NULL, &d) == RCSCM_EINVAL, "objective NULL");
    expect(rcscm_backward(NULL, &f, &f, NULL, NULL, NULL) == RCSCM_EINVAL, "backward NULL");
    expect(rcscm_backproject(NULL, &f, &f, &i0, &f, &f, &f, NULL, NULL) == RCSCM_EINVAL,
           "backproject NULL");
    expect(rcscm_get_schedule(NULL, &i0, &i1, &i2) == RCSCM_EINVAL, "get_schedule NULL");
    expect(rcscm_set_run_classes(NULL, 1, tab) == RCSCM_EINVAL, "set_run_classes NULL");
    expect(rcscm_get_run_classes(NULL, 0, NULL, &i0) == RCSCM_EINVAL, "get_run_classes NULL");
    rcscm_destroy(NULL);
    printf("null context ok\n");
  }

  /* the no-allocation entry point rejects what it cannot run before any device work */
  {
    float f = 0.0f;
    rcscm_params p = params();
    expect(rcscm_run_noalloc(RCSCM_NOALLOC_MAX_ROWS + 1, 100, 4, &p, NULL, &f, &f, &f, &f, NULL,
                             NULL, NULL, 1, &f, &f, &f, NULL, 0) == RCSCM_ESHAPE,
           "noalloc too many rows");
    expect(rcscm_run_noalloc(4, 9000, 4, &p, NULL, &f, &f, &f, &f, NULL, NULL, NULL, 1, &f, &f,
                             &f, NULL, 0) == RCSCM_ESHAPE,
           "noalloc row too long");
    expect(rcscm_run_noalloc(4, 100, 4, &p, NULL, NULL, &f, &f, &f, NULL, NULL, NULL, 1, &f, &f,
                             &f, NULL, 0) == RCSCM_EINVAL,
           "noalloc NULL x");
    expect(rcscm_run_noalloc(4, 100, 4, &p, NULL, &f, &f, &f, &f, NULL, NULL, NULL, -1, &f, &f,
                             &f, NULL, 0) == RCSCM_ESHAPE,
           "noalloc K < 0");
    p.rule = RCSCM_RULE_NAIVE;
    expect(rcscm_run_noalloc(4, 100, 4, &p, NULL, &f, &f, &f, &f, NULL, NULL, NULL, 1, &f, &f,
                             &f, NULL, 0) != RCSCM_OK,
           "noalloc naive rule");
    p = params();
    p.flags = RCSCM_FLAG_CHECKPOINT;
    expect(rcscm_run_noalloc(4, 100, 4, &p, NULL, &f, &f, &f, &f, NULL, NULL, NULL, 1, &f, &f,
                             &f, NULL, 0) != RCSCM_OK,
           "noalloc checkpoint");
    expect(strlen(rcscm_last_error(NULL)) > 0, "noalloc message");
    printf("noalloc ok\n");
  }

  printf(failures ? "abi_host FAILED %d\n" : "abi_host done\n", failures);
  return failures ? 1 : 0;
}
