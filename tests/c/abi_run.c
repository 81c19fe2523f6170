/* A plain C99 user of include/rcscm.h: loads x (complex64 [I][J][M]) and a, R', b
 * (complex128) from raw little-endian files in DIR, runs rcscm_run for K
 * iterations on device buffers it allocates itself, and writes r^h, r^u,
 * lambda and s_hat back to DIR.  Exit status 0 on success; the rcscm status
 * of rcscm_sync is printed.  Then the resume round trip: rcscm_get_state must
 * equal the run's r^h, r^u, lambda bitwise, and a second context initialised
 * with the same inputs and given that state by rcscm_set_state must reach the
 * bitwise same state as the first after 3 more iterations ("get_state 1",
 * "resume 1" on stdout).
 *
 *   abi_run DIR I J M K
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "rcscm.h"

static void* load(const char* dir, const char* name, size_t bytes) {
  char path[4096];
  snprintf(path, sizeof path, "%s/%s", dir, name);
  FILE* f = fopen(path, "rb");
  if (!f) return NULL;
  void* h = malloc(bytes);
  size_t n = h ? fread(h, 1, bytes, f) : 0;
  fclose(f);
  if (n != bytes) {
    free(h);
    return NULL;
  }
  void* d = NULL;
  if (hipMalloc(&d, bytes) != hipSuccess || hipMemcpy(d, h, bytes, hipMemcpyHostToDevice) != hipSuccess) {
    free(h);
    return NULL;
  }
  free(h);
  return d;
}

/* 1 when the device arrays d1 and d2 of the given size hold the same bytes. */
static int same_bytes(const void* d1, const void* d2, size_t bytes) {
  void* h1 = malloc(bytes);
  void* h2 = malloc(bytes);
  int eq = h1 && h2 && hipMemcpy(h1, d1, bytes, hipMemcpyDeviceToHost) == hipSuccess &&
           hipMemcpy(h2, d2, bytes, hipMemcpyDeviceToHost) == hipSuccess &&
           memcmp(h1, h2, bytes) == 0;
  free(h1);
  free(h2);
  return eq;
}

/* get_state after the run, then set_state into a second context; 0 on success. */
static int resume_round_trip(rcscm_ctx* ctx, const void* x, const void* a, const void* Rp,
                             const void* b, int I, int J, int M, const float* rh, const float* ru,
                             const float* lam) {
  const size_t nb = (size_t)I * J;
  float *srh = NULL, *sru = NULL, *slam = NULL, *trh = NULL, *tru = NULL, *tlam = NULL;
  if (hipMalloc((void**)&srh, nb * 4) != hipSuccess || hipMalloc((void**)&sru, nb * 4) != hipSuccess ||
      hipMalloc((void**)&slam, (size_t)I * 4) != hipSuccess ||
      hipMalloc((void**)&trh, nb * 4) != hipSuccess || hipMalloc((void**)&tru, nb * 4) != hipSuccess ||
      hipMalloc((void**)&tlam, (size_t)I * 4) != hipSuccess)
    return 1;
  rcscm_status st = rcscm_get_state(ctx, srh, sru, slam);
  if (st == RCSCM_OK) st = rcscm_sync(ctx);
  if (st != RCSCM_OK) return 1;
  printf("get_state %d\n", same_bytes(srh, rh, nb * 4) && same_bytes(sru, ru, nb * 4) &&
                               same_bytes(slam, lam, (size_t)I * 4));
  rcscm_ctx* c2 = NULL;
  rcscm_params p;
  rcscm_default_params(&p);
  if (rcscm_create(&c2, I, J, M, &p, NULL) != RCSCM_OK) return 1;
  st = rcscm_init(c2, x, a, Rp, b, NULL, NULL, NULL);
  if (st == RCSCM_OK) st = rcscm_set_state(c2, srh, sru, slam);
  if (st == RCSCM_OK) st = rcscm_iterate(c2, 3);
  if (st == RCSCM_OK) st = rcscm_extract(c2, trh, tru, tlam, NULL);
  if (st == RCSCM_OK) st = rcscm_sync(c2);
  if (st == RCSCM_OK) st = rcscm_iterate(ctx, 3);
  if (st == RCSCM_OK) st = rcscm_get_state(ctx, srh, sru, slam);
  if (st == RCSCM_OK) st = rcscm_sync(ctx);
  if (st != RCSCM_OK) return 1;
  printf("resume %d\n", same_bytes(srh, trh, nb * 4) && same_bytes(sru, tru, nb * 4) &&
                             same_bytes(slam, tlam, (size_t)I * 4));
  rcscm_destroy(c2);
  hipFree(srh);
  hipFree(sru);
  hipFree(slam);
  hipFree(trh);
  hipFree(tru);
  hipFree(tlam);
  return 0;
}

static int save(const char* dir, const char* name, const void* d, size_t bytes) {
  char path[4096];
  snprintf(path, sizeof path, "%s/%s", dir, name);
  void* h = malloc(bytes);
  if (!h || hipMemcpy(h, d, bytes, hipMemcpyDeviceToHost) != hipSuccess) return 1;
  FILE* f = fopen(path, "wb");
  if (!f) return 1;
  size_t n = fwrite(h, 1, bytes, f);
  fclose(f);
  free(h);
  return n == bytes ? 0 : 1;
}

int main(int argc, char** argv) {
  if (argc != 6) {
    fprintf(stderr, "usage: %s DIR I J M K\n", argv[0]);
    return 2;
  }
  const char* dir = argv[1];
  const int I = atoi(argv[2]), J = atoi(argv[3]), M = atoi(argv[4]), K = atoi(argv[5]);
  const size_t nb = (size_t)I * J;
  void* x = load(dir, "x.bin", nb * M * 8);
  void* a = load(dir, "a.bin", (size_t)I * M * 16);
  void* Rp = load(dir, "Rp.bin", (size_t)I * M * M * 16);
  void* b = load(dir, "b.bin", (size_t)I * M * 16);
  if (!x || !a || !Rp || !b) {
    fprintf(stderr, "abi_run: could not load the inputs\n");
    return 1;
  }
  float *rh = NULL, *ru = NULL, *lam = NULL;
  void* s_hat = NULL;
  if (hipMalloc((void**)&rh, nb * 4) != hipSuccess || hipMalloc((void**)&ru, nb * 4) != hipSuccess ||
      hipMalloc((void**)&lam, (size_t)I * 4) != hipSuccess || hipMalloc(&s_hat, nb * 8) != hipSuccess)
    return 1;
  rcscm_params p;
  rcscm_default_params(&p);
  rcscm_ctx* ctx = NULL;
  rcscm_status st = rcscm_create(&ctx, I, J, M, &p, NULL);
  if (st != RCSCM_OK) {
    fprintf(stderr, "rcscm_create: %d %s\n", (int)st, rcscm_last_error(NULL));
    return 1;
  }
  st = rcscm_run(ctx, x, a, Rp, b, NULL, NULL, NULL, K, rh, ru, lam, s_hat);
  if (st == RCSCM_OK) st = rcscm_sync(ctx);
  printf("rcscm status %d\n", (int)st);
  if (st != RCSCM_OK) {
    fprintf(stderr, "%s\n", rcscm_last_error(ctx));
    rcscm_destroy(ctx);
    return 1;
  }
  int err = save(dir, "out_rh.bin", rh, nb * 4) | save(dir, "out_ru.bin", ru, nb * 4) |
            save(dir, "out_lam.bin", lam, (size_t)I * 4) | save(dir, "out_shat.bin", s_hat, nb * 8);
  err |= resume_round_trip(ctx, x, a, Rp, b, I, J, M, rh, ru, lam);
  rcscm_destroy(ctx);
  hipFree(x);
  hipFree(a);
  hipFree(Rp);
  hipFree(b);
  hipFree(rh);
  hipFree(ru);
  hipFree(lam);
  hipFree(s_hat);
  return err;
}
