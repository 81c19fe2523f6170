/* A plain C99 user of include/rcscm.h: loads x (complex64 [I][J][M]) and a, R', b
 * (complex128) from raw little-endian files in DIR, runs rcscm_run for K
 * iterations on device buffers it allocates itself, and writes r^h, r^u,
 * lambda and s_hat back to DIR.  Exit status 0 on success; the rcscm status
 * of rcscm_sync is printed.
 *
 *   abi_run DIR I J M K
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

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
