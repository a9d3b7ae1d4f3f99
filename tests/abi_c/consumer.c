/* A plain C99 consumer of the C ABI in include/vemg.h: it creates a
 * handle (host-only, device -1, unless argv[2] names a HIP device), sets up
 * the mesh read from the file named by argv[1] and prints the setup's sizes,
 * the checksum of one exported array and the memory footprint.
 *
 * Mesh file (native endianness): int64 n_nodes, int64 n_tets, then
 * double xyz[n_nodes][3], int64 tets[n_tets][4], uint8 top[n_nodes]. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "vemg.h"

static void *read_block(FILE *f, size_t size) {
  void *p = malloc(size ? size : 1);
  if (!p || fread(p, 1, size, f) != size) {
    fprintf(stderr, "short mesh file\n");
    exit(2);
  }
  return p;
}

int main(int argc, char **argv) {
  if (argc != 2 && argc != 3) return 2;
  const int device = argc == 3 ? atoi(argv[2]) : -1;
  FILE *f = fopen(argv[1], "rb");
  if (!f) return 2;
  int64_t nn = 0, nt = 0;
  if (fread(&nn, sizeof nn, 1, f) != 1 || fread(&nt, sizeof nt, 1, f) != 1) return 2;
  double *xyz = read_block(f, (size_t)nn * 3 * sizeof(double));
  int64_t *tets = read_block(f, (size_t)nt * 4 * sizeof(int64_t));
  uint8_t *top = read_block(f, (size_t)nn);
  fclose(f);

  vemg_options o;
  vemg_default_options(&o);
  o.coarse_max = 16;
  vemg_solver s = NULL;
  vemg_status st = vemg_create(&o, device, NULL, &s);
  if (st != VEMG_OK) {
    printf("create %s\n", vemg_status_string(st));
    return 1;
  }
  st = vemg_setup(s, nn, xyz, nt, tets, top);
  if (st != VEMG_OK) {
    printf("setup %s: %s\n", vemg_status_string(st), vemg_last_error(s));
    return 1;
  }
  vemg_info info;
  if (vemg_get_info(s, &info) != VEMG_OK) return 1;
  size_t bytes = 0;
  if (vemg_export(s, "perm", NULL, &bytes) != VEMG_OK) return 1;
  int64_t *perm = malloc(bytes);
  if (!perm || vemg_export(s, "perm", perm, &bytes) != VEMG_OK) return 1;
  int64_t sum = 0;
  for (size_t i = 0; i < bytes / sizeof(int64_t); ++i) sum += perm[i] * (int64_t)(i + 1);
  size_t fp0 = 0, fp3 = 0;
  if (vemg_footprint(s, 0, &fp0) != VEMG_OK || vemg_footprint(s, 3, &fp3) != VEMG_OK) return 1;
  /* solving needs a device: a host-only handle refuses it before touching
   * the (here host) vectors */
  st = device < 0 ? vemg_solve(s, 1, xyz, xyz, 1e-8, 10, NULL, NULL) : VEMG_OK;
  printf("n=%lld n_top=%lld nnz_offdiag=%lld s_levels=%d abar_levels=%d perm_checksum=%lld solve=%d "
         "footprint0=%llu footprint3=%llu device_bytes=%llu\n",
         (long long)info.n, (long long)info.n_top, (long long)info.nnz_offdiag, info.s_levels,
         info.abar_levels, (long long)sum, (int)st, (unsigned long long)fp0, (unsigned long long)fp3,
         (unsigned long long)info.device_bytes);
  vemg_destroy(s);
  free(perm);
  free(xyz);
  free(tets);
  free(top);
  return 0;
}
