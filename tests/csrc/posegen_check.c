/* Drives the synthetic pose generator (synth/csrc/posegen.c) outside Python so that
 * it can be built with AddressSanitizer / UndefinedBehaviorSanitizer: each pose gets
 * a work buffer and output arrays of exactly the documented sizes, and the program
 * prints an FNV-1a 64 digest of all outputs, which the test compares with the
 * digest of the same poses generated through the normal build.
 * usage: posegen_check seed stream mode lim0 lim1 lim2 lim3 pose0 n_poses */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void cfgen_pose_sizes(uint64_t seed, uint64_t stream, int64_t pose0, int64_t n_poses, int mode,
                      const int32_t *lim, int32_t *n_lig_out, int32_t *n_pock_out);
size_t cfgen_work_bytes(int n);
double cfgen_pose(uint64_t seed, uint64_t stream, int64_t pose, int n_lig, int n_pock, double r_in, double r_out,
                  int jam, void *work, int32_t *xyz, float *feat, uint8_t *is_lig);

static uint64_t fnv(uint64_t h, const void *p, size_t n) {
  const unsigned char *b = (const unsigned char *)p;
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 0x100000001b3ULL;
  }
  return h;
}

int main(int argc, char **argv) {
  if (argc != 10) return 2;
  const uint64_t seed = strtoull(argv[1], 0, 10), stream = strtoull(argv[2], 0, 10);
  const int mode = atoi(argv[3]);
  const int32_t lim[4] = {atoi(argv[4]), atoi(argv[5]), atoi(argv[6]), atoi(argv[7])};
  const int64_t pose0 = atoll(argv[8]), np = atoll(argv[9]);
  int32_t *nl = malloc(sizeof(int32_t) * np), *npk = malloc(sizeof(int32_t) * np);
  cfgen_pose_sizes(seed, stream, pose0, np, mode, lim, nl, npk);
  uint64_t h = 0xcbf29ce484222325ULL;
  for (int64_t p = 0; p < np; ++p) {
    const int n = nl[p] + npk[p];
    void *work = malloc(cfgen_work_bytes(n));
    int32_t *xyz = malloc(sizeof(int32_t) * 3 * n);
    float *feat = malloc(sizeof(float) * 19 * n);
    uint8_t *lig = malloc(n);
    if (cfgen_pose(seed, stream, pose0 + p, nl[p], npk[p], 4.0, 10.0, 2000, work, xyz, feat, lig) < 0) return 3;
    h = fnv(h, xyz, sizeof(int32_t) * 3 * n);
    h = fnv(h, feat, sizeof(float) * 19 * n);
    h = fnv(h, lig, n);
    free(work);
    free(xyz);
    free(feat);
    free(lig);
  }
  free(nl);
  free(npk);
  printf("%016llx\n", (unsigned long long)h);
  return 0;
}
