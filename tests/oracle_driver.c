/*
 * Test-only driver: runs the CPU oracle on one event read from a binary
 * file and prints its item counts.  Built by tests/test_oracle_sanitized.py
 * with gcc and -fsanitize=address,undefined to check the oracle's memory
 * handling; it is not part of the library.
 *
 * File layout (little endian): orc_config (raw struct), uint32 n_hits,
 * float x[n], float y[n], float z[n], int16 layer[n].
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "../oracle/pxt_oracle.c"

int main(int argc, char** argv) {
  if (argc != 2) return 2;
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 3;
  orc_config cfg;
  uint32_t n = 0;
  if (fread(&cfg, sizeof(cfg), 1, f) != 1 || fread(&n, 4, 1, f) != 1) return 4;
  float* x = (float*)malloc(4ull * n + 4);
  float* y = (float*)malloc(4ull * n + 4);
  float* z = (float*)malloc(4ull * n + 4);
  int16_t* l = (int16_t*)malloc(2ull * n + 2);
  if (fread(x, 4, n, f) != n || fread(y, 4, n, f) != n || fread(z, 4, n, f) != n ||
      fread(l, 2, n, f) != n)
    return 5;
  fclose(f);
  orc_result* r = orc_run(&cfg, n, x, y, z, l);
  if (!r) return 6;
  printf("%d", orc_status(r));
  for (int i = 0; i < ORC_NITEMS; ++i) printf(" %llu", (unsigned long long)orc_count(r, i));
  printf("\n");
  orc_free(r);
  free(x); free(y); free(z); free(l);
  return 0;
}
