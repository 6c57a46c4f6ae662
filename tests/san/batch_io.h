/* Reads a chain-set batch that tests/test_sanitizers.py wrote as raw arrays
 * (one file per field, native byte order) into malloc'd buffers.  Test
 * infrastructure for the sanitizer drivers only. */
#ifndef SAN_BATCH_IO_H
#define SAN_BATCH_IO_H
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

static void *san_read(const char *dir, const char *name, long *n_bytes) {
  char path[4096];
  snprintf(path, sizeof path, "%s/%s.bin", dir, name);
  FILE *f = fopen(path, "rb");
  if (!f) {
    fprintf(stderr, "cannot open %s\n", path);
    exit(3);
  }
  fseek(f, 0, SEEK_END);
  long n = ftell(f);
  fseek(f, 0, SEEK_SET);
  void *p = malloc(n > 0 ? (size_t)n : 1);
  if (n > 0 && fread(p, 1, (size_t)n, f) != (size_t)n) {
    fprintf(stderr, "short read %s\n", path);
    exit(3);
  }
  fclose(f);
  if (n_bytes) *n_bytes = n;
  return p;
}
#endif
