/* Test driver of the three-dimensional oracle built with AddressSanitizer and
   UndefinedBehaviorSanitizer: the oracle's source is compiled into this program.  Reads
   [o3_params][int64 steps][rho, ux, uy, uz, T as double[nz][ny][nx] each] from argv[1], runs the
   steps, writes [int32 status][rho, ux, uy, uz, T][f, g, history] to argv[2].  Exit status 0
   unless the files cannot be read or written (a sanitizer finding aborts the program). */
#include "../../oracle/lbm3d_oracle.c"

#include <stdio.h>

static int read_all(FILE* fp, void* dst, size_t bytes) { return fread(dst, 1, bytes, fp) == bytes; }

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  FILE* in = fopen(argv[1], "rb");
  if (!in) return 2;
  o3_params p;
  int64_t steps = 0;
  if (!read_all(in, &p, sizeof(p)) || !read_all(in, &steps, sizeof(steps))) return 2;
  const size_t n = (size_t)p.nx * (size_t)p.ny * (size_t)p.nz;
  double* fields = (double*)malloc(5 * n * sizeof(double));
  if (!fields || !read_all(in, fields, 5 * n * sizeof(double))) return 2;
  fclose(in);
  o3_state* s = o3_new(&p);
  if (!s) return 3;
  o3_init(s, fields, fields + n, fields + 2 * n, fields + 3 * n, fields + 4 * n);
  int32_t status = (int32_t)o3_step(s, (long)steps);
  if (status == 0) status = (int32_t)o3_fields(s, fields, fields + n, fields + 2 * n, fields + 3 * n, fields + 4 * n);
  double* st = (double*)malloc((19 + 7 + 2) * n * sizeof(double));
  if (!st) return 2;
  o3_get_state(s, st, st + 19 * n, st + 26 * n);
  FILE* out = fopen(argv[2], "wb");
  if (!out) return 2;
  fwrite(&status, sizeof(status), 1, out);
  fwrite(fields, sizeof(double), 5 * n, out);
  fwrite(st, sizeof(double), 28 * n, out);
  fclose(out);
  o3_free(s);
  free(st);
  free(fields);
  return 0;
}
