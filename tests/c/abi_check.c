/* Plain-C client of libdop: compiles include/dop.h as C99, prints the layout
 * of dop_problem, and exercises the host-only paths of the ABI (status
 * strings, argument validation, workspace sizes) without touching a GPU.
 * Output: one "key value" pair per line, read by tests/test_c_abi_cpu.py. */
#include <stddef.h>
#include <stdio.h>
#include <string.h>

#include "dop.h"

static dop_problem problem(int ny, int n, int my, int m, const double *lam, const double *nidx) {
  dop_problem p;
  memset(&p, 0, sizeof(p));
  p.n = n;
  p.m = m;
  p.ny = ny;
  p.my = my;
  p.dx = 0.5;
  p.z = 1000.0;
  p.n_lambda = 1;
  p.lambda = lam;
  p.n_index = nidx;
  p.weight = NULL;
  p.out_mode = DOP_OUT_CROP;
  p.flags = 0;
  p.upsample = 0;
  return p;
}

int main(void) {
  const double lam[1] = {0.55}, nidx[1] = {1.46};
  size_t bytes = 0;
  dop_status st;
  dop_problem p;

  printf("sizeof %zu\n", sizeof(dop_problem));
  printf("off_n %zu\noff_m %zu\noff_dx %zu\noff_z %zu\noff_n_lambda %zu\n", offsetof(dop_problem, n),
         offsetof(dop_problem, m), offsetof(dop_problem, dx), offsetof(dop_problem, z),
         offsetof(dop_problem, n_lambda));
  printf("off_lambda %zu\noff_n_index %zu\noff_weight %zu\noff_out_mode %zu\noff_flags %zu\n",
         offsetof(dop_problem, lambda), offsetof(dop_problem, n_index),
         offsetof(dop_problem, weight), offsetof(dop_problem, out_mode),
         offsetof(dop_problem, flags));
  printf("off_upsample %zu\noff_ny %zu\noff_my %zu\n", offsetof(dop_problem, upsample),
         offsetof(dop_problem, ny), offsetof(dop_problem, my));
  printf("status_ok %s\nstatus_unsupported %s\n", dop_status_string(DOP_OK),
         dop_status_string(DOP_ERR_UNSUPPORTED));

  /* square power of two: 8 M (M + 16) bytes */
  p = problem(0, 512, 0, 1024, lam, nidx);
  st = dop_workspace_size(NULL, &p, DOP_OP_PSF, &bytes);
  printf("ws_1024 %d %zu\n", (int)st, bytes);
  /* the paper's rectangular grid: 8 My (Mx + 16) bytes */
  p = problem(64320, 42880, 128640, 85760, lam, nidx);
  st = dop_workspace_size(NULL, &p, DOP_OP_PSF, &bytes);
  printf("ws_paper %d %zu\n", (int)st, bytes);
  /* a grid with no plan */
  p = problem(0, 500, 0, 1000, lam, nidx);
  st = dop_workspace_size(NULL, &p, DOP_OP_PSF, &bytes);
  printf("ws_1000 %d\n", (int)st);
  printf("err_1000_mentions_paper_grid %d\n", strstr(dop_last_error(), "128640x85760") != NULL);
  /* DOE larger than the grid */
  p = problem(0, 2048, 0, 1024, lam, nidx);
  st = dop_workspace_size(NULL, &p, DOP_OP_PSF, &bytes);
  printf("ws_n_gt_m %d\n", (int)st);
  /* a NULL context is rejected before any device access */
  st = dop_psf(NULL, &p, NULL, NULL, NULL, NULL, NULL, 0, NULL);
  printf("psf_null_ctx %d\n", (int)st);
  return 0;
}
