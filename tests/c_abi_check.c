/* The C-ABI used from plain C (C99, no C++): a host-only mesh (device -1)
 * of 3 x 3 periodic squares is uploaded, precomputed in FP64 and inspected;
 * error paths return their documented codes.  Prints "ok" on success. */
#include <stdio.h>
#include <string.h>

#include "uweno.h"

#define CHECK(cond, what)                                          \
  do {                                                             \
    if (!(cond)) {                                                 \
      printf("FAIL %s: %s\n", what, uw_last_error());              \
      return 1;                                                    \
    }                                                              \
  } while (0)

int main(void) {
  /* 4 x 4 nodes on [0,3]^2; the last row and column duplicate the first */
  double xy[32];
  int32_t node_id[16];
  for (int j = 0; j < 4; ++j)
    for (int i = 0; i < 4; ++i) {
      xy[2 * (4 * j + i)] = i;
      xy[2 * (4 * j + i) + 1] = j;
      node_id[4 * j + i] = (j % 3) * 3 + (i % 3);
    }
  int32_t cells[36];
  for (int j = 0; j < 3; ++j)
    for (int i = 0; i < 3; ++i) {
      int32_t* c = cells + 4 * (3 * j + i);
      c[0] = 4 * j + i;
      c[1] = 4 * j + i + 1;
      c[2] = 4 * (j + 1) + i + 1;
      c[3] = 4 * (j + 1) + i;
    }
  uw_mesh_desc d;
  memset(&d, 0, sizeof d);
  d.n_nodes = 16;
  d.node_xy = xy;
  d.n_cells = 9;
  d.cell_nodes = cells;
  d.node_id = node_id;
  d.bc = UW_BC_PERIODIC;
  uw_mesh* m = NULL;
  CHECK(uw_mesh_upload(&d, -1, &m) == UW_OK && m != NULL, "upload");
  int64_t n = 0, nq = 0, nfaces = 0;
  int32_t new_of_old[9];
  CHECK(uw_mesh_info(m, &n, &nq, &nfaces, new_of_old) == UW_OK, "info");
  CHECK(n == 9 && nq == 9 && nfaces == 18, "sizes");
  uw_scheme s = {1e-14, 3.0, 1e-3, 1, UW_D_PER_GP, UW_WENO, UW_CONSERVED};
  uw_diag diag;
  CHECK(uw_precompute_geometry(m, &s, &diag) == UW_OK, "precompute");
  CHECK(diag.sum_dev < 1e-12, "sum of the linear weights");
  double gamma[9 * 8 * 12];
  CHECK(uw_mesh_table(m, 0, gamma) == UW_OK, "table");
  for (int c = 0; c < 9; ++c)
    for (int g = 0; g < 8; ++g) {
      double sum = 0.0;
      for (int j = 0; j < 12; ++j) sum += gamma[(c * 8 + g) * 12 + j];
      CHECK(sum > 1.0 - 1e-12 && sum < 1.0 + 1e-12, "weights sum to 1");
    }
  /* a host-only mesh has no device state */
  uw_physics p = {UW_EULER, 1.0, 1.0, 1.4, UW_FP64};
  double W[36], L[36];
  CHECK(uw_residual(m, &p, W, L, NULL) == UW_ESTATE, "residual on a host-only mesh");
  /* documented argument errors */
  s.theta = 1.0;
  CHECK(uw_precompute_geometry(m, &s, NULL) == UW_EINVAL, "theta = 1");
  CHECK(uw_mesh_upload(NULL, -1, &m) == UW_EINVAL, "null description");
  uw_mesh_destroy(m);
  printf("ok\n");
  return 0;
}
