/* Host-only use of the C ABI from plain C99: the headers compile as C, the
 * library links, and calls that need no device behave as documented
 * (descriptor, validation, sizing, argument errors before any launch). */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "sa.h"
#include "sa_runtime.h"
#include "sa_workload.h"

static int failures = 0;
#define CHECK(cond)                                              \
  do {                                                           \
    if (!(cond)) {                                               \
      fprintf(stderr, "%s:%d: %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                \
    }                                                            \
  } while (0)

int main(void) {
  sa_arch a;
  CHECK(sa_arch_gfx950(&a) == SA_OK);
  CHECK(a.wave_size == 64 && a.max_threads_per_block == 1024);
  CHECK(sa_arch_validate(&a) == SA_OK);
  sa_arch bad = a;
  bad.wave_size = 48;
  CHECK(sa_arch_validate(&bad) != SA_OK);
  CHECK(strcmp(sa_status_string(SA_ERR_ARG), "SA_ERR_ARG") == 0);

  /* sizing */
  CHECK(sa_workspace_bytes(10, 100000, 8, 0) > 0);
  CHECK(sa_workspace_bytes(10, 0, 8, 0) == 0);
  CHECK(sa_product_workspace_bytes(3, 16384, 8) > 0);

  /* argument errors return before any launch */
  sa_variants v;
  memset(&v, 0, sizeof v);
  sa_configs c;
  memset(&c, 0, sizeof c);
  CHECK(sa_occupancy(&a, &v, &c, 1, 1, NULL, NULL) != SA_OK);
  CHECK(sa_score(&a, NULL, &c, 1, 1, NULL, NULL, 8, NULL, NULL, NULL, NULL, 0, NULL) == SA_ERR_ARG);
  CHECK(sa_topk(NULL, NULL, 1, 1, 8, NULL, NULL, NULL, 0, NULL) == SA_ERR_ARG);
  CHECK(sa_headroom(&a, NULL, NULL, 4, NULL, NULL, NULL) == SA_ERR_ARG);
  CHECK(sa_score_product(&a, &v, 1, NULL, NULL, NULL, 8, NULL, NULL, NULL, 0, NULL) != SA_OK);
  CHECK(sa_last_error()[0] != '\0');

  /* the measured families' launch rules */
  CHECK(sa_rt_grid(SA_RT_MATVEC, 1680, 64, 1, 256) == 54);
  CHECK(sa_rt_grid(SA_RT_REDUCE, 100, 64, 9, 256) == -1);
  CHECK(sa_rt_cpi(SA_CPI_FP, 0, NULL, NULL, NULL, NULL) == -1);
  CHECK(sa_gen_configs(1, 0, -1, 256, NULL, NULL, NULL, NULL, NULL) == -1);

  if (failures) return 1;
  printf("ok\n");
  return 0;
}
