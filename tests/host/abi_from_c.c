/* The C ABI used from plain C99: host-side calls only (no device needed).
 * Prints the workspace size of a small problem, then the status and the
 * thread-local message of a refused call. */
#include <stdint.h>
#include <stdio.h>

#include "../../include/lp.h"

int main(void) {
  const int64_t offsets[5] = {0, 500, 1000, 1500, 2000};
  size_t bytes = 0;
  lp_status s = lp_workspace_size(LP_F64, 2000, 100, offsets, 4, 5, &bytes);
  printf("%d %zu\n", (int)s, bytes);
  const int64_t bad[4] = {0, 500, 500, 2000};   /* an empty partition */
  s = lp_workspace_size(LP_F64, 2000, 100, bad, 3, 5, &bytes);
  printf("%d %s\n", (int)s, lp_strerror(s));
  printf("%s\n", lp_last_error());
  return 0;
}
