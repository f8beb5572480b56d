/* Prints sizeof and field offsets of the option and job structs of lp.h, so the
 * Python binding's ctypes layouts can be checked against the C compiler's. */
#include <stddef.h>
#include <stdio.h>

#include "lp.h"

#define F(T, f) printf(#T "." #f " %zu\n", offsetof(T, f))

int main(void) {
  printf("lp_run_opts %zu\n", sizeof(lp_run_opts));
  F(lp_run_opts, U_ref); F(lp_run_opts, sin_hist); F(lp_run_opts, signs_out);
  F(lp_run_opts, z0_orthonormal); F(lp_run_opts, use_graph); F(lp_run_opts, time_local);
  F(lp_run_opts, split_rounds); F(lp_run_opts, k_ref); F(lp_run_opts, rho_out); F(lp_run_opts, seed);
  printf("lp_solve_opts %zu\n", sizeof(lp_solve_opts));
  F(lp_solve_opts, p0); F(lp_solve_opts, target); F(lp_solve_opts, max_rounds);
  F(lp_solve_opts, z0_orthonormal); F(lp_solve_opts, p_used); F(lp_solve_opts, change_out);
  F(lp_solve_opts, seed);
  printf("lp_run_stats %zu\n", sizeof(lp_run_stats));
  printf("lp_solve_stats %zu\n", sizeof(lp_solve_stats));
  printf("lp_tuning %zu\n", sizeof(lp_tuning));
  F(lp_tuning, local_kernel); F(lp_tuning, chunk_rows); F(lp_tuning, cached_loads);
  F(lp_tuning, split_operands);
  printf("lp_job %zu\n", sizeof(lp_job));
  F(lp_job, A); F(lp_job, dtype); F(lp_job, n); F(lp_job, d); F(lp_job, lda); F(lp_job, offsets);
  F(lp_job, m); F(lp_job, k); F(lp_job, p0); F(lp_job, mode); F(lp_job, target);
  F(lp_job, max_rounds); F(lp_job, Y0); F(lp_job, Z_out); F(lp_job, stream); F(lp_job, gen_seed);
  F(lp_job, gen_gap); F(lp_job, gen_decay); F(lp_job, single_bf16);
  printf("lp_job_result %zu\n", sizeof(lp_job_result));
  return 0;
}
