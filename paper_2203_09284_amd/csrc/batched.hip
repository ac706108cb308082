// Batched personalized PageRank (k-column pull).
#include "internal.h"

extern "C" int pr_solve_batched(pr_graph *, double, double, int, int, const int32_t *, int, float *,
                                int *, double *, void *) {
  return pr_fail(PR_EINVAL, "pr_solve_batched: not available in this build");
}

extern "C" int pr_autotune_batched(pr_graph *, int, const char *, int *, void *) {
  return pr_fail(PR_EINVAL, "pr_autotune_batched: not available in this build");
}
