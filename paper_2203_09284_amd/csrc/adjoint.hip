// Adjoint of the PageRank fixed point.
#include "internal.h"

extern "C" int pr_adjoint(pr_graph *, double, const double *, const double *, double, int, double *,
                          double *, double *, int *, double *, void *) {
  return pr_fail(PR_EINVAL, "pr_adjoint: not available in this build");
}
