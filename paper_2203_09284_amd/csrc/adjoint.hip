// Gradients of the PageRank fixed point from the converged adjoint lam.
//
// With (I - dP)^T lam = dL/dx solved by pr_adjoint (the transposed pull runs
// in the sweep kernel's adjoint mode), the loss gradients are
//   dL/dp_u     = (1-d) lam_u
//   dL/dw(v->u) = d x_v / W_v (lam_u - (P^T lam)_v),
//   (P^T lam)_v = sum_{v->u'} w(v->u') lam_u' / W_v,
// since P[i][v] = w(v->i) / W_v gives dP[i][v]/dw(v->u) = [i = u]/W_v - w(v->i)/W_v^2.
// One wavefront per vertex pushes over its out-edges (pr_csr out order):
// lanes stride the list, first to form (P^T lam)_v, then to write the
// gradient of every out-edge.
#include <algorithm>

#include "device_common.h"
#include "internal.h"

using namespace fpr;
using namespace fpr::dev;

namespace {

__global__ __launch_bounds__(kBlock) void k_adj_grad(int64_t n, const uint32_t *out_ptr,
                                                     const int32_t *out_dst, const double *out_w,
                                                     const double *inv_w, const double *x,
                                                     const double *lam, double d, double *dLdp,
                                                     double *dLdw) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * kWaves;
  for (int64_t v = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); v < n; v += waves) {
    if (dLdp && lane == 0) dLdp[v] = (1.0 - d) * lam[v];
    const double iw = inv_w[v];
    if (iw == 0.0 || !dLdw) continue;
    const uint32_t b = out_ptr[v], e = out_ptr[v + 1];
    double t = 0.0;
    for (uint32_t j = b + lane; j < e; j += 64) t += (out_w ? out_w[j] : 1.0) * lam[out_dst[j]];
    t = wave_sum(t) * iw;
    const double scale = d * x[v] * iw;
    for (uint32_t j = b + lane; j < e; j += 64) dLdw[j] = scale * (lam[out_dst[j]] - t);
  }
}

}  // namespace

int fpr_adjoint_gradients(pr_graph *g, double d, const double *x, const double *lam, double *dLdp,
                          double *dLdw, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>(65535, (g->n + kWaves - 1) / kWaves);
  hipLaunchKernelGGL(k_adj_grad, dim3((unsigned)blocks), dim3(kBlock), 0, s, g->n,
                     (const uint32_t *)g->out_ptr, (const int32_t *)g->out_dst, (const double *)g->out_w,
                     (const double *)g->inv_w, x, lam, d, dLdp, dLdw);
  PR_HIP(hipGetLastError());
  return PR_OK;
}
