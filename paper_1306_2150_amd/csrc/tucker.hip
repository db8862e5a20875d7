// 3D Tucker solve (placeholder until the Tucker cross kernels land).
#include "host.h"

extern "C" lrp_status lrpoisson_solve3d(lrp_ctx *ctx, int64_t n, const int32_t rank[3],
                                        const double *U1, const double *U2,
                                        const double *U3, int64_t ld, const double *G,
                                        double eps, const lrp_opts *opts,
                                        double *U1x, double *U2x, double *U3x,
                                        int64_t ldx, double *Gx, const int32_t rmax[3],
                                        int32_t rank_out[3], lrp_info *info, void *stream) {
  return LRP_EINVAL;
}
