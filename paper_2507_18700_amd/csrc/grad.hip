// Backward pass (placeholder until the BPTT kernels land).
#include "kernels.h"

namespace vmc {

void grad_sizes(const Dims &d, int64_t ns, int *G, size_t *part_floats, size_t *gst_doubles) {
    *G = 1;
    *part_floats = 16;
    *gst_doubles = 16;
}

hipError_t launch_grad(const Dims &d, const void *BcT, const void *BgT, const float *E, const float *Hd,
                       int64_t ns, const uint8_t *cfg, const float *hcache, const float *act,
                       const double *eloc, const double *weights, double *stats, float *dcell,
                       float *dglu, float *dhead, void *dcol, float *part, int G, double *grad_st,
                       double *grad, hipStream_t st) {
    return hipErrorNotSupported;
}

}  // namespace vmc
