// Forward-engine instantiations: F32, 1D chains.
#include "engine_impl.h"

namespace vmc {

hipError_t launch_engine_f32_1d(const FwdArgs &a, const BatchInfo &bi, int mode, int sh, int sl, int sa, int grid,
                              hipStream_t st) {
    return launch_engine_d<F32, 1>(a, bi, mode, sh, sl, sa, grid, st);
}

int chain_occupancy_f32_1d(int DH, int N) { return chain_occupancy_d<F32, 1>(DH, N); }

}  // namespace vmc
