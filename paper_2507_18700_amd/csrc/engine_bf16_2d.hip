// Forward-engine instantiations: BF16, 2D chains.
#include "engine_impl.h"

namespace vmc {

hipError_t launch_engine_bf16_2d(const FwdArgs &a, const BatchInfo &bi, int mode, int sh, int sl, int sa, int grid,
                              hipStream_t st) {
    return launch_engine_d<BF16, 2>(a, bi, mode, sh, sl, sa, grid, st);
}

int chain_occupancy_bf16_2d(int DH, int N) { return chain_occupancy_d<BF16, 2>(DH, N); }

}  // namespace vmc
