// Forward-engine dispatch (the kernel template is in engine_impl.h, its
// instantiations in engine_{bf16,f32}_{1,2}d.hip, compiled in parallel).
#include "engine_impl.h"

namespace vmc {

hipError_t launch_engine_bf16_1d(const FwdArgs &a, const BatchInfo &bi, int mode, int sh, int sl, int sa, int grid,
                              hipStream_t st);
hipError_t launch_engine_bf16_2d(const FwdArgs &a, const BatchInfo &bi, int mode, int sh, int sl, int sa, int grid,
                              hipStream_t st);
hipError_t launch_engine_f32_1d(const FwdArgs &a, const BatchInfo &bi, int mode, int sh, int sl, int sa, int grid,
                              hipStream_t st);
hipError_t launch_engine_f32_2d(const FwdArgs &a, const BatchInfo &bi, int mode, int sh, int sl, int sa, int grid,
                              hipStream_t st);

int chain_occupancy_bf16_1d(int DH, int N);
int chain_occupancy_bf16_2d(int DH, int N);
int chain_occupancy_f32_1d(int DH, int N);
int chain_occupancy_f32_2d(int DH, int N);

// Work-groups of the suffix-chain launch per compute unit (0: unknown).
int chain_occupancy(const Dims &d) {
    if (d.prec == VMC_BF16)
        return d.dims == 1 ? chain_occupancy_bf16_1d(d.DH, d.N) : chain_occupancy_bf16_2d(d.DH, d.N);
    return d.dims == 1 ? chain_occupancy_f32_1d(d.DH, d.N) : chain_occupancy_f32_2d(d.DH, d.N);
}

// bi: NULL, or the batch of vmc_step_batched (1D chain and sampling launches)
hipError_t launch_forward(const FwdArgs &a, int mode, int store_h, int store_lpc, int store_act, int grid,
                          hipStream_t st, const BatchInfo *bi) {
    BatchInfo none;
    none.n = 0;
    const BatchInfo &b = bi ? *bi : none;
    if (b.n > 0 && a.d.dims != 1) return hipErrorInvalidValue;
    if (a.d.prec == VMC_BF16)
        return a.d.dims == 1 ? launch_engine_bf16_1d(a, b, mode, store_h, store_lpc, store_act, grid, st)
                             : launch_engine_bf16_2d(a, b, mode, store_h, store_lpc, store_act, grid, st);
    return a.d.dims == 1 ? launch_engine_f32_1d(a, b, mode, store_h, store_lpc, store_act, grid, st)
                         : launch_engine_f32_2d(a, b, mode, store_h, store_lpc, store_act, grid, st);
}

// Rows per tile of tile class tc (0, 1 or 2, see Eng) for this model.
static int tile_rows(const Dims &d, int tc) {
#define VMC_T(PP, D) (tc == 0 ? tile_rows_d<PP, D, 0>(d.DH) : tc == 1 ? tile_rows_d<PP, D, 1>(d.DH) : tile_rows_d<PP, D, 2>(d.DH))
    if (d.prec == VMC_BF16) return d.dims == 1 ? VMC_T(BF16, 1) : VMC_T(BF16, 2);
    return d.dims == 1 ? VMC_T(F32, 1) : VMC_T(F32, 2);
#undef VMC_T
}

// Rows per tile of the sampling / log psi launches (the tuned choice) and of
// the suffix-chain launch.
int forward_tile_rows(const Dims &d) { return tile_rows(d, d.row_alt ? 2 : 0); }
int chain_tile_rows(const Dims &d) { return tile_rows(d, 1); }

// The row-tile heights a model can run with: the built-in one first, then
// the alternative where one exists.  Returns the count (1 or 2).
int row_tile_options(const Dims &d, int out[2]) {
    out[0] = tile_rows(d, 0);
    out[1] = tile_rows(d, 2);
    return out[1] != out[0] ? 2 : 1;
}

// LDS of one engine workgroup (static tiles + the tile's configurations).
size_t engine_lds(const Dims &d) {
    if (d.prec == VMC_BF16)
        return d.dims == 1 ? engine_lds_d<BF16, 1>(d.DH, d.N) : engine_lds_d<BF16, 2>(d.DH, d.N);
    return d.dims == 1 ? engine_lds_d<F32, 1>(d.DH, d.N) : engine_lds_d<F32, 2>(d.DH, d.N);
}

// Row length of the staged forward cell weights [3*DH][kpx] for this model.
int engine_kpx(const Dims &d) {
    const int ks = d.prec == VMC_BF16 ? 32 : 16;
    const int khb = cround(d.DH, ks);
    return ((d.dims == 1 ? 1 : 2) * (khb / ks) + 1) * ks;
}

}  // namespace vmc
