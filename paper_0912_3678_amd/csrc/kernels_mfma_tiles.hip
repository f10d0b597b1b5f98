// FP64 instantiation of the matrix-core kernels of kernels_mfma_tiles.h and
// the public launchers, which hand FP32 work to kernels_mfma_tiles32.hip.
#include "kernels_mfma_tiles.h"

namespace pf {

hipError_t launch_mfma32_factor(const LevelArgs &a, bool f32, hipStream_t s)
{
    return f32 ? fp32::launch_mfma32_factor(a, s) : Tiles<double>::mfma32_factor(a, s);
}
hipError_t launch_mfma32_factor_batch(bool add, bool f32, const LevelArgs *tab, const int4 *work,
                                      int nwg, hipStream_t s)
{
    return f32 ? fp32::launch_mfma32_factor_batch(add, tab, work, nwg, s)
               : Tiles<double>::mfma32_factor_batch(add, tab, work, nwg, s);
}
hipError_t launch_mfma16_factor(const LevelArgs &a, const SolveArgs *sv, bool f32, hipStream_t s)
{
    return f32 ? fp32::launch_mfma16_factor(a, sv, s) : Tiles<double>::mfma16_factor(a, sv, s);
}
hipError_t launch_mfma16_factor_batch(bool add, bool f32, const LevelArgs *tab, const int4 *work,
                                      int nwg, hipStream_t s)
{
    return f32 ? fp32::launch_mfma16_factor_batch(add, tab, work, nwg, s)
               : Tiles<double>::mfma16_factor_batch(add, tab, work, nwg, s);
}
hipError_t launch_mfma_babd16_factor(const LevelArgs &a, const SolveArgs *sv, bool f32, hipStream_t s)
{
    return f32 ? fp32::launch_mfma_babd16_factor(a, sv, s) : Tiles<double>::babd16_factor(a, sv, s);
}
hipError_t launch_mfma_babd16_factor_batch(bool f32, const LevelArgs *tab, const int4 *work, int nwg,
                                           hipStream_t s)
{
    return f32 ? fp32::launch_mfma_babd16_factor_batch(tab, work, nwg, s)
               : Tiles<double>::babd16_factor_batch(tab, work, nwg, s);
}

// columns a workgroup of the tiled solve kernels covers: 16 or 32, and 64
// in launches of at least kWideParts partitions (the factor blocks of a block
// row then read once for up to 64 columns) for 16 x 16 blocks, FP32 factors
// of 32 x 32 blocks and, with FP64 32 x 32 factors, block tridiagonal sweeps
// of one right-hand side (wide64: not a bidiagonal level, whose sweeps would
// not fit the registers, nor a forward sweep that adds a second one)
int solve32_cols(int M, bool f32, bool wide64, int nrhs, int64_t parts)
{
    if (nrhs <= 16) return 16;
    if (nrhs <= 32 || parts < kWideParts) return 32;
    return (M == 16 || f32 || wide64) ? 64 : 32;
}

hipError_t launch_solvet(int M, int kind, bool fwd, bool add, bool f32, const SolveArgs &a,
                         hipStream_t s)
{
    return f32 ? fp32::launch_solvet(M, kind, fwd, add, a, s)
               : Tiles<double>::solvet(M, kind, fwd, add, a, s);
}
hipError_t launch_solvet_batch(int M, int kind, bool fwd, bool add, bool f32, int cols,
                               const SolveArgs *tab, const int4 *work, int nwg, hipStream_t s)
{
    return f32 ? fp32::launch_solvet_batch(M, kind, fwd, add, cols, tab, work, nwg, s)
               : Tiles<double>::solvet_batch(M, kind, fwd, add, cols, tab, work, nwg, s);
}

}  // namespace pf
