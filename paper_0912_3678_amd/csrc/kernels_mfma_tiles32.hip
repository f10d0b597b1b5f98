// FP32 instantiation of the matrix-core kernels of kernels_mfma_tiles.h
// (v_mfma_f32_16x16x4f32 with FP32 accumulation): the finest level of
// PF_FP32_IR factorizations with 16 x 16 and 32 x 32 blocks and the sweeps
// over those FP32 factors.  Reached through the launchers of
// kernels_mfma_tiles.hip.
#include "kernels_mfma_tiles.h"

namespace pf {
namespace fp32 {

hipError_t launch_mfma32_factor(const LevelArgs &a, hipStream_t s)
{
    return Tiles<float>::mfma32_factor(a, s);
}
hipError_t launch_mfma32_factor_batch(bool add, const LevelArgs *tab, const int4 *work, int nwg,
                                      hipStream_t s)
{
    return Tiles<float>::mfma32_factor_batch(add, tab, work, nwg, s);
}
hipError_t launch_mfma16_factor(const LevelArgs &a, const SolveArgs *sv, hipStream_t s)
{
    return Tiles<float>::mfma16_factor(a, sv, s);
}
hipError_t launch_mfma16_factor_batch(bool add, const LevelArgs *tab, const int4 *work, int nwg,
                                      hipStream_t s)
{
    return Tiles<float>::mfma16_factor_batch(add, tab, work, nwg, s);
}
hipError_t launch_mfma_babd16_factor(const LevelArgs &a, const SolveArgs *sv, hipStream_t s)
{
    return Tiles<float>::babd16_factor(a, sv, s);
}
hipError_t launch_mfma_babd16_factor_batch(const LevelArgs *tab, const int4 *work, int nwg,
                                           hipStream_t s)
{
    return Tiles<float>::babd16_factor_batch(tab, work, nwg, s);
}
hipError_t launch_solvet(int M, int kind, bool fwd, bool add, const SolveArgs &a, hipStream_t s)
{
    return Tiles<float>::solvet(M, kind, fwd, add, a, s);
}
hipError_t launch_solvet_batch(int M, int kind, bool fwd, bool add, int cols, const SolveArgs *tab,
                               const int4 *work, int nwg, hipStream_t s)
{
    return Tiles<float>::solvet_batch(M, kind, fwd, add, cols, tab, work, nwg, s);
}

}  // namespace fp32
}  // namespace pf
