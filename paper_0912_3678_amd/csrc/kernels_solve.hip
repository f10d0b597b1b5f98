// Solve kernels of the partition method (gfx950): the kernels and launchers
// around the bodies of kernels_solve.h.
#include "kernels_solve.h"

namespace pf {
namespace {

template <int KIND, int M, int KC, typename T, bool ADD>
__global__ __launch_bounds__(WG) void k_fwd(SolveArgs a)
{
    __shared__ __align__(16) T lds[fwd_lds<M, KC, T>()];
    fwd_body<KIND, M, KC, T, ADD>(a, blockIdx.x, blockIdx.y, threadIdx.x, lds);
}
template <int KIND, int M, int KC, typename T, bool ADD>
__global__ __launch_bounds__(WG) void kb_fwd(const SolveArgs *tab, const int4 *work)
{
    __shared__ __align__(16) T lds[fwd_lds<M, KC, T>()];
    const int4 w = work[blockIdx.x];
    const SolveArgs a = tab[w.x];
    fwd_body<KIND, M, KC, T, ADD>(a, w.y, w.z, threadIdx.x, lds);
}
template <int KIND, int M, int KC, typename T>
__global__ __launch_bounds__(WG) void k_bwd(SolveArgs a)
{
    __shared__ __align__(16) T lds[bwd_lds<M, KC, T>()];
    bwd_body<KIND, M, KC, T>(a, blockIdx.x, blockIdx.y, threadIdx.x, lds);
}
template <int KIND, int M, int KC, typename T>
__global__ __launch_bounds__(WG) void kb_bwd(const SolveArgs *tab, const int4 *work)
{
    __shared__ __align__(16) T lds[bwd_lds<M, KC, T>()];
    const int4 w = work[blockIdx.x];
    const SolveArgs a = tab[w.x];
    bwd_body<KIND, M, KC, T>(a, w.y, w.z, threadIdx.x, lds);
}

}  // namespace

int groups_per_wg(int M) { return WG / M; }
int rhs_chunk(int nrhs, int64_t parts)
{
    return nrhs == 1 ? 1 : (nrhs <= 4 || parts < kWideParts) ? 4 : 8;
}

template <int KIND, bool FWD>
static hipError_t launch_solve(int M, bool f32, const SolveArgs &a, hipStream_t s)
{
    if (solve_tiled(M, f32)) return launch_solvet(M, KIND, FWD, KIND == 0 && a.Fadd, f32, a, s);
    return dispatch_M(M, [&](auto mc) {
        constexpr int MV = decltype(mc)::value;
        return dispatch_KC(rhs_chunk(a.nrhs, a.p), [&](auto kcc) {
            constexpr int KC = decltype(kcc)::value;
            const dim3 grid = grid_for(MV, a.p, a.nrhs, KC);
            const bool add = KIND == 0 && a.Fadd;
            if (FWD) {
                if (add) {
                    if (f32) launch_k((k_fwd<KIND, MV, KC, float, true>), grid, dim3(WG), s, a);
                    else launch_k((k_fwd<KIND, MV, KC, double, true>), grid, dim3(WG), s, a);
                } else {
                    if (f32) launch_k((k_fwd<KIND, MV, KC, float, false>), grid, dim3(WG), s, a);
                    else launch_k((k_fwd<KIND, MV, KC, double, false>), grid, dim3(WG), s, a);
                }
            } else {
                if (f32) launch_k((k_bwd<KIND, MV, KC, float>), grid, dim3(WG), s, a);
                else launch_k((k_bwd<KIND, MV, KC, double>), grid, dim3(WG), s, a);
            }
            return hipGetLastError();
        });
    });
}

hipError_t launch_btri_fwd(int M, bool f32, const SolveArgs &a, hipStream_t s)
{
    return launch_solve<0, true>(M, f32, a, s);
}
hipError_t launch_btri_bwd(int M, bool f32, const SolveArgs &a, hipStream_t s)
{
    return launch_solve<0, false>(M, f32, a, s);
}
hipError_t launch_babd_fwd(int M, bool f32, const SolveArgs &a, hipStream_t s)
{
    return launch_solve<1, true>(M, f32, a, s);
}
hipError_t launch_babd_bwd(int M, bool f32, const SolveArgs &a, hipStream_t s)
{
    return launch_solve<1, false>(M, f32, a, s);
}

template <int KIND>
static hipError_t launch_solve_batch_k(bool fwd, int M, bool f32, bool add, int KC,
                                       const SolveArgs *tab, const int4 *work, int nwg,
                                       hipStream_t s)
{
    return dispatch_M(M, [&](auto mc) {
        constexpr int MV = decltype(mc)::value;
        return dispatch_KC(KC, [&](auto kcc) {
            constexpr int K = decltype(kcc)::value;
            const dim3 grid(nwg);
            if (fwd) {
                if (KIND == 0 && add) {
                    if (f32) launch_k((kb_fwd<KIND, MV, K, float, true>), grid, dim3(WG), s, tab, work);
                    else launch_k((kb_fwd<KIND, MV, K, double, true>), grid, dim3(WG), s, tab, work);
                } else {
                    if (f32) launch_k((kb_fwd<KIND, MV, K, float, false>), grid, dim3(WG), s, tab, work);
                    else launch_k((kb_fwd<KIND, MV, K, double, false>), grid, dim3(WG), s, tab, work);
                }
            } else {
                if (f32) launch_k((kb_bwd<KIND, MV, K, float>), grid, dim3(WG), s, tab, work);
                else launch_k((kb_bwd<KIND, MV, K, double>), grid, dim3(WG), s, tab, work);
            }
            return hipGetLastError();
        });
    });
}

hipError_t launch_solve_batch(int kind, bool fwd, int M, bool f32, bool add, int KC,
                              const SolveArgs *tab, const int4 *work, int nwg, hipStream_t s)
{
    if (nwg <= 0) return hipSuccess;
    if (solve_tiled(M, f32)) return launch_solvet_batch(M, kind, fwd, add, f32, KC, tab, work, nwg, s);
    return kind == 0 ? launch_solve_batch_k<0>(fwd, M, f32, add, KC, tab, work, nwg, s)
                     : launch_solve_batch_k<1>(fwd, M, f32, add, KC, tab, work, nwg, s);
}

}  // namespace pf
