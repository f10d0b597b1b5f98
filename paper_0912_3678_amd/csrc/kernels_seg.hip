// Partition-method factor kernels, segment lane mapping (gfx950): the
// kernels and launchers around the bodies of kernels_seg.h.
#include "kernels_seg.h"

namespace pf {
namespace {

// ---- kernels ----------------------------------------------------------------
template <int M, int E, typename T, bool ADD, bool RHS>
__global__ __launch_bounds__(WG) void k_btri_seg(LevelArgs a, SolveArgs sv)
{
    __shared__ __align__(16) T lds[seg_btri_lds<M, E, T, RHS>()];
    btri_seg_body<M, E, T, ADD, RHS>(a, sv, blockIdx.x, threadIdx.x, lds);
}
template <int M, int E, typename T, bool RHS>
__global__ __launch_bounds__(WG) void k_babd_seg(LevelArgs a, SolveArgs sv)
{
    __shared__ __align__(16) T lds[seg_babd_lds<M, E, T, RHS>()];
    babd_seg_body<M, E, T, RHS>(a, sv, blockIdx.x, threadIdx.x, lds);
}
// batched (factor only): workgroup w serves table entry work[w].x, partition
// block work[w].y
template <int M, int E, typename T, bool ADD>
__global__ __launch_bounds__(WG) void kb_btri_seg(const LevelArgs *tab, const int4 *work)
{
    __shared__ __align__(16) T lds[seg_btri_lds<M, E, T, false>()];
    const int4 w = work[blockIdx.x];
    const LevelArgs a = tab[w.x];
    btri_seg_body<M, E, T, ADD, false>(a, SolveArgs{}, w.y, threadIdx.x, lds);
}
template <int M, int E, typename T>
__global__ __launch_bounds__(WG) void kb_babd_seg(const LevelArgs *tab, const int4 *work)
{
    __shared__ __align__(16) T lds[seg_babd_lds<M, E, T, false>()];
    const int4 w = work[blockIdx.x];
    const LevelArgs a = tab[w.x];
    babd_seg_body<M, E, T, false>(a, SolveArgs{}, w.y, threadIdx.x, lds);
}

// the (M, E) pairs with kernels
template <typename F>
hipError_t dispatch_ME(int M, int E, F &&f)
{
    using std::integral_constant;
    if (M == 1 && E == 1) return f(integral_constant<int, 1>{}, integral_constant<int, 1>{});
    if (M == 2 && E == 1) return f(integral_constant<int, 2>{}, integral_constant<int, 1>{});
    if (M == 4 && E == 1) return f(integral_constant<int, 4>{}, integral_constant<int, 1>{});
    if (M == 8 && E == 1) return f(integral_constant<int, 8>{}, integral_constant<int, 1>{});
    if (M == 8 && E == 2) return f(integral_constant<int, 8>{}, integral_constant<int, 2>{});
    if (M == 8 && E == 4) return f(integral_constant<int, 8>{}, integral_constant<int, 4>{});
    if (M == 16 && E == 4) return f(integral_constant<int, 16>{}, integral_constant<int, 4>{});
    return hipErrorInvalidValue;
}

}  // namespace

bool seg_ok(int M, int E)
{
    return (M == 1 && E == 1) || (M == 2 && E == 1) || (M == 4 && E == 1) || (M == 8 && E == 1) ||
           (M == 8 && E == 2) || (M == 8 && E == 4) || (M == 16 && E == 4);
}

int seg_partitions_per_wg(int M, int E) { return WG / (M * M / E); }

hipError_t launch_seg_factor(int kind, int M, int E, bool f32, const LevelArgs &a,
                             const SolveArgs *sv, hipStream_t s)
{
    if (sv && (sv->nrhs < 1 || sv->nrhs > M)) return hipErrorInvalidValue;
    return dispatch_ME(M, E, [&](auto mc, auto ec) {
        constexpr int MV = decltype(mc)::value, EV = decltype(ec)::value;
        const int ppw = seg_partitions_per_wg(MV, EV);
        const dim3 grid((unsigned)((a.p + ppw - 1) / ppw));
        const SolveArgs none{};
        const SolveArgs &v = sv ? *sv : none;
        if (kind == 1) {
            if (sv) {
                if (f32) launch_k((k_babd_seg<MV, EV, float, true>), grid, dim3(WG), s, a, v);
                else launch_k((k_babd_seg<MV, EV, double, true>), grid, dim3(WG), s, a, v);
            } else {
                if (f32) launch_k((k_babd_seg<MV, EV, float, false>), grid, dim3(WG), s, a, v);
                else launch_k((k_babd_seg<MV, EV, double, false>), grid, dim3(WG), s, a, v);
            }
        } else if (a.Dadd) {
            if (sv) {
                if (f32) launch_k((k_btri_seg<MV, EV, float, true, true>), grid, dim3(WG), s, a, v);
                else launch_k((k_btri_seg<MV, EV, double, true, true>), grid, dim3(WG), s, a, v);
            } else {
                if (f32) launch_k((k_btri_seg<MV, EV, float, true, false>), grid, dim3(WG), s, a, v);
                else launch_k((k_btri_seg<MV, EV, double, true, false>), grid, dim3(WG), s, a, v);
            }
        } else {
            if (sv) {
                if (f32) launch_k((k_btri_seg<MV, EV, float, false, true>), grid, dim3(WG), s, a, v);
                else launch_k((k_btri_seg<MV, EV, double, false, true>), grid, dim3(WG), s, a, v);
            } else {
                if (f32) launch_k((k_btri_seg<MV, EV, float, false, false>), grid, dim3(WG), s, a, v);
                else launch_k((k_btri_seg<MV, EV, double, false, false>), grid, dim3(WG), s, a, v);
            }
        }
        return hipGetLastError();
    });
}

hipError_t launch_seg_factor_batch(int kind, int M, int E, bool f32, bool add, const LevelArgs *tab,
                                   const int4 *work, int nwg, hipStream_t s)
{
    if (nwg <= 0) return hipSuccess;
    return dispatch_ME(M, E, [&](auto mc, auto ec) {
        constexpr int MV = decltype(mc)::value, EV = decltype(ec)::value;
        const dim3 grid(nwg);
        if (kind == 1) {
            if (f32) launch_k((kb_babd_seg<MV, EV, float>), grid, dim3(WG), s, tab, work);
            else launch_k((kb_babd_seg<MV, EV, double>), grid, dim3(WG), s, tab, work);
        } else if (add) {
            if (f32) launch_k((kb_btri_seg<MV, EV, float, true>), grid, dim3(WG), s, tab, work);
            else launch_k((kb_btri_seg<MV, EV, double, true>), grid, dim3(WG), s, tab, work);
        } else {
            if (f32) launch_k((kb_btri_seg<MV, EV, float, false>), grid, dim3(WG), s, tab, work);
            else launch_k((kb_btri_seg<MV, EV, double, false>), grid, dim3(WG), s, tab, work);
        }
        return hipGetLastError();
    });
}

}  // namespace pf
