// In-place Gauss-Jordan inversion of the pivot blocks, segment lane mapping
// (gfx950, wave64), shared by the factor kernels.
//
// One partition is owned by M*M/E lanes; lane (r, g) holds the E entries
// (r, g*E .. g*E+E-1) of the tableau, the M lanes of one segment column g
// being consecutive.  Step j of the inversion exchanges unknown j with the
// equation of its pivot row p_j (row partial pivoting inside the block, the
// pivot ranked by pivot_key): with v = b(p_j, j) the tableau becomes
// b(p_j, j) = 1/v, b(p_j, l) = b(p_j, l)/v, b(i, j) = -b(i, j)/v and
// b(i, l) = b(i, l) - b(i, j) b(p_j, l)/v.  After the M steps entry (r, c) of
// the tableau is entry (sigma(r), p_c) of the inverse, sigma(r) being the step
// at which row r was the pivot.  The pivot search of step j+1 is a DPP
// reduction in the segment column holding column j+1, right after step j's
// update, so a step costs one LDS round trip.
#pragma once
#include "kernels_common.h"

namespace pf {
namespace {

template <int M, int E> constexpr int seg_lanes() { return M * M / E; }

// E consecutive T in LDS <-> registers (16- or 8-byte accesses when the
// size and the alignment of segment starts allow)
template <int E, typename T>
__device__ __forceinline__ void lds_put(T *p, const T (&v)[E])
{
    if constexpr (sizeof(T) == 8 && E % 2 == 0) {
#pragma unroll
        for (int e = 0; e < E; e += 2) *reinterpret_cast<double2 *>(p + e) = make_double2(v[e], v[e + 1]);
    } else if constexpr (sizeof(T) == 4 && E % 4 == 0) {
#pragma unroll
        for (int e = 0; e < E; e += 4)
            *reinterpret_cast<float4 *>(p + e) = make_float4(v[e], v[e + 1], v[e + 2], v[e + 3]);
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) p[e] = v[e];
    }
}
template <int E, typename T>
__device__ __forceinline__ void lds_get(T (&v)[E], const T *p)
{
    lds_row<E, T>(v, p);
}

// pivot row of column j: reduce in the segment column holding column j,
// then broadcast to the partition's lanes
template <int M, int E, typename T>
__device__ __forceinline__ int seg_pivot(T bj, bool used, int r, int j)
{
    constexpr int LP = seg_lanes<M, E>();
    const int idx = group_pivot<M>(pivot_key(bj, r, used));
    if constexpr (LP == WG) return __builtin_amdgcn_readlane(idx, (j / E) * M);
    else return __shfl(idx, (int)((threadIdx.x / LP) * LP) + (j / E) * M, WG);
}

// In-place Gauss-Jordan of the tableau b = D'(r, c0 .. c0+E-1), c0 = gc E;
// returns sigma(r) and p_c of the lane's columns through the references.
// tau > 0: the block also fails (ill-conditioned) when its smallest pivot
// is below tau times its largest (or a pivot is not finite).
template <int M, int E, typename T>
__device__ __forceinline__ void seg_invert(T (&b)[E], int r, int gc, T *S, int &sigma,
                                           int (&pc)[E], bool &sing, T tau = T(0))
{
    constexpr int RS = M + kPad<T>;
    const int c0 = gc * E;
    bool used = false;
    T pmin = T(0), pmax = T(0);
    int pr = seg_pivot<M, E, T>(b[0], used, r, 0);
#pragma unroll
    for (int j = 0; j < M; ++j) {
        T prow[E], mcol, pv;
        if constexpr (E == M) {
            // whole rows per lane: only the pivot row goes through LDS (to
            // row 0 of the block's area), column j is in the lane's registers
            if (r == pr) lds_put<E, T>(S, b);
            wave_sync();
            lds_get<E, T>(prow, S);
            mcol = b[j];
            pv = prow[j];
        } else {
            lds_put<E, T>(S + r * RS + c0, b);
            wave_sync();
            lds_get<E, T>(prow, S + __umul24(pr, RS) + c0);
            mcol = S[r * RS + j];
            pv = S[__umul24(pr, RS) + j];
        }
        sing = sing || (pv == T(0));
        const T apv = fabs(pv);
        pmin = j == 0 ? apv : fmin(pmin, apv);
        pmax = j == 0 ? apv : fmax(pmax, apv);
        const T inv = recip(pv);
        const bool isr = (r == pr);
        // exchange step as selects of computed values (no divergent code):
        // q = 1/v in the pivot row and -b(i,j)/v elsewhere; entries off
        // column j become q b(p_j, l) + [row is not the pivot] b(i, l).
        // Column j is entry j % E of segment column j / E.
        const T q = isr ? inv : -(mcol * inv);
        const T keep = isr ? T(0) : T(1);   // one select per step, a product per entry
        const bool inc = (gc == j / E);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const T sb = E >= 4 ? b[e] * keep : (isr ? T(0) : b[e]);
            const T w = fma(q, prow[e], sb);
            if (e == j % E) {
                b[e] = inc ? q : w;
                pc[e] = inc ? pr : pc[e];
            } else {
                b[e] = w;
            }
        }
        used = used || isr;
        sigma = isr ? j : sigma;
        wave_sync();
        if (j + 1 < M) pr = seg_pivot<M, E, T>(b[(j + 1) % E], used, r, j + 1);
    }
    if (tau > T(0)) sing = sing || !(pmin > tau * pmax);
}

}  // namespace
}  // namespace pf
