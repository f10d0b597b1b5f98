// Solve bodies of the partition method (gfx950): the forward sweep (the F
// solve of Sec. 2: t and the reduced right-hand side of every partition) and
// the back substitution (the G solve; for the bidiagonal-plus-corner form
// the independent updates of eq. (pups)), for factors stored by either
// factor mapping (row-major blocks E, X, Zh, R per block row).  A partition
// is a group of M lanes, lane i owning row i of a chunk of right-hand-side
// columns.
#pragma once
#include "kernels_common.h"

namespace pf {
namespace {

// ---------------------------------------------------------------------------
// Forward sweep of a solve (the F solve): t_k and the reduced right-hand side.
// Lane i owns row i of KC right-hand-side columns.  ADD: the right-hand side
// is the sum of two arrays (reduced levels of block tridiagonal matrices).
template <int M, int KC, typename T> constexpr int fwd_lds()
{
    return (WG / M) * group_stride<T>(KC * (M + kPad<T>));
}
template <int M, int KC, typename T> constexpr int bwd_lds()
{
    return (WG / M) * group_stride<T>(2 * KC * (M + kPad<T>));
}

// lane: 0..63 within the wave; lds: the wave's fwd_lds elements
template <int KIND, int M, int KC, typename T, bool ADD>
__device__ __forceinline__ void fwd_body(const SolveArgs &a, int64_t pblock, int cblock, int lane,
                                         T *lds)
{
    constexpr int GPW = WG / M;
    constexpr size_t MM = (size_t)M * M;
    const int tid = lane, grp = tid / M, i = tid % M;
    constexpr int CS = M + kPad<T>;                   // padded column stride
    constexpr int GS = group_stride<T>(KC * CS);
    T *SV = lds + grp * GS;                           // M x KC block vector, by columns
    const int64_t part = pblock * GPW + grp;
    const Geo G = geometry<KIND>(a.nb, a.p, part, a.sep);
    const int c0 = cblock * KC;
    const int kc = (a.nrhs - c0) < KC ? (a.nrhs - c0) : KC;
    const T *E = (const T *)a.E, *R = (const T *)a.R;
    double *dump = a.dump + tid;

    int64_t col[KC];   // column offsets, clamped to existing columns
#pragma unroll
    for (int c = 0; c < KC; ++c) col[c] = (int64_t)(c0 + (c < kc ? c : kc - 1));

    T fp[KC], gl[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) {
        fp[c] = T(0);
        gl[c] = T(0);
        if (G.valid) {
            double v = a.F[G.start * M + i + col[c] * a.ldf];
            if constexpr (ADD) v += a.Fadd[G.start * M + i + col[c] * a.ldf];
            fp[c] = (T)v;
        }
    }
    // Row i of E_g, R_g and A(g+1,g) and row i of the next right-hand side,
    // loaded one block row ahead (before the current row's stores); missing
    // operands come from the zero block.
    const T *zt = (const T *)a.zero + i * M;
    // (the right-hand side stays in FP64 and its two addends apart until the
    // row that uses them: converting or summing early would wait for this
    // row's own prefetch)
    auto load_row = [&](int64_t g, bool ok, T (&er)[M], T (&rr)[M], T (&lr)[M],
                        double (&fn)[KC], double (&fa)[KC]) {
        const bool nx = ok && (g + 1 < a.nb);
        ld_fac<M, T>(er, ok ? E + g * MM + i * M : zt);
        if constexpr (KIND == 0) ld_fac<M, T>(rr, (ok && G.hasL) ? R + g * MM + i * M : zt);
        ld_row_d<M, T>(lr, nx ? a.Lo + g * MM : a.zero, i);
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            const int64_t o = (g + 1) * M + i + col[c] * a.ldf;
            fn[c] = *(nx ? a.F + o : a.zero);
            if constexpr (ADD) fa[c] = *(nx ? a.Fadd + o : a.zero);
        }
    };
    T ec[M], rc[M], lc[M];
    double fc[KC], fca[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) fca[c] = 0.0;
    load_row(G.start, G.len > 0, ec, rc, lc, fc, fca);
    for (int k = 0; k < G.len; ++k) {
        const int64_t g = G.start + k;
        T er[M], lr[M], rr[M];
        double fn[KC], fna[KC];
#pragma unroll
        for (int l = 0; l < M; ++l) {
            er[l] = ec[l];
            lr[l] = lc[l];
            if constexpr (KIND == 0) rr[l] = rc[l];
        }
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            fn[c] = fc[c];
            fna[c] = fca[c];
        }
        load_row(g + 1, k + 1 < G.len, ec, rc, lc, fc, fca);
#pragma unroll
        for (int c = 0; c < KC; ++c) SV[i + c * CS] = fp[c];
        wave_sync();
        T t[KC];
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            T s = T(0);
#pragma unroll
            for (int l = 0; l < M; ++l) s = fma(er[l], SV[l + c * CS], s);
            t[c] = s;
        }
        wave_sync();
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            double *dst = (c < kc) ? a.Y + g * M + i + col[c] * a.ldy : dump;
            *dst = (double)t[c];
        }
#pragma unroll
        for (int c = 0; c < KC; ++c) SV[i + c * CS] = t[c];
        wave_sync();
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            T sl = T(0), sr = T(0);
#pragma unroll
            for (int l = 0; l < M; ++l) {
                const T tv = SV[l + c * CS];
                sl = fma(lr[l], tv, sl);
                if constexpr (KIND == 0) sr = fma(rr[l], tv, sr);
            }
            fp[c] = (T)(ADD ? fn[c] + fna[c] : fn[c]) - sl;
            if constexpr (KIND == 0) gl[c] -= sr;
        }
        wave_sync();
    }
#pragma unroll
    for (int c = 0; c < KC; ++c) {
        if (c >= kc) continue;
        const int64_t cn = col[c] * a.ldn;
        if (KIND == 0) {
            if (G.hasR) a.nF[part * M + i + cn] = (double)fp[c];
            if (G.hasL) a.nFadd[(part - 1) * M + i + cn] = (double)gl[c];
        } else if (G.valid) {
            a.nF[(part + 1) * M + i + cn] = (double)fp[c];
            if (part == 0) a.nF[i + cn] = a.F[i + col[c] * a.ldf];
        }
    }
}

// ---------------------------------------------------------------------------
// Back substitution (the G solve / the parallel updates of eq. (pups)).
// lane: 0..63 within the wave; lds: the wave's bwd_lds elements
template <int KIND, int M, int KC, typename T>
__device__ __forceinline__ void bwd_body(const SolveArgs &a, int64_t pblock, int cblock, int lane,
                                         T *lds)
{
    constexpr int GPW = WG / M;
    constexpr size_t MM = (size_t)M * M;
    const int tid = lane, grp = tid / M, i = tid % M;
    constexpr int CS = M + kPad<T>;                   // padded column stride
    constexpr int GS = group_stride<T>(2 * KC * CS);
    T *SV = lds + grp * GS;                           // x of the row below (M x KC)
    T *SL = SV + KC * CS;                             // x at the left separator
    const int64_t part = pblock * GPW + grp;
    const Geo G = geometry<KIND>(a.nb, a.p, part, a.sep);
    const int c0 = cblock * KC;
    const int kc = (a.nrhs - c0) < KC ? (a.nrhs - c0) : KC;
    const T *Zs = (const T *)a.Z, *Xs = (const T *)a.X;
    double *dump = a.dump + tid;
    const int64_t sR = G.start + G.len;
    // reduced-solution indices of the two separators
    const int64_t jl = (KIND == 0) ? part - 1 : part;
    const int64_t jr = (KIND == 0) ? part : part + 1;

    int64_t col[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) col[c] = (int64_t)(c0 + (c < kc ? c : kc - 1));

    // Row i of Zh_g and X_g and row i of t_g, loaded PD block rows ahead of
    // their use (the chain runs from the last block row up; k < 0 reads the
    // zero block); the first rows are requested before the separators'
    // solution, so the waits overlap.  A row costs 2M + KC registers per lane,
    // which bounds the depth for the larger blocks.
    constexpr int PD = M <= 4 ? 4 : (M <= 8 ? 3 : (M <= 16 ? 1 : 0));
    struct Row {
        T zr[M], xr[M];
        double t[KC];
    };
    const T *zt = (const T *)a.zero + i * M;
    auto load_row = [&](int k, Row &w) {
        const bool ok = k >= 0;
        const int64_t g = G.start + (ok ? k : 0);
        ld_fac<M, T>(w.zr, ok ? Zs + g * MM + i * M : zt);
        if constexpr (KIND == 0) ld_fac<M, T>(w.xr, ok ? Xs + g * MM + i * M : zt);
#pragma unroll
        for (int c = 0; c < KC; ++c) w.t[c] = *(ok ? a.Y + g * M + i + col[c] * a.ldy : a.zero);
    };
    Row buf[PD + 1];   // buf[0]: the row in use
#pragma unroll
    for (int d = 0; d < PD; ++d) load_row(G.len - 1 - d, buf[d]);

#pragma unroll
    for (int c = 0; c < KC; ++c) {
        T xl = T(0), xr = T(0);
        if (c < kc) {
            const int64_t cn = col[c] * a.ldn;
            if (G.hasL) xl = (T)a.Xsep[jl * M + i + cn];
            if (G.hasR) {
                const double v = a.Xsep[jr * M + i + cn];
                xr = (T)v;
                a.Y[sR * M + i + col[c] * a.ldy] = v;
            }
            if (KIND == 1 && G.valid && part == 0) a.Y[i + col[c] * a.ldy] = a.Xsep[i + cn];
        }
        SL[i + c * CS] = xl;
        SV[i + c * CS] = xr;
    }
    wave_sync();
    for (int k = G.len - 1; k >= 0; --k) {
        const int64_t g = G.start + k;
        load_row(k - PD, buf[PD]);
        const Row &cur = buf[0];
        T xk[KC];
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            T s = (T)cur.t[c];
#pragma unroll
            for (int l = 0; l < M; ++l) {
                s = fma(-cur.zr[l], SL[l + c * CS], s);
                if constexpr (KIND == 0) s = fma(-cur.xr[l], SV[l + c * CS], s);
            }
            xk[c] = s;
        }
        if constexpr (KIND == 0) wave_sync();
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            double *dst = (c < kc) ? a.Y + g * M + i + col[c] * a.ldy : dump;
            *dst = (double)xk[c];
            if constexpr (KIND == 0) SV[i + c * CS] = xk[c];
        }
        if constexpr (KIND == 0) wave_sync();
#pragma unroll
        for (int d = 0; d < PD; ++d) buf[d] = buf[d + 1];
    }
}

}  // namespace
}  // namespace pf
