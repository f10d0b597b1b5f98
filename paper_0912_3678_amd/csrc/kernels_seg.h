// Partition-method factor bodies, segment lane mapping (gfx950).
//
// One partition is owned by M*M/E lanes; lane (r, g) holds the E entries
// (r, g*E .. g*E+E-1) of row r of every block of its chain, the M lanes of
// one segment column g being consecutive.  E = 1 puts one block entry in each
// lane: the chain row's work is spread over M*M lanes and its latency is
// lowest, which is what bounds the reduced levels of the recursion (few
// partitions).  Larger E spends fewer instructions per partition and suits
// the finest level (many partitions, bound by issue and bandwidth).
//
// Pivot blocks are inverted in place by the Gauss-Jordan exchange steps of
// kernels_gj.h.  Block products read rows of the left operand and columns of
// the right operand from the partition's LDS slice; the factor kernels can
// also sweep up to M right-hand sides forward in the same pass
// (factor-and-solve: the F solve of Sec. 2 alongside the factorization), lane
// (r, g) carrying right-hand-side columns g*E .. g*E+E-1.
//
// Outputs and recurrences are those of the row mapping (kernels_rows.hip):
// row-major factor blocks E, X, Zh, R per block row, the reduced matrix of
// eq. (redmatr) / (redmatr1), and for the forward sweep t and the reduced
// right-hand side.
#pragma once
#include "kernels_gj.h"

namespace pf {
namespace {

// prefetch depth of the chain loops (block rows): a row's operands take 6E
// registers per lane, which bounds the depth for the widest segments
template <int E> constexpr int seg_prefetch() { return E <= 2 ? 2 : 1; }

// entries (r, c0 .. c0+E-1) of a column-major M x M block (FP64)
template <int M, int E>
__device__ __forceinline__ void ld_ent(double (&v)[E], const double *blk, int r, int c0)
{
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = blk[r + (c0 + e) * M];
}

// Block tridiagonal factor, segment mapping.  RHS: the forward sweep of up to
// M right-hand sides runs in the same pass.
// LDS elements of a wave's partitions (BTRI and BABD bodies)
template <int M, int E, typename T, bool RHS> constexpr int seg_btri_lds()
{
    return (WG / seg_lanes<M, E>()) * group_stride<T>((RHS ? 6 : 5) * M * (M + kPad<T>));
}
template <int M, int E, typename T, bool RHS> constexpr int seg_babd_lds()
{
    return (WG / seg_lanes<M, E>()) * group_stride<T>((RHS ? 5 : 4) * M * (M + kPad<T>));
}

// lane: 0..63 within the wave; lds: the wave's seg_btri_lds elements
template <int M, int E, typename T, bool ADD, bool RHS>
__device__ __forceinline__ void btri_seg_body(const LevelArgs &a, const SolveArgs &sv,
                                              int64_t pblock, int lane, T *lds)
{
    constexpr int LP = seg_lanes<M, E>(), PPW = WG / LP;
    constexpr size_t MM = (size_t)M * M;
    const int tid = lane, grp = tid / LP, t = tid % LP;
    const int r = t % M, c0 = (t / M) * E;
    constexpr int RS = M + kPad<T>;
    constexpr int NS = RHS ? 6 : 5;
    constexpr int GS = group_stride<T>(NS * M * RS);
    T *S0 = lds + grp * GS;   // tableau; then E by rows; then R by rows
    T *S1 = S0 + M * RS;      // Z' by columns; then X by columns
    T *S2 = S1 + M * RS;      // A(g+1,g) by rows
    T *S3 = S2 + M * RS;      // Zh by columns
    T *S5 = S3 + M * RS;      // A(g,g+1) by columns
    T *S4 = S5 + M * RS;      // (RHS) f' by columns; then t by columns
    constexpr int PD = seg_prefetch<E>();

    const int64_t nb = a.nb;
    const int64_t part = pblock * PPW + grp;
    const Geo G = geometry<0>(nb, a.p, part, a.sep);
    const int gc = t / M;   // segment column

    // Block arrays and factors through raw buffers based one block row before
    // the workgroup's first partition: every row a partition touches lies at
    // or past the base (its left separator's couplings included), and rows
    // past an array's end read zero, as a missing operand must.
    const int64_t s0 = geometry_wave<0>(nb, a.p, pblock * PPW, a.sep).start;
    const int64_t gb = s0 > 0 ? s0 - 1 : 0;
    constexpr uint32_t BB = MM * 8, BT = MM * sizeof(T);
    const uint64_t nr = (uint64_t)(nb - gb), nr1 = nb - 1 > gb ? (uint64_t)(nb - 1 - gb) : 0;
    const auto rD = buf_rsrc(a.D + gb * MM, nr * BB);
    const auto rDa = buf_rsrc(ADD ? a.Dadd + gb * MM : a.D, ADD ? nr * BB : 0);
    const auto rL = buf_rsrc(a.Lo + gb * MM, nr1 * BB);
    const auto rU = buf_rsrc(a.Up + gb * MM, nr1 * BB);
    const auto rE = buf_rsrc((T *)a.E + gb * MM, nr * BT);
    const auto rR = buf_rsrc((T *)a.R + gb * MM, nr * BT);
    const auto rZ = buf_rsrc((T *)a.Z + gb * MM, nr * BT);
    const auto rX = buf_rsrc((T *)a.X + gb * MM, nr * BT);
    const uint32_t rel = (uint32_t)(G.start - gb);          // partition start, relative
    const uint32_t ent = (uint32_t)(r + c0 * M) * 8;        // entry (r, c0), column-major FP64
    const uint32_t fen = (uint32_t)(r * M + c0) * sizeof(T);   // entry (r, c0), row-major factor
    auto ld_blk = [&](double (&v)[E], __amdgpu_buffer_rsrc_t rs, uint32_t row) {
        const uint32_t o = row * BB + ent;
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = buf_ld(rs, o + (uint32_t)(e * M * 8));
    };

    double *ydump = (double *)a.dump + 2048 + tid * E;
    const double *zero = a.zero;
    // right-hand-side columns of this lane's entries (clamped to column 0
    // when there is none; their loads then read the zero block)
    bool act[E];
    int64_t fo[E], yo[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        act[e] = RHS && (c0 + e < sv.nrhs);
        fo[e] = (int64_t)r + (int64_t)(act[e] ? c0 + e : 0) * sv.ldf;
        yo[e] = (int64_t)r + (int64_t)(act[e] ? c0 + e : 0) * sv.ldy;
    }

    T d[E], z[E], rr[E], a1[E], fp[E], gl[E];
#pragma unroll
    for (int e = 0; e < E; ++e) { d[e] = z[e] = rr[e] = a1[e] = fp[e] = gl[e] = T(0); }
    if (G.valid) {
        double v[E];
        ld_blk(v, rD, rel);
        if constexpr (ADD) {
            double w[E];
            ld_blk(w, rDa, rel);
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] += w[e];
        }
#pragma unroll
        for (int e = 0; e < E; ++e) d[e] = (T)v[e];
        if constexpr (RHS) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                double w = *(act[e] ? sv.F + G.start * M + fo[e] : zero);
                if constexpr (ADD) w += *(act[e] ? sv.Fadd + G.start * M + fo[e] : zero);
                fp[e] = (T)w;
            }
        }
    }
    if (G.hasL) {
        double v[E], w[E];
        ld_blk(v, rL, rel - 1);   // A(g_1, sL)
        ld_blk(w, rU, rel - 1);   // A(sL, g_1)
#pragma unroll
        for (int e = 0; e < E; ++e) { z[e] = (T)v[e]; rr[e] = (T)w[e]; }
    }
    unsigned long long bad = ~0ull;

    // Operands of block row g that do not depend on the chain -- A(g,g+1),
    // A(g+1,g), D[g+1] and f[g+1] at the lane's entries -- loaded PD block
    // rows ahead and kept in FP64 (the two addends of a sum apart) until the
    // row that uses them.  Rows past the partition's end are loaded too
    // (never used); rows past the matrix read zero.
    struct Next {
        double up[E], lo[E], dn[E], da[E], fn[E], fa[E];
    };
    auto load_next = [&](int k, Next &n) {
        const uint32_t row = rel + (uint32_t)k;
        ld_blk(n.up, rU, row);
        ld_blk(n.lo, rL, row);
        ld_blk(n.dn, rD, row + 1);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            n.da[e] = 0.0;
            n.fn[e] = 0.0;
            n.fa[e] = 0.0;
        }
        if constexpr (ADD) ld_blk(n.da, rDa, row + 1);
        if constexpr (RHS) {
            const int64_t g = G.start + k;
            const bool ok = k < G.len && g + 1 < nb;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                n.fn[e] = *((ok && act[e]) ? sv.F + (g + 1) * M + fo[e] : zero);
                if constexpr (ADD) n.fa[e] = *((ok && act[e]) ? sv.Fadd + (g + 1) * M + fo[e] : zero);
            }
        }
    };
    Next buf[PD + 1];   // buf[0]: the operands of the row in use
#pragma unroll
    for (int d = 0; d < PD; ++d) load_next(d, buf[d]);

    for (int k = 0; k < G.len; ++k) {
        const int64_t g = G.start + k;
        const uint32_t frow = (rel + (uint32_t)k) * BT;   // this block row's factors
        load_next(k + PD, buf[PD]);
        const Next &cur = buf[0];

        T b[E];
        int sigma = 0, pc[E];
#pragma unroll
        for (int e = 0; e < E; ++e) { b[e] = d[e]; pc[e] = 0; }
        bool sing = false;
        seg_invert<M, E, T>(b, r, gc, S0, sigma, pc, sing, (T)a.tau);
        const unsigned long long code = status_code(a.level, g);
        bad = (sing && code < bad) ? code : bad;

        T lo[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            S0[sigma * RS + pc[e]] = b[e];           // E_k by (logical) rows
            S1[(c0 + e) * RS + r] = z[e];            // Z'_k by columns
            S5[(c0 + e) * RS + r] = (T)cur.up[e];    // A(g,g+1) by columns
            if constexpr (RHS) S4[(c0 + e) * RS + r] = fp[e];   // f'_k by columns
            lo[e] = (T)cur.lo[e];
        }
        lds_put<E, T>(S2 + r * RS + c0, lo);         // A(g+1,g) by rows
        wave_sync();
        T er[M];
        lds_row<M, T>(er, S0 + r * RS);
        T x[E], zh[E], tk[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            T col[M];
            lds_row<M, T>(col, S5 + (c0 + e) * RS);
            x[e] = dot<M, T>(er, col);               // X_k = E_k A(g,g+1)
            lds_row<M, T>(col, S1 + (c0 + e) * RS);
            zh[e] = dot<M, T>(er, col);              // Zh_k = E_k Z'_k
            tk[e] = T(0);
            if constexpr (RHS) {
                lds_row<M, T>(col, S4 + (c0 + e) * RS);
                tk[e] = dot<M, T>(er, col);          // t_k = E_k f'_k
                *(act[e] ? sv.Y + g * M + yo[e] : ydump + e) = (double)tk[e];
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e)
            buf_st(rE, frow + (uint32_t)(sigma * M + pc[e]) * (uint32_t)sizeof(T), b[e]);
        buf_st_row<E, T>(rR, G.hasL ? frow + fen : kOffNone, rr);
        buf_st_row<E, T>(rX, frow + fen, x);
        buf_st_row<E, T>(rZ, frow + fen, zh);
        wave_sync();
        lds_put<E, T>(S0 + r * RS + c0, rr);          // R_k by rows
#pragma unroll
        for (int e = 0; e < E; ++e) {
            S1[(c0 + e) * RS + r] = x[e];            // X_k by columns
            S3[(c0 + e) * RS + r] = zh[e];           // Zh_k by columns
            if constexpr (RHS) S4[(c0 + e) * RS + r] = tk[e];   // t_k by columns
        }
        wave_sync();
        T rw[M], lr[M];
        lds_row<M, T>(rw, S0 + r * RS);
        lds_row<M, T>(lr, S2 + r * RS);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            T xc[M], hc[M];
            lds_row<M, T>(xc, S1 + (c0 + e) * RS);
            lds_row<M, T>(hc, S3 + (c0 + e) * RS);
            a1[e] -= dot<M, T>(rw, hc);                                         // alpha_1
            rr[e] = -dot<M, T>(rw, xc);                                         // R_{k+1}
            d[e] = (T)(ADD ? cur.dn[e] + cur.da[e] : cur.dn[e]) - dot<M, T>(lr, xc);   // D'_{k+1}
            z[e] = -dot<M, T>(lr, hc);                                          // Z'_{k+1}
            if constexpr (RHS) {
                T tc[M];
                lds_row<M, T>(tc, S4 + (c0 + e) * RS);
                gl[e] -= dot<M, T>(rw, tc);                                     // g_sL -= R_k t_k
                fp[e] = (T)(ADD ? cur.fn[e] + cur.fa[e] : cur.fn[e]) - dot<M, T>(lr, tc);
            }
        }
#pragma unroll
        for (int d = 0; d < PD; ++d) buf[d] = buf[d + 1];
        wave_sync();
    }
    report_bad(a, bad);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int cm = r + (c0 + e) * M;
        if (G.hasR) {
            a.nD[part * MM + cm] = (double)d[e];                       // D[sR] + alpha_2
            if (G.hasL) a.nLo[(part - 1) * MM + cm] = (double)z[e];    // beta
        }
        if (G.hasL) {
            a.nDadd[(part - 1) * MM + cm] = (double)a1[e];             // alpha_1
            if (G.hasR) a.nUp[(part - 1) * MM + cm] = (double)rr[e];   // gamma
        }
        if constexpr (RHS) {
            if (act[e]) {
                const int64_t no = (int64_t)r + (int64_t)(c0 + e) * sv.ldn;
                if (G.hasR) sv.nF[part * M + no] = (double)fp[e];           // f[sR] - A(sR,g_n) t_n
                if (G.hasL) sv.nFadd[(part - 1) * M + no] = (double)gl[e];  // - sum R_k t_k
            }
        }
    }
}

// Bidiagonal-plus-corner factor, segment mapping (D' = D: the inversion of
// a block row does not wait for the chain).
template <int M, int E, typename T, bool RHS>
__device__ __forceinline__ void babd_seg_body(const LevelArgs &a, const SolveArgs &sv,
                                              int64_t pblock, int lane, T *lds)
{
    constexpr int LP = seg_lanes<M, E>(), PPW = WG / LP;
    constexpr size_t MM = (size_t)M * M;
    const int tid = lane, grp = tid / LP, t = tid % LP;
    const int r = t % M, c0 = (t / M) * E;
    constexpr int RS = M + kPad<T>;
    constexpr int NS = RHS ? 5 : 4;
    constexpr int GS = group_stride<T>(NS * M * RS);
    T *S0 = lds + grp * GS;   // tableau; then E by rows
    T *S1 = S0 + M * RS;      // Z' by columns
    T *S2 = S1 + M * RS;      // A(g+1,g) by rows
    T *S3 = S2 + M * RS;      // Zh by columns
    T *S4 = S3 + M * RS;      // (RHS) f' by columns; then t by columns
    constexpr int PD = seg_prefetch<E>();

    const int64_t part = pblock * PPW + grp;
    const Geo G = geometry<1>(a.nb, a.p, part, a.sep);
    const int gc = t / M;   // segment column
    // raw buffers based one block row before the workgroup's first partition
    // (its left separator); rows past an array's end read zero
    const int64_t nb = a.nb;
    const int64_t gb = geometry_wave<1>(nb, a.p, pblock * PPW, a.sep).start - 1;
    constexpr uint32_t BB = MM * 8, BT = MM * sizeof(T);
    const uint64_t nr = (uint64_t)(nb - gb), nr1 = nb - 1 > gb ? (uint64_t)(nb - 1 - gb) : 0;
    const auto rD = buf_rsrc(a.D + gb * MM, nr * BB);
    const auto rL = buf_rsrc(a.Lo + gb * MM, nr1 * BB);
    const auto rE = buf_rsrc((T *)a.E + gb * MM, nr * BT);
    const auto rZ = buf_rsrc((T *)a.Z + gb * MM, nr * BT);
    const uint32_t rel = (uint32_t)(G.start - gb);
    const uint32_t ent = (uint32_t)(r + c0 * M) * 8;
    const uint32_t fen = (uint32_t)(r * M + c0) * sizeof(T);
    auto ld_blk = [&](double (&v)[E], __amdgpu_buffer_rsrc_t rs, uint32_t row) {
        const uint32_t o = row * BB + ent;
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = buf_ld(rs, o + (uint32_t)(e * M * 8));
    };
    double *ydump = (double *)a.dump + 2048 + tid * E;
    const double *zero = a.zero;
    bool act[E];
    int64_t fo[E], yo[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        act[e] = RHS && (c0 + e < sv.nrhs);
        fo[e] = (int64_t)r + (int64_t)(act[e] ? c0 + e : 0) * sv.ldf;
        yo[e] = (int64_t)r + (int64_t)(act[e] ? c0 + e : 0) * sv.ldy;
    }

    T z[E], fp[E];
    {
        double v[E];
        ld_blk(v, rL, rel - 1);   // A(g_1, sL) (read for invalid partitions too: unused)
#pragma unroll
        for (int e = 0; e < E; ++e) {
            z[e] = (T)v[e];
            fp[e] = (RHS && G.valid && act[e]) ? (T)sv.F[G.start * M + fo[e]] : T(0);
        }
    }
    unsigned long long bad = ~0ull;
    // D[g], A(g+1,g) and f[g+1] at the lane's entries, PD block rows ahead
    struct Next {
        double dc[E], lc[E], fc[E];
    };
    auto load_next = [&](int k, Next &n) {
        const uint32_t row = rel + (uint32_t)k;
        ld_blk(n.dc, rD, row);
        ld_blk(n.lc, rL, row);
        const int64_t g = G.start + k;
        const bool ok = k < G.len;
#pragma unroll
        for (int e = 0; e < E; ++e)
            n.fc[e] = RHS ? *((ok && act[e]) ? sv.F + (g + 1) * M + fo[e] : zero) : 0.0;
    };
    Next buf[PD + 1];
#pragma unroll
    for (int d = 0; d < PD; ++d) load_next(d, buf[d]);
    for (int k = 0; k < G.len; ++k) {
        const int64_t g = G.start + k;
        const uint32_t frow = (rel + (uint32_t)k) * BT;
        load_next(k + PD, buf[PD]);
        const Next &cur = buf[0];

        T b[E], lo[E];
        int sigma = 0, pc[E];
#pragma unroll
        for (int e = 0; e < E; ++e) { b[e] = (T)cur.dc[e]; lo[e] = (T)cur.lc[e]; pc[e] = 0; }
        bool sing = false;
        seg_invert<M, E, T>(b, r, gc, S0, sigma, pc, sing, (T)a.tau);
        const unsigned long long code = status_code(a.level, g);
        bad = (sing && code < bad) ? code : bad;

#pragma unroll
        for (int e = 0; e < E; ++e) {
            S0[sigma * RS + pc[e]] = b[e];
            S1[(c0 + e) * RS + r] = z[e];
            if constexpr (RHS) S4[(c0 + e) * RS + r] = fp[e];
        }
        lds_put<E, T>(S2 + r * RS + c0, lo);
        wave_sync();
        T er[M];
        lds_row<M, T>(er, S0 + r * RS);
        T zh[E], tk[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            T col[M];
            lds_row<M, T>(col, S1 + (c0 + e) * RS);
            zh[e] = dot<M, T>(er, col);
            tk[e] = T(0);
            if constexpr (RHS) {
                lds_row<M, T>(col, S4 + (c0 + e) * RS);
                tk[e] = dot<M, T>(er, col);
                *(act[e] ? sv.Y + g * M + yo[e] : ydump + e) = (double)tk[e];
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e)
            buf_st(rE, frow + (uint32_t)(sigma * M + pc[e]) * (uint32_t)sizeof(T), b[e]);
        buf_st_row<E, T>(rZ, frow + fen, zh);
        wave_sync();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            S3[(c0 + e) * RS + r] = zh[e];
            if constexpr (RHS) S4[(c0 + e) * RS + r] = tk[e];
        }
        wave_sync();
        T lr[M];
        lds_row<M, T>(lr, S2 + r * RS);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            T hc[M];
            lds_row<M, T>(hc, S3 + (c0 + e) * RS);
            z[e] = -dot<M, T>(lr, hc);
            if constexpr (RHS) {
                T tc[M];
                lds_row<M, T>(tc, S4 + (c0 + e) * RS);
                fp[e] = (T)cur.fc[e] - dot<M, T>(lr, tc);
            }
        }
#pragma unroll
        for (int d = 0; d < PD; ++d) buf[d] = buf[d + 1];
        wave_sync();
    }
    report_bad(a, bad);
    if (G.valid) {
        const int64_t sR = G.start + G.len;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int cm = r + (c0 + e) * M;
            a.nLo[part * MM + cm] = (double)z[e];                      // beta
            a.nD[(part + 1) * MM + cm] = a.D[sR * MM + cm];
            if (part == 0) {
                a.nD[cm] = a.D[cm];
                a.nC[cm] = a.C[cm];
            }
            if constexpr (RHS) {
                if (act[e]) {
                    const int64_t no = (int64_t)r + (int64_t)(c0 + e) * sv.ldn;
                    sv.nF[(part + 1) * M + no] = (double)fp[e];
                    if (part == 0) sv.nF[no] = sv.F[fo[e]];
                }
            }
        }
    }
}

}  // namespace
}  // namespace pf
