// Partition-method factor kernels, row lane mapping (gfx950, CDNA4).
//
// Method (Amodio & Brugnano, Sec. 2): the block rows are split into p
// partitions separated by single separator block rows (eq. (parpart) for a
// block tridiagonal matrix, eq. (parpart1) for the bidiagonal-plus-corner
// form).  Each partition factors its local block M^(i) of eq. (Mi0) with the
// LU variant of eq. (parblock): a block Gaussian elimination down the
// partition that also carries the two fill-in spikes -- the left-separator
// column spike (paper z) and, for block tridiagonal matrices, the
// left-separator row spike (paper w) -- and ends with the partition's
// contributions alpha_1, alpha_2, beta, gamma to the reduced matrix of
// eq. (redmatr) / (redmatr1).
//
// GPU mapping.  A workgroup is one wave64.  A partition is owned by a group
// of M consecutive lanes (M = block size; 64/M partitions per wave) and lane
// i holds row i of every block the partition works on.  The pivot block is
// inverted by a row-distributed Gauss-Jordan elimination whose pivot search
// is a DPP reduction inside the group; operands that every lane needs in
// full go through the group's own, bank-padded slice of LDS.  This mapping
// serves the block sizes without a segment kernel (32) and runs on request
// (PF_FLAG_MAP_ROWS); kernels_seg.hip has the others.
//
// Factor storage: per block row g, row-major M x M blocks E (inverse of the
// eliminated pivot block D'), X = E A(g,g+1), Zh (left spike column) and R
// (left spike row) -- exactly the quantities the solve needs, laid out so the
// solve kernels load contiguous rows.
//
// Recurrences of one partition (global blocks g_1..g_n between the
// separators sL = g_1 - 1 and sR = g_n + 1), block tridiagonal case:
//   D'_1 = D[g_1],  Z'_1 = A(g_1, sL),  R_1 = A(sL, g_1)
//   for k = 1..n:
//     E_k = D'_k^{-1}                    (Gauss-Jordan, row partial pivoting)
//     X_k = E_k A(g_k, g_k+1),  Zh_k = E_k Z'_k
//     alpha_1 -= R_k Zh_k,      R_{k+1} = -R_k X_k
//     D'_{k+1} = D[g_k+1] - A(g_k+1, g_k) X_k,   Z'_{k+1} = -A(g_k+1, g_k) Zh_k
// At k = n the "next" quantities are the partition's contributions to the
// right separator: D'_{n+1} = D[sR] + alpha_2 (written as the reduced
// diagonal), Z'_{n+1} = beta, and R_{n+1} = gamma.
// Solve:  t_k = E_k (f_k - A(g_k, g_k-1) t_{k-1}),  g_sL -= sum R_k t_k,
//         g_sR -= A(sR, g_n) t_n;  then
//         x_k = t_k - Zh_k x_sL - X_k x_{k+1}  (x_{n+1} = x_sR).
// In the bidiagonal-plus-corner case A(g, g+1) = 0, so X = R = 0 and the
// back substitution is independent row by row (eq. (pups)).
#include "kernels_common.h"

namespace pf {
namespace {

// ---- Gauss-Jordan inversion of the pivot block with row partial pivoting --
// Row-distributed and swap-free: lane i holds row i of D' in d (consumed) and
// starts with row i of the identity in e.  At step c the pivot is the row
// with the largest |D'(r,c)| among rows not yet used as pivots (ranked by
// pivot_key), found by a DPP max-reduction; the pivot lane's row [d | e] is read
// from the group's LDS, the pivot row is scaled by 1/pivot and column c is
// eliminated from every other row.  Rows never move: the lane chosen at step
// c ends with row c of D'^{-1} in e, and sigma (the return value) is c.
// Only the columns > c of d are still needed after step c.
// tau > 0: the block also fails (ill-conditioned) when its smallest pivot
// is below tau times its largest (or a pivot is not finite).
template <int M, typename T>
__device__ __forceinline__ int gj_rows(T (&d)[M], T (&e)[M], int i, T *SP, bool &sing,
                                       T tau = T(0))
{
    constexpr int PR = 2 * M + kPad<T>;   // padded row stride of SP
    T pmin = T(0), pmax = T(0);
#pragma unroll
    for (int l = 0; l < M; ++l) e[l] = (l == i) ? T(1) : T(0);
    bool used = false;
    int sigma = 0;
#pragma unroll
    for (int c = 0; c < M; ++c) {
        const int pr = group_pivot<M>(pivot_key(d[c], i, used));
        T *row = SP + i * PR;
#pragma unroll
        for (int l = c; l < M; ++l) row[l] = d[l];
#pragma unroll
        for (int l = 0; l < M; ++l) row[M + l] = e[l];
        wave_sync();
        const T *prow = SP + pr * PR;
        T pd[M], pe[M];
#pragma unroll
        for (int l = c; l < M; ++l) pd[l] = prow[l];
#pragma unroll
        for (int l = 0; l < M; ++l) pe[l] = prow[M + l];
        const T pv = pd[c];
        sing = sing || (pv == T(0));
        const T apv = fabs(pv);
        pmin = c == 0 ? apv : fmin(pmin, apv);
        pmax = c == 0 ? apv : fmax(pmax, apv);
        const T inv = recip(pv);
        const bool isp = (i == pr);
        const T f = isp ? -inv : d[c] * inv;
        const T s = isp ? T(0) : T(1);
#pragma unroll
        for (int l = c + 1; l < M; ++l) d[l] = fma(-f, pd[l], s * d[l]);
#pragma unroll
        for (int l = 0; l < M; ++l) e[l] = fma(-f, pe[l], s * e[l]);
        used = used || isp;
        sigma = isp ? c : sigma;
        wave_sync();
    }
    if (tau > T(0)) sing = sing || !(pmin > tau * pmax);
    return sigma;
}

// store row i of an M x M column-major FP64 block
template <int M, typename T>
__device__ __forceinline__ void st_row_d(double *__restrict__ blk, int i, const T (&v)[M])
{
#pragma unroll
    for (int l = 0; l < M; ++l) blk[i + l * M] = (double)v[l];
}

// ---------------------------------------------------------------------------
// Block tridiagonal factor: one level.  Lane i of a group holds row i of the
// running blocks D', Z', R and alpha_1.  ADD: the diagonal blocks are the sum
// of two arrays (the two neighbours' contributions of the level above).
template <int M, typename T, bool ADD>
__device__ __forceinline__ void btri_factor_body(const LevelArgs &a, int64_t pblock)
{
    constexpr int GPW = WG / M;
    constexpr size_t MM = (size_t)M * M;
    const int tid = threadIdx.x, grp = tid / M, i = tid % M;
    constexpr int RS = M + kPad<T>, PR = 2 * M + kPad<T>;
    constexpr int GS = group_stride<T>(M * PR + 2 * M * RS);
    __shared__ __align__(16) T lds[GPW * GS];
    T *SP = lds + grp * GS;   // Gauss-Jordan pivot rows (M x PR)
    T *SU = SP + M * PR;      // A(g,g+1)^T, then the rows of X (M x RS)
    T *SZ = SU + M * RS;      // Z'^T, then the rows of Zh (M x RS)

    const int64_t nb = a.nb;
    const int64_t part = pblock * GPW + grp;
    const Geo G = geometry<0>(nb, a.p, part, a.sep);
    T *E = (T *)a.E, *R = (T *)a.R, *Zs = (T *)a.Z, *Xs = (T *)a.X;
    T *dump = (T *)a.dump + tid * M;

    T d[M], z[M], rr[M], a1[M];
    zero<M, T>(d); zero<M, T>(z); zero<M, T>(rr); zero<M, T>(a1);
    if (G.valid) {
        ld_row_d<M, T>(d, a.D + G.start * MM, i);
        if constexpr (ADD) {
            T w[M];
            ld_row_d<M, T>(w, a.Dadd + G.start * MM, i);
#pragma unroll
            for (int l = 0; l < M; ++l) d[l] += w[l];
        }
    }
    if (G.hasL) {
        ld_row_d<M, T>(z, a.Lo + (G.start - 1) * MM, i);   // A(g_1, sL)
        ld_row_d<M, T>(rr, a.Up + (G.start - 1) * MM, i);  // A(sL, g_1)
    }
    unsigned long long bad = ~0ull;

    // Operands of block row g that do not depend on the chain: column i of
    // A(g,g+1), row i of A(g+1,g) and of D[g+1].  They are loaded one row
    // ahead (before the stores of the current row), and from the zero block
    // when they do not exist.
    auto load_next = [&](int64_t g, bool ok, T (&upc)[M], T (&lor)[M], T (&dn)[M]) {
        ld_vec<M, T>(upc, (ok ? a.Up + g * MM : a.zero) + i * M);
        ld_row_d<M, T>(lor, ok ? a.Lo + g * MM : a.zero, i);
        ld_row_d<M, T>(dn, ok ? a.D + (g + 1) * MM : a.zero, i);
        if constexpr (ADD) {
            T w[M];
            ld_row_d<M, T>(w, ok ? a.Dadd + (g + 1) * MM : a.zero, i);
#pragma unroll
            for (int l = 0; l < M; ++l) dn[l] += w[l];
        }
    };
    T upc[M], lor[M], dn[M];
    load_next(G.start, G.len > 0 && G.start + 1 < nb, upc, lor, dn);

    for (int k = 0; k < G.len; ++k) {
        const int64_t g = G.start + k;
        T upn[M], lon[M], dnn[M];
        load_next(g + 1, k + 1 < G.len && g + 2 < nb, upn, lon, dnn);

        T e[M];
        bool sing = false;
        const int sig = gj_rows<M, T>(d, e, i, SP, sing, (T)a.tau);
        const unsigned long long code = status_code(a.level, g);
        bad = (sing && code < bad) ? code : bad;
        st_fac<M, T>(E + g * MM + sig * M, e);             // row sig of E_k
        st_fac<M, T>(G.hasL ? R + g * MM + i * M : dump, rr);   // row i of R_k
#pragma unroll
        for (int l = 0; l < M; ++l) {
            SU[i * RS + l] = upc[l];                       // row i of A(g,g+1)^T
            SZ[l * RS + i] = z[l];                         // column i of Z'^T
        }
        wave_sync();
        T x[M], zh[M];
#pragma unroll
        for (int c = 0; c < M; ++c) {                      // row sig of X_k and Zh_k
            T sx = T(0), sz = T(0);
#pragma unroll
            for (int l = 0; l < M; ++l) {
                sx = fma(e[l], SU[c * RS + l], sx);
                sz = fma(e[l], SZ[c * RS + l], sz);
            }
            x[c] = sx;
            zh[c] = sz;
        }
        st_fac<M, T>(Xs + g * MM + sig * M, x);
        st_fac<M, T>(Zs + g * MM + sig * M, zh);
        wave_sync();
#pragma unroll
        for (int c = 0; c < M; ++c) {
            SU[sig * RS + c] = x[c];
            SZ[sig * RS + c] = zh[c];
        }
        wave_sync();
        T rn[M], t1[M], dl[M], zl[M];
        zero<M, T>(rn); zero<M, T>(t1); zero<M, T>(dl); zero<M, T>(zl);
#pragma unroll
        for (int l = 0; l < M; ++l) {                      // R_k X_k, R_k Zh_k, Lo X_k, Lo Zh_k
#pragma unroll
            for (int c = 0; c < M; ++c) {
                const T xv = SU[l * RS + c], zv = SZ[l * RS + c];
                rn[c] = fma(rr[l], xv, rn[c]);
                t1[c] = fma(rr[l], zv, t1[c]);
                dl[c] = fma(lor[l], xv, dl[c]);
                zl[c] = fma(lor[l], zv, zl[c]);
            }
        }
#pragma unroll
        for (int c = 0; c < M; ++c) {
            a1[c] -= t1[c];
            rr[c] = -rn[c];
            d[c] = dn[c] - dl[c];
            z[c] = -zl[c];
            upc[c] = upn[c];
            lor[c] = lon[c];
            dn[c] = dnn[c];
        }
        wave_sync();
    }
    report_bad(a, bad);
    // contributions to the reduced matrix (eq. (redmatr)); separator j sits
    // between partitions j and j+1
    if (G.hasR) {
        st_row_d<M, T>(a.nD + part * MM, i, d);                    // D[sR] + alpha_2
        if (G.hasL) st_row_d<M, T>(a.nLo + (part - 1) * MM, i, z); // beta
    }
    if (G.hasL) {
        st_row_d<M, T>(a.nDadd + (part - 1) * MM, i, a1);          // alpha_1
        if (G.hasR) st_row_d<M, T>(a.nUp + (part - 1) * MM, i, rr); // gamma
    }
}

// ---------------------------------------------------------------------------
// Bidiagonal-plus-corner factor: one level.  Separators s_0 = 0 < s_1 < ... <
// s_p = nb-1; partition `part` lies between s_part and s_{part+1}.  The
// reduced matrix (eq. (redmatr1) with gamma = 0) has the same form:
// diagonal D[s_i], sub-diagonal beta, corner unchanged.
template <int M, typename T>
__device__ __forceinline__ void babd_factor_body(const LevelArgs &a, int64_t pblock)
{
    constexpr int GPW = WG / M;
    constexpr size_t MM = (size_t)M * M;
    const int tid = threadIdx.x, grp = tid / M, i = tid % M;
    constexpr int RS = M + kPad<T>, PR = 2 * M + kPad<T>;
    constexpr int GS = group_stride<T>(M * PR + M * RS);
    __shared__ __align__(16) T lds[GPW * GS];
    T *SP = lds + grp * GS;   // Gauss-Jordan pivot rows
    T *SZ = SP + M * PR;      // Z'^T, then the rows of Zh

    const int64_t part = pblock * GPW + grp;
    const Geo G = geometry<1>(a.nb, a.p, part, a.sep);
    T *E = (T *)a.E, *Zs = (T *)a.Z;

    T z[M];
    zero<M, T>(z);
    if (G.valid) ld_row_d<M, T>(z, a.Lo + (G.start - 1) * MM, i);   // A(g_1, sL)
    unsigned long long bad = ~0ull;

    // rows i of D[g] and A(g+1,g), loaded one block row ahead
    T dc[M], lc[M];
    ld_row_d<M, T>(dc, G.len > 0 ? a.D + G.start * MM : a.zero, i);
    ld_row_d<M, T>(lc, G.len > 0 ? a.Lo + G.start * MM : a.zero, i);
    for (int k = 0; k < G.len; ++k) {
        const int64_t g = G.start + k;
        const bool more = k + 1 < G.len;
        T d[M], lor[M];
#pragma unroll
        for (int l = 0; l < M; ++l) {
            d[l] = dc[l];
            lor[l] = lc[l];
        }
        ld_row_d<M, T>(dc, more ? a.D + (g + 1) * MM : a.zero, i);
        ld_row_d<M, T>(lc, more ? a.Lo + (g + 1) * MM : a.zero, i);
        T e[M];
        bool sing = false;
        const int sig = gj_rows<M, T>(d, e, i, SP, sing, (T)a.tau);
        const unsigned long long code = status_code(a.level, g);
        bad = (sing && code < bad) ? code : bad;
        st_fac<M, T>(E + g * MM + sig * M, e);
#pragma unroll
        for (int l = 0; l < M; ++l) SZ[l * RS + i] = z[l];   // column i of Z'^T
        wave_sync();
        T zh[M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            T s = T(0);
#pragma unroll
            for (int l = 0; l < M; ++l) s = fma(e[l], SZ[c * RS + l], s);
            zh[c] = s;
        }
        st_fac<M, T>(Zs + g * MM + sig * M, zh);
        wave_sync();
#pragma unroll
        for (int c = 0; c < M; ++c) SZ[sig * RS + c] = zh[c];
        wave_sync();
        T zl[M];
        zero<M, T>(zl);
#pragma unroll
        for (int l = 0; l < M; ++l)
#pragma unroll
            for (int c = 0; c < M; ++c) zl[c] = fma(lor[l], SZ[l * RS + c], zl[c]);
#pragma unroll
        for (int c = 0; c < M; ++c) z[c] = -zl[c];
        wave_sync();
    }
    report_bad(a, bad);
    if (G.valid) {
        const int64_t sR = G.start + G.len;
        st_row_d<M, T>(a.nLo + part * MM, i, z);                     // beta
        const double *ds = a.D + sR * MM + i * M;                    // copy column i
        double *od = a.nD + (part + 1) * MM + i * M;
#pragma unroll
        for (int r = 0; r < M; ++r) od[r] = ds[r];
        if (part == 0) {
#pragma unroll
            for (int r = 0; r < M; ++r) {
                a.nD[i * M + r] = a.D[i * M + r];
                a.nC[i * M + r] = a.C[i * M + r];
            }
        }
    }
}

// ---- kernels: one system (the grid covers its partitions) and batched (a
// table of per-system arguments and a work list whose entry w says: system
// table[w.x], partition block w.y, right-hand-side block w.z) -----------------
template <int M, typename T, bool ADD>
__global__ __launch_bounds__(WG) void k_btri_factor(LevelArgs a)
{
    btri_factor_body<M, T, ADD>(a, blockIdx.x);
}
template <int M, typename T, bool ADD>
__global__ __launch_bounds__(WG) void kb_btri_factor(const LevelArgs *tab, const int4 *work)
{
    const int4 w = work[blockIdx.x];
    const LevelArgs a = tab[w.x];
    btri_factor_body<M, T, ADD>(a, w.y);
}
template <int M, typename T>
__global__ __launch_bounds__(WG) void k_babd_factor(LevelArgs a)
{
    babd_factor_body<M, T>(a, blockIdx.x);
}
template <int M, typename T>
__global__ __launch_bounds__(WG) void kb_babd_factor(const LevelArgs *tab, const int4 *work)
{
    const int4 w = work[blockIdx.x];
    const LevelArgs a = tab[w.x];
    babd_factor_body<M, T>(a, w.y);
}
}  // namespace

hipError_t launch_btri_factor(int M, bool f32, const LevelArgs &a, hipStream_t s)
{
    return dispatch_M(M, [&](auto mc) {
        constexpr int MV = decltype(mc)::value;
        const dim3 grid = grid_for(MV, a.p, 1, 1);
        if (a.Dadd) {
            if (f32) launch_k((k_btri_factor<MV, float, true>), grid, dim3(WG), s, a);
            else launch_k((k_btri_factor<MV, double, true>), grid, dim3(WG), s, a);
        } else {
            if (f32) launch_k((k_btri_factor<MV, float, false>), grid, dim3(WG), s, a);
            else launch_k((k_btri_factor<MV, double, false>), grid, dim3(WG), s, a);
        }
        return hipGetLastError();
    });
}

hipError_t launch_babd_factor(int M, bool f32, const LevelArgs &a, hipStream_t s)
{
    return dispatch_M(M, [&](auto mc) {
        constexpr int MV = decltype(mc)::value;
        const dim3 grid = grid_for(MV, a.p, 1, 1);
        if (f32) launch_k((k_babd_factor<MV, float>), grid, dim3(WG), s, a);
        else launch_k((k_babd_factor<MV, double>), grid, dim3(WG), s, a);
        return hipGetLastError();
    });
}

hipError_t launch_factor_batch(int kind, int M, bool f32, bool add, const LevelArgs *tab,
                               const int4 *work, int nwg, hipStream_t s)
{
    if (nwg <= 0) return hipSuccess;
    return dispatch_M(M, [&](auto mc) {
        constexpr int MV = decltype(mc)::value;
        const dim3 grid(nwg);
        if (kind == 1) {
            if (f32) launch_k((kb_babd_factor<MV, float>), grid, dim3(WG), s, tab, work);
            else launch_k((kb_babd_factor<MV, double>), grid, dim3(WG), s, tab, work);
        } else if (add) {
            if (f32) launch_k((kb_btri_factor<MV, float, true>), grid, dim3(WG), s, tab, work);
            else launch_k((kb_btri_factor<MV, double, true>), grid, dim3(WG), s, tab, work);
        } else {
            if (f32) launch_k((kb_btri_factor<MV, float, false>), grid, dim3(WG), s, tab, work);
            else launch_k((kb_btri_factor<MV, double, false>), grid, dim3(WG), s, tab, work);
        }
        return hipGetLastError();
    });
}

}  // namespace pf
